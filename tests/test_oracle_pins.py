"""Pins of the FP64 oracle to facts the paper and the mathematics fix.

None of these re-types an oracle formula: each compares the oracle with an
independent fact -- an exact discrete identity, a closed-form spectrum, a
conservation (energy) identity, an invariance, a brute-force dense solve or a
count that follows from the geometry.  The mutation tests at the end plant
plausible mistakes in the oracle and check that some pin catches each.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from tests import _helpers as H

SHAPES = [(3, 4, 5), (5, 2, 3), (4, 4, 4)]


# --- Sec. II eq. (CP): topology --------------------------------------------

@pytest.mark.parametrize("n", SHAPES)
def test_curl_annihilates_gradients_and_divergence_annihilates_curl(n):
    """div curl = 0 and curl grad = 0 hold exactly in integers (the discrete
    de Rham identities behind C~ = C^T, Sec. II)."""
    c, g, s = O.curl(*n), O.gradient(*n), O.divergence(*n)
    assert c.dtype.kind == "i"
    assert abs(c @ g).max() == 0
    assert abs(s @ c).max() == 0
    # dual identity S~ C~ = -(C G)^T = 0 with S~ = -G^T
    assert abs((-g.T) @ c.T).max() == 0


@pytest.mark.parametrize("n", SHAPES)
def test_partial_difference_rows_have_one_plus_one_minus(n):
    """P_w has exactly one +1 and one -1 per row (Sec. II), except the last
    node along w, which has no successor (ghost row, zero)."""
    nx, ny, nz = n
    for p, m in zip(O.partials(nx, ny, nz), (nx, ny, nz)):
        p = p.tocsr()
        counts = np.diff(p.indptr)
        assert set(np.unique(counts)) <= {0, 2}
        assert (counts == 0).sum() == nx * ny * nz // m
        for r in np.nonzero(counts == 2)[0][:50]:
            assert sorted(p.data[p.indptr[r]:p.indptr[r + 1]].tolist()) == [-1, 1]


def test_curl_has_four_entries_per_facet_row():
    """Four nonzeros per row of C (Sec. III preallocation), +-1 valued."""
    c = O.curl(6, 5, 4).tocsr()
    counts = np.diff(c.indptr)
    assert counts.max() == 4
    assert set(np.unique(np.abs(c.data))) == {1}


# --- Sec. II/III: the assembled system ----------------------------------------

def _small_layered(seed=11, graded=True):
    return D.layered_device(10, 9, 8, n_layers=3, n_strips=1, n_ports=1, seed=seed,
                            graded=graded)


def test_system_has_at_most_13_entries_per_row_and_is_symmetric():
    """Sec. II: 13 nonzeros per row; Table I: the operator is (complex)
    symmetric A = A^T since the dual curl is C^T."""
    for dev in (D.cavity(6, 5, 4), _small_layered()):
        a = O.system_matrix(dev, 2 * np.pi * 7e9).tocsr()
        counts = np.diff(a.indptr)
        assert counts.max() == 13
        assert (counts == 13).sum() > 0
        assert abs(a - a.T).max() == 0.0


def test_free_edge_count_of_closed_box_matches_geometry():
    """Electric walls on all faces: x-edges survive only strictly inside the
    y and z ranges, and likewise for y and z (Sec. II boundary condition)."""
    ncx, ncy, ncz = 5, 4, 3
    f = O.free_edges(D.cavity(ncx, ncy, ncz))
    expected = (ncx * (ncy - 1) * (ncz - 1) + ncy * (ncx - 1) * (ncz - 1)
                + ncz * (ncx - 1) * (ncy - 1))
    assert f.sum() == expected


def test_pec_cell_removes_exactly_its_twelve_edges():
    dev = D.cavity(6, 6, 6)
    base = O.free_edges(dev).sum()
    dev.materials.append(D.Material(is_pec=True))
    dev.cell_mat[3, 3, 3] = 1  # an interior cell: all 12 of its edges are free before
    assert base - O.free_edges(dev).sum() == 12


def test_open_walls_keep_boundary_edges():
    """Without electric walls only the ghost edges are removed."""
    dev = D.cavity(3, 4, 5)
    dev.pec_walls = 0
    nx, ny, nz = dev.nodes
    expected = 3 * nx * ny * nz - (ny * nz + nx * nz + nx * ny)
    assert O.free_edges(dev).sum() == expected


# --- Sec. IV: cavity eigenmodes (closed forms) -------------------------------

def _discrete_cavity_spectrum(ncx, ncy, ncz, hx, hy, hz):
    """Exact FIT/Yee spectrum of a homogeneous vacuum PEC box: modes (m, n, p)
    with 0 <= m < ncx etc., at most one index zero, two polarisations when all
    three are non-zero, omega^2 = c^2 sum (2/h)^2 sin^2(m pi / (2 nc))."""
    vals = []
    for m in range(ncx):
        for n in range(ncy):
            for p in range(ncz):
                z = (m == 0) + (n == 0) + (p == 0)
                if z >= 2:
                    continue
                w2 = O.C0 ** 2 * ((2 / hx) ** 2 * np.sin(m * np.pi / (2 * ncx)) ** 2
                                  + (2 / hy) ** 2 * np.sin(n * np.pi / (2 * ncy)) ** 2
                                  + (2 / hz) ** 2 * np.sin(p * np.pi / (2 * ncz)) ** 2)
                vals += [w2] * (2 if z == 0 else 1)
    return np.sort(vals)


@pytest.mark.parametrize("dims", [((4, 3, 5), (1e-3, 1.3e-3, 0.7e-3)),
                                  ((3, 3, 3), (2e-3, 2e-3, 2e-3))])
def test_full_discrete_cavity_spectrum(dims):
    (ncx, ncy, ncz), (hx, hy, hz) = dims
    dev = D.cavity(ncx, ncy, ncz, hx, hy, hz)
    lam = O.cavity_omega2(dev)
    interior = (ncx - 1) * (ncy - 1) * (ncz - 1)
    tiny = np.abs(lam) <= 1e-9 * lam.max()
    assert tiny.sum() == interior  # gradient null space: one per interior node
    ref = _discrete_cavity_spectrum(ncx, ncy, ncz, hx, hy, hz)
    got = np.sort(lam[~tiny])
    assert got.shape == ref.shape
    np.testing.assert_allclose(got, ref, rtol=1e-10)


def _axis_indices(n, pair):
    """Mode indices of one axis with n cells for (tangential components,
    normal component, node potentials).  pair = the axis' two wall bits:
    both electric -> sines vanishing at both walls (tangential, nodes) and
    cosines (normal); both open -> cosines (tangential, nodes) and sines
    (normal), with the half dual cells at the walls; one of each ->
    quarter-wave (half-integer) indices for all three."""
    if pair == 3:
        return list(range(1, n)), list(range(0, n)), list(range(1, n))
    if pair == 0:
        return list(range(0, n + 1)), list(range(1, n + 1)), list(range(0, n + 1))
    half = [m + 0.5 for m in range(n)]
    return half, half, half


def _discrete_box_spectrum(ns, hs, walls):
    """Exact FIT spectrum of a homogeneous vacuum box with any mix of
    electric and open (magnetic) walls: the operator separates into sine and
    cosine series per axis, and an index triple mu carries
    omega^2 = c^2 sum_a (2/h_a)^2 sin^2(mu_a pi / (2 n_a)) once per field
    component whose index sets contain it, minus one gradient (node
    potential) mode.  Returns (curl eigenvalues, null-space dimension); the
    null space holds the gradients and the uniform fields that are curl-free
    but no node gradient (omega^2 = 0, e.g. E_z between two electric plates
    with open sides)."""
    rs = [_axis_indices(ns[a], (walls >> (2 * a)) & 3) for a in range(3)]
    w2 = lambda mu: O.C0 ** 2 * sum((2 / hs[a]) ** 2 * np.sin(mu[a] * np.pi / (2 * ns[a])) ** 2
                                    for a in range(3))
    comps = {}
    for w in range(3):
        sets = [rs[a][1] if a == w else rs[a][0] for a in range(3)]
        for m in sets[0]:
            for n in sets[1]:
                for p in sets[2]:
                    comps[(m, n, p)] = comps.get((m, n, p), 0) + 1
    nodes = {(m, n, p) for m in rs[0][2] for n in rs[1][2] for p in rs[2][2]}
    curl, null = [], 0
    for mu, k in comps.items():
        v = w2(mu)
        if v == 0.0:
            null += k
            continue
        g = 1 if mu in nodes else 0
        null += g
        curl += [v] * (k - g)
    return np.sort(curl), null


@pytest.mark.parametrize("walls", [0b000000, 0b110000, 0b001111, 0b010110, 0b000001, 0b100111,
                                   0b011001])
def test_discrete_spectrum_with_open_and_mixed_walls(walls):
    """Walls left open (the magnetic, natural boundary of the dual grid) and
    every mix with electric walls: the oracle's generalized eigenproblem
    K e = omega^2 M_eps e on the free edges reproduces the closed form, null
    space included."""
    ns, hs = (3, 4, 2), (1e-3, 1.3e-3, 0.7e-3)
    dev = D.cavity(*ns, *hs)
    dev.pec_walls = walls
    lam = O.cavity_omega2(dev)
    tiny = np.abs(lam) <= 1e-9 * np.abs(lam).max()
    curl, null = _discrete_box_spectrum(ns, hs, walls)
    assert tiny.sum() == null
    np.testing.assert_allclose(np.sort(lam[~tiny]), curl, rtol=1e-9)


def test_box_spectrum_closed_form_reduces_to_the_electric_box():
    """With six electric walls the general closed form is the PEC cavity
    spectrum above, null space = interior nodes."""
    ns, hs = (4, 3, 5), (1e-3, 1.3e-3, 0.7e-3)
    curl, null = _discrete_box_spectrum(ns, hs, 0x3F)
    assert null == 3 * 2 * 4
    ref = _discrete_cavity_spectrum(*ns, *hs)
    np.testing.assert_allclose(curl, ref[ref > 0], rtol=1e-12)


def test_tiny_cavity_first_resonance_matches_closed_forms():
    """16^3 cells of 1 mm: TE101/TE011/TE110 are degenerate at the discrete
    value, within O(h^2) of the continuous f = (c/2) sqrt(2)/a."""
    dev = D.cavity(16, 16, 16, 1e-3)
    f = O.cavity_eigenfrequencies(dev, k=4, sigma_f=13.0e9)
    disc = O.C0 / (2 * np.pi) * np.sqrt(2) * (2 / 1e-3) * np.sin(np.pi / 32)
    np.testing.assert_allclose(f[:3], disc, rtol=1e-9)
    cont = 0.5 * O.C0 * np.sqrt(2) / 16e-3
    assert abs(f[0] / cont - 1) < 2e-3
    assert f[3] > f[0] * 1.1


def test_homogeneous_permittivity_scales_frequencies():
    a = O.cavity_omega2(D.cavity(3, 4, 3, 1e-3, 0.9e-3, 1.2e-3))
    b = O.cavity_omega2(D.cavity(3, 4, 3, 1e-3, 0.9e-3, 1.2e-3, eps_r=4.0))
    nz = a > 1e-9 * a.max()
    np.testing.assert_allclose(np.sort(b[nz]), np.sort(a[nz]) / 4.0, rtol=1e-10)


# --- Sec. II material averaging: energy identities ----------------------------

def _open_random_device(seed=3):
    rng = np.random.default_rng(seed)
    ncx, ncy, ncz = 5, 4, 6
    mats = [D.Material(eps_r=float(rng.uniform(1, 12)), mu_r=float(rng.uniform(1, 3)),
                       sigma=float(rng.uniform(0, 5)), tan_delta=float(rng.uniform(0, 0.05)))
            for _ in range(4)]
    dev = D.Device(dx=rng.uniform(1e-4, 5e-4, ncx), dy=rng.uniform(1e-4, 5e-4, ncy),
                   dz=rng.uniform(1e-4, 5e-4, ncz),
                   cell_mat=rng.integers(0, 4, (ncz, ncy, ncx)).astype(np.uint8),
                   materials=mats, ports=[], pec_walls=0)
    return dev


def test_permittivity_energy_of_uniform_field_equals_cell_sum():
    """A uniform field E0 along w gives e = E0 * L on every w-edge; the
    electric energy e^T M_eps e must equal E0^2 sum_cells eps_cell V_cell --
    the defining property of averaging over dual facets with half cells at
    the boundary (graded, inhomogeneous, lossy)."""
    dev = _open_random_device()
    m_eps, m_sig = O.edge_materials(dev)
    nx, ny, nz = dev.nodes
    vol = dev.dz[:, None, None] * dev.dy[None, :, None] * dev.dx[None, None, :]
    mats = dev.materials
    eps_c = np.array([O.EPS0 * m.eps_r * (1 - 1j * m.tan_delta) for m in mats])[dev.cell_mat]
    sig_c = np.array([m.sigma for m in mats])[dev.cell_mat]
    lengths = [dev.dx, dev.dy, dev.dz]
    for w in range(3):
        L = np.zeros((nz, ny, nx))
        idx = [slice(None)] * 3
        ax = 2 - w
        shape = [1, 1, 1]
        shape[ax] = len(lengths[w])
        sl = [slice(None)] * 3
        sl[ax] = slice(0, len(lengths[w]))
        L[tuple(sl)] = lengths[w].reshape(shape)
        e2 = np.zeros(dev.n_edges)
        e2[w::3] = (L ** 2).ravel()
        np.testing.assert_allclose((m_eps * e2).sum(), (eps_c * vol).sum(), rtol=1e-12)
        np.testing.assert_allclose((m_sig * e2).sum(), (sig_c * vol).sum(), rtol=1e-12)


def test_reluctance_energy_of_uniform_flux_equals_cell_sum():
    """A uniform B0 along w gives b = B0 * area on every w-facet; the magnetic
    energy b^T M_nu b must equal B0^2 sum_cells V_cell / mu_cell (series
    combination along the dual edge)."""
    dev = _open_random_device()
    nu = O.facet_reluctance(dev)
    nx, ny, nz = dev.nodes
    vol = dev.dz[:, None, None] * dev.dy[None, :, None] * dev.dx[None, None, :]
    inv_mu = np.array([1 / (O.MU0 * m.mu_r) for m in dev.materials])[dev.cell_mat]
    ncx, ncy, ncz = dev.ncx, dev.ncy, dev.ncz
    for w in range(3):
        # facet area on every existing w-facet (all nodes along w)
        a = np.zeros((nz, ny, nx))
        if w == 0:
            a[:ncz, :ncy, :] = (dev.dz[:, None] * dev.dy[None, :])[:, :, None]
        elif w == 1:
            a[:ncz, :, :ncx] = (dev.dz[:, None] * dev.dx[None, :])[:, None, :]
        else:
            a[:, :ncy, :ncx] = (dev.dy[:, None] * dev.dx[None, :])[None, :, :]
        b2 = np.zeros(dev.n_edges)
        b2[w::3] = (a ** 2).ravel()
        np.testing.assert_allclose((nu * b2).sum(), (inv_mu * vol).sum(), rtol=1e-12)


def test_interface_edge_averages_two_permittivities():
    """On equal spacings an x-edge lying on the interface between eps1 (below)
    and eps2 (above) sees eps0 (eps1 + eps2)/2 over its full dual facet."""
    dev = D.cavity(4, 4, 4, 1e-3)
    dev.materials = [D.Material(eps_r=2.0), D.Material(eps_r=7.0)]
    dev.cell_mat[2:] = 1
    m_eps, _ = O.edge_materials(dev)
    e = dev.edge_index(0, 1, 2, 2)  # x-edge in plane z = 2 (interface), interior in y
    np.testing.assert_allclose(m_eps[e].real, O.EPS0 * 4.5 * 1e-3 * 1e-3 / 1e-3, rtol=1e-14)


def test_length_scaling_invariance():
    """M_eps ~ length and M_nu ~ 1/length, so A(omega/lam; lam*grid) = A/lam."""
    dev = _small_layered()
    lam = 3.7
    dev2 = D.Device(dx=dev.dx * lam, dy=dev.dy * lam, dz=dev.dz * lam, cell_mat=dev.cell_mat,
                    materials=dev.materials, ports=dev.ports, pec_walls=dev.pec_walls)
    om = 2 * np.pi * 9e9
    a1 = O.system_matrix(dev, om)
    a2 = O.system_matrix(dev2, om / lam)
    # port conductances do not scale with length; compare without ports
    dev.ports, dev2.ports = [], []
    a1 = O.system_matrix(dev, om)
    a2 = O.system_matrix(dev2, om / lam)
    diff = abs(a2 * lam - a1).max()
    assert diff <= 1e-13 * abs(a1).max()


def test_gradients_are_in_the_static_null_space_on_graded_meshes():
    """K (grad phi) = 0 for any nodal potential that vanishes on the walls
    (graded, inhomogeneous, lossy, mu_r != 1, closed electric box)."""
    dev = _open_random_device(5)
    dev.pec_walls = 0x3F
    nx, ny, nz = dev.nodes
    rng = np.random.default_rng(0)
    phi = rng.standard_normal((nz, ny, nx))
    phi[0], phi[-1], phi[:, 0], phi[:, -1], phi[:, :, 0], phi[:, :, -1] = 0, 0, 0, 0, 0, 0
    e = O.gradient(nx, ny, nz).astype(float) @ phi.ravel()
    f = O.free_edges(dev)
    e[~f] = 0.0
    k = O.stiffness(dev)
    y = (k @ e)[f]
    assert np.linalg.norm(y) <= 1e-12 * abs(k).max() * np.linalg.norm(e)


def test_sym_scaled_operator_has_unit_mass():
    """Eq. (e2t): S A S = S K S - omega^2 I, so for a lossless cavity the
    eigenvalues of S A S + omega^2 I are the cavity's omega_mnp^2."""
    dev = D.cavity(3, 3, 4, 1e-3, 1e-3, 1.5e-3)
    om = 2 * np.pi * 50e9
    a = O.system_matrix(dev, om).toarray()
    s = O.sym_scaling(dev, om)
    hat = s[:, None] * a * s[None, :] + om ** 2 * np.eye(len(s))
    lam = np.sort(np.linalg.eigvalsh(0.5 * (hat + hat.T).real))
    ref = O.cavity_omega2(dev)
    np.testing.assert_allclose(lam, np.sort(ref), rtol=1e-9, atol=1e-9 * ref.max())


# --- The paper's factorized form and its diagonal preconditioner ------------

@pytest.mark.parametrize("walls", [0x3F, 0b000000, 0b010110])
def test_paper_diagonal_preconditioner_closed_form(walls):
    """Eq. (Precond) on a homogeneous box of uniform cells: every free edge
    along axis w has P = 2 c^2 / eps_r * sum over the two other axes a of
    1/h_a^2, also at open walls (half dual cells halve both the facet
    reluctances and the edge's permittivity integral)."""
    hs = (1.0e-3, 1.3e-3, 0.7e-3)
    dev = D.cavity(4, 3, 5, *hs, eps_r=2.5)
    dev.pec_walls = walls
    om = 2 * np.pi * 7e9
    p = O.paper_diag_preconditioner(dev, om)
    w = (np.arange(dev.n_edges) % 3)[O.free_edges(dev)]
    inv2 = np.array([1 / h ** 2 for h in hs])
    ref = 2 * O.C0 ** 2 / 2.5 * (inv2.sum() - inv2[w])
    np.testing.assert_allclose(p, ref, rtol=1e-12)


def test_factorized_form_equals_the_scaled_operator():
    """Eq. (e2tt): calA^T calA - omega^2 I is S A S (eq. (e2t)); the column
    sums of calA's squares are the diagonal of S K S."""
    dev = D.layered_device(9, 8, 6, n_layers=3, n_strips=1, n_ports=1, seed=3)
    om = 2 * np.pi * 11e9
    x = (np.random.default_rng(4).uniform(-1, 1, dev.n_edges)
         + 1j * np.random.default_rng(5).uniform(-1, 1, dev.n_edges)) * O.free_edges(dev)
    y_fact = O.matvec(dev, om, x, scaling="fact")
    y_sym = O.matvec(dev, om, x, scaling="sym")
    assert np.linalg.norm(y_fact - y_sym) <= 1e-13 * np.linalg.norm(y_sym)
    f = O.free_edges(dev)
    kd = O.stiffness(dev).diagonal()[f]
    s = O.sym_scaling(dev, om)
    np.testing.assert_allclose(O.paper_diag_preconditioner(dev, om), kd * s * s, rtol=1e-13)


def test_paper_preconditioned_cocg_is_unscaled_cocg_with_inverse_curl_diagonal():
    """COCG on S A S preconditioned by 1/P produces the iterates of COCG on
    A preconditioned by S (1/P) S = 1/K_ee (x = S x_hat)."""
    dev = D.layered_device(10, 9, 8, n_layers=3, n_strips=1, n_ports=1, seed=11)
    om = 2 * np.pi * 7e9
    s = O.sym_scaling(dev, om)
    a0 = O.system_matrix(dev, om)
    b0 = O.rhs(dev, om, D.port_source(dev, 0))
    p = O.paper_diag_preconditioner(dev, om)
    xs, _, _, hs = O.cocg(sp.diags(s) @ a0 @ sp.diags(s), s * b0, tol=1e-30, maxiter=40,
                          history=True, m=1.0 / p)
    kd = O.stiffness(dev).diagonal()[O.free_edges(dev)]
    xu, _, _, hu = O.cocg(a0, b0, tol=1e-30, maxiter=40, history=True, m=1.0 / kd)
    assert np.linalg.norm(xu - s * xs) <= 1e-8 * np.linalg.norm(xu)


# --- Solves ------------------------------------------------------------------

@pytest.mark.parametrize("graded", [False, True])
def test_parallel_plate_solution_has_the_closed_form(graded):
    """Pins the magnitude, phase and frequency dependence of b = -j omega j
    and of the diagonal term: the oracle's direct solution equals the
    closed-form uniform field of a z-layered parallel-plate device."""
    dev = H.plate_device(graded)
    for f in (0.3e9, 2e9):
        om = 2 * np.pi * f
        x = O.solve_direct(dev, om, H.plate_source(dev))
        ref = H.plate_closed_form(dev, om)
        assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_direct_solve_matches_dense_brute_force():
    dev = D.layered_device(5, 4, 4, n_layers=2, n_strips=1, n_ports=1, seed=1)
    om = 2 * np.pi * 12e9
    j = D.port_source(dev, 0)
    x = O.solve_direct(dev, om, j)
    a = O.system_matrix(dev, om).toarray()
    b = O.rhs(dev, om, j)
    xd = np.linalg.solve(a, b)
    assert np.linalg.norm(x[O.free_edges(dev)] - xd) <= 1e-9 * np.linalg.norm(xd)
    assert O.relative_residual(dev, om, j, x) < 1e-12


@pytest.mark.parametrize("method", ["bicgstab", "gmres"])
def test_textbook_krylov_reaches_direct_solution(method):
    dev, om, j = D.tiny_cavity_case()
    a = O.system_matrix(dev, om)
    b = O.rhs(dev, om, j)
    ref = O.solve_direct(dev, om, j)[O.free_edges(dev)]
    if method == "bicgstab":
        x, it, rr = O.bicgstab(a, b, tol=1e-10)
    else:
        x, it, rr = O.gmres(a, b, restart=30, tol=1e-10)
    assert rr <= 1e-10
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-7


def test_flexible_gmres_with_exact_inverse_converges_in_one_step():
    dev = D.layered_device(4, 4, 3, n_layers=2, n_strips=1, n_ports=1, seed=2)
    om = 2 * np.pi * 5e9
    a = O.system_matrix(dev, om).tocsc()
    b = O.rhs(dev, om, D.port_source(dev, 0))
    import scipy.sparse.linalg as spla
    lu = spla.splu(a)
    x, it, rr = O.gmres(a, b, restart=5, tol=1e-12, precond=lu.solve)
    assert it == 1 and rr < 1e-12


def test_reciprocity_and_passivity_of_two_port():
    """Z_pq = Z_qp (complex symmetry of A) and Re Z_pp >= 0 for a lossy
    device, with Z = -u/I (u = sum of edge voltages along the port, Sec. IV;
    the minus sign because e integrates E from the ground end upward)."""
    dev = D.layered_device(12, 10, 6, n_layers=2, n_strips=2, n_ports=2, seed=4)
    assert len(dev.ports) == 2
    om = 2 * np.pi * 6e9
    z = np.zeros((2, 2), complex)
    for q in range(2):
        x = O.solve_direct(dev, om, D.port_source(dev, q))
        z[:, q] = -O.port_voltages(dev, x) / 1.0
    assert abs(z[0, 1] - z[1, 0]) <= 1e-9 * abs(z).max()
    assert z[0, 0].real >= 0 and z[1, 1].real >= 0


def test_scattering_matrix_equals_its_closed_form_in_the_loaded_impedance():
    """With Norton ports loaded by z0, S = (Z - z0)(Z + z0)^-1 computed from
    its definition (two inversions to Z, one more for S) equals
    2 zl / z0 - I: on the two-port device and on random matrices."""
    dev = D.layered_device(12, 10, 6, n_layers=2, n_strips=2, n_ports=2, seed=4)
    zl = O.loaded_impedance(dev, 2 * np.pi * 6e9)
    rng = np.random.default_rng(3)
    for m in [zl] + [rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n)) for n in (1, 3, 5)]:
        _, s = O.port_network(m, 50.0)
        np.testing.assert_allclose(s, 2 * m / 50.0 - np.eye(m.shape[0]), rtol=0, atol=1e-10 * max(1, abs(s).max()))


@pytest.mark.parametrize("z, s_ref", [(50.0, 0.0), (150.0, 0.5), (50.0 / 3, -0.5), (50j, 1j)])
def test_one_port_network_round_trip_and_reflection(z, s_ref):
    """A one-port of impedance z loaded by z0 = 50 Ohm shows zl = z || z0;
    the oracle recovers z, and S = (z - z0)/(z + z0) (0 matched, +-1/2,
    a pure reactance j z0 reflects with S = j)."""
    zl = np.array([[1.0 / (1.0 / z + 1.0 / 50.0)]], dtype=np.complex128)
    zz, s = O.port_network(zl, 50.0)
    np.testing.assert_allclose(zz[0, 0], z, rtol=1e-12)
    np.testing.assert_allclose(s[0, 0], s_ref, atol=1e-12)


def test_two_port_network_is_reciprocal_and_passive():
    """Z and S of the lossy two-port are symmetric (complex symmetry of A)
    and S is contractive (no singular value above 1: the device absorbs)."""
    dev = D.layered_device(12, 10, 6, n_layers=2, n_strips=2, n_ports=2, seed=4)
    z, s = O.port_network(O.loaded_impedance(dev, 2 * np.pi * 6e9), 50.0)
    assert abs(z[0, 1] - z[1, 0]) <= 1e-8 * abs(z).max()
    assert abs(s[0, 1] - s[1, 0]) <= 1e-9
    assert np.linalg.svd(s, compute_uv=False).max() <= 1.0 + 1e-12


def test_tiny_cavity_case_bicgstab_reaches_1e8():
    dev, om, j = D.tiny_cavity_case()
    a = O.system_matrix(dev, om)
    b = O.rhs(dev, om, j)
    assert a.shape[0] == 10800 and dev.n_edges == 14739
    x, it, rr = O.bicgstab(a, b, tol=1e-8)
    assert rr <= 1e-8 and it < 200


def test_splitmix64_matches_published_sequence():
    """SplitMix64 from state 0 yields 0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
    0x06C45D188009454F (the published reference outputs)."""
    out = O.splitmix64(np.arange(3, dtype=np.uint64), 0)
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    v = O.shadow_vector(1000)
    assert np.all(np.abs(v.real) <= 1) and np.all(np.abs(v.imag) <= 1)
    assert abs(v.real.mean()) < 0.1 and abs(np.var(v.imag) - 1 / 3) < 0.05


def test_textbook_bicgstab_with_dense_shadow_vector():
    dev = D.layered_device(10, 9, 8, n_layers=3, n_strips=1, n_ports=1, seed=11)
    om = 2 * np.pi * 7e9
    s = O.sym_scaling(dev, om)
    a = sp.diags(s) @ O.system_matrix(dev, om) @ sp.diags(s)
    b = s * O.rhs(dev, om, D.port_source(dev, 0))
    rh = O.shadow_vector(dev.n_edges)[O.free_edges(dev)]
    x, it, rr = O.bicgstab(a, b, tol=1e-10, rhat=rh)
    assert rr <= 1e-10
    xc, itc, rrc = O.cocg(a, b, tol=1e-10)
    assert rrc <= 3e-10  # recursive residual stops at 1e-10; true one within a small gap
    assert np.linalg.norm(xc - x) <= 1e-6 * np.linalg.norm(x)
    # COCG on S A S equals COCG on A preconditioned by S^2 (x = S x_hat)
    a0 = O.system_matrix(dev, om)
    b0 = O.rhs(dev, om, D.port_source(dev, 0))
    _, _, _, h_scaled = O.cocg(a, b, tol=1e-30, maxiter=40, history=True)
    xp, _, _, h_pre = O.cocg(a0, b0, tol=1e-30, maxiter=40, history=True, m=s * s)
    xh, _, _ = O.cocg(a, b, tol=1e-30, maxiter=40)
    assert np.linalg.norm(xp - s * xh) <= 1e-8 * np.linalg.norm(xp)


# --- Mutation tests: plant mistakes in the oracle, the pins must notice ------

def _run_pins():
    fails = []
    for name, fn in [
        ("spectrum", lambda: test_full_discrete_cavity_spectrum(((4, 3, 5), (1e-3, 1.3e-3, 0.7e-3)))),
        ("topology", lambda: test_curl_annihilates_gradients_and_divergence_annihilates_curl((3, 4, 5))),
        ("eps_energy", test_permittivity_energy_of_uniform_field_equals_cell_sum),
        ("nu_energy", test_reluctance_energy_of_uniform_flux_equals_cell_sum),
        ("count", test_free_edge_count_of_closed_box_matches_geometry),
        ("pec12", test_pec_cell_removes_exactly_its_twelve_edges),
        ("passive", test_reciprocity_and_passivity_of_two_port),
        ("open_walls", lambda: test_discrete_spectrum_with_open_and_mixed_walls(0b010110)),
        ("plate", lambda: test_parallel_plate_solution_has_the_closed_form(True)),
    ]:
        try:
            fn()
        except (AssertionError, np.linalg.LinAlgError):  # a pin that no longer holds
            fails.append(name)
    return fails


def test_mutation_wrong_curl_sign_is_caught(monkeypatch):
    real = O.curl

    def bad(nx, ny, nz):
        px, py, pz = O.partials(nx, ny, nz)
        blk = sp.bmat([[None, pz, py], [pz, None, -px], [-py, px, None]], format="csr")
        q = O.interleave(nx * ny * nz)
        return (q @ blk @ q.T).tocsr()

    monkeypatch.setattr(O, "curl", bad)
    assert _run_pins()
    monkeypatch.setattr(O, "curl", real)


def test_mutation_dropped_averaging_term_is_caught(monkeypatch):
    real = O._sum_pairs

    def bad(w, axes):
        for ax in axes[:1]:  # forgets the second axis of the dual-facet sum
            w = real(w, (ax,))
        if len(axes) > 1:
            pad = [(0, 0)] * w.ndim
            pad[axes[1]] = (0, 1)
            w = np.pad(w, pad)
        return w

    monkeypatch.setattr(O, "_sum_pairs", bad)
    assert _run_pins()


def test_mutation_mask_ignoring_pec_cells_is_caught(monkeypatch):
    real = O._cell_props

    def bad(dev):
        eps_c, sigma, inv_mu, pec = real(dev)
        return eps_c, sigma, inv_mu, np.zeros_like(pec)

    monkeypatch.setattr(O, "_cell_props", bad)
    assert "pec12" in _run_pins()


def test_mutation_wrong_loss_sign_is_caught(monkeypatch):
    real = O.diagonal

    def bad(dev, omega):
        m_eps, m_sig = O.edge_materials(dev)
        return -omega * omega * np.conj(m_eps) - 1j * omega * m_sig

    monkeypatch.setattr(O, "diagonal", bad)
    assert "passive" in _run_pins()


def test_mutation_half_cell_at_boundary_is_caught(monkeypatch):
    real = O.facet_reluctance

    def bad(dev):
        nu = real(dev)
        return nu * 1.0000001  # tiny global scale error of the reluctances
    monkeypatch.setattr(O, "facet_reluctance", bad)
    assert {"spectrum", "nu_energy"} <= set(_run_pins())


def test_mutation_full_dual_cells_at_walls_is_caught(monkeypatch):
    """Cells outside the grid taking the boundary cell's value gives the wall
    edges whole dual facets instead of halves; with electric walls those
    edges are masked, so only the open-wall spectrum can notice."""
    def bad(w, axes):
        for ax in axes:
            pad = [(0, 0)] * w.ndim
            pad[ax] = (1, 1)
            wp = np.pad(w, pad, mode="edge")
            lo = [slice(None)] * w.ndim
            hi = [slice(None)] * w.ndim
            lo[ax] = slice(0, -1)
            hi[ax] = slice(1, None)
            w = wp[tuple(lo)] + wp[tuple(hi)]
        return w

    monkeypatch.setattr(O, "_sum_pairs", bad)
    assert "open_walls" in _run_pins()


def test_mutation_rhs_without_omega_is_caught(monkeypatch):
    """b = -j j (a dropped factor omega) leaves every invariant pin intact;
    only the parallel-plate closed form sees it."""
    def bad(dev, omega, jsrc):
        return (-1j * jsrc)[O.free_edges(dev)]

    monkeypatch.setattr(O, "rhs", bad)
    assert _run_pins() == ["plate"]


def test_mutation_rhs_sign_is_caught(monkeypatch):
    def bad(dev, omega, jsrc):
        return (1j * omega * jsrc)[O.free_edges(dev)]

    monkeypatch.setattr(O, "rhs", bad)
    assert "plate" in _run_pins()


def _paper_edge_counts():
    rows = []
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_edge_counts.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        *_, nx, ny, nz, ne = line.split()
        rows.append((int(nx), int(ny), int(nz), int(ne)))
    return rows


def test_edge_count_reading_matches_the_paper():
    """n_e printed in Sec. IV equals 3 Nx Ny Nz with N counted in nodes; for
    the meshes small enough to assemble, the oracle's curl has exactly that
    many rows and columns, and a device of N-1 cells per axis reports it."""
    rows = _paper_edge_counts()
    assert len(rows) == 4
    for nx, ny, nz, ne in rows:
        assert 3 * nx * ny * nz == ne
        if ne < 1_000_000:
            c = O.curl(nx, ny, nz)
            assert c.shape == (ne, ne)
            dev = D.cavity(nx - 1, ny - 1, nz - 1)
            assert dev.n_edges == ne


def test_mutation_scaled_curl_without_square_root_is_caught(monkeypatch):
    """calA built with M_nu instead of M_nu^{1/2}: only the closed form of
    eq. (Precond) notices."""
    def bad(dev, omega):
        nx, ny, nz = dev.nodes
        f = O.free_edges(dev)
        c = O.curl(nx, ny, nz).astype(np.float64).tocsc()[:, f]
        return (sp.diags(O.facet_reluctance(dev)) @ c @ sp.diags(O.sym_scaling(dev, omega))).tocsr()

    monkeypatch.setattr(O, "scaled_curl", bad)
    with pytest.raises(AssertionError):
        test_paper_diagonal_preconditioner_closed_form(0x3F)


@pytest.mark.parametrize("method", ["cocr", "tfqmr", "cgs"])
def test_cocr_and_tfqmr_reach_the_direct_solution(method):
    """The further methods of the paper's solver comparison (Sec. IV: CR in
    complex symmetric form, TFQMR and CGS) on a small lossy graded device,
    scaled as in eq. (e2t): the iterate reaches the sparse direct solution."""
    dev = D.layered_device(9, 8, 7, n_layers=3, n_strips=1, n_ports=1, seed=13)
    om = 2 * np.pi * 9e9
    s = O.sym_scaling(dev, om)
    a = (sp.diags(s) @ O.system_matrix(dev, om) @ sp.diags(s)).tocsr()
    src = D.port_source(dev, 0)
    b = s * O.rhs(dev, om, src)
    rhat = O.shadow_vector(dev.n_edges)[O.free_edges(dev)]
    if method == "cocr":
        x, it, rr = O.cocr(a, b, tol=1e-11)
    elif method == "tfqmr":
        x, it, rr = O.tfqmr(a, b, rhat, tol=1e-11)
    else:
        x, it, rr = O.cgs(a, b, rhat, tol=1e-11)
    ref = O.solve_direct(dev, om, src)[O.free_edges(dev)]
    assert rr <= 1e-9
    assert np.linalg.norm(s * x - ref) <= 1e-6 * np.linalg.norm(ref)


def test_cocr_minimises_the_residual_on_a_hermitian_positive_system():
    """On a real symmetric positive definite matrix COCR is CR, which
    minimises ||b - A x|| over the Krylov space: its residual norms never
    increase and, after k steps, do not exceed GMRES(k)'s by more than
    rounding."""
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    a = (q * np.linspace(1, 50, 60)) @ q.T
    b = rng.standard_normal(60).astype(np.complex128)
    _, _, _, h = O.cocr(sp.csr_matrix(a.astype(np.complex128)), b, tol=1e-14, maxiter=25,
                        history=True)
    assert np.all(np.diff(h) <= 1e-12)
    for k in (5, 10, 20):
        _, _, rg = O.gmres(sp.csr_matrix(a.astype(np.complex128)), b, restart=k, tol=1e-16, maxiter=k)
        assert h[k - 1] <= rg * (1 + 1e-8)


def test_cgs_residual_is_the_squared_bicg_polynomial():
    """CGS applies the BiCG residual polynomial twice: on a real symmetric
    positive definite matrix with the shadow vector r0 (where BiCG is CG),
    ||r_k^CGS|| = ||phi_k(A)^2 r0|| with phi_k from CG's own recurrence."""
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.linspace(1, 9, 40)
    a = (q * lam) @ q.T
    b = rng.standard_normal(40).astype(np.complex128)
    am = sp.csr_matrix(a.astype(np.complex128))
    _, _, _, h = O.cgs(am, b, b.copy(), tol=1e-30, maxiter=6, history=True)
    # CG's residual polynomial through the Lanczos recurrence, as a matrix
    r = b.copy(); p = r.copy(); rr = np.vdot(r, r)
    phis = []
    poly_r = np.eye(40); poly_p = np.eye(40)
    for k in range(6):
        ap = a @ p
        alpha = rr / np.vdot(p, ap)
        poly_r_new = poly_r - alpha * (a @ poly_p)
        r = r - alpha * ap
        rr_new = np.vdot(r, r)
        beta = rr_new / rr
        poly_p = poly_r_new + beta * poly_p
        p = r + beta * p
        poly_r, rr = poly_r_new, rr_new
        phis.append(np.linalg.norm(poly_r @ poly_r @ b) / np.linalg.norm(b))
    np.testing.assert_allclose(h, phis, rtol=1e-8)


def test_graded_mesh_conditioning_rules_out_complex64_inner_solves():
    """Why complex64 inner iterations stall on the graded meshes (the
    precision form's evidence, Sec. III's scaled operator of eq. (e2t)): the
    largest eigenvalue of S K S (S = M_eps^{-1/2}) relative to the shift
    omega^2 bounds the condition number of S A S from below (its gradient
    cluster sits at -omega^2).  At 1 GHz it exceeds 1/u32 on the graded
    10-200 um mesh and stays two orders below it on a uniform 100 um mesh;
    the ratio scales as omega^-2."""
    import scipy.sparse.linalg as spla
    u32 = 2.0 ** -24
    ratio = {}
    for graded in (True, False):
        dev = D.layered_device(24, 24, 16, n_layers=4, n_strips=3, n_ports=1, seed=2, graded=graded)
        f = O.free_edges(dev)
        k = O.stiffness(dev)[f][:, f]
        m_eps, _ = O.edge_materials(dev)
        s = 1.0 / np.sqrt(m_eps[f].real)
        sks = (sp.diags(s) @ k @ sp.diags(s)).tocsr()
        lmax = spla.eigsh(sks, k=1, which="LA", return_eigenvectors=False)[0]
        ratio[graded] = lmax / (2 * np.pi * 1e9) ** 2
    assert ratio[True] * u32 > 1.0
    assert ratio[False] * u32 < 0.1
    assert ratio[True] > 50 * ratio[False]
