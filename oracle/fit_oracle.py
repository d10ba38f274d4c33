"""FP64 CPU oracle for the frequency-domain FIT operator and its solvers.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library and must never be used as a fallback by the product path.

What it computes, and where the paper defines it (Geranmayeh, "Parallel
Matrix-Free Implementation of Frequency-Domain Finite Difference Methods for
Cluster Computing"):

* Sec. II, eq. (CP): the primal curl ``C`` built from the partial-difference
  blocks ``P_x, P_y, P_z`` (two entries +1/-1 per row), with the dual curl
  equal to ``C^T``;
* Sec. II, eq. (Material) and the averaging rule that follows it: diagonal
  ``M_eps`` (permittivity averaged over the dual facet of each primal edge,
  complex for lossy dielectrics) and ``M_nu = M_mu^{-1}`` (permeability
  combined along the dual edge through each primal facet);
* Sec. II, eq. (e2) with ``s = j*omega``: the curl-curl system
  ``(C^T M_nu C - omega^2 M_eps + j omega M_sigma) e = -j omega j``;
* Sec. II, the electric (PEC) boundary condition: tangential electric
  voltages vanish on electric walls and on perfectly conducting cells;
* Sec. II/III, eqs. (e2s)/(e2t): the symmetric scaling by ``M_eps^{-1/2}``;
* Sec. IV: probe voltages are sums of edge voltages along the port segments.

The assembled matrix is deliberately the "explicit A" of Sec. III (13 entries
per row); nothing here is blocked, fused or reordered beyond those
definitions.  Readings where the paper is silent (sign convention, ghost
edges, averaging, port loading, stop criterion) are listed in the project's
design notes and restated next to the code that takes them.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# SI constants.  mu0 uses the classical defined value 4*pi*1e-7 H/m.
MU0 = 4.0e-7 * np.pi
C0 = 299_792_458.0
EPS0 = 1.0 / (MU0 * C0 * C0)

WALL_XM, WALL_XP, WALL_YM, WALL_YP, WALL_ZM, WALL_ZP = (1 << b for b in range(6))


# ---------------------------------------------------------------------------
# O1  Topology: partial differences and the primal curl (Sec. II, eq. (CP)).
# ---------------------------------------------------------------------------

def diff_1d(n: int) -> sp.csr_matrix:
    """``D_n``: ``(D f)_i = f_{i+1} - f_i`` for ``i < n-1``; the last row is zero
    (reading: a node with no successor has no outgoing primal edge)."""
    rows = np.repeat(np.arange(n - 1), 2)
    cols = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1).ravel()
    vals = np.tile([-1, 1], n - 1)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n), dtype=np.int64)


def partials(nx: int, ny: int, nz: int):
    """``P_x, P_y, P_z`` on the node lattice, node ``n = i + nx*(j + ny*k)``."""
    ix, iy, iz = (sp.identity(m, dtype=np.int64, format="csr") for m in (nx, ny, nz))
    px = sp.kron(iz, sp.kron(iy, diff_1d(nx)), format="csr")
    py = sp.kron(iz, sp.kron(diff_1d(ny), ix), format="csr")
    pz = sp.kron(diff_1d(nz), sp.kron(iy, ix), format="csr")
    return px, py, pz


def interleave(np_: int) -> sp.csr_matrix:
    """Permutation from component-block order ``(w*Np + n)`` to the paper's
    cell-by-cell order ``(3*n + w)`` (Sec. II, eq. (e12Nxyz))."""
    n = np.arange(np_)
    rows = np.concatenate([3 * n + w for w in range(3)])
    cols = np.concatenate([w * np_ + n for w in range(3)])
    return sp.csr_matrix((np.ones(3 * np_, dtype=np.int64), (rows, cols)),
                         shape=(3 * np_, 3 * np_))


def curl(nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """Primal curl of eq. (CP), rows and columns in interleaved order."""
    px, py, pz = partials(nx, ny, nz)
    z = None
    blk = sp.bmat([[z, -pz, py], [pz, z, -px], [-py, px, z]], format="csr")
    q = interleave(nx * ny * nz)
    return (q @ blk @ q.T).tocsr()


def gradient(nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """Primal gradient ``[P_x; P_y; P_z]`` (nodes -> edges), interleaved rows."""
    px, py, pz = partials(nx, ny, nz)
    q = interleave(nx * ny * nz)
    return (q @ sp.vstack([px, py, pz], format="csr")).tocsr()


def divergence(nx: int, ny: int, nz: int) -> sp.csr_matrix:
    """Primal-facet divergence ``[P_x, P_y, P_z]`` (facets -> cells)."""
    px, py, pz = partials(nx, ny, nz)
    q = interleave(nx * ny * nz)
    return (sp.hstack([px, py, pz], format="csr") @ q.T).tocsr()


# ---------------------------------------------------------------------------
# O2/O3  Material matrices (Sec. II, eq. (Material) and the averaging rule).
# ---------------------------------------------------------------------------

def _cell_props(dev):
    mats = dev.materials
    eps_r = np.array([m.eps_r for m in mats], np.float64)[dev.cell_mat]
    tand = np.array([m.tan_delta for m in mats], np.float64)[dev.cell_mat]
    sigma = np.array([m.sigma for m in mats], np.float64)[dev.cell_mat]
    mu_r = np.array([m.mu_r for m in mats], np.float64)[dev.cell_mat]
    pec = np.array([bool(m.is_pec) for m in mats])[dev.cell_mat]
    # complex permittivity eps0*eps_r*(1 - j tan(delta)) for e^{+j omega t}
    eps_c = EPS0 * eps_r * (1.0 - 1j * tand)
    return eps_c, sigma, 1.0 / (MU0 * mu_r), pec


def _sum_pairs(w: np.ndarray, axes) -> np.ndarray:
    """For each node index ``n`` along each listed cell axis, add the cell
    values at ``n-1`` and ``n`` that lie inside the grid.  A cell axis of
    length ``m`` becomes a node axis of length ``m + 1``."""
    for ax in axes:
        pad = [(0, 0)] * w.ndim
        pad[ax] = (1, 1)
        wp = np.pad(w, pad)  # zero outside the grid
        lo = [slice(None)] * w.ndim
        hi = [slice(None)] * w.ndim
        lo[ax] = slice(0, -1)
        hi[ax] = slice(1, None)
        w = wp[tuple(lo)] + wp[tuple(hi)]
    return w


def _to_nodes(arr: np.ndarray, shape) -> np.ndarray:
    """Place an array defined on a sub-box at the start of a node array."""
    out = np.zeros(shape, dtype=arr.dtype)
    out[: arr.shape[0], : arr.shape[1], : arr.shape[2]] = arr
    return out


def edge_materials(dev):
    """``M_eps`` (complex) and ``M_sigma`` (real, ports included) per primal
    edge, interleaved order.  Each is the material coefficient integrated over
    the dual facet of the edge (quarters of the up-to-4 adjacent cells) and
    divided by the edge length: ``M = (1/L_n) * sum_cells coef * (quarter area)``."""
    eps_c, sigma, _, _ = _cell_props(dev)
    dx, dy, dz = dev.dx, dev.dy, dev.dz
    nx, ny, nz = dev.nodes
    shape = (nz, ny, nx)
    # weights of each cell's quarter of the dual facet, arrays indexed [c, b, a]
    q_yz = (dz[:, None, None] / 2) * (dy[None, :, None] / 2) * np.ones_like(sigma)
    q_xz = (dz[:, None, None] / 2) * (dx[None, None, :] / 2) * np.ones_like(sigma)
    q_xy = (dy[None, :, None] / 2) * (dx[None, None, :] / 2) * np.ones_like(sigma)
    out = []
    for coef in (eps_c, sigma.astype(np.complex128)):
        # x-edges (i < ncx): cells (i, j-1..j, k-1..k); sum over b and c
        mx = _sum_pairs(coef * q_yz, axes=(0, 1)) / dx[None, None, :]
        # y-edges (j < ncy): cells (i-1..i, j, k-1..k); sum over a and c
        my = _sum_pairs(coef * q_xz, axes=(0, 2)) / dy[None, :, None]
        # z-edges (k < ncz): cells (i-1..i, j-1..j, k); sum over a and b
        mz = _sum_pairs(coef * q_xy, axes=(1, 2)) / dz[:, None, None]
        m = np.stack([_to_nodes(mx, shape), _to_nodes(my, shape), _to_nodes(mz, shape)],
                     axis=-1).ravel()
        out.append(m)
    m_eps, m_sig = out[0], out[1].real.copy()
    # Lumped ports: a port of k edges in series with total internal impedance
    # z0 puts a conductance k/z0 on each of its edges.
    for p in range(len(dev.ports)):
        e = dev.port_edges(p)
        m_sig[e] += len(e) / dev.ports[p].z0
    return m_eps, m_sig


def facet_reluctance(dev):
    """``M_nu = M_mu^{-1}`` per primal facet, interleaved order: the dual-edge
    integral of ``1/mu`` (halves of the up-to-2 adjacent cells) divided by the
    facet area.  Facets outside the grid (ghost facets) get 0."""
    _, _, inv_mu, _ = _cell_props(dev)
    dx, dy, dz = dev.dx, dev.dy, dev.dz
    nx, ny, nz = dev.nodes
    shape = (nz, ny, nx)
    # x-facets (j < ncy, k < ncz): cells (i-1..i, j, k)
    fx = _sum_pairs(inv_mu * (dx[None, None, :] / 2), axes=(2,)) \
        / (dy[None, :, None] * dz[:, None, None])
    # y-facets (i < ncx, k < ncz): cells (i, j-1..j, k)
    fy = _sum_pairs(inv_mu * (dy[None, :, None] / 2), axes=(1,)) \
        / (dx[None, None, :] * dz[:, None, None])
    # z-facets (i < ncx, j < ncy): cells (i, j, k-1..k)
    fz = _sum_pairs(inv_mu * (dz[:, None, None] / 2), axes=(0,)) \
        / (dx[None, None, :] * dy[None, :, None])
    return np.stack([_to_nodes(fx, shape), _to_nodes(fy, shape), _to_nodes(fz, shape)],
                    axis=-1).ravel()


# ---------------------------------------------------------------------------
# O4  Boundary condition (Sec. II): which edges carry unknowns.
# ---------------------------------------------------------------------------

def free_edges(dev) -> np.ndarray:
    """Boolean per edge: it exists, is not tangential to an electric wall and
    touches no PEC cell."""
    _, _, _, pec = _cell_props(dev)
    nx, ny, nz = dev.nodes
    ncx, ncy, ncz = dev.ncx, dev.ncy, dev.ncz
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    w = dev.pec_walls

    def on_wall(idx, n_cells, bit_lo, bit_hi):
        return ((idx == 0) & bool(w & bit_lo)) | ((idx == n_cells) & bool(w & bit_hi))

    wall_x = on_wall(i, ncx, WALL_XM, WALL_XP)
    wall_y = on_wall(j, ncy, WALL_YM, WALL_YP)
    wall_z = on_wall(k, ncz, WALL_ZM, WALL_ZP)
    pec_f = pec.astype(np.int64)
    shape = (nz, ny, nx)
    touch_x = _to_nodes(_sum_pairs(pec_f, axes=(0, 1)), shape) > 0
    touch_y = _to_nodes(_sum_pairs(pec_f, axes=(0, 2)), shape) > 0
    touch_z = _to_nodes(_sum_pairs(pec_f, axes=(1, 2)), shape) > 0
    fx = (i < ncx) & ~wall_y & ~wall_z & ~touch_x
    fy = (j < ncy) & ~wall_x & ~wall_z & ~touch_y
    fz = (k < ncz) & ~wall_x & ~wall_y & ~touch_z
    return np.stack([fx, fy, fz], axis=-1).ravel()


# ---------------------------------------------------------------------------
# O5  The system of eq. (e2) with s = j*omega, restricted to free edges.
# ---------------------------------------------------------------------------

def stiffness(dev) -> sp.csr_matrix:
    """``K = C^T diag(M_nu) C`` on all edges (ghost rows included)."""
    nx, ny, nz = dev.nodes
    c = curl(nx, ny, nz).astype(np.float64)
    return (c.T @ sp.diags(facet_reluctance(dev)) @ c).tocsr()


def diagonal(dev, omega: float) -> np.ndarray:
    """``d = -omega^2 M_eps + j omega M_sigma`` per edge."""
    m_eps, m_sig = edge_materials(dev)
    return -omega * omega * m_eps + 1j * omega * m_sig


def system_matrix(dev, omega: float) -> sp.csr_matrix:
    """``A(omega)`` restricted to free edges (rows and columns)."""
    f = free_edges(dev)
    a = (stiffness(dev) + sp.diags(diagonal(dev, omega))).tocsr()
    return a[f][:, f].tocsr()


def rhs(dev, omega: float, jsrc: np.ndarray) -> np.ndarray:
    """``b = -j omega j`` on free edges (eq. (e2), s = j*omega)."""
    return (-1j * omega * jsrc)[free_edges(dev)]


def sym_scaling(dev, omega: float) -> np.ndarray:
    """``diag(M_eps,c^{-1/2})`` on free edges with ``M_eps,c = M_eps - j M_sigma/omega``
    (principal square root), the scaling of eqs. (e2s)/(e2t)."""
    f = free_edges(dev)
    m_eps, m_sig = edge_materials(dev)
    return 1.0 / np.sqrt((m_eps - 1j * m_sig / omega)[f])


def scaled_curl(dev, omega: float) -> sp.csr_matrix:
    """``calA = M_mu^{-1/2} C M_eps,c^{-1/2}`` of Sec. III (the factor before
    eq. (e2tt)): rows are primal facets, columns the free edges; the
    reluctance enters as its square root, the permittivity as the symmetric
    scaling of :func:`sym_scaling`."""
    nx, ny, nz = dev.nodes
    f = free_edges(dev)
    c = curl(nx, ny, nz).astype(np.float64).tocsc()[:, f]
    return (sp.diags(np.sqrt(facet_reluctance(dev))) @ c @ sp.diags(sym_scaling(dev, omega))).tocsr()


def paper_diag_preconditioner(dev, omega: float) -> np.ndarray:
    """Eq. (Precond): ``P_ii = sum_k [calA]_ki^2``, the column sums of the
    squared (unconjugated) entries of ``calA``, on the free edges.  The
    preconditioner of the scaled system is ``1/P``."""
    a = scaled_curl(dev, omega)
    return np.asarray(a.multiply(a).sum(axis=0)).ravel()


def matvec(dev, omega: float, x: np.ndarray, scaling: str = "none") -> np.ndarray:
    """``y = A(omega) x`` on all edges: free-edge rows of the assembled
    matrix applied to the free-edge part of ``x``; ``y`` is zero elsewhere.
    ``scaling='sym'`` applies ``S A S`` instead (eq. (e2t)); ``scaling='fact'``
    applies the factorized form of eq. (e2tt), ``calA^T (calA x) - omega^2 x``."""
    f = free_edges(dev)
    xf = np.asarray(x, np.complex128)[f]
    if scaling == "fact":
        a = scaled_curl(dev, omega)
        yf = a.T @ (a @ xf) - omega * omega * xf
        y = np.zeros(dev.n_edges, np.complex128)
        y[f] = yf
        return y
    a = system_matrix(dev, omega)
    if scaling == "sym":
        s = sym_scaling(dev, omega)
        yf = s * (a @ (s * xf))
    else:
        yf = a @ xf
    y = np.zeros(dev.n_edges, np.complex128)
    y[f] = yf
    return y


def embed(dev, xf: np.ndarray) -> np.ndarray:
    x = np.zeros(dev.n_edges, np.complex128)
    x[free_edges(dev)] = xf
    return x


# ---------------------------------------------------------------------------
# O6/O7  Outputs and reference solutions.
# ---------------------------------------------------------------------------

def port_voltages(dev, x: np.ndarray) -> np.ndarray:
    """Probe rule of Sec. IV: the sum of edge voltages along each port."""
    return np.array([x[dev.port_edges(p)].sum() for p in range(len(dev.ports))],
                    dtype=np.complex128)


def loaded_impedance(dev, omega: float) -> np.ndarray:
    """Loaded port impedance matrix: column q is ``-u`` (port voltages,
    Sec. IV probe rule) of the direct solve driven by a unit current at
    port q, every port loaded by its internal impedance (reading of the
    lumped port as a Norton source)."""
    n = len(dev.ports)
    zl = np.zeros((n, n), dtype=np.complex128)
    for q in range(n):
        jsrc = np.zeros(dev.n_edges)
        jsrc[dev.port_edges(q)] = 1.0
        zl[:, q] = -port_voltages(dev, solve_direct(dev, omega, jsrc))
    return zl


def port_network(zl: np.ndarray, z0: float):
    """Network parameters from the loaded impedance matrix, by their
    definitions: the ports' own admittance is the loaded one minus the
    loads, ``Y = zl^-1 - I/z0``, ``Z = Y^-1``, and the scattering matrix for
    reference impedance z0 is ``S = (Z - z0 I)(Z + z0 I)^-1``.  Returns
    ``(Z, S)``."""
    n = zl.shape[0]
    eye = np.eye(n)
    y = np.linalg.inv(zl) - eye / z0
    z = np.linalg.inv(y)
    s = (z - z0 * eye) @ np.linalg.inv(z + z0 * eye)
    return z, s


def solve_direct(dev, omega: float, jsrc: np.ndarray) -> np.ndarray:
    """Sparse direct solve of ``A x = b``; returns ``x`` on all edges."""
    a = system_matrix(dev, omega).tocsc()
    b = rhs(dev, omega, jsrc)
    return embed(dev, spla.spsolve(a, b))


def relative_residual(dev, omega: float, jsrc: np.ndarray, x: np.ndarray) -> float:
    """``||b - A x||_2 / ||b||_2`` on free edges, unscaled FP64 system."""
    a = system_matrix(dev, omega)
    b = rhs(dev, omega, jsrc)
    xf = np.asarray(x, np.complex128)[free_edges(dev)]
    return float(np.linalg.norm(b - a @ xf) / np.linalg.norm(b))


# ---------------------------------------------------------------------------
# Textbook Krylov methods (the paper's KSP choices, Sec. IV), plain NumPy.
# ---------------------------------------------------------------------------

SPLITMIX_GAMMA = 0x9E3779B97F4A7C15


def splitmix64(counter: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 (Steele, Lea & Flood 2014) evaluated at ``seed + (counter+1)
    * gamma``: a counter-based generator, one 64-bit output per counter."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * np.uint64(SPLITMIX_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def shadow_vector(n_edges: int, seed: int = 0x5EED) -> np.ndarray:
    """Dense pseudo-random BiCGStab shadow vector over all edge indices:
    re, im uniform in [-1, 1) from counters 2e and 2e+1 (top 53 bits)."""
    e = np.arange(n_edges, dtype=np.uint64)
    u = (splitmix64(2 * e, seed) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    v = (splitmix64(2 * e + np.uint64(1), seed) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return (2.0 * u - 1.0) + 1j * (2.0 * v - 1.0)


def bicgstab(a, b, tol=1e-8, maxiter=100000, x0=None, rhat=None):
    """Complex BiCGStab (van der Vorst, 1992) with conjugated inner products;
    the shadow vector is ``r_hat = r_0`` unless ``rhat`` is given (any vector
    with <r_hat, r_0> != 0 is admissible).  Stops when the recursively
    updated residual satisfies ``||r|| <= tol ||b||`` and the true residual
    agrees, restarting from the current iterate otherwise.  Returns
    ``(x, iterations, relres)``."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    it = 0
    while it < maxiter:
        r = b - a @ x
        if np.linalg.norm(r) <= tol * nb:
            break
        rh = r.copy() if rhat is None else np.asarray(rhat, np.complex128).copy()
        rho_old = alpha = omg = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while it < maxiter:
            it += 1
            rho = np.vdot(rh, r)
            if rho == 0:
                break
            beta = (rho / rho_old) * (alpha / omg)
            p = r + beta * (p - omg * v)
            v = a @ p
            alpha = rho / np.vdot(rh, v)
            s = r - alpha * v
            t = a @ s
            tt = np.vdot(t, t)
            omg = np.vdot(t, s) / tt if tt != 0 else 0.0
            x = x + alpha * p + omg * s
            r = s - omg * t
            rho_old = rho
            if np.linalg.norm(r) <= tol * nb or omg == 0:
                break
        if np.linalg.norm(b - a @ x) <= tol * nb:
            break
    return x, it, float(np.linalg.norm(b - a @ x) / nb)


def cocg(a, b, tol=1e-8, maxiter=100000, x0=None, history=False, m=None):
    """Conjugate orthogonal conjugate gradients (van der Vorst & Melissen,
    1990): the CG recurrences with the unconjugated bilinear form x^T y,
    valid for complex symmetric A; ``m`` is an optional diagonal
    (complex symmetric) preconditioner, z = m * r.  Stops when
    ``||r|| <= tol ||b||`` (recursive residual, checked against the true one
    at the end).  Returns ``(x, iterations, relres)`` and, with ``history``,
    the recursive relative residual after every iteration."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    r = b - a @ x
    p = np.zeros_like(b)
    z = r if m is None else m * r
    rho = r @ z
    beta = 0.0
    hist = []
    it = 0
    while it < maxiter and np.linalg.norm(r) > tol * nb:
        it += 1
        p = z + beta * p
        q = a @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        z = r if m is None else m * r
        rho_new = r @ z
        beta = rho_new / rho
        rho = rho_new
        hist.append(np.linalg.norm(r) / nb)
    rr = float(np.linalg.norm(b - a @ x) / nb)
    if history:
        return x, it, rr, np.array(hist)
    return x, it, rr


def cocr(a, b, tol=1e-8, maxiter=100000, history=False):
    """Conjugate orthogonal conjugate residual method (Sogabe & Zhang, 2007):
    the conjugate residual recurrences with the unconjugated bilinear form
    x^T y, valid for complex symmetric A (the paper's "cr", Sec. IV).  Stops
    when the recursive ``||r|| <= tol ||b||``.  Returns ``(x, iterations,
    relres)`` and, with ``history``, the recursive relative residual after
    every iteration."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    w = a @ r
    q = w.copy()
    rho = r @ w
    hist = []
    it = 0
    while it < maxiter and np.linalg.norm(r) > tol * nb:
        it += 1
        alpha = rho / (q @ q)
        x = x + alpha * p
        r = r - alpha * q
        hist.append(np.linalg.norm(r) / nb)
        w = a @ r
        rho_new = r @ w
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
        q = w + beta * q
    rr = float(np.linalg.norm(b - a @ x) / nb)
    if history:
        return x, it, rr, np.array(hist)
    return x, it, rr


def tfqmr(a, b, rhat, tol=1e-8, maxiter=100000, history=False):
    """Transpose-free QMR (Freund, 1993) in its half-step form: per
    iteration two half-steps m (even: new alpha, u_{m+1} = u_m - alpha v_m;
    both: w -= alpha A u_m, d = u_m + (theta^2/alpha) eta d, theta =
    ||w||/tau, c = (1+theta^2)^{-1/2}, tau = tau theta c, eta = c^2 alpha,
    x += eta d; odd: rho' = <rhat, w>, beta = rho'/rho, u_{m+1} = w + beta
    u_m, v = A u_{m+1} + beta (A u_m + beta v)), with conjugated inner
    products.  Stops on the QMR bound tau sqrt(m+1) <= tol ||b||.  Returns
    ``(x, iterations, relres)`` and, with ``history``, the relative bound
    after every iteration."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    w = b.copy()
    u = b.copy()
    au = a @ u
    v = au.copy()
    d = np.zeros_like(b)
    tau = nb
    theta = 0.0
    eta = 0.0
    rho = np.vdot(rhat, b)
    alpha = 0.0
    hist = []
    it = 0
    m = 0
    while it < maxiter:
        # even half-step
        alpha = rho / np.vdot(rhat, v)
        u_next = u - alpha * v
        w = w - alpha * au
        d = u + (theta ** 2 / alpha) * eta * d
        theta = np.linalg.norm(w) / tau
        c2 = 1.0 / (1.0 + theta ** 2)
        tau = tau * theta * np.sqrt(c2)
        eta = c2 * alpha
        x = x + eta * d
        m += 1
        # odd half-step
        u = u_next
        au_odd = a @ u
        w = w - alpha * au_odd
        d = u + (theta ** 2 / alpha) * eta * d
        theta = np.linalg.norm(w) / tau
        c2 = 1.0 / (1.0 + theta ** 2)
        tau = tau * theta * np.sqrt(c2)
        eta = c2 * alpha
        x = x + eta * d
        m += 1
        it += 1
        bound = tau * np.sqrt(m + 1)
        hist.append(bound / nb)
        if bound <= tol * nb:
            break
        rho_new = np.vdot(rhat, w)
        beta = rho_new / rho
        rho = rho_new
        u_even = w + beta * u
        au = a @ u_even
        v = au + beta * (au_odd + beta * v)
        u = u_even
    rr = float(np.linalg.norm(b - a @ x) / nb)
    if history:
        return x, it, rr, np.array(hist)
    return x, it, rr


def cgs(a, b, rhat, tol=1e-8, maxiter=100000, history=False):
    """Conjugate gradients squared (Sonneveld, 1989) with conjugated inner
    products against the shadow vector ``rhat`` (one of the methods of the
    paper's comparison, Sec. IV): per iteration rho = <rhat, r>, beta =
    rho/rho_old (0 at the start), u = r + beta q, p = u + beta (q + beta p),
    alpha = rho/<rhat, A p>, q = u - alpha A p, x += alpha (u + q),
    r -= alpha A (u + q).  Stops when the recursive ``||r|| <= tol ||b||``.
    Returns ``(x, iterations, relres)`` and, with ``history``, the recursive
    relative residual after every iteration."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    p = np.zeros_like(b)
    q = np.zeros_like(b)
    rho = np.vdot(rhat, r)
    beta = 0.0
    hist = []
    it = 0
    while it < maxiter and np.linalg.norm(r) > tol * nb:
        it += 1
        u = r + beta * q
        p = u + beta * (q + beta * p)
        v = a @ p
        alpha = rho / np.vdot(rhat, v)
        q = u - alpha * v
        w = u + q
        x = x + alpha * w
        r = r - alpha * (a @ w)
        hist.append(np.linalg.norm(r) / nb)
        rho_new = np.vdot(rhat, r)
        beta = rho_new / rho
        rho = rho_new
    rr = float(np.linalg.norm(b - a @ x) / nb)
    if history:
        return x, it, rr, np.array(hist)
    return x, it, rr


def gmres(a, b, restart=30, tol=1e-8, maxiter=100000, precond=None, x0=None):
    """Restarted GMRES(m) with classical Gram-Schmidt applied twice and
    Givens rotations; with ``precond`` it is flexible GMRES (right
    preconditioning, the preconditioned directions are stored).  Returns
    ``(x, iterations, relres)``."""
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else x0.astype(np.complex128).copy()
    it = 0
    m = restart
    while it < maxiter:
        r = b - a @ x
        beta = np.linalg.norm(r)
        if beta <= tol * nb:
            break
        v = np.zeros((m + 1, b.size), np.complex128)
        z = np.zeros((m, b.size), np.complex128) if precond is not None else None
        h = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m, np.complex128)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        v[0] = r / beta
        k_used = 0
        for jj in range(m):
            it += 1
            zj = precond(v[jj]) if precond is not None else v[jj]
            if z is not None:
                z[jj] = zj
            w = a @ zj
            for _ in range(2):  # CGS2
                hh = v[: jj + 1].conj() @ w
                w = w - hh @ v[: jj + 1]
                h[: jj + 1, jj] += hh
            h[jj + 1, jj] = np.linalg.norm(w)
            if h[jj + 1, jj] != 0:
                v[jj + 1] = w / h[jj + 1, jj]
            # Givens rotations G_i = [[conj(c_i), conj(s_i)], [-s_i, c_i]] with
            # c = a/rho, s = b/rho map (a, b) to (rho, 0) and are unitary.
            for i in range(jj):
                t = np.conj(cs[i]) * h[i, jj] + np.conj(sn[i]) * h[i + 1, jj]
                h[i + 1, jj] = -sn[i] * h[i, jj] + cs[i] * h[i + 1, jj]
                h[i, jj] = t
            rho = np.sqrt(abs(h[jj, jj]) ** 2 + abs(h[jj + 1, jj]) ** 2)
            cs[jj] = h[jj, jj] / rho if rho != 0 else 1.0
            sn[jj] = h[jj + 1, jj] / rho if rho != 0 else 0.0
            h[jj, jj] = rho
            h[jj + 1, jj] = 0.0
            g[jj + 1] = -sn[jj] * g[jj]
            g[jj] = np.conj(cs[jj]) * g[jj]
            k_used = jj + 1
            if abs(g[jj + 1]) <= tol * nb or it >= maxiter:
                break
        y = np.linalg.solve(np.triu(h[:k_used, :k_used]), g[:k_used]) if k_used else []
        basis = z if z is not None else v
        for i in range(k_used):
            x = x + y[i] * basis[i]
        if np.linalg.norm(b - a @ x) <= tol * nb:
            break
    return x, it, float(np.linalg.norm(b - a @ x) / nb)


# ---------------------------------------------------------------------------
# Generalised eigenproblem of the lossless cavity (Sec. IV, first check).
# ---------------------------------------------------------------------------

def cavity_omega2(dev) -> np.ndarray:
    """Every generalised eigenvalue ``omega^2`` [rad^2/s^2] of
    ``K e = omega^2 M_eps e`` on the free edges of a lossless device, in
    ascending order, the gradient null space included (one zero per interior
    node potential).  Dense: for grids of at most a few thousand free edges."""
    import scipy.linalg as sla
    f = free_edges(dev)
    kk = stiffness(dev)[f][:, f]
    m_eps, _ = edge_materials(dev)
    return np.sort(sla.eigh(kk.toarray(), np.diag(m_eps[f].real), eigvals_only=True))


def cavity_eigenfrequencies(dev, k: int = 6, sigma_f: float = 1e9) -> np.ndarray:
    """The ``k`` resonance frequencies [Hz] of ``K e = omega^2 M_eps e`` on
    the free edges closest to ``sigma_f`` [Hz] (shift-invert Lanczos), in
    ascending order."""
    import scipy.sparse.linalg as ssl
    f = free_edges(dev)
    kk = stiffness(dev)[f][:, f]
    m_eps, _ = edge_materials(dev)
    sig = (2 * np.pi * sigma_f) ** 2
    lam = ssl.eigsh(kk.tocsc(), k=k, M=sp.diags(m_eps[f].real).tocsc(), sigma=sig,
                    which="LM", return_eigenvectors=False)
    return np.sort(np.sqrt(np.abs(lam)) / (2 * np.pi))
