"""Parity of the HIP operator with the FP64 oracle (Sec. II eq. (e2) with
losses; Sec. III eq. (e2t) for the symmetric scaling).

Bars: complex128 <= 1e-12 relative 2-norm, complex64 <= 1e-5 (the oracle is
fed the FP32-rounded input), masks bit-exact, material diagonals <= 1e-14.
"""
import numpy as np
import pytest

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests._helpers import crop, crop_vector, rand_c, parity_devices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DEVS = parity_devices()
OMEGA = 2 * np.pi * 13.7e9
TILES = [(64, 8, 16), (48, 8, 3), (32, 8, 1), (32, 16, 5)]


def _grid(name):
    return fit.Grid(DEVS[name])


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("name", sorted(DEVS))
def test_edge_mask_bit_exact(name):
    g = _grid(name)
    m = g.edge_mask().cpu().numpy().astype(bool)
    np.testing.assert_array_equal(m, O.free_edges(DEVS[name]))


@pytest.mark.parametrize("name", sorted(DEVS))
def test_material_diagonals(name):
    dev = DEVS[name]
    g = _grid(name)
    m_eps, m_sig = O.edge_materials(dev)
    nu = O.facet_reluctance(dev)
    for kind, ref in ((0, m_eps), (1, m_sig.astype(complex)), (2, nu.astype(complex))):
        got = g.material_diag(kind).cpu().numpy()
        scale = np.abs(ref).max()
        assert np.abs(got - ref).max() <= 1e-14 * scale, kind


@pytest.mark.parametrize("scaling", ["none", "sym"])
@pytest.mark.parametrize("name", sorted(DEVS))
@pytest.mark.parametrize("tile", TILES)
def test_matvec_c128_parity(name, scaling, tile):
    dev = DEVS[name]
    g = _grid(name)
    g.set_tile("c128", *tile)
    x = rand_c(dev.n_edges, 11)
    y = g.matvec(OMEGA, _cuda(x), scaling=scaling).cpu().numpy()
    ref = O.matvec(dev, OMEGA, x, scaling=scaling)
    f = O.free_edges(dev)
    assert np.all(y[~f] == 0)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert rel <= 1e-12, rel


@pytest.mark.parametrize("scaling", ["none", "sym"])
@pytest.mark.parametrize("name", sorted(DEVS))
def test_matvec_c64_parity(name, scaling):
    dev = DEVS[name]
    g = _grid(name)
    g.set_tile("c64", 48, 8, 7)
    x = rand_c(dev.n_edges, 12, np.complex64)
    y = g.matvec(OMEGA, _cuda(x), scaling=scaling).cpu().numpy().astype(np.complex128)
    ref = O.matvec(dev, OMEGA, x.astype(np.complex128), scaling=scaling)
    f = O.free_edges(dev)
    assert np.all(y[~f] == 0)
    rel = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    assert rel <= 1e-5, rel


def test_matvec_zero_frequency_is_the_curl_curl():
    dev = DEVS["layered_pec"]
    g = _grid("layered_pec")
    x = rand_c(dev.n_edges, 13)
    y = g.matvec(0.0, _cuda(x)).cpu().numpy()
    ref = O.matvec(dev, 0.0, x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)


def test_complex_symmetry_on_gpu():
    """u^T (A v) = v^T (A u) (unconjugated): Table I's symmetric operator."""
    dev = DEVS["layered_sigma"]
    g = _grid("layered_sigma")
    u, v = rand_c(dev.n_edges, 1), rand_c(dev.n_edges, 2)
    f = O.free_edges(dev)
    u[~f] = 0
    v[~f] = 0
    for scaling in ("none", "sym"):
        av = g.matvec(OMEGA, _cuda(v), scaling=scaling).cpu().numpy()
        au = g.matvec(OMEGA, _cuda(u), scaling=scaling).cpu().numpy()
        a, b = u @ av, v @ au
        assert abs(a - b) <= 1e-13 * np.linalg.norm(u) * np.linalg.norm(av)


def test_gradient_fields_are_annihilated_at_zero_frequency():
    dev = D.layered_device(40, 30, 20, n_layers=3, n_strips=0, n_ports=0, seed=3)
    g = fit.Grid(dev)
    nx, ny, nz = dev.nodes
    rng = np.random.default_rng(4)
    phi = rng.standard_normal((nz, ny, nx))
    phi[[0, -1]] = 0
    phi[:, [0, -1]] = 0
    phi[:, :, [0, -1]] = 0
    e = (O.gradient(nx, ny, nz).astype(float) @ phi.ravel()).astype(complex)
    y = g.matvec(0.0, _cuda(e)).cpu().numpy()
    ref_scale = np.linalg.norm(O.matvec(dev, 0.0, rand_c(dev.n_edges, 5)))
    assert np.linalg.norm(y) <= 1e-12 * ref_scale * np.linalg.norm(e) / np.sqrt(dev.n_edges)


def test_ignores_input_on_masked_edges():
    dev = DEVS["layered_pec"]
    g = _grid("layered_pec")
    x = rand_c(dev.n_edges, 21)
    f = O.free_edges(dev)
    x2 = x.copy()
    x2[~f] = 1e30
    y1 = g.matvec(OMEGA, _cuda(x)).cpu().numpy()
    y2 = g.matvec(OMEGA, _cuda(x2)).cpu().numpy()
    np.testing.assert_array_equal(y1, y2)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_128_cubed_sampled_parity(dtype):
    """The 128^3-cell graded layered device at full size, default launch:
    sampled nodes checked one by one against the oracle on local crops."""
    dev = D.plain_device_128(2)
    g = fit.Grid(dev)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    x = rand_c(dev.n_edges, 31, npdt)
    y = g.matvec(OMEGA, _cuda(x), scaling="sym").cpu().numpy().astype(np.complex128)
    x = x.astype(np.complex128)
    rng = np.random.default_rng(6)
    nx, ny, nz = dev.nodes
    pts = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)))
           for _ in range(120)]
    pts += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (63, 3, 15), (64, 4, 16), (65, 5, 17), (61, 5, 15), (62, 6, 16)]
    p0 = dev.ports[0]
    pts.append((p0.i, p0.j, (p0.k0 + p0.k1) // 2))
    worst = 0.0
    for (i, j, k) in pts:
        sub, off = crop(dev, i, j, k)
        xs = crop_vector(dev, sub, off, x)
        ys = O.matvec(sub, OMEGA, xs, scaling="sym")
        li, lj, lk = i - off[0], j - off[1], k - off[2]
        for w in range(3):
            ref = ys[sub.edge_index(w, li, lj, lk)]
            got = y[dev.edge_index(w, i, j, k)]
            scale = max(np.abs(ys).max(), 1e-300)
            worst = max(worst, abs(got - ref) / scale)
    assert worst <= (1e-12 if dtype == "c128" else 1e-5), worst


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_full_size_256_interconnect_sampled_parity(dtype):
    """The 256x256x128-cell interconnect (25.6M unknowns) at full size,
    default launch, in both precisions: sampled nodes, tile seams and the
    port column checked one by one against the oracle on local crops."""
    dev = D.interconnect_256(3)
    g = fit.Grid(dev)
    npdt = np.complex128 if dtype == "c128" else np.complex64
    x = rand_c(dev.n_edges, 37, npdt)
    om = 2 * np.pi * 10e9
    y = g.matvec(om, _cuda(x)).cpu().numpy().astype(np.complex128)
    x = x.astype(np.complex128)
    rng = np.random.default_rng(8)
    nx, ny, nz = dev.nodes
    pts = [(int(rng.integers(0, nx)), int(rng.integers(0, ny)), int(rng.integers(0, nz)))
           for _ in range(80)]
    pts += [(0, 0, 0), (nx - 1, ny - 1, nz - 1), (nx // 2, ny // 2, nz // 2), (31, 7, 64), (32, 8, 65)]
    p0 = dev.ports[0]
    pts.append((p0.i, p0.j, (p0.k0 + p0.k1) // 2))
    worst = 0.0
    for (i, j, k) in pts:
        sub, off = crop(dev, i, j, k)
        xs = crop_vector(dev, sub, off, x)
        ys = O.matvec(sub, om, xs)
        li, lj, lk = i - off[0], j - off[1], k - off[2]
        for w in range(3):
            ref = ys[sub.edge_index(w, li, lj, lk)]
            got = y[dev.edge_index(w, i, j, k)]
            scale = max(np.abs(ys).max(), 1e-300)
            worst = max(worst, abs(got - ref) / scale)
    assert worst <= (1e-12 if dtype == "c128" else 1e-5), worst


def test_autotune_records_a_shape():
    dev = DEVS["layered_pec"]
    g = _grid("layered_pec")
    (tx, ty, zc), us = g.autotune("c128", "sym", OMEGA, reps=3)
    assert (tx, ty) in {(64, 8), (48, 8), (32, 8), (32, 16)} and zc >= 1 and us > 0
