"""Degenerate grids on the GPU against the oracle: one cell thick along an
axis, a single cell, open walls, and a device whose cells are all PEC (every
edge masked)."""
import numpy as np
import pytest

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests._helpers import rand_c

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _open(dev):
    dev.pec_walls = 0
    return dev


def _devices():
    pec = D.cavity(6, 5, 4)
    pec.materials = [D.Material(is_pec=True)]
    lossy = D.cavity(9, 1, 7, 1e-3, 0.3e-3, 2e-3, eps_r=4.0)
    lossy.materials = [D.Material(eps_r=4.0, sigma=0.5, tan_delta=0.01)]
    return {
        "thin_x_pec": D.cavity(1, 6, 5),
        "thin_x_open": _open(D.cavity(1, 6, 5)),
        "thin_yz_open": _open(D.cavity(7, 1, 1)),
        "single_cell_open": _open(D.cavity(1, 1, 1)),
        "thin_y_lossy_open": _open(lossy),
        "all_pec": pec,
    }


DEVS = _devices()


@pytest.mark.parametrize("name", sorted(DEVS))
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_degenerate_matvec_and_mask(name, dtype):
    dev = DEVS[name]
    g = fit.Grid(dev)
    f = O.free_edges(dev)
    np.testing.assert_array_equal(g.edge_mask().cpu().numpy().astype(bool), f)
    om = 2 * np.pi * 7e9
    npdt = np.complex128 if dtype == "c128" else np.complex64
    x = rand_c(dev.n_edges, 3, npdt)
    for scaling in ("none", "sym"):
        y = g.matvec(om, _cuda(x), scaling=scaling).cpu().numpy().astype(np.complex128)
        ref = O.matvec(dev, om, x.astype(np.complex128), scaling=scaling)
        assert np.all(y[~f] == 0)
        nr = np.linalg.norm(ref)
        if nr == 0:
            assert np.all(y == 0)
        else:
            tol = 1e-12 if dtype == "c128" else 1e-5
            assert np.linalg.norm(y - ref) <= tol * nr, (name, scaling)


@pytest.mark.parametrize("name", ["thin_x_open", "single_cell_open", "thin_y_lossy_open"])
def test_degenerate_solves(name):
    dev = DEVS[name]
    g = fit.Grid(dev)
    f = O.free_edges(dev)
    src = np.zeros(dev.n_edges, complex)
    src[np.flatnonzero(f)[len(np.flatnonzero(f)) // 2]] = 1.0
    om = 2 * np.pi * 5e9
    for solver in ("cocg", "bicgstab", "gmres"):
        x, info = g.solve(om, _cuda(src), tol=1e-8, solver=solver, raise_on_error=False)
        rr = O.relative_residual(dev, om, src, x.cpu().numpy())
        assert info["status_name"] == "FIT_OK" and rr <= 1e-8, (solver, info)


def test_all_pec_device():
    dev = DEVS["all_pec"]
    g = fit.Grid(dev)
    assert not O.free_edges(dev).any()
    x, info = g.solve(2 * np.pi * 5e9, _cuda(np.zeros(dev.n_edges, complex)), tol=1e-8,
                      solver="cocg")
    assert info["true_relres"] == 0.0 and torch.count_nonzero(x).item() == 0
    src = np.zeros(dev.n_edges, complex)
    src[0] = 1.0
    with pytest.raises(fit.FitError):
        g.solve(2 * np.pi * 5e9, _cuda(src), tol=1e-8)
