"""The C ABI library loads and exports every entry point declared in
include/fit.h; host-side argument validation needs no GPU."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

from paper_1705_08849_amd import fit
from paper_1705_08849_amd import devices as D

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "fit.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fit_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = fit.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fit.exported_symbols())


def test_version_and_error_string():
    assert fit.lib().fit_version().decode().startswith("fit-mi355x")
    assert isinstance(fit.last_error(), str)


def _desc(dev, **over):
    dx = np.ascontiguousarray(dev.dx)
    dy = np.ascontiguousarray(dev.dy)
    dz = np.ascontiguousarray(dev.dz)
    cm = np.ascontiguousarray(dev.cell_mat).ravel()
    mats = (fit.Material * len(dev.materials))(*[
        fit.Material(m.eps_r, m.mu_r, m.sigma, m.tan_delta, int(m.is_pec), 0)
        for m in dev.materials])
    ports = (fit.Port * max(1, len(dev.ports)))(*[fit.Port(p.i, p.j, p.k0, p.k1, p.z0)
                                                   for p in dev.ports])
    d = fit.GridDesc(len(dx), len(dy), len(dz), len(dev.materials),
                     dx.ctypes.data_as(C.POINTER(C.c_double)),
                     dy.ctypes.data_as(C.POINTER(C.c_double)),
                     dz.ctypes.data_as(C.POINTER(C.c_double)),
                     cm.ctypes.data_as(C.POINTER(C.c_uint8)), mats, len(dev.ports),
                     dev.pec_walls, ports)
    for k, v in over.items():
        setattr(d, k, v)
    return d, (dx, dy, dz, cm, mats, ports)


@pytest.mark.parametrize("bad", [
    dict(ncx=0), dict(nmat=0), dict(nmat=255), dict(pec_walls=0x40), dict(nports=65),
])
def test_grid_create_rejects_invalid_descriptors(bad):
    dev = D.layered_device(6, 5, 4, n_layers=2, n_strips=1, n_ports=1, seed=1)
    d, keep = _desc(dev, **bad)
    h = C.c_void_p()
    st = fit.lib().fit_grid_create(C.byref(d), 0, C.byref(h))
    assert st == fit.E_INVALID and not h.value
    assert fit.last_error()


def test_grid_create_rejects_bad_geometry_and_ports():
    dev = D.cavity(4, 4, 4)
    dev.dx[1] = -1.0
    d, keep = _desc(dev)
    h = C.c_void_p()
    assert fit.lib().fit_grid_create(C.byref(d), 0, C.byref(h)) == fit.E_INVALID
    dev = D.cavity(4, 4, 4)
    dev.cell_mat[1, 1, 1] = 3
    d, keep = _desc(dev)
    assert fit.lib().fit_grid_create(C.byref(d), 0, C.byref(h)) == fit.E_INVALID
    dev = D.cavity(4, 4, 4)
    dev.ports = [D.Port(1, 1, 0, 2), D.Port(1, 1, 2, 4)]  # two ports on one column
    d, keep = _desc(dev)
    assert fit.lib().fit_grid_create(C.byref(d), 0, C.byref(h)) == fit.E_INVALID
    assert "column" in fit.last_error()
    dev.ports = [D.Port(1, 1, 2, 6)]  # beyond ncz
    d, keep = _desc(dev)
    assert fit.lib().fit_grid_create(C.byref(d), 0, C.byref(h)) == fit.E_INVALID


def test_null_arguments_are_rejected():
    L = fit.lib()
    assert L.fit_matvec(None, 1.0, 0, 0, None, None, None) == fit.E_INVALID
    assert L.fit_edge_mask(None, None, None) == fit.E_INVALID
    assert L.fit_num_edges(None) == -1
    L.fit_grid_destroy(None)
    assert L.fit_tile_set(None, 0, 64, 8, 8) == fit.E_INVALID


def test_batched_and_sweep_argument_checks():
    """Argument validation of the batched entry points needs no device."""
    L = fit.lib()
    om = (C.c_double * 2)(1e9, 2e9)
    assert L.fit_matvec_batched(None, 2, om, 0, 0, None, None, None) == fit.E_INVALID
    assert L.fit_sweep(None, 1, om, 2, None, 1, 1e-8, None, None, None, None) == fit.E_INVALID
    gh = (C.c_void_p * 1)(None)
    src = (C.c_void_p * 1)(None)
    assert L.fit_sweep(gh, 1, om, 2, src, 1, 1e-8, None, None, None, None) == fit.E_INVALID
    assert "NULL" in fit.last_error()
    assert L.fit_sweep(gh, 1, om, 2, src, 1, 2.0, None, None, None, None) == fit.E_INVALID
    bad = (C.c_double * 2)(1e9, -1.0)
    assert L.fit_sweep(gh, 1, bad, 2, src, 1, 1e-8, None, None, None, None) == fit.E_INVALID


def test_port_network_host_matches_the_oracle():
    """fit_port_network (host code in the library) against the oracle's
    definitions on random loaded impedance matrices of 1 to 6 ports."""
    from oracle import fit_oracle as O
    rng = np.random.default_rng(11)
    for n in (1, 2, 4, 6):
        zl = 40 * (rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))) + 30 * np.eye(n)
        z, s = fit.port_network(zl, 50.0)
        z_ref, s_ref = O.port_network(zl, 50.0)
        np.testing.assert_allclose(z, z_ref, rtol=1e-10, atol=1e-10 * abs(z_ref).max())
        np.testing.assert_allclose(s, s_ref, rtol=1e-10, atol=1e-10 * abs(s_ref).max())


def test_port_network_rejects_bad_arguments_and_writes_nothing():
    L = fit.lib()
    buf = (C.c_double * 8)(*([7.0] * 8))
    out = (C.c_double * 8)(*([-3.0] * 8))
    assert L.fit_port_network(0, 50.0, buf, out, out) == fit.E_INVALID
    assert L.fit_port_network(2, 0.0, buf, out, out) == fit.E_INVALID
    assert L.fit_port_network(65, 50.0, buf, out, out) == fit.E_INVALID
    assert L.fit_port_network(2, 50.0, None, out, out) == fit.E_INVALID
    # all-equal entries: zl is singular, so the unloaded Z does not exist
    assert L.fit_port_network(2, 50.0, buf, out, None) == fit.E_INVALID
    assert list(out) == [-3.0] * 8
    # S alone needs no inversion
    assert L.fit_port_network(2, 50.0, buf, None, out) == fit.OK
    assert abs(out[0] - (2 * 7.0 / 50.0 - 1.0)) < 1e-15 and abs(out[2] - 2 * 7.0 / 50.0) < 1e-15
