"""fit_port_voltages_noalloc (static device scratch, no allocation) against
fit_port_voltages, which allocates a device buffer per call: the same
kernel writes every value, so the two must agree bit for bit, also when a
second call with fewer vectors follows a larger one in the shared array."""
import ctypes as C

import numpy as np
import pytest

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests._helpers import rand_c

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _call_noalloc(g, x, nvec):
    n = len(g.dev.ports)
    out = (C.c_double * (2 * n * nvec))()
    st = fit.lib().fit_port_voltages_noalloc(g.h, C.c_void_p(x.data_ptr()), nvec, out, None)
    return st, np.frombuffer(out, dtype=np.float64).copy().view(np.complex128).reshape(nvec, n)


def test_noalloc_port_voltages_match_the_allocating_entry_point():
    dev = D.layered_device(20, 17, 13, n_layers=4, n_strips=3, n_ports=3, seed=8,
                           strip_kind="sigma")
    assert len(dev.ports) == 3
    g = fit.Grid(dev)
    free = O.free_edges(dev)
    xs = np.concatenate([rand_c(dev.n_edges, 300 + v) * free for v in range(5)])
    x = torch.from_numpy(xs).to("cuda:0")
    # two calls in a row through the C ABI, the second with a smaller input
    for nvec in (5, 2):
        st, got = _call_noalloc(g, x, nvec)
        assert st == fit.OK
        ref = g.port_voltages(x, nvec=nvec)
        np.testing.assert_array_equal(got, ref)
        for v in range(nvec):
            np.testing.assert_allclose(
                got[v], O.port_voltages(dev, xs[v * dev.n_edges:(v + 1) * dev.n_edges]),
                rtol=1e-12, atol=1e-14 * np.abs(xs).max())


def test_noalloc_port_voltages_reject_oversized_calls():
    dev = D.layered_device(20, 17, 13, n_layers=4, n_strips=3, n_ports=3, seed=8,
                           strip_kind="sigma")
    g = fit.Grid(dev)
    x = torch.zeros(dev.n_edges, dtype=torch.complex128, device="cuda:0")
    nvec = 65536 // 3 + 1  # 3 ports: one value over the scratch array
    out = (C.c_double * 2)()
    st = fit.lib().fit_port_voltages_noalloc(g.h, C.c_void_p(x.data_ptr()), nvec, out, None)
    assert st == fit.E_INVALID
    assert "65536" in fit.last_error()
