"""Thin ctypes binding of ``libfit.so`` (the C ABI declared in ``include/fit.h``).

Only argument marshalling lives here: every step of the operator and the
solvers runs in the library's HIP kernels.  PyTorch supplies device memory
and streams (``tensor.data_ptr()``, ``torch.cuda.current_stream()``).  If the
shared library is missing the binding raises; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path
from typing import Optional, Sequence

import numpy as np

_HERE = Path(__file__).resolve().parent
LIB_PATH = _HERE / "libfit.so"

# status codes (fit_status)
OK, E_INVALID, E_NOMEM, E_DEVICE, E_NOT_CONVERGED, E_BREAKDOWN, E_NAN, E_UNSUPPORTED = range(8)
STATUS_NAMES = ["FIT_OK", "FIT_E_INVALID", "FIT_E_NOMEM", "FIT_E_DEVICE", "FIT_E_NOT_CONVERGED",
                "FIT_E_BREAKDOWN", "FIT_E_NAN", "FIT_E_UNSUPPORTED"]
C128, C64 = 0, 1
SCALE_NONE, SCALE_SYM, SCALE_FACT = 0, 1, 2
BICGSTAB, GMRES, FGMRES, COCG, COCR, TFQMR, CGS = 0, 1, 2, 3, 4, 5, 6
PREC_FP64, PREC_MIXED = 0, 1
DIAG_AUTO, DIAG_MASS, DIAG_PAPER, DIAG_JACOBI = 0, 1, 2, 3

SOLVERS = {"bicgstab": BICGSTAB, "gmres": GMRES, "fgmres": FGMRES, "cocg": COCG, "cocr": COCR,
           "tfqmr": TFQMR, "cgs": CGS}
SCALINGS = {"none": SCALE_NONE, "sym": SCALE_SYM, "fact": SCALE_FACT}
PRECISIONS = {"fp64": PREC_FP64, "mixed": PREC_MIXED}
DIAGS = {"auto": DIAG_AUTO, "mass": DIAG_MASS, "paper": DIAG_PAPER, "jacobi": DIAG_JACOBI}
TILE_BATCHED_C128 = 2  # tile-table key of batched (sweep) launches in complex128
_TILE_KEYS = {"c128": C128, "c64": C64, "c128_batched": TILE_BATCHED_C128}


class FitError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 8 else status}: {msg}")
        self.status = status


class Material(C.Structure):
    _fields_ = [("eps_r", C.c_double), ("mu_r", C.c_double), ("sigma", C.c_double),
                ("tan_delta", C.c_double), ("is_pec", C.c_int32), ("reserved", C.c_int32)]


class Port(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k0", C.c_int32), ("k1", C.c_int32),
                ("z0", C.c_double)]


class GridDesc(C.Structure):
    _fields_ = [("ncx", C.c_int32), ("ncy", C.c_int32), ("ncz", C.c_int32), ("nmat", C.c_int32),
                ("dx", C.POINTER(C.c_double)), ("dy", C.POINTER(C.c_double)),
                ("dz", C.POINTER(C.c_double)), ("cell_mat", C.POINTER(C.c_uint8)),
                ("mats", C.POINTER(Material)), ("nports", C.c_int32),
                ("pec_walls", C.c_uint32), ("ports", C.POINTER(Port))]


class SolveOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("restart", C.c_int32), ("max_iters", C.c_int32),
                ("check_every", C.c_int32), ("precision", C.c_int32), ("scaling", C.c_int32),
                ("inner_tol", C.c_double), ("precond", C.c_void_p), ("stream", C.c_void_p),
                ("resid_history", C.POINTER(C.c_double)), ("resid_history_len", C.c_int32),
                ("use_graph", C.c_int32), ("diag", C.c_int32), ("reserved", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("refinements", C.c_int32),
                ("fell_back", C.c_int32), ("matvecs", C.c_int32), ("reserved", C.c_int32),
                ("true_relres", C.c_double), ("time_ms", C.c_double),
                ("bytes_moved", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_int64), ("total_ms", C.c_double)]


def profile_start():
    check(lib().fit_profile_start(), "fit_profile_start")


def profile_stop():
    """Per kernel family: {name: (launches, total_ms)} since profile_start()."""
    n = C.c_int()
    buf = (KernelStat * 64)()
    check(lib().fit_profile_stop(buf, 64, C.byref(n)), "fit_profile_stop")
    return {buf[i].name.decode(): (buf[i].launches, buf[i].total_ms) for i in range(min(n.value, 64))}


def tune_save(path: str):
    """Write the process-wide tile table (fit_tune_save)."""
    check(lib().fit_tune_save(os.fsencode(path)), "fit_tune_save")


def tune_load(path: str):
    """Merge a saved tile table into the process-wide one (fit_tune_load)."""
    check(lib().fit_tune_load(os.fsencode(path)), "fit_tune_load")


class PrecondCfg(C.Structure):
    _fields_ = [("base_channels", C.c_int32), ("steps", C.c_int32), ("batch", C.c_int32),
                ("crop", C.c_int32), ("pairs_per_system", C.c_int32), ("seed", C.c_int32),
                ("lr", C.c_double), ("weight_decay", C.c_double), ("stream", C.c_void_p)]


# (name, restype, argtypes) of every exported entry point.
_SIGS = [
    ("fit_grid_create", C.c_int, [C.POINTER(GridDesc), C.c_int, C.POINTER(C.c_void_p)]),
    ("fit_grid_destroy", None, [C.c_void_p]),
    ("fit_num_edges", C.c_int64, [C.c_void_p]),
    ("fit_edge_mask", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("fit_material_diag", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]),
    ("fit_matvec", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_void_p, C.c_void_p,
                             C.c_void_p]),
    ("fit_matvec_batched", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.c_int,
                                     C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]),
    ("fit_solve", C.c_int, [C.c_void_p, C.c_double, C.c_void_p, C.c_double,
                            C.POINTER(SolveOpts), C.c_void_p, C.POINTER(SolveInfo)]),
    ("fit_sweep", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_double), C.c_int,
                            C.POINTER(C.c_void_p), C.c_int, C.c_double, C.POINTER(SolveOpts),
                            C.POINTER(C.c_double), C.POINTER(C.c_void_p), C.POINTER(SolveInfo)]),
    ("fit_port_voltages", C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                    C.c_void_p]),
    ("fit_port_voltages_noalloc", C.c_int, [C.c_void_p, C.c_void_p, C.c_int,
                                            C.POINTER(C.c_double), C.c_void_p]),
    ("fit_port_network", C.c_int, [C.c_int, C.c_double, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("fit_precond_train", C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_double),
                                    C.c_int, C.POINTER(PrecondCfg), C.POINTER(C.c_void_p)]),
    ("fit_precond_create", C.c_int, [C.POINTER(PrecondCfg), C.c_int, C.POINTER(C.c_void_p)]),
    ("fit_precond_save", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_size_t)]),
    ("fit_precond_load", C.c_int, [C.c_void_p, C.c_size_t, C.c_int, C.POINTER(C.c_void_p)]),
    ("fit_precond_apply", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                    C.c_void_p]),
    ("fit_precond_destroy", None, [C.c_void_p]),
    ("fit_precond_loss_grad", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                        C.POINTER(C.c_double), C.c_void_p, C.c_void_p]),
    ("fit_precond_train_history", C.c_int, [C.POINTER(C.c_double), C.c_int, C.POINTER(C.c_int)]),
    ("fit_precond_harvest", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_int, C.c_double,
                                      C.c_void_p, C.c_void_p, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]),
    ("fit_tile_set", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]),
    ("fit_tile_get", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_int32)]),
    ("fit_autotune_solver", C.c_int, [C.c_void_p, C.c_double, C.c_int, C.c_void_p,
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("fit_sweep_set_batch", C.c_int, [C.c_int]),
    ("fit_autotune_sweep", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int, C.c_int,
                                     C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    ("fit_autotune", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int, C.c_void_p,
                               C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    ("fit_tune_save", C.c_int, [C.c_char_p]),
    ("fit_tune_load", C.c_int, [C.c_char_p]),
    ("fit_profile_start", C.c_int, []),
    ("fit_profile_stop", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int)]),
    ("fit_last_error", C.c_char_p, []),
    ("fit_version", C.c_char_p, []),
]

_lib = None


def lib():
    """Load ``libfit.so`` (built in-tree by ``paper_1705_08849_amd.build``)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1705_08849_amd.build` (no fallback exists)")
        L = C.CDLL(str(LIB_PATH))
        for name, res, args in _SIGS:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [s[0] for s in _SIGS]


def last_error() -> str:
    return lib().fit_last_error().decode()


def check(status: int, what: str = ""):
    if status != OK:
        raise FitError(status, f"{what}: {last_error()}")


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


class Grid:
    """A device-resident FIT grid (``fit_grid_create``).

    ``dev`` is any object with ``dx, dy, dz`` (cell widths, m), ``cell_mat``
    (uint8, shape ``(ncz, ncy, ncx)``), ``materials`` (objects with
    ``eps_r, mu_r, sigma, tan_delta, is_pec``), ``ports`` (objects with
    ``i, j, k0, k1, z0``) and ``pec_walls``.
    """

    def __init__(self, dev, device: int = 0):
        L = lib()
        self.dev = dev
        self.device = device
        self._keep = []
        dx = np.ascontiguousarray(dev.dx, np.float64)
        dy = np.ascontiguousarray(dev.dy, np.float64)
        dz = np.ascontiguousarray(dev.dz, np.float64)
        cm = np.ascontiguousarray(dev.cell_mat, np.uint8).ravel()
        mats = (Material * len(dev.materials))(*[
            Material(m.eps_r, m.mu_r, m.sigma, m.tan_delta, int(bool(m.is_pec)), 0)
            for m in dev.materials])
        nports = len(dev.ports)
        ports = (Port * max(nports, 1))(*[Port(p.i, p.j, p.k0, p.k1, p.z0) for p in dev.ports])
        self._keep = [dx, dy, dz, cm, mats, ports]
        desc = GridDesc(len(dx), len(dy), len(dz), len(dev.materials),
                        dx.ctypes.data_as(C.POINTER(C.c_double)),
                        dy.ctypes.data_as(C.POINTER(C.c_double)),
                        dz.ctypes.data_as(C.POINTER(C.c_double)),
                        cm.ctypes.data_as(C.POINTER(C.c_uint8)), mats, nports,
                        int(dev.pec_walls), ports)
        h = C.c_void_p()
        check(L.fit_grid_create(C.byref(desc), device, C.byref(h)), "fit_grid_create")
        self.h = h
        self.n_edges = int(L.fit_num_edges(h))
        self.nodes = (len(dx) + 1, len(dy) + 1, len(dz) + 1)

    def close(self):
        if getattr(self, "h", None):
            lib().fit_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- launch shapes --------------------------------------------------------
    def set_tile(self, dtype: str, tx: int, ty: int, zc: int):
        check(lib().fit_tile_set(self.h, _TILE_KEYS[dtype], tx, ty, zc),
              "fit_tile_set")

    def tile(self, dtype: str = "c128"):
        """``fit_tile_get``: the (tx, ty, zc) that launches on this grid use now."""
        tx, ty, zc = C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().fit_tile_get(self.h, _TILE_KEYS[dtype], C.byref(tx), C.byref(ty),
                                 C.byref(zc)), "fit_tile_get")
        return tx.value, ty.value, zc.value

    def autotune(self, dtype: str = "c128", scaling: str = "none", omega: float = 2e10,
                 reps: int = 10, stream=None):
        tx, ty, zc, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        check(lib().fit_autotune(self.h, _TILE_KEYS[dtype], SCALINGS[scaling],
                                 float(omega), reps, _stream_ptr(stream), C.byref(tx),
                                 C.byref(ty), C.byref(zc), C.byref(us)), "fit_autotune")
        return (tx.value, ty.value, zc.value), us.value

    def autotune_solver(self, omega: float, iters: int = 200, stream=None):
        """``fit_autotune_solver``: tile tuned on the COCG iteration itself;
        returns ((tx, ty, zc), microseconds per iteration)."""
        tx, ty, zc, us = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
        check(lib().fit_autotune_solver(self.h, float(omega), iters, _stream_ptr(stream),
                                        C.byref(tx), C.byref(ty), C.byref(zc), C.byref(us)),
              "fit_autotune_solver")
        return (tx.value, ty.value, zc.value), us.value

    def autotune_sweep(self, omegas: Sequence[float], iters: int = 100, stream=None):
        """``fit_autotune_sweep``: systems per batch for sweeps on grids like
        this one; returns (batch, system-iterations per second)."""
        om = (C.c_double * len(omegas))(*[float(o) for o in omegas])
        b, rate = C.c_int32(), C.c_double()
        check(lib().fit_autotune_sweep(self.h, om, len(omegas), iters, _stream_ptr(stream),
                                       C.byref(b), C.byref(rate)), "fit_autotune_sweep")
        return b.value, rate.value

    # -- debug exports ------------------------------------------------------
    def edge_mask(self, stream=None):
        torch = _torch()
        m = torch.empty(self.n_edges, dtype=torch.uint8, device=f"cuda:{self.device}")
        check(lib().fit_edge_mask(self.h, _dptr(m), _stream_ptr(stream)), "fit_edge_mask")
        return m

    def material_diag(self, kind: int, stream=None):
        torch = _torch()
        d = torch.empty(self.n_edges, dtype=torch.complex128, device=f"cuda:{self.device}")
        check(lib().fit_material_diag(self.h, kind, _dptr(d), _stream_ptr(stream)),
              "fit_material_diag")
        return d

    # -- operator -----------------------------------------------------------
    def matvec(self, omega: float, x, y=None, scaling: str = "none", stream=None):
        torch = _torch()
        dt = {torch.complex128: C128, torch.complex64: C64}[x.dtype]
        assert x.is_contiguous() and x.numel() == self.n_edges
        if y is None:
            y = torch.empty_like(x)
        check(lib().fit_matvec(self.h, float(omega), dt, SCALINGS[scaling], _dptr(x), _dptr(y),
                               _stream_ptr(stream)), "fit_matvec")
        return y

    def matvec_batched(self, omegas: Sequence[float], x, y=None, scaling: str = "none",
                       stream=None):
        torch = _torch()
        dt = {torch.complex128: C128, torch.complex64: C64}[x.dtype]
        nb = len(omegas)
        assert x.is_contiguous() and x.numel() == nb * self.n_edges
        if y is None:
            y = torch.empty_like(x)
        om = (C.c_double * nb)(*[float(o) for o in omegas])
        check(lib().fit_matvec_batched(self.h, nb, om, dt, SCALINGS[scaling], _dptr(x), _dptr(y),
                                       _stream_ptr(stream)), "fit_matvec_batched")
        return y

    # -- solve --------------------------------------------------------------
    def solve(self, omega: float, source, tol: float = 1e-8, solver: str = "bicgstab",
              restart: int = 30, max_iters: int = 0, check_every: int = 0,
              precision: str = "fp64", scaling: str = "sym", inner_tol: float = 0.0,
              precond=None, history: int = 0, use_graph: bool = False, x=None,
              stream=None, raise_on_error: bool = True, diag: str = "auto"):
        """Solve ``A(omega) e = -j omega j`` (``source`` = j, complex128 on the
        device).  Returns ``(e, info_dict)``."""
        torch = _torch()
        assert source.dtype == torch.complex128 and source.numel() == self.n_edges
        if x is None:
            x = torch.empty_like(source)
        hist = (C.c_double * history)() if history else None
        opts = SolveOpts(SOLVERS[solver], restart, max_iters, check_every,
                         PRECISIONS[precision], SCALINGS[scaling], inner_tol,
                         C.c_void_p(precond.h.value if precond is not None else None),
                         _stream_ptr(stream),
                         C.cast(hist, C.POINTER(C.c_double)) if hist else None,
                         history, int(bool(use_graph)), DIAGS[diag])
        info = SolveInfo()
        st = lib().fit_solve(self.h, float(omega), _dptr(source), float(tol), C.byref(opts),
                             _dptr(x), C.byref(info))
        d = info.as_dict()
        d["status_name"] = STATUS_NAMES[st] if 0 <= st < 8 else str(st)
        if hist is not None:
            d["history"] = np.array(hist[: min(history, max(info.iterations, 0))])
        if st == E_INVALID or (raise_on_error and st not in (OK,)):
            raise FitError(st, f"fit_solve: {last_error()} (info={d})")
        return x, d

    def port_voltages(self, x, nvec: int = 1, stream=None, noalloc: bool = False) -> np.ndarray:
        """Port sums of ``nvec`` fields stored back to back; ``noalloc`` calls
        ``fit_port_voltages_noalloc`` (static device scratch, no allocation)."""
        n = len(self.dev.ports)
        out = (C.c_double * (2 * max(1, n * nvec)))()
        fn = lib().fit_port_voltages_noalloc if noalloc else lib().fit_port_voltages
        check(fn(self.h, _dptr(x), nvec, out, _stream_ptr(stream)),
              "fit_port_voltages_noalloc" if noalloc else "fit_port_voltages")
        a = np.frombuffer(out, dtype=np.float64)[: 2 * n * nvec].copy()
        return a.view(np.complex128).reshape(nvec, n)


def sweep_set_batch(systems: int):
    """``fit_sweep_set_batch``: systems per batch of ``sweep`` (1..64)."""
    check(lib().fit_sweep_set_batch(int(systems)), "fit_sweep_set_batch")


def port_network(zl, z0: float = 50.0):
    """Unloaded impedance matrix Z and scattering matrix S of the ports from
    the loaded impedance matrix ``zl`` (``zl[p, q] = -u_p`` for a unit
    current at port q); see ``fit_port_network``.  Returns ``(z, s)``."""
    a = np.ascontiguousarray(np.asarray(zl, dtype=np.complex128))
    n = a.shape[0] if a.ndim == 2 else 0
    if a.ndim != 2 or a.shape[1] != n:
        raise ValueError("port_network: zl must be a square matrix")
    zin = a.view(np.float64).ctypes.data_as(C.POINTER(C.c_double))
    zo = (C.c_double * (2 * n * n))()
    so = (C.c_double * (2 * n * n))()
    check(lib().fit_port_network(n, float(z0), zin, zo, so), "fit_port_network")
    z = np.frombuffer(zo, dtype=np.float64).copy().view(np.complex128).reshape(n, n)
    s_ = np.frombuffer(so, dtype=np.float64).copy().view(np.complex128).reshape(n, n)
    return z, s_


def sweep(grids: Sequence[Grid], omegas: Sequence[float], sources, tol: float = 1e-8,
          solver: str = "cocg", precision: str = "fp64", scaling: str = "sym",
          max_iters: int = 0, check_every: int = 0, inner_tol: float = 0.0, xs=None,
          restart: int = 30, stream=None, use_graph: bool = True):
    """``fit_sweep``: solve every (grid, omega, rhs) system.  ``sources[g]`` is
    a complex128 tensor of shape ``(nrhs, n_e(g))``.  Returns
    ``(status, port_voltages list per grid [nomega, nrhs, nports], infos)``."""
    ng, nf = len(grids), len(omegas)
    nrhs = int(sources[0].shape[0])
    gh = (C.c_void_p * ng)(*[g.h.value for g in grids])
    om = (C.c_double * nf)(*[float(o) for o in omegas])
    src = (C.c_void_p * ng)(*[s.data_ptr() for s in sources])
    npts = [len(g.dev.ports) for g in grids]
    tot = sum(nf * nrhs * p for p in npts)
    pv = (C.c_double * (2 * max(tot, 1)))()
    xp = (C.c_void_p * ng)(*[x.data_ptr() for x in xs]) if xs is not None else None
    infos = (SolveInfo * (ng * nf * nrhs))()
    opts = SolveOpts(SOLVERS[solver], restart, max_iters, check_every, PRECISIONS[precision],
                     SCALINGS[scaling], inner_tol, None, _stream_ptr(stream), None, 0,
                     int(bool(use_graph)))
    st = lib().fit_sweep(gh, ng, om, nf, src, nrhs, float(tol), C.byref(opts), pv, xp, infos)
    if st == E_INVALID:
        raise FitError(st, f"fit_sweep: {last_error()}")
    a = np.frombuffer(pv, dtype=np.float64)[: 2 * tot].copy().view(np.complex128)
    out, off = [], 0
    for p in npts:
        out.append(a[off: off + nf * nrhs * p].reshape(nf, nrhs, p))
        off += nf * nrhs * p
    return st, out, [infos[q].as_dict() for q in range(ng * nf * nrhs)]


PRECOND_MAGIC = 0x3154454E55544946


class Precond:
    """The learned FGMRES right preconditioner (``fit_precond_*``)."""

    def __init__(self, h: C.c_void_p, device: int = 0):
        self.h = h
        self.device = device

    @staticmethod
    def _cfg(base_channels=16, steps=0, batch=0, crop=0, seed=0, lr=0.0, weight_decay=0.0,
             stream=None, pairs_per_system=0):
        return PrecondCfg(base_channels, steps, batch, crop, pairs_per_system, seed, lr,
                          weight_decay, _stream_ptr(stream))

    @staticmethod
    def harvest(grid: "Grid", omega: float, port: int = 0, npairs: int = 8, tol: float = 1e-8):
        """``fit_precond_harvest``: solver-generated pairs (e, r), each a
        complex128 tensor of shape (made, n_e); returns (e, r, iterations)."""
        torch = _torch()
        n = grid.n_edges
        e = torch.empty(npairs * n, dtype=torch.complex128, device=f"cuda:{grid.device}")
        r = torch.empty_like(e)
        made, iters = C.c_int(), C.c_int()
        check(lib().fit_precond_harvest(grid.h, float(omega), port, npairs, float(tol), _dptr(e),
                                        _dptr(r), C.byref(made), C.byref(iters)),
              "fit_precond_harvest")
        m = made.value
        return e[: m * n].view(m, n), r[: m * n].view(m, n), iters.value

    @classmethod
    def create(cls, base_channels: int = 16, seed: int = 0, device: int = 0):
        h = C.c_void_p()
        cfg = cls._cfg(base_channels=base_channels, seed=seed)
        check(lib().fit_precond_create(C.byref(cfg), device, C.byref(h)), "fit_precond_create")
        return cls(h, device)

    @classmethod
    def train(cls, grids: Sequence["Grid"], omegas: Sequence[float], **kw):
        gh = (C.c_void_p * len(grids))(*[g.h.value for g in grids])
        om = (C.c_double * len(omegas))(*[float(o) for o in omegas])
        cfg = cls._cfg(**kw)
        h = C.c_void_p()
        check(lib().fit_precond_train(gh, len(grids), om, len(omegas), C.byref(cfg), C.byref(h)),
              "fit_precond_train")
        return cls(h, grids[0].device)

    @staticmethod
    def train_history() -> np.ndarray:
        n = C.c_int()
        check(lib().fit_precond_train_history(None, 0, C.byref(n)), "fit_precond_train_history")
        out = (C.c_double * max(n.value, 1))()
        check(lib().fit_precond_train_history(out, n.value, C.byref(n)), "fit_precond_train_history")
        return np.array(out[: n.value])

    def save(self) -> bytes:
        n = C.c_size_t()
        check(lib().fit_precond_save(self.h, None, C.byref(n)), "fit_precond_save")
        buf = (C.c_char * n.value)()
        check(lib().fit_precond_save(self.h, buf, C.byref(n)), "fit_precond_save")
        return bytes(buf)

    @classmethod
    def load(cls, blob: bytes, device: int = 0):
        h = C.c_void_p()
        check(lib().fit_precond_load(blob, len(blob), device, C.byref(h)), "fit_precond_load")
        return cls(h, device)

    @staticmethod
    def blob_from_params(base_channels: int, params: np.ndarray) -> bytes:
        p = np.ascontiguousarray(params, dtype=np.float32)
        head = np.array([PRECOND_MAGIC], np.uint64).tobytes() + \
            np.array([base_channels, 0], np.int32).tobytes() + np.array([p.size], np.int64).tobytes()
        return head + p.tobytes()

    def params(self) -> np.ndarray:
        return np.frombuffer(self.save()[24:], dtype=np.float32).copy()

    def apply(self, grid: "Grid", omega: float, v, z=None, stream=None):
        torch = _torch()
        if z is None:
            z = torch.empty_like(v)
        check(lib().fit_precond_apply(self.h, grid.h, float(omega), _dptr(v), _dptr(z),
                                      _stream_ptr(stream)), "fit_precond_apply")
        return z

    def loss_grad(self, grid: "Grid", omega: float, r, e, stream=None):
        loss = C.c_double()
        n = self.params().size
        g = np.zeros(n, np.float32)
        check(lib().fit_precond_loss_grad(self.h, grid.h, float(omega), _dptr(r), _dptr(e),
                                          C.byref(loss), g.ctypes.data_as(C.c_void_p),
                                          _stream_ptr(stream)), "fit_precond_loss_grad")
        return loss.value, g

    def close(self):
        if getattr(self, "h", None):
            lib().fit_precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
