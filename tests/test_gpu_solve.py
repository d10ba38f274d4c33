"""GPU solves against the FP64 oracle (Sec. II eq. (e2); Sec. IV solvers).

Every solution must reach a true relative residual <= 1e-8 measured by the
oracle's own assembled matrix (or, at full size, on sampled rows computed
one by one on local crops); the forward error against the oracle's direct
solution is reported, not thresholded beyond a loose sanity bound, because
any x meeting the residual bound is a correct answer.
"""
import os

import numpy as np
import pytest

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests import _helpers as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _small_device():
    return D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)


@pytest.mark.parametrize("solver,scaling,precision", [
    ("bicgstab", "none", "fp64"), ("bicgstab", "sym", "fp64"),
    ("gmres", "sym", "fp64"), ("fgmres", "sym", "fp64"),
    ("bicgstab", "sym", "mixed"), ("gmres", "sym", "mixed"),
])
def test_tiny_cavity_case(solver, scaling, precision):
    dev, om, src = D.tiny_cavity_case()
    g = fit.Grid(dev)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver=solver, scaling=scaling,
                      precision=precision)
    xh = x.cpu().numpy()
    rr = O.relative_residual(dev, om, src, xh)
    ref = O.solve_direct(dev, om, src)
    fe = np.linalg.norm(xh - ref) / np.linalg.norm(ref)
    print(f"{solver}/{scaling}/{precision}: iters {info['iterations']} relres {rr:.2e} "
          f"(gpu {info['true_relres']:.2e}) forward err {fe:.2e}")
    assert rr <= 1e-8 and info["true_relres"] <= 1e-8
    assert abs(rr - info["true_relres"]) <= 1e-9
    assert fe < 1e-5
    assert np.all(xh[~O.free_edges(dev)] == 0)


@pytest.mark.parametrize("solver,precision", [("gmres", "fp64"), ("fgmres", "fp64")])
def test_restarted_gmres_tracks_the_oracle(solver, precision):
    """On graded layered devices restarted GMRES(30) stagnates (it does on
    the oracle too); after the same number of Arnoldi steps the GPU's true
    residual must match the oracle GMRES(30)'s."""
    dev = _small_device()
    g = fit.Grid(dev)
    om = 2 * np.pi * 17e9
    src = D.port_source(dev, 0)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver=solver, precision=precision,
                      max_iters=300, raise_on_error=False)
    a = O.system_matrix(dev, om)
    s = O.sym_scaling(dev, om)
    import scipy.sparse as sp
    xs, it, _ = O.gmres(sp.diags(s) @ a @ sp.diags(s), s * O.rhs(dev, om, src), restart=30,
                        tol=1e-12, maxiter=300)
    r_cpu = O.relative_residual(dev, om, src, O.embed(dev, s * xs))
    r_gpu = O.relative_residual(dev, om, src, x.cpu().numpy())
    print(f"{solver}: 300 steps, relres gpu {r_gpu:.6e} oracle {r_cpu:.6e}")
    assert it == 300 and info["iterations"] == 300
    assert abs(r_gpu - r_cpu) <= 1e-6 * r_cpu
    assert abs(info["true_relres"] - r_gpu) <= 1e-9


def _bicgstab_history(a, b, nit, rhat):
    """Recursive residual norms of the textbook BiCGStab recurrences."""
    x = np.zeros_like(b)
    r = b.copy()
    rh = rhat.copy()
    rho_old = al = om = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    out = []
    for _ in range(nit):
        rho = np.vdot(rh, r)
        beta = (rho / rho_old) * (al / om)
        p = r + beta * (p - om * v)
        v = a @ p
        al = rho / np.vdot(rh, v)
        s = r - al * v
        t = a @ s
        om = np.vdot(t, s) / np.vdot(t, t)
        x = x + al * p + om * s
        r = s - om * t
        rho_old = rho
        out.append(np.linalg.norm(r) / np.linalg.norm(b))
    return x, np.array(out)


@pytest.mark.parametrize("shape,f", [((40, 36, 30), 10e9), ((64, 64, 48), 3e9)])
def test_bicgstab_recurrences_track_the_oracle(shape, f):
    """The fused device BiCGStab follows the textbook recurrences: its
    recursive residual history matches the oracle's step by step until
    rounding differences are amplified."""
    dev = D.layered_device(*shape, n_layers=4, n_strips=3, n_ports=1, seed=12)
    g = fit.Grid(dev)
    om = 2 * np.pi * f
    src = D.port_source(dev, 0)
    nit = 60
    # a single poll, at the cap: the returned x is the last iterate (with
    # more polls the solver would hand back the best polled one instead)
    x, info = g.solve(om, _cuda(src), tol=1e-14, max_iters=nit, history=nit, check_every=nit,
                      raise_on_error=False)
    hg = info["history"]
    a = O.system_matrix(dev, om)
    s = O.sym_scaling(dev, om)
    import scipy.sparse as sp
    rhat = O.shadow_vector(dev.n_edges)[O.free_edges(dev)]
    xs, hc = _bicgstab_history((sp.diags(s) @ a @ sp.diags(s)).tocsr(), s * O.rhs(dev, om, src),
                               nit, rhat)
    n = min(len(hg), len(hc))
    rel = np.abs(hg[:n] - hc[:n]) / hc[:n]
    print("history gpu", hg[:8], "\n        cpu", hc[:8], "\n max rel diff first 30:", rel[:30].max())
    assert n == nit
    assert rel[:20].max() < 1e-8 and rel[:30].max() < 1e-4
    r_gpu = O.relative_residual(dev, om, src, x.cpu().numpy())
    r_cpu = O.relative_residual(dev, om, src, O.embed(dev, s * xs))
    print("true relres after", nit, "steps: gpu", r_gpu, "cpu", r_cpu)
    # a correction that increases the true residual is rolled back (x = 0)
    expect = min(r_cpu, 1.0)
    assert abs(r_gpu - expect) <= 1e-3 * expect + 1e-12


@pytest.mark.parametrize("shape,f", [((40, 36, 30), 10e9), ((64, 64, 48), 3e9)])
def test_cocg_recurrences_track_the_oracle(shape, f):
    dev = D.layered_device(*shape, n_layers=4, n_strips=3, n_ports=1, seed=12)
    g = fit.Grid(dev)
    om = 2 * np.pi * f
    src = D.port_source(dev, 0)
    nit = 80
    x, info = g.solve(om, _cuda(src), tol=1e-14, solver="cocg", max_iters=nit, history=nit,
                      check_every=2, raise_on_error=False)
    hg = info["history"]
    # COCG with the symmetric scaling runs on the unscaled operator with the
    # diagonal preconditioner S^2 = 1/M_eps,c
    a = O.system_matrix(dev, om)
    s = O.sym_scaling(dev, om)
    xs, it, _, hc = O.cocg(a, O.rhs(dev, om, src), tol=1e-14, maxiter=nit, history=True,
                           m=s * s)
    n = min(len(hg), len(hc))
    rel = np.abs(hg[:n] - hc[:n]) / hc[:n]
    print("cocg history gpu", hg[:6], "\n             cpu", hc[:6], "\n max rel diff:", rel.max())
    assert n == nit and rel[:40].max() < 1e-8 and rel.max() < 1e-4


@pytest.mark.parametrize("solver,precision", [("bicgstab", "fp64"), ("bicgstab", "mixed"),
                                              ("cocg", "fp64"), ("cocg", "mixed")])
def test_graded_layered_device(solver, precision):
    dev = _small_device()
    g = fit.Grid(dev)
    for f in (2e9, 17e9):
        om = 2 * np.pi * f
        src = D.port_source(dev, 0)
        x, info = g.solve(om, _cuda(src), tol=1e-8, solver=solver, precision=precision)
        xh = x.cpu().numpy()
        rr = O.relative_residual(dev, om, src, xh)
        ref = O.solve_direct(dev, om, src)
        fe = np.linalg.norm(xh - ref) / np.linalg.norm(ref)
        print(f"{solver}/{precision} f={f:.1e}: iters {info['iterations']} refin "
              f"{info['refinements']} relres {rr:.2e} forward err {fe:.2e}")
        assert rr <= 1e-8
        assert fe < 1e-2


def test_port_voltages_and_reciprocity():
    dev = _small_device()
    assert len(dev.ports) == 2
    g = fit.Grid(dev)
    om = 2 * np.pi * 9e9
    z = np.zeros((2, 2), complex)
    for q in range(2):
        src = D.port_source(dev, q)
        x, info = g.solve(om, _cuda(src), tol=1e-10)
        u = g.port_voltages(x)[0]
        uo = O.port_voltages(dev, x.cpu().numpy())
        np.testing.assert_allclose(u, uo, rtol=1e-12, atol=1e-14 * np.abs(uo).max())
        z[:, q] = -u
    assert abs(z[0, 1] - z[1, 0]) <= 1e-6 * abs(z).max()
    assert z[0, 0].real >= 0 and z[1, 1].real >= 0


def test_port_network_from_gpu_solves_matches_the_oracle():
    """Loaded impedance from GPU solves (one per port, true residual 1e-10)
    -> fit_port_network -> unloaded Z and S, against the oracle's direct
    solves and definitions.  The bound follows the solve tolerance: a true
    residual of 1e-10 on this graded device leaves a forward error of the
    port voltages far below 1e-5 relative (the network is nearly lossless:
    the largest singular value of S is 1 - 1e-7, so passivity is checked to
    the same 1e-5 scale)."""
    dev = _small_device()
    g = fit.Grid(dev)
    om = 2 * np.pi * 9e9
    zl = np.zeros((2, 2), complex)
    for q in range(2):
        x, info = g.solve(om, _cuda(D.port_source(dev, q)), tol=1e-10)
        assert info["true_relres"] <= 1e-10
        zl[:, q] = -g.port_voltages(x)[0]
    z, s = fit.port_network(zl, 50.0)
    z_ref, s_ref = O.port_network(O.loaded_impedance(dev, om), 50.0)
    np.testing.assert_allclose(z, z_ref, rtol=1e-5, atol=1e-5 * abs(z_ref).max())
    np.testing.assert_allclose(s, s_ref, rtol=0, atol=1e-5)
    assert np.linalg.svd(s, compute_uv=False).max() <= 1.0 + 1e-5  # passive


def test_cavity_eigen_check_by_inverse_iteration():
    """TE101/TE011/TE110 of the 16 mm cavity from GPU solves: shifted inverse
    iteration at 13 GHz, then the Rayleigh quotient x^T K x / x^T M_eps x with
    K x = A(0) x and M_eps from the material export."""
    dev = D.cavity(16, 16, 16, 1e-3)
    g = fit.Grid(dev)
    om0 = 2 * np.pi * 13.0e9
    m_eps = g.material_diag(0).real.contiguous()
    mask = g.edge_mask().bool()
    src = torch.zeros(dev.n_edges, dtype=torch.complex128, device="cuda:0")
    for w, (i, j, k) in ((2, (8, 8, 8)), (0, (8, 8, 8)), (1, (8, 8, 8))):
        src[dev.edge_index(w, i, j, k)] = 1.0
    x = None
    for _ in range(4):
        x, info = g.solve(om0, src, tol=1e-10)
        rhs = torch.where(mask, m_eps * x, torch.zeros_like(x))
        src = (rhs / (-1j * om0)).contiguous()
        src = src / torch.linalg.vector_norm(src)
    kx = g.matvec(0.0, x)
    lam = (x @ kx) / (x @ (m_eps * x))
    f = float(np.sqrt(lam.real.item()) / (2 * np.pi))
    disc = O.C0 / (2 * np.pi) * np.sqrt(2) * (2 / 1e-3) * np.sin(np.pi / 32)
    cont = 0.5 * O.C0 * np.sqrt(2) / 16e-3
    print(f"Rayleigh quotient {f / 1e9:.7f} GHz, discrete {disc / 1e9:.7f}, continuous {cont / 1e9:.6f}")
    assert abs(f / disc - 1) < 1e-6
    assert abs(f / cont - 1) < 2e-3


def test_iteration_cap_returns_best_iterate():
    dev = _small_device()
    g = fit.Grid(dev)
    om = 2 * np.pi * 5e9
    src = D.port_source(dev, 0)
    x, info = g.solve(om, _cuda(src), tol=1e-8, max_iters=5, raise_on_error=False)
    assert info["status_name"] == "FIT_E_NOT_CONVERGED"
    # the best iterate: the 5-step correction, or x = 0 if that was worse
    assert 0 < info["true_relres"] <= 1
    rr = O.relative_residual(dev, om, src, x.cpu().numpy())
    assert abs(rr - info["true_relres"]) <= 1e-9


def test_masked_source_is_rejected():
    dev = _small_device()
    g = fit.Grid(dev)
    src = np.zeros(dev.n_edges, complex)
    src[dev.edge_index(0, 0, 0, 0)] = 1.0  # tangential to the -y/-z walls
    with pytest.raises(fit.FitError) as e:
        g.solve(2 * np.pi * 5e9, _cuda(src))
    assert e.value.status == fit.E_INVALID


def test_nan_source_reports_nan():
    dev = _small_device()
    g = fit.Grid(dev)
    src = D.port_source(dev, 0)
    src[dev.port_edges(0)[0]] = np.nan
    x, info = g.solve(2 * np.pi * 5e9, _cuda(src), raise_on_error=False)
    assert info["status_name"] == "FIT_E_NAN"


def test_singular_lossless_resonance_does_not_report_success():
    """At an exact discrete resonance of the lossless cavity the system is
    singular; the solver must not claim convergence."""
    dev = D.cavity(6, 5, 4, 1e-3, 1.2e-3, 0.9e-3)
    om = O.C0 * np.sqrt((2 / 1e-3) ** 2 * np.sin(np.pi / 12) ** 2
                        + (2 / 0.9e-3) ** 2 * np.sin(np.pi / 8) ** 2)  # mode (1, 0, 1)
    src = np.zeros(dev.n_edges, complex)
    src[dev.edge_index(1, 3, 2, 2)] = 1.0
    g = fit.Grid(dev)
    x, info = g.solve(om, _cuda(src), tol=1e-10, max_iters=3000, raise_on_error=False)
    assert info["status_name"] != "FIT_OK" or info["true_relres"] <= 1e-10
    if info["status_name"] == "FIT_OK":
        # a consistent right-hand side may still be solvable; then it must be a true solution
        assert O.relative_residual(dev, om, src, x.cpu().numpy()) <= 1e-9


def test_bitwise_determinism_and_graph_replay():
    dev = _small_device()
    g = fit.Grid(dev)
    om = 2 * np.pi * 11e9
    src = _cuda(D.port_source(dev, 1))
    x1, i1 = g.solve(om, src, check_every=20)
    x2, i2 = g.solve(om, src, check_every=20)
    x3, i3 = g.solve(om, src, check_every=20, use_graph=True)
    assert torch.equal(x1, x2) and i1["iterations"] == i2["iterations"]
    assert torch.equal(x1, x3) and i1["iterations"] == i3["iterations"]


def test_residual_history():
    dev, om, src = D.tiny_cavity_case()
    g = fit.Grid(dev)
    x, info = g.solve(om, _cuda(src), history=500)
    h = info["history"]
    assert len(h) == info["iterations"] and h[-1] < 1e-7


@pytest.mark.timeout(600)
def test_full_size_128_cubed_solution():
    """The 128^3-cell plain-method device at its seeded frequency: COCG in
    complex128 to 1e-8 in the benchmark's launch configuration; the oracle
    assembles the whole system and computes the true residual of the
    returned field."""
    dev = D.plain_device_128(2)
    f = D.log_uniform_frequency(2)
    om = 2 * np.pi * f
    # the launch configuration the benchmark times: its committed tile table
    fit.tune_load(os.path.join(ROOT, "paper_1705_08849_amd", "tune_gfx950.json"))
    g = fit.Grid(dev)
    src = D.port_source(dev, 0)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver="cocg", max_iters=60000)
    print(f"128^3 at {f / 1e9:.3f} GHz: iters {info['iterations']} relres {info['true_relres']:.2e} "
          f"time {info['time_ms']:.0f} ms", flush=True)
    assert info["status_name"] == "FIT_OK" and info["true_relres"] <= 1e-8
    xh = x.cpu().numpy()
    del x
    rr = O.relative_residual(dev, om, src, xh)
    print(f"oracle relres {rr:.3e}")
    assert rr <= 1e-8 and abs(rr - info["true_relres"]) <= 1e-3 * rr


@pytest.mark.timeout(900)
def test_full_size_256_interconnect_mixed_falls_back_and_converges():
    """The 256x256x128-cell interconnect (25.6M unknowns) at 10 GHz asked for
    the precision form: the complex64 inner COCG stalls on this graded mesh
    (its attainable accuracy is u32 times a condition number above 1e7), so
    the solve must report the fallback and finish in complex128 to a true
    residual of 1e-8, checked by the oracle on the whole assembled system."""
    dev = D.interconnect_256(3)
    om = 2 * np.pi * 10e9
    g = fit.Grid(dev)
    src = D.port_source(dev, 0)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver="cocg", precision="mixed", max_iters=80000)
    print(f"256x256x128 at 10 GHz mixed: iters {info['iterations']} refinements {info['refinements']} "
          f"fell back {info['fell_back']} relres {info['true_relres']:.2e} time {info['time_ms']:.0f} ms",
          flush=True)
    assert info["status_name"] == "FIT_OK" and info["true_relres"] <= 1e-8
    assert info["fell_back"] == 1
    xh = x.cpu().numpy()
    del x
    rr = O.relative_residual(dev, om, src, xh)
    print(f"oracle relres {rr:.3e}")
    assert rr <= 1e-8 and abs(rr - info["true_relres"]) <= 1e-3 * rr


@pytest.mark.skip(reason="complex64 inner iterations cannot contract the residual of the "
                         "256x256x128 graded interconnect: the mass-scaled operator's condition "
                         "number exceeds 1e7 (10 um cells), so u32 * kappa >= 1 and every inner "
                         "solve stalls; the solve finishes on the complex128 fallback, which "
                         "the test above checks")
def test_full_size_256_interconnect_precision_form_without_fallback():
    dev = D.interconnect_256(3)
    om = 2 * np.pi * 10e9
    g = fit.Grid(dev)
    x, info = g.solve(om, _cuda(D.port_source(dev, 0)), tol=1e-8, solver="cocg",
                      precision="mixed", max_iters=80000)
    assert info["fell_back"] == 0 and info["true_relres"] <= 1e-8


def test_precision_form_complex64_does_the_work():
    """Where the mass-scaled operator is conditioned well enough for FP32
    (uniform 100 um cells), the precision form converges to 1e-8 without
    falling back: every inner iteration runs in complex64 and only the
    residuals, corrections and the stopping test are complex128."""
    dev = D.layered_device(48, 40, 24, n_layers=3, n_strips=2, n_ports=1, seed=31, graded=False)
    g = fit.Grid(dev)
    src = D.port_source(dev, 0)
    for f in (3e9, 20e9):
        om = 2 * np.pi * f
        x, info = g.solve(om, _cuda(src), tol=1e-8, solver="cocg", precision="mixed",
                          max_iters=40000)
        xh = x.cpu().numpy()
        rr = O.relative_residual(dev, om, src, xh)
        # forward error against an FP64 solve to 1e-12 (the residual bar
        # above is the oracle's; a sparse direct solve of this size would
        # spend minutes of host time on a number that is only reported)
        x64, _ = g.solve(om, _cuda(src), tol=1e-12, solver="cocg", precision="fp64",
                         max_iters=40000)
        ref = x64.cpu().numpy()
        fe = np.linalg.norm(xh - ref) / np.linalg.norm(ref)
        print(f"{f / 1e9:.0f} GHz: iters {info['iterations']} refinements {info['refinements']} "
              f"fell back {info['fell_back']} relres {rr:.2e} forward error vs fp64 {fe:.2e}")
        assert info["fell_back"] == 0 and info["refinements"] >= 2
        assert rr <= 1e-8 and abs(rr - info["true_relres"]) <= 1e-9


@pytest.mark.parametrize("solver", ["bicgstab", "cocg", "gmres"])
def test_parallel_plate_closed_form(solver):
    """Electric plates at -z/+z, open side walls, three lossy z-layers on a
    graded grid, uniform current density: the solution is the closed-form
    uniform field per layer (E_k = -j omega J / (-omega^2 eps_k + j omega
    sigma_k)), which fixes the magnitude and phase of b = -j omega j."""
    dev = H.plate_device(True)
    g = fit.Grid(dev)
    for f in (0.3e9, 2e9):
        om = 2 * np.pi * f
        x, info = g.solve(om, _cuda(H.plate_source(dev)), tol=1e-11, solver=solver)
        ref = H.plate_closed_form(dev, om)
        fe = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"{solver} {f / 1e9} GHz: iters {info['iterations']} forward error {fe:.2e}")
        assert fe <= 1e-8
