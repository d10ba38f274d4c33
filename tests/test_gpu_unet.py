"""The learned FGMRES preconditioner on the GPU against its FP64 oracle.

Forward: the device applies z = s U(v/s) with bf16 storage and fp32
accumulation; the oracle takes the same storage roundings (bf16=True), so the
two agree up to the fp32 accumulation order (a rounding-boundary flip of a
stored bf16 value now and then), bar 1e-2 relative 2-norm.  Gradient: the
device back-propagates in bf16 (ReLU masks and per-layer gradients stored in
bf16), the oracle in fp64 through the same forward roundings; bar 3e-2
relative 2-norm per layer.
"""
import numpy as np
import pytest

from oracle import fit_oracle as O
from oracle import unet_oracle as U
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests._helpers import rand_c

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _dev():
    return D.layered_device(14, 11, 9, n_layers=3, n_strips=2, n_ports=1, seed=31)


def _params(c, seed):
    p = U.init_params(c, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    # nonzero biases so that every ReLU sees both signs
    off = 0
    for _, _, t, ci, co in U.layer_shapes(c):
        off += t * ci * co
        p[off: off + co] = rng.uniform(-0.1, 0.1, co)
        off += co
    return p.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("c", [8, 16])
def test_forward_matches_oracle(c):
    dev = _dev()
    g = fit.Grid(dev)
    p = _params(c, 3)
    pre = fit.Precond.load(fit.Precond.blob_from_params(c, p))
    np.testing.assert_array_equal(pre.params(), p.astype(np.float32))
    free = O.free_edges(dev)
    v = rand_c(dev.n_edges, 5) * free
    om = 2 * np.pi * 7e9
    z = pre.apply(g, om, _cuda(v)).cpu().numpy()
    ref = U.apply(dev, om, p, v, free, c=c, bf16=True)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print(f"c={c}: forward rel err {err:.2e}")
    assert err <= 1e-2
    assert np.all(z[~free] == 0)
    # degree-1 homogeneity holds on the device too (s scales, v/s does not)
    z2 = pre.apply(g, om, _cuda(4.0 * v)).cpu().numpy()
    assert np.linalg.norm(z2 - 4.0 * z) <= 1e-6 * np.linalg.norm(z2)


def test_gradient_matches_oracle():
    dev = _dev()
    g = fit.Grid(dev)
    c = 8
    p = _params(c, 7)
    pre = fit.Precond.load(fit.Precond.blob_from_params(c, p))
    free = O.free_edges(dev)
    e = rand_c(dev.n_edges, 8) * free
    om = 2 * np.pi * 4e9
    r = O.matvec(dev, om, e)
    loss, grad = pre.loss_grad(g, om, _cuda(r), _cuda(e))
    ref_loss, ref_grad = U.loss_and_grad(dev, om, p, r, e, free, c=c, bf16=True)
    print(f"loss gpu {loss:.6e} oracle {ref_loss:.6e}")
    assert abs(loss - ref_loss) <= 1e-2 * ref_loss
    off = 0
    for name, _, t, ci, co in U.layer_shapes(c):
        n = t * ci * co + co
        gg, rr = grad[off: off + n].astype(np.float64), ref_grad[off: off + n]
        err = np.linalg.norm(gg - rr) / max(np.linalg.norm(rr), 1e-30)
        print(f"{name:6s} grad rel err {err:.2e} (|g| {np.linalg.norm(rr):.3e})")
        assert err <= 3e-2, name
        off += n


def test_save_load_roundtrip_and_determinism():
    dev = _dev()
    g = fit.Grid(dev)
    pre = fit.Precond.create(base_channels=8, seed=11)
    blob = pre.save()
    pre2 = fit.Precond.load(blob)
    assert pre2.save() == blob
    v = _cuda(rand_c(dev.n_edges, 3) * O.free_edges(dev))
    z1 = pre.apply(g, 1e10, v)
    z2 = pre2.apply(g, 1e10, v)
    assert torch.equal(z1, z2)
    with pytest.raises(fit.FitError):
        fit.Precond.load(blob[:100])


def test_training_reduces_the_loss():
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    omegas = list(D.log_spaced_omegas(4, 2e9, 20e9))
    pre = fit.Precond.train([g], omegas, base_channels=8, steps=200, batch=2, crop=12, seed=5,
                            lr=5e-3)
    h = fit.Precond.train_history()
    assert h.size == 200 and np.all(np.isfinite(h))
    first, last = h[:20].mean(), h[-20:].mean()
    print(f"training loss: first 20 steps {first:.4f}, last 20 steps {last:.4f}")
    assert last < 0.95 * first
    # same seed, same history: the training step is deterministic
    pre2 = fit.Precond.train([g], omegas, base_channels=8, steps=5, batch=2, crop=12, seed=5,
                             lr=5e-3)
    np.testing.assert_array_equal(fit.Precond.train_history(), h[:5])


def test_fgmres_with_the_network_tracks_the_oracle():
    """FGMRES(30) with the network as right preconditioner follows the
    oracle's flexible GMRES with the oracle network: same true residual
    after 20 Arnoldi steps (up to the bf16 accumulation-order noise)."""
    dev = _dev()
    g = fit.Grid(dev)
    c = 8
    p = _params(c, 13)
    pre = fit.Precond.load(fit.Precond.blob_from_params(c, p))
    om = 2 * np.pi * 6e9
    src = D.port_source(dev, 0)
    nit = 20
    x, info = g.solve(om, _cuda(src), tol=1e-14, solver="fgmres", precond=pre, scaling="none",
                      max_iters=nit, raise_on_error=False)
    free = O.free_edges(dev)

    def m(vf):
        return U.apply(dev, om, p, O.embed(dev, vf), free, c=c, bf16=True)[free]

    xs, it, rc = O.gmres(O.system_matrix(dev, om), O.rhs(dev, om, src), restart=30, tol=1e-14,
                         maxiter=nit, precond=m)
    xg = x.cpu().numpy()
    r_gpu = O.relative_residual(dev, om, src, xg)
    xe = O.embed(dev, xs)
    dx = np.linalg.norm(xg - xe) / np.linalg.norm(xe)
    print(f"FGMRES+U-Net after {nit} steps: relres gpu {r_gpu:.9e} oracle {rc:.9e}; x diff {dx:.2e}")
    assert it == nit and info["iterations"] == nit
    # The residual after a fixed number of steps is the well-conditioned
    # quantity (the iterate of a slowly converging run is not): bar 1e-3,
    # the size of one bf16 storage flip in a preconditioner output.  Plain
    # GMRES reaches a very different residual, so the bar tells them apart.
    assert abs(r_gpu - rc) <= 1e-3 * rc
    _, _, r_plain = O.gmres(O.system_matrix(dev, om), O.rhs(dev, om, src), restart=30, tol=1e-14,
                            maxiter=nit)
    assert abs(r_plain - rc) > 0.1 * rc


@pytest.mark.timeout(600)
def test_full_size_family_device():
    """The 192x192x96-cell family device at full size, the application the
    benchmark times (c = 16): element by element against the oracle's FP64
    forward pass over the whole padded grid (the same bf16 storage
    roundings), and exactly equivariant to a power-of-two scaling of the
    input (z = s U(v / s) with s the rms of v, so v -> 2 v gives z -> 2 z
    bit for bit)."""
    dev = D.learned_family_device(9000)
    g = fit.Grid(dev)
    c = 16
    p = U.init_params(c, seed=1).astype(np.float32).astype(np.float64)
    pre = fit.Precond.load(fit.Precond.blob_from_params(c, p))
    free = O.free_edges(dev)
    v = rand_c(dev.n_edges, 41) * free
    om = 2 * np.pi * 1e10
    vd = _cuda(v)
    z1 = pre.apply(g, om, vd).cpu().numpy()
    z2 = pre.apply(g, om, 2 * vd).cpu().numpy()
    assert np.all(np.isfinite(z1))
    assert np.all(z1[~free] == 0)
    assert np.linalg.norm(z1) > 0
    np.testing.assert_array_equal(z2, 2 * z1)
    zr = U.apply(dev, om, p, v, free, c=c, bf16=True)
    rel = np.linalg.norm(z1 - zr) / np.linalg.norm(zr)
    print(f"192x192x96 c=16 application vs oracle: rel err {rel:.3e}")
    # the small-grid bar: fp32 accumulation order can flip a stored bf16 value
    assert rel <= 1e-2


def test_solver_generated_pairs_are_residual_error_pairs():
    """fit_precond_harvest: e_k = x* - x_k from COCG iterates of the port
    excitation and r_k = A e_k, checked by the oracle (r_k against its own
    operator applied to e_k, x* against its residual), with the errors taken
    strictly before convergence (every pair nonzero)."""
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    om = 2 * np.pi * 9e9
    e, r, iters = fit.Precond.harvest(g, om, port=1, npairs=6, tol=1e-9)
    assert e.shape[0] == 6 and iters > 0
    eh, rh = e.cpu().numpy(), r.cpu().numpy()
    src = D.port_source(dev, 1)
    b = np.zeros(dev.n_edges, complex)
    b[O.free_edges(dev)] = O.rhs(dev, om, src)
    for k in range(6):
        ref = O.matvec(dev, om, eh[k])
        assert np.linalg.norm(rh[k] - ref) <= 1e-12 * np.linalg.norm(ref)
        assert np.linalg.norm(eh[k]) > 0 and np.all(eh[k][~O.free_edges(dev)] == 0)
        # x_k = x* - e_k is an iterate: b - A x_k = r(x*) + r_k with r(x*) <= 1e-9 |b|
        assert np.linalg.norm(rh[k]) > 1e-6 * np.linalg.norm(b)
    # x* itself: the last error plus the iterate it came from is a solution
    x, _ = g.solve(om, _cuda(src), tol=1e-9, solver="cocg")
    assert O.relative_residual(dev, om, src, x.cpu().numpy()) <= 1e-9


def test_training_on_solver_generated_pairs_lowers_the_loss():
    devs = [D.layered_device(28, 24, 16, n_layers=3, n_strips=2, n_ports=1, seed=s)
            for s in (1000, 1001)]
    grids = [fit.Grid(d) for d in devs]
    pre = fit.Precond.train(grids, [2 * np.pi * 5e9, 2 * np.pi * 20e9], base_channels=8,
                            steps=120, batch=4, crop=16, seed=5, pairs_per_system=4)
    h = fit.Precond.train_history()
    assert len(h) == 120 and np.all(np.isfinite(h))
    assert h[-20:].mean() < h[:10].mean()


def test_learned_fgmres_falls_back_to_cocg_on_stagnation():
    """A network that does not precondition (seeded random weights) makes
    FGMRES(30) stall; after 10 restart cycles without halving the true
    residual the solve continues with the mass-preconditioned COCG from the
    current iterate and meets the tolerance, reporting the fallback."""
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    pre = fit.Precond.create(base_channels=8, seed=1)
    om = 2 * np.pi * 9e9
    src = D.port_source(dev, 0)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver="fgmres", precond=pre, max_iters=20000)
    rr = O.relative_residual(dev, om, src, x.cpu().numpy())
    print(f"fgmres+net: iters {info['iterations']} fell back {info['fell_back']} relres {rr:.2e}")
    assert info["status_name"] == "FIT_OK" and info["fell_back"] == 1
    assert rr <= 1e-8 and abs(rr - info["true_relres"]) <= 1e-9
    # the learned stage spent at most the stall window before handing over
    _, plain = g.solve(om, _cuda(src), tol=1e-8, solver="cocg")
    assert info["iterations"] <= plain["iterations"] + 30 * 12


def test_what_the_trained_network_gains_on_a_held_out_device():
    """The network trained on solver-generated pairs of two seeded devices,
    used on a third (held out) as FGMRES(30)'s right preconditioner: the
    residual after 60 steps beside plain GMRES(30)'s, and the iterations to
    1e-8 beside COCG's.  What it gains is reported, not assumed (on these
    graded devices it gains nothing, see the printed line); what the test
    asserts is the contract around it: the learned solve meets the
    tolerance (through its COCG fallback if FGMRES stalls), and a
    correction that would raise the true residual is never kept."""
    devs = [D.layered_device(28, 24, 16, n_layers=3, n_strips=2, n_ports=1, seed=s)
            for s in (1000, 1001, 1002)]
    om = 2 * np.pi * 8e9
    pre = fit.Precond.train([fit.Grid(d) for d in devs[:2]], [om], base_channels=8, steps=150,
                            batch=4, crop=16, seed=7, pairs_per_system=6)
    dev = devs[2]
    g = fit.Grid(dev)
    src = _cuda(D.port_source(dev, 0))
    _, learned60 = g.solve(om, src, tol=1e-8, solver="fgmres", precond=pre, max_iters=60,
                           raise_on_error=False)
    _, plain60 = g.solve(om, src, tol=1e-8, solver="gmres", max_iters=60, raise_on_error=False)
    x, learned = g.solve(om, src, tol=1e-8, solver="fgmres", precond=pre, max_iters=40000)
    _, cocg = g.solve(om, src, tol=1e-8, solver="cocg", max_iters=40000)
    rr = O.relative_residual(dev, om, D.port_source(dev, 0), x.cpu().numpy())
    print(f"after 60 steps: FGMRES+net {learned60['true_relres']:.3e}, GMRES(30) "
          f"{plain60['true_relres']:.3e}; to 1e-8: FGMRES+net {learned['iterations']} it "
          f"(fell back {learned['fell_back']}), COCG {cocg['iterations']} it; gain "
          f"{cocg['iterations'] - learned['iterations']} iterations")
    assert learned["status_name"] == "FIT_OK" and rr <= 1e-8
    assert learned60["true_relres"] <= 1.0 and plain60["true_relres"] <= 1.0
