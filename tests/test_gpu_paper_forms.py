"""The paper's factorized operator and its diagonal preconditioner on the
GPU against the FP64 oracle (Sec. III: eq. (e2tt), the factor
calA = M_mu^{-1/2} C M_eps^{-1/2}, and eq. (Precond), the squared column
norms of calA), together with the other diagonal preconditioners of COCG
(the mass scaling of eq. (e2t) kept as a stored vector, and Jacobi).
"""
import numpy as np
import pytest

from oracle import fit_oracle as O
from paper_1705_08849_amd import devices as D
from paper_1705_08849_amd import fit
from tests._helpers import parity_devices, rand_c

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("name", sorted(parity_devices()))
def test_curl_curl_diagonal_matches_the_oracle(name):
    """K_ee = sum of M_nu over the four facets of edge e, every index."""
    dev = parity_devices()[name]
    g = fit.Grid(dev)
    kd = g.material_diag(3).cpu().numpy()
    ref = O.stiffness(dev).diagonal()
    assert np.all(kd.imag == 0)
    np.testing.assert_allclose(kd.real, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("name", sorted(parity_devices()))
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_factorized_operator_matches_the_oracle(name, dtype):
    """calA^T (calA x) - omega^2 x (eq. (e2tt)) element by element."""
    dev = parity_devices()[name]
    g = fit.Grid(dev)
    om = 2 * np.pi * 13e9
    x = rand_c(dev.n_edges, 7)
    if dtype == "c64":
        x = x.astype(np.complex64).astype(np.complex128)
        xd = _cuda(x.astype(np.complex64))
    else:
        xd = _cuda(x)
    y = g.matvec(om, xd, scaling="fact").cpu().numpy().astype(np.complex128)
    ref = O.matvec(dev, om, x, scaling="fact")
    tol = 1e-12 if dtype == "c128" else 1e-5
    assert np.linalg.norm(y - ref) <= tol * np.linalg.norm(ref)
    # the same operator as the symmetric scaling, up to rounding
    ys = g.matvec(om, xd, scaling="sym").cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(y - ys) <= 10 * tol * np.linalg.norm(ys)


def _oracle_diag(dev, om, kind):
    f = O.free_edges(dev)
    kd = O.stiffness(dev).diagonal()[f]
    if kind == "paper":
        # 1/P on the scaled system is S (1/P) S = 1/K_ee on the unscaled one
        s = O.sym_scaling(dev, om)
        return s * s / O.paper_diag_preconditioner(dev, om)
    if kind == "mass":
        s = O.sym_scaling(dev, om)
        return s * s
    return 1.0 / (kd + O.diagonal(dev, om)[f])


@pytest.mark.parametrize("kind", ["paper", "mass", "jacobi"])
def test_cocg_with_stored_diagonal_tracks_the_oracle(kind):
    """COCG with a stored diagonal preconditioner follows the oracle's
    preconditioned COCG step by step (recursive residual history)."""
    dev = D.layered_device(40, 36, 30, n_layers=4, n_strips=3, n_ports=1, seed=12)
    g = fit.Grid(dev)
    om = 2 * np.pi * 10e9
    src = D.port_source(dev, 0)
    nit = 80
    x, info = g.solve(om, _cuda(src), tol=1e-14, solver="cocg", diag=kind, max_iters=nit,
                      history=nit, check_every=2, raise_on_error=False)
    hg = info["history"]
    a = O.system_matrix(dev, om)
    _, _, _, hc = O.cocg(a, O.rhs(dev, om, src), tol=1e-14, maxiter=nit, history=True,
                         m=_oracle_diag(dev, om, kind))
    n = min(len(hg), len(hc))
    rel = np.abs(hg[:n] - hc[:n]) / hc[:n]
    print(f"{kind}: history gpu {hg[:4]} cpu {hc[:4]} max rel diff {rel.max():.2e}")
    assert n == nit and rel[:40].max() < 1e-8 and rel.max() < 1e-4


@pytest.mark.parametrize("kind", ["paper", "mass", "jacobi"])
def test_cocg_with_stored_diagonal_solves(kind):
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    for f in (2e9, 17e9):
        om = 2 * np.pi * f
        src = D.port_source(dev, 1)
        x, info = g.solve(om, _cuda(src), tol=1e-8, solver="cocg", diag=kind, max_iters=60000)
        rr = O.relative_residual(dev, om, src, x.cpu().numpy())
        print(f"{kind} {f / 1e9:.0f} GHz: iters {info['iterations']} relres {rr:.2e}")
        assert info["status_name"] == "FIT_OK" and rr <= 1e-8
        assert abs(rr - info["true_relres"]) <= 1e-9


def test_stored_mass_diagonal_follows_the_fused_path():
    """The stored mass diagonal and the fused symmetric-scaling path apply
    the same preconditioner (bit-level differences only from the order of
    the recomputation): equal iteration counts within a few per cent."""
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    om = 2 * np.pi * 9e9
    src = _cuda(D.port_source(dev, 0))
    x1, i1 = g.solve(om, src, tol=1e-8, solver="cocg")
    x2, i2 = g.solve(om, src, tol=1e-8, solver="cocg", diag="mass")
    print("fused", i1["iterations"], "stored", i2["iterations"])
    assert abs(i1["iterations"] - i2["iterations"]) <= 0.05 * i1["iterations"] + 2
    assert (torch.linalg.vector_norm(x1 - x2) / torch.linalg.vector_norm(x1)).item() < 1e-5


def test_stored_diagonal_needs_cocg():
    dev = D.layered_device(12, 10, 8, n_layers=2, n_strips=1, n_ports=1, seed=2)
    g = fit.Grid(dev)
    with pytest.raises(fit.FitError) as e:
        g.solve(2 * np.pi * 5e9, _cuda(D.port_source(dev, 0)), solver="bicgstab", diag="paper")
    assert e.value.status == fit.E_UNSUPPORTED


@pytest.mark.parametrize("method", ["cocr", "tfqmr", "cgs"])
def test_cocr_and_tfqmr_recurrences_track_the_oracle(method):
    """The further methods of the paper's comparison (Sec. IV) follow the
    oracle's textbook recurrences step by step on the scaled system:
    COCR's and CGS's recursive residuals, TFQMR's QMR bound tau
    sqrt(m + 1)."""
    dev = D.layered_device(40, 36, 30, n_layers=4, n_strips=3, n_ports=1, seed=12)
    g = fit.Grid(dev)
    om = 2 * np.pi * 10e9
    src = D.port_source(dev, 0)
    nit = 40
    x, info = g.solve(om, _cuda(src), tol=1e-14, solver=method, max_iters=nit, history=nit,
                      check_every=nit, raise_on_error=False)
    hg = info["history"]
    import scipy.sparse as sp
    s = O.sym_scaling(dev, om)
    a = (sp.diags(s) @ O.system_matrix(dev, om) @ sp.diags(s)).tocsr()
    b = s * O.rhs(dev, om, src)
    if method == "cocr":
        xs, _, _, hc = O.cocr(a, b, tol=1e-14, maxiter=nit, history=True)
    elif method == "tfqmr":
        rhat = O.shadow_vector(dev.n_edges)[O.free_edges(dev)]
        xs, _, _, hc = O.tfqmr(a, b, rhat, tol=1e-14, maxiter=nit, history=True)
    else:
        rhat = O.shadow_vector(dev.n_edges)[O.free_edges(dev)]
        xs, _, _, hc = O.cgs(a, b, rhat, tol=1e-14, maxiter=nit, history=True)
    n = min(len(hg), len(hc))
    rel = np.abs(hg[:n] - hc[:n]) / hc[:n]
    print(f"{method}: gpu {hg[:4]} cpu {hc[:4]} max rel diff {rel.max():.2e}")
    assert n == nit and rel[:20].max() < 1e-8 and rel.max() < 1e-4


@pytest.mark.parametrize("method", ["cocr", "tfqmr", "cgs"])
def test_cocr_and_tfqmr_solve(method):
    dev = D.layered_device(24, 20, 12, n_layers=3, n_strips=2, n_ports=2, seed=21)
    g = fit.Grid(dev)
    for f in (2e9, 17e9):
        om = 2 * np.pi * f
        src = D.port_source(dev, 0)
        x, info = g.solve(om, _cuda(src), tol=1e-8, solver=method, max_iters=60000)
        rr = O.relative_residual(dev, om, src, x.cpu().numpy())
        print(f"{method} {f / 1e9:.0f} GHz: iters {info['iterations']} refin "
              f"{info['refinements']} relres {rr:.2e}")
        assert info["status_name"] == "FIT_OK" and rr <= 1e-8
        assert abs(rr - info["true_relres"]) <= 1e-9
    # the tiny cavity against the direct solution
    dev, om, src = D.tiny_cavity_case()
    g = fit.Grid(dev)
    x, info = g.solve(om, _cuda(src), tol=1e-8, solver=method)
    xh = x.cpu().numpy()
    ref = O.solve_direct(dev, om, src)
    assert O.relative_residual(dev, om, src, xh) <= 1e-8
    assert np.linalg.norm(xh - ref) <= 1e-5 * np.linalg.norm(ref)
