"""Pins of the U-Net preconditioner oracle (CPU).

The library-backed layers are checked against brute-force loops written from
their index definitions, against adjoint identities that tie the strided,
transposed and flipped forms to each other, and the autograd gradient
against central finite differences; the bf16 emulation against torch's own
bfloat16 conversion.
"""
import numpy as np
import pytest
import torch

from oracle import fit_oracle as O
from oracle import unet_oracle as U
from paper_1705_08849_amd import devices as D


def _rand(shape, seed):
    return np.random.Generator(np.random.PCG64(seed)).uniform(-1, 1, shape)


def _brute_conv3(x, w, b):
    Z, Y, X, ci = x.shape
    co = w.shape[2]
    out = np.tile(b, (Z, Y, X, 1)).astype(float)
    for z in range(Z):
        for y in range(Y):
            for xx in range(X):
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            zz, yy, x2 = z + dz, y + dy, xx + dx
                            if 0 <= zz < Z and 0 <= yy < Y and 0 <= x2 < X:
                                tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                out[z, y, xx] += x[zz, yy, x2] @ w[tap]
    return out


def test_conv3_matches_brute_force():
    x, w, b = _rand((3, 4, 5, 2), 1), _rand((27, 2, 3), 2), _rand(3, 3)
    got = U.conv3(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    np.testing.assert_allclose(got, _brute_conv3(x, w, b), rtol=0, atol=1e-12)


def test_down2_and_up2_match_brute_force():
    x, w, b = _rand((4, 2, 6, 3), 4), _rand((8, 3, 2), 5), _rand(2, 6)
    got = U.down2(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b)).numpy()
    ref = np.zeros((2, 1, 3, 2)) + b
    for z in range(2):
        for y in range(1):
            for xx in range(3):
                for t in range(8):
                    dz, dy, dx = t // 4, (t // 2) % 2, t % 2
                    ref[z, y, xx] += x[2 * z + dz, 2 * y + dy, 2 * xx + dx] @ w[t]
    np.testing.assert_allclose(got, ref, atol=1e-12)
    xs, wu, bu = _rand((2, 1, 3, 3), 7), _rand((8, 3, 2), 8), _rand(2, 9)
    got = U.up2(torch.from_numpy(xs), torch.from_numpy(wu), torch.from_numpy(bu)).numpy()
    ref = np.zeros((4, 2, 6, 2)) + bu
    for z in range(2):
        for y in range(1):
            for xx in range(3):
                for t in range(8):
                    dz, dy, dx = t // 4, (t // 2) % 2, t % 2
                    ref[2 * z + dz, 2 * y + dy, 2 * xx + dx] += xs[z, y, xx] @ wu[t]
    np.testing.assert_allclose(got, ref, atol=1e-12)


def test_adjoint_identities():
    """<up2(x; w), y> = <x, down2(y; w^T)> and <conv3(x; w), y> =
    <x, conv3(y; flip(w)^T)>: the backward-data forms used by training."""
    T = torch.from_numpy
    x, y = _rand((2, 3, 2, 4), 10), _rand((4, 6, 4, 3), 11)
    w = _rand((8, 4, 3), 12)
    z0 = np.zeros(3)
    lhs = np.sum(U.up2(T(x), T(w), T(z0)).numpy() * y)
    rhs = np.sum(x * U.down2(T(y), T(w.transpose(0, 2, 1).copy()), T(np.zeros(4))).numpy())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    x, y = _rand((3, 4, 5, 2), 13), _rand((3, 4, 5, 3), 14)
    w = _rand((27, 2, 3), 15)
    wf = w[::-1].transpose(0, 2, 1).copy()
    lhs = np.sum(U.conv3(T(x), T(w), T(z0)).numpy() * y)
    rhs = np.sum(x * U.conv3(T(y), T(wf), T(np.zeros(2))).numpy())
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_bf16_rounding_matches_torch():
    v = np.concatenate([_rand(10000, 16) * 10.0 ** np.arange(-20, 20, 4).repeat(1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(U.bf16_round(v), ref)


def _tiny_dev():
    return D.layered_device(6, 5, 4, n_layers=2, n_strips=1, n_ports=1, seed=3)


def test_gradient_matches_finite_differences():
    dev = _tiny_dev()
    c = 2
    p = U.init_params(c, seed=1)
    p += 0.05 * _rand(p.size, 2)  # nonzero biases
    free = O.free_edges(dev)
    r = (_rand(dev.n_edges, 3) + 1j * _rand(dev.n_edges, 4)) * free
    e = (_rand(dev.n_edges, 5) + 1j * _rand(dev.n_edges, 6)) * free
    om = 2 * np.pi * 5e9
    loss, g = U.loss_and_grad(dev, om, p, r, e, free, c=c, bf16=False)
    rng = np.random.Generator(np.random.PCG64(9))
    for idx in rng.choice(p.size, 12, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        lp, _ = U.loss_and_grad(dev, om, pp, r, e, free, c=c, bf16=False)
        lm, _ = U.loss_and_grad(dev, om, pm, r, e, free, c=c, bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(fd)), (idx, fd, g[idx])


def test_features_and_homogeneity():
    dev = D.cavity(4, 4, 4)
    free = O.free_edges(dev)
    v = (_rand(dev.n_edges, 20) + 1j * _rand(dev.n_edges, 21)) * free
    om = 2 * np.pi * 10e9
    x, s = U.features(dev, om, v, free)
    assert np.allclose(x[..., 6], 1.0 / 12.0) and np.allclose(x[..., 7], 0.0)
    assert np.allclose(x[..., 8], 1.0 / 1.6)
    assert np.allclose(x[..., 9:12], 1.0)  # 1 mm cells: log10(1 mm / 100 um)
    assert abs(np.mean(np.sum(x[..., :6] ** 2, -1)) * 125 / free.sum() - 1.0) < 1e-12
    p = U.init_params(4, seed=3)
    z1 = U.apply(dev, om, p, v, free, c=4, bf16=False)
    z2 = U.apply(dev, om, p, 3.7 * v, free, c=4, bf16=False)
    assert np.allclose(z2, 3.7 * z1, rtol=1e-12, atol=0)
    assert np.all(z1[~free] == 0)


def test_parameter_layout():
    assert U.n_params(16) == sum(t * ci * co + co for _, _, t, ci, co in U.layer_shapes(16))
    shapes = {n: (t, ci, co) for n, _, t, ci, co in U.layer_shapes(16)}
    assert shapes["enc1a"] == (27, 12, 16) and shapes["dec2a"] == (27, 64, 32)
    assert shapes["up2"] == (8, 64, 32) and shapes["head"] == (1, 16, 6)
