"""FP64 CPU oracle of the learned right preconditioner (a 3-level 3D U-Net).

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports or calls this
module; only the tests, the smoke check and the benchmark's CPU baseline do.

The paper applies its Krylov solvers without a learned component; this
network is the learned preconditioner that the flexible GMRES of the paper's
solver comparison (Sec. IV) accepts as its right preconditioner: any
nonlinear map z = M(v) is admissible there because FGMRES stores the
preconditioned directions.  Its definition is this module:

  * Spatial layout: the node grid (Nz, Ny, Nx) of the edge vector, channels
    last; the three edge components of a node are its channels.
  * Input, 12 channels per node: Re/Im of the x, y and z edge values of v/s
    with s = rms of v over the free edges; eps_r / 12 and
    (log10(sigma + 1e-3) + 3) / 11 of the cell owned by the node (cell
    (min(i, ncx-1), min(j, ncy-1), min(k, ncz-1))); log10(f / 1 GHz) / 1.6;
    log10(h / 100 um) of that cell's widths h = dx, dy, dz (the local mesh
    scale, which sets the size of the curl-curl term).
  * Network (c = base channels): enc1a, enc1b (conv3, 12->c->c);
    down1 (2x2x2 stride 2, c->2c); enc2a, enc2b (conv3, 2c); down2 (2c->4c);
    bot_a, bot_b (conv3, 4c); up2 (transposed 2x2x2 stride 2, 4c->2c);
    dec2a (conv3 on [up2, enc2b] = 4c -> 2c), dec2b (2c); up1 (2c->c);
    dec1a (conv3 on [up1, enc1b] = 2c -> c), dec1b (c); head (1x1x1, c->6).
    ReLU after every layer but the head.  conv3 pads with zeros.
  * Output: z = s * (y0 + j y1, y2 + j y3, y4 + j y5) per node, 0 on masked
    edges.  The spatial grid is zero-padded at its upper end to a multiple
    of 4 before the network and cropped back after it.
  * Weights: per layer w[tap][ci][co] and b[co]; conv3 tap =
    (dz+1)*9 + (dy+1)*3 + (dx+1), 2x2x2 tap t = dz*4 + dy*2 + dx (z slowest).
    The flat parameter vector is every layer's w then b, in the order above.
  * Storage precision of the device network: bf16 activations and weights,
    fp32 accumulation and biases, fp32 head output.  `bf16=True` rounds at
    exactly those points (round to nearest even) so that the oracle takes
    the same storage decisions.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

LAYERS = [
    # name, kind, cin multiplier (of c; 0 = the 12 input channels), cout multiplier (0 = 6 outputs)
    ("enc1a", "conv3", 0, 1), ("enc1b", "conv3", 1, 1), ("down1", "down2", 1, 2),
    ("enc2a", "conv3", 2, 2), ("enc2b", "conv3", 2, 2), ("down2", "down2", 2, 4),
    ("bot_a", "conv3", 4, 4), ("bot_b", "conv3", 4, 4), ("up2", "up2", 4, 2),
    ("dec2a", "conv3", 4, 2), ("dec2b", "conv3", 2, 2), ("up1", "up2", 2, 1),
    ("dec1a", "conv3", 2, 1), ("dec1b", "conv3", 1, 1), ("head", "pw", 1, 0),
]
TAPS = {"conv3": 27, "down2": 8, "up2": 8, "pw": 1}
N_IN, N_OUT = 12, 6


def layer_shapes(c: int = 16):
    """[(name, kind, taps, cin, cout)] for base channels c."""
    out = []
    for name, kind, mi, mo in LAYERS:
        cin = N_IN if mi == 0 else mi * c
        cout = N_OUT if mo == 0 else mo * c
        out.append((name, kind, TAPS[kind], cin, cout))
    return out


def n_params(c: int = 16) -> int:
    return sum(t * ci * co + co for _, _, t, ci, co in layer_shapes(c))


def unflatten(flat: np.ndarray, c: int = 16):
    """Flat parameter vector -> {name: (w[tap][ci][co], b[co])} (float64)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, off = {}, 0
    for name, _, t, ci, co in layer_shapes(c):
        w = flat[off: off + t * ci * co].reshape(t, ci, co)
        off += t * ci * co
        b = flat[off: off + co]
        off += co
        out[name] = (w, b)
    assert off == flat.size
    return out


def init_params(c: int = 16, seed: int = 0) -> np.ndarray:
    """He-uniform weights, zero biases (a seeded starting point for tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, _, t, ci, co in layer_shapes(c):
        lim = np.sqrt(6.0 / (t * ci))
        parts.append(rng.uniform(-lim, lim, t * ci * co))
        parts.append(np.zeros(co))
    return np.concatenate(parts)


def bf16_round(a) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), as float64."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    bias = 0x7FFF + ((bits >> 16) & 1)
    r = ((bits + bias) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out


# ---------------------------------------------------------------------------
# Layers on (Z, Y, X, C) float64 tensors.
# ---------------------------------------------------------------------------
def _nc(x):  # (Z, Y, X, C) -> (1, C, Z, Y, X)
    return x.permute(3, 0, 1, 2).unsqueeze(0)


def _cl(x):  # (1, C, Z, Y, X) -> (Z, Y, X, C)
    return x.squeeze(0).permute(1, 2, 3, 0)


def conv3(x, w, b):
    """out[z,y,x,co] = b[co] + sum_{taps, ci} x[z+dz, y+dy, x+dx, ci] w[tap, ci, co]."""
    t, ci, co = w.shape
    wt = w.reshape(3, 3, 3, ci, co).permute(4, 3, 0, 1, 2)  # (co, ci, kz, ky, kx)
    return _cl(F.conv3d(_nc(x), wt, b, padding=1))


def down2(x, w, b):
    """out[z,y,x,co] = b[co] + sum_{t, ci} x[2z+dz, 2y+dy, 2x+dx, ci] w[t, ci, co]."""
    t, ci, co = w.shape
    wt = w.reshape(2, 2, 2, ci, co).permute(4, 3, 0, 1, 2)
    return _cl(F.conv3d(_nc(x), wt, b, stride=2))


def up2(x, w, b):
    """out[2z+dz, 2y+dy, 2x+dx, co] = b[co] + sum_ci x[z, y, x, ci] w[t, ci, co]."""
    t, ci, co = w.shape
    wt = w.reshape(2, 2, 2, ci, co).permute(3, 4, 0, 1, 2)  # (ci, co, kz, ky, kx)
    return _cl(F.conv_transpose3d(_nc(x), wt, b, stride=2))


def pw(x, w, b):
    return x @ w[0] + b


LAYER_FN = {"conv3": conv3, "down2": down2, "up2": up2, "pw": pw}


def forward(params, x, bf16: bool = False):
    """U-Net forward on x (Z, Y, X, 12) with Z, Y, X multiples of 4 (torch
    float64 tensors; params from unflatten, as torch tensors or arrays).
    Returns the (Z, Y, X, 6) head output."""
    rnd = (lambda t: torch.from_numpy(bf16_round(t.detach().numpy())) + (t - t.detach())) if bf16 \
        else (lambda t: t)
    p = {k: (torch.as_tensor(w), torch.as_tensor(b)) for k, (w, b) in params.items()}
    if bf16:
        p = {k: (rnd(w), b) for k, (w, b) in p.items()}

    def lay(name, kind, h, relu=True):
        w, b = p[name]
        o = LAYER_FN[kind](h, w, b)
        return rnd(torch.relu(o)) if relu else o

    h = rnd(x)
    e1 = lay("enc1b", "conv3", lay("enc1a", "conv3", h))
    e2 = lay("enc2b", "conv3", lay("enc2a", "conv3", lay("down1", "down2", e1)))
    b3 = lay("bot_b", "conv3", lay("bot_a", "conv3", lay("down2", "down2", e2)))
    d2 = lay("dec2b", "conv3", lay("dec2a", "conv3", torch.cat([lay("up2", "up2", b3), e2], -1)))
    d1 = lay("dec1b", "conv3", lay("dec1a", "conv3", torch.cat([lay("up1", "up2", d2), e1], -1)))
    return lay("head", "pw", d1, relu=False)


# ---------------------------------------------------------------------------
# Preconditioner application on a device.
# ---------------------------------------------------------------------------
def node_materials(dev):
    """(eps_r, sigma) of the cell owned by each node, arrays (Nz, Ny, Nx)."""
    nx, ny, nz = dev.nodes
    i = np.minimum(np.arange(nx), dev.ncx - 1)
    j = np.minimum(np.arange(ny), dev.ncy - 1)
    k = np.minimum(np.arange(nz), dev.ncz - 1)
    ids = dev.cell_mat[np.ix_(k, j, i)]
    eps = np.array([m.eps_r for m in dev.materials])[ids]
    sig = np.array([m.sigma for m in dev.materials])[ids]
    return eps, sig


def features(dev, omega: float, v: np.ndarray, free: np.ndarray):
    """The 12 input channels (Nz, Ny, Nx, 12) for the edge vector v, and s."""
    nx, ny, nz = dev.nodes
    vf = np.where(free, v, 0.0)
    s = np.sqrt(np.sum(np.abs(vf) ** 2) / max(int(free.sum()), 1))
    vs = (vf / s if s > 0 else vf).reshape(nz, ny, nx, 3)
    eps, sig = node_materials(dev)
    x = np.zeros((nz, ny, nx, N_IN))
    x[..., 0:6:2] = vs.real
    x[..., 1:6:2] = vs.imag
    x[..., 6] = eps / 12.0
    x[..., 7] = (np.log10(sig + 1e-3) + 3.0) / 11.0
    x[..., 8] = np.log10(omega / (2 * np.pi) / 1e9) / 1.6
    i = np.minimum(np.arange(nx), dev.ncx - 1)
    j = np.minimum(np.arange(ny), dev.ncy - 1)
    k = np.minimum(np.arange(nz), dev.ncz - 1)
    x[..., 9] = np.log10(dev.dx[i] / 1e-4)[None, None, :]
    x[..., 10] = np.log10(dev.dy[j] / 1e-4)[None, :, None]
    x[..., 11] = np.log10(dev.dz[k] / 1e-4)[:, None, None]
    return x, s


def pad4(x):
    z, y, w = x.shape[:3]
    pz, py, px = (-z) % 4, (-y) % 4, (-w) % 4
    return np.pad(x, ((0, pz), (0, py), (0, px), (0, 0)))


def apply(dev, omega: float, flat_params: np.ndarray, v: np.ndarray, free: np.ndarray,
          c: int = 16, bf16: bool = True) -> np.ndarray:
    """z = s * U(v / s) on the free edges (Sec. IV flexible GMRES right
    preconditioner), as an n_e complex vector."""
    nx, ny, nz = dev.nodes
    x, s = features(dev, omega, v, free)
    if s == 0:
        return np.zeros_like(v)
    y = forward(unflatten(flat_params, c), torch.from_numpy(pad4(x)), bf16=bf16).detach().numpy()
    y = y[:nz, :ny, :nx]
    z = (y[..., 0:6:2] + 1j * y[..., 1:6:2]).reshape(-1) * s
    return np.where(free, z, 0.0)


def loss_and_grad(dev, omega: float, flat_params: np.ndarray, r: np.ndarray, e: np.ndarray,
                  free: np.ndarray, c: int = 16, bf16: bool = True):
    """Training objective for one (residual r, error e) pair: the mean over
    free edges of |U(r / s_r) - e / s_e|^2 (real and imaginary parts summed),
    and its gradient with respect to the flat parameters.  With bf16=True the
    storage roundings are applied in the forward pass and passed straight
    through in the backward pass."""
    nx, ny, nz = dev.nodes
    x, _ = features(dev, omega, r, free)
    fe = np.where(free, e, 0.0)
    se = np.sqrt(np.sum(np.abs(fe) ** 2) / max(int(free.sum()), 1))
    t = (fe / se).reshape(nz, ny, nx, 3)
    tgt = np.zeros((nz, ny, nx, N_OUT))
    tgt[..., 0:6:2] = t.real
    tgt[..., 1:6:2] = t.imag
    m = np.repeat(free.reshape(nz, ny, nx, 3), 2, axis=-1).astype(np.float64)
    flat = torch.tensor(flat_params, dtype=torch.float64, requires_grad=True)
    params = {}
    off = 0
    for name, _, tp, ci, co in layer_shapes(c):
        w = flat[off: off + tp * ci * co].reshape(tp, ci, co)
        off += tp * ci * co
        params[name] = (w, flat[off: off + co])
        off += co
    y = forward(params, torch.from_numpy(pad4(x)), bf16=bf16)[:nz, :ny, :nx]
    mt = torch.from_numpy(m)
    nfree = float(m.sum() / 2)
    loss = torch.sum(mt * (y - torch.from_numpy(tgt)) ** 2) / nfree
    loss.backward()
    return float(loss.detach()), flat.grad.numpy().copy()
