"""Seeded synthetic FIT devices: problem *inputs* only.

This module describes problems; it computes nothing of the method itself.  A
device is the data the solver is handed in the paper's problem statement
(Sec. II, solution stages; Sec. IV, port excitation): the cell spacings of a
non-equidistant Cartesian grid, a material id per cell, the material table,
the lumped ports and which outer walls are electric (PEC) walls.  Both the
CPU oracle and the GPU path consume these objects, so nothing here may hold
the operator's arithmetic (no curl, no material averaging, no masks).

Shapes follow the paper's workloads (Sec. IV): strips over layered
substrates inside a PEC box, relative permittivities between 2 and 12,
lossy dielectrics, lumped ports from the ground wall to a strip, graded
meshes refined around every geometric feature.  All randomness comes from a
NumPy PCG64 generator seeded by the caller.

Index conventions (the paper's cell-by-cell (x, y, z) interleaving, eq.
(e12Nxyz)): nodes ``(i, j, k)`` with ``0 <= i < Nx = ncx + 1``; edge
``(w, i, j, k)`` (``w`` = 0, 1, 2 for x, y, z) sits at
``3 * (i + Nx * (j + Ny * k)) + w``.  ``cell_mat`` is stored as a C-ordered
``(ncz, ncy, ncx)`` array, i.e. cell ``(a, b, c)`` at ``a + ncx * (b + ncy * c)``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Speed of light in vacuum (exact SI value).  Only used here to place the
# tiny cavity case's frequency relative to its first continuous resonance.
C0 = 299_792_458.0


@dataclass
class Material:
    """One entry of the material table (Sec. II, material relations)."""

    eps_r: float = 1.0
    mu_r: float = 1.0
    sigma: float = 0.0  # S/m
    tan_delta: float = 0.0
    is_pec: bool = False


@dataclass
class Port:
    """Lumped port: the z-directed edges ``(i, j, k)`` for ``k0 <= k < k1``.

    The port drives 1 A through each of its edges and loads them with an
    internal impedance ``z0`` split evenly over the edges (Sec. IV)."""

    i: int
    j: int
    k0: int
    k1: int
    z0: float = 50.0


@dataclass
class Device:
    dx: np.ndarray
    dy: np.ndarray
    dz: np.ndarray
    cell_mat: np.ndarray  # uint8, shape (ncz, ncy, ncx)
    materials: List[Material]
    ports: List[Port] = field(default_factory=list)
    pec_walls: int = 0x3F  # bits: -x, +x, -y, +y, -z, +z
    name: str = "device"

    def __post_init__(self):
        self.dx = np.ascontiguousarray(self.dx, dtype=np.float64)
        self.dy = np.ascontiguousarray(self.dy, dtype=np.float64)
        self.dz = np.ascontiguousarray(self.dz, dtype=np.float64)
        self.cell_mat = np.ascontiguousarray(self.cell_mat, dtype=np.uint8)
        assert self.cell_mat.shape == (len(self.dz), len(self.dy), len(self.dx))

    @property
    def ncx(self) -> int:
        return len(self.dx)

    @property
    def ncy(self) -> int:
        return len(self.dy)

    @property
    def ncz(self) -> int:
        return len(self.dz)

    @property
    def nodes(self) -> Tuple[int, int, int]:
        return (self.ncx + 1, self.ncy + 1, self.ncz + 1)

    @property
    def n_nodes(self) -> int:
        nx, ny, nz = self.nodes
        return nx * ny * nz

    @property
    def n_edges(self) -> int:
        return 3 * self.n_nodes

    def edge_index(self, w: int, i: int, j: int, k: int) -> int:
        nx, ny, _ = self.nodes
        return 3 * (i + nx * (j + ny * k)) + w

    def port_edges(self, p: int) -> np.ndarray:
        port = self.ports[p]
        return np.array([self.edge_index(2, port.i, port.j, k)
                         for k in range(port.k0, port.k1)], dtype=np.int64)


# ---------------------------------------------------------------------------
# Excitation vectors (impressed currents per edge, in A).
# ---------------------------------------------------------------------------

def edge_source(dev: Device, edges: Sequence[Tuple[int, int, int, int, complex]]) -> np.ndarray:
    """Impressed current vector with the given ``(w, i, j, k, current)`` entries."""
    j = np.zeros(dev.n_edges, dtype=np.complex128)
    for w, i, jj, k, cur in edges:
        j[dev.edge_index(w, i, jj, k)] += cur
    return j


def port_source(dev: Device, p: int, current: complex = 1.0) -> np.ndarray:
    """1 A (or ``current``) through every edge of port ``p`` (Sec. IV)."""
    j = np.zeros(dev.n_edges, dtype=np.complex128)
    j[dev.port_edges(p)] = current
    return j


# ---------------------------------------------------------------------------
# Canonical problems.
# ---------------------------------------------------------------------------

def cavity(ncx: int = 16, ncy: int = 16, ncz: int = 16,
           hx: float = 1e-3, hy: Optional[float] = None, hz: Optional[float] = None,
           eps_r: float = 1.0) -> Device:
    """Homogeneous rectangular box with electric walls on all six faces."""
    hy = hx if hy is None else hy
    hz = hx if hz is None else hz
    return Device(dx=np.full(ncx, hx), dy=np.full(ncy, hy), dz=np.full(ncz, hz),
                  cell_mat=np.zeros((ncz, ncy, ncx), np.uint8),
                  materials=[Material(eps_r=eps_r)], ports=[], pec_walls=0x3F,
                  name=f"cavity{ncx}x{ncy}x{ncz}")


def tiny_cavity_case():
    """16^3 uniform vacuum PEC box, 1 mm cells, driven at 0.8x its first
    continuous resonance by 1 A on the z-edge owned by the centre node.

    Returns ``(device, omega, source)``.
    """
    dev = cavity(16, 16, 16, 1e-3)
    a = 16e-3
    f101 = 0.5 * C0 * np.sqrt(2.0) / a
    omega = 2.0 * np.pi * 0.8 * f101
    src = edge_source(dev, [(2, 8, 8, 8, 1.0)])
    return dev, omega, src


# ---------------------------------------------------------------------------
# Layered strip devices with graded meshes.
# ---------------------------------------------------------------------------

def graded_axis(n: int, features: Sequence[int], hmin: float = 10e-6,
                hmax: float = 200e-6, ratio: float = 1.2) -> np.ndarray:
    """Cell sizes ``h_i = min(hmax, hmin * ratio**dist_i)`` where ``dist_i`` is
    the distance (in cells) from cell ``i`` (nodes ``i``, ``i+1``) to the nearest
    feature node.  Adjacent cells therefore differ by at most ``ratio``."""
    feats = np.asarray(sorted(set(int(f) for f in features)), dtype=np.int64)
    i = np.arange(n)
    if feats.size == 0:
        return np.full(n, hmax)
    d = np.minimum(np.abs(i[:, None] - feats[None, :]),
                   np.abs(i[:, None] + 1 - feats[None, :])).min(axis=1)
    return np.minimum(hmax, hmin * ratio ** d.astype(np.float64))


def _layer_bounds(rng, ncz: int, n_layers: int) -> List[Tuple[int, int]]:
    n_layers = max(1, min(n_layers, ncz // 2))
    extra = ncz - 2 * n_layers
    add = rng.multinomial(extra, np.full(n_layers, 1.0 / n_layers))
    th = 2 + add
    z = np.concatenate([[0], np.cumsum(th)])
    return [(int(z[l]), int(z[l + 1])) for l in range(n_layers)]


def layered_device(ncx: int, ncy: int, ncz: int, n_layers: int, n_strips: int,
                   n_ports: int, seed: int, strip_kind: str = "pec",
                   graded: bool = True, name: Optional[str] = None) -> Device:
    """Strips over a stack of lossy dielectric layers inside a PEC box.

    * layers: contiguous z ranges, >= 2 cells thick, eps_r ~ U[2, 12],
      tan(delta) ~ U[0.001, 0.02];
    * strips: along x or y, width U{4..20} cells, one cell thick, lying on the
      top face of a randomly chosen (non-top) layer, >= 2 cells from the side
      walls; ``strip_kind='pec'`` makes them electric conductors,
      ``'sigma'`` gives each its own conductivity ~ log-U[1e6, 5.8e7] S/m;
    * ports: one per strip (first ``n_ports`` strips that admit one), a column
      of z-edges from the bottom wall to the strip's underside at the strip's
      start, centred across its width;
    * mesh: graded around strip edges (x, y) and layer interfaces and strip
      planes (z), 10-200 um, adjacent ratio <= 1.2.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = _layer_bounds(rng, ncz, n_layers)
    mats: List[Material] = []
    for _ in layers:
        mats.append(Material(eps_r=float(rng.uniform(2.0, 12.0)),
                             tan_delta=float(rng.uniform(0.001, 0.02))))
    cell = np.zeros((ncz, ncy, ncx), np.uint8)
    for l, (z0, z1) in enumerate(layers):
        cell[z0:z1] = l

    pec_id = None
    if strip_kind == "pec":
        mats.append(Material(eps_r=1.0, is_pec=True))
        pec_id = len(mats) - 1

    strips = []  # (axis, a0, a1, b0, b1, zc)
    fx, fy, fz = [0, ncx], [0, ncy], [0, ncz]
    for (z0, z1) in layers:
        fz += [z0, z1]
    cand_layers = [l for l in range(len(layers) - 1)] or [0]
    for s in range(n_strips):
        axis = int(rng.integers(0, 2))  # 0: runs along x, 1: along y
        n_len, n_wid = (ncx, ncy) if axis == 0 else (ncy, ncx)
        width = int(rng.integers(4, 21))
        width = max(1, min(width, n_wid - 4))
        b0 = int(rng.integers(2, max(3, n_wid - 2 - width + 1)))
        b1 = b0 + width
        length = int(rng.integers(max(2, n_len // 4), max(3, n_len - 4 + 1)))
        length = min(length, n_len - 4)
        a0 = int(rng.integers(2, max(3, n_len - 2 - length + 1)))
        a1 = a0 + length
        l = int(cand_layers[int(rng.integers(0, len(cand_layers)))])
        zc = layers[l][1] if layers[l][1] < ncz else layers[l][1] - 1
        if strip_kind == "pec":
            mid = pec_id
        else:
            sig = float(np.exp(rng.uniform(np.log(1e6), np.log(5.8e7))))
            mats.append(Material(eps_r=1.0, sigma=sig))
            mid = len(mats) - 1
        if axis == 0:
            cell[zc, b0:b1, a0:a1] = mid
            fx += [a0, a1]
            fy += [b0, b1]
        else:
            cell[zc, a0:a1, b0:b1] = mid
            fy += [a0, a1]
            fx += [b0, b1]
        fz += [zc, zc + 1]
        strips.append((axis, a0, a1, b0, b1, zc))

    is_pec = np.array([m.is_pec for m in mats])

    def column_clear(i, j, k1):
        # cells touching the z-edges (i, j, k), k < k1: (i-1..i, j-1..j, k)
        for k in range(k1):
            for b in (j - 1, j):
                for a in (i - 1, i):
                    if 0 <= a < ncx and 0 <= b < ncy and is_pec[cell[k, b, a]]:
                        return False
        return True

    ports: List[Port] = []
    for (axis, a0, a1, b0, b1, zc) in strips:
        if len(ports) >= n_ports:
            break
        bc = (b0 + b1) // 2
        for end in (a0, a1):
            i, j = (end, bc) if axis == 0 else (bc, end)
            if zc >= 1 and column_clear(i, j, zc) and all((q.i, q.j) != (i, j) for q in ports):
                ports.append(Port(i=i, j=j, k0=0, k1=zc, z0=50.0))
                break

    if graded:
        dx = graded_axis(ncx, fx)
        dy = graded_axis(ncy, fy)
        dz = graded_axis(ncz, fz)
    else:
        dx, dy, dz = (np.full(ncx, 100e-6), np.full(ncy, 100e-6), np.full(ncz, 100e-6))
    return Device(dx=dx, dy=dy, dz=dz, cell_mat=cell, materials=mats, ports=ports,
                  pec_walls=0x3F, name=name or f"layered{ncx}x{ncy}x{ncz}s{seed}")


def log_uniform_frequency(seed: int, fmin: float = 1e9, fmax: float = 40e9) -> float:
    """One frequency ``10**U[log10 fmin, log10 fmax]`` drawn from ``seed``."""
    rng = np.random.Generator(np.random.PCG64(seed + 7919))
    return float(10.0 ** rng.uniform(np.log10(fmin), np.log10(fmax)))


def log_spaced_omegas(n: int, fmin: float = 1e9, fmax: float = 40e9) -> np.ndarray:
    return 2.0 * np.pi * np.logspace(np.log10(fmin), np.log10(fmax), n)


# ---------------------------------------------------------------------------
# The workloads: the tiny cavity, the 128^3 plain-method device, the
# 256x256x128 precision-form interconnect, the six uneven sweep devices and
# the 192x192x96 learned-form device family.
# ---------------------------------------------------------------------------

def plain_device_128(seed: int = 2) -> Device:
    return layered_device(128, 128, 128, n_layers=6, n_strips=4, n_ports=1, seed=seed,
                          name=f"layered128^3 s{seed}")


def interconnect_256(seed: int = 3) -> Device:
    return layered_device(256, 256, 128, n_layers=8, n_strips=12, n_ports=1, seed=seed,
                          name=f"interconnect256x256x128 s{seed}")


SWEEP_SHAPES = [(64, 64, 32), (96, 96, 48), (128, 128, 64), (144, 144, 72),
                (160, 160, 80), (192, 192, 96)]


def sweep_devices(seeds=range(40, 46), shapes=SWEEP_SHAPES) -> List[Device]:
    out = []
    for s, (nx, ny, nz) in zip(seeds, shapes):
        out.append(layered_device(nx, ny, nz, n_layers=6, n_strips=4, n_ports=4, seed=s,
                                  strip_kind="sigma", name=f"sweep{nx}x{ny}x{nz} s{s}"))
    return out


def learned_family_device(seed: int, shape=(192, 192, 96)) -> Device:
    nx, ny, nz = shape
    return layered_device(nx, ny, nz, n_layers=6, n_strips=4, n_ports=1, seed=seed,
                          name=f"family{nx}x{ny}x{nz} s{seed}")
