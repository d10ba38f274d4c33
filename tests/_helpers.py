"""Test-side helpers: seeded vectors and local crops of a device.

A crop keeps the cells within two of a node, so the oracle can evaluate the
operator's rows at that node exactly on a tiny system (the operator only
couples a node's edges to cells and edges within one cell of it).  This lets
parity tests check full-size launches at sampled nodes.
"""
import numpy as np

from paper_1705_08849_amd import devices as D

# vacuum permittivity from the defined mu0 = 4 pi 1e-7 H/m and the exact c0
EPS0 = 1.0 / (4.0e-7 * np.pi * D.C0 ** 2)


def rand_c(n, seed, dtype=np.complex128):
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.uniform(-1, 1, n) + 1j * rng.uniform(-1, 1, n)).astype(dtype)


def crop(dev, i, j, k, r=2):
    """Sub-device of the cells [i-r, i+r) x [j-r, j+r) x [k-r, k+r) (clipped),
    with the original electric walls kept only where the window touches them,
    ports clipped to the window with their per-edge conductance preserved.
    Returns (sub_device, (a0, b0, c0)) -- the node offset of the window."""
    a0, a1 = max(0, i - r), min(dev.ncx, i + r)
    b0, b1 = max(0, j - r), min(dev.ncy, j + r)
    c0, c1 = max(0, k - r), min(dev.ncz, k + r)
    walls = 0
    for bit, touch in ((1, a0 == 0), (2, a1 == dev.ncx), (4, b0 == 0), (8, b1 == dev.ncy),
                       (16, c0 == 0), (32, c1 == dev.ncz)):
        if touch and (dev.pec_walls & bit):
            walls |= bit
    ports = []
    for p in dev.ports:
        pi, pj = p.i - a0, p.j - b0
        if 0 <= pi <= a1 - a0 and 0 <= pj <= b1 - b0:
            k0, k1 = max(p.k0, c0) - c0, min(p.k1, c1) - c0
            if k1 > k0:
                g = (p.k1 - p.k0) / p.z0
                ports.append(D.Port(pi, pj, k0, k1, (k1 - k0) / g))
    sub = D.Device(dx=dev.dx[a0:a1], dy=dev.dy[b0:b1], dz=dev.dz[c0:c1],
                   cell_mat=dev.cell_mat[c0:c1, b0:b1, a0:a1], materials=dev.materials,
                   ports=ports, pec_walls=walls)
    return sub, (a0, b0, c0)


def crop_vector(dev, sub, off, x):
    """Restrict a full edge vector to the crop's nodes."""
    a0, b0, c0 = off
    nx, ny, nz = dev.nodes
    sx, sy, sz = sub.nodes
    x4 = x.reshape(nz, ny, nx, 3)
    return np.ascontiguousarray(x4[c0:c0 + sz, b0:b0 + sy, a0:a0 + sx]).ravel()


def parity_devices():
    """Small devices spanning several 64x4 tiles with ragged tails, graded
    meshes, lossy layers, PEC and conducting strips, ports, open walls and
    mu_r != 1."""
    out = {}
    out["cavity16"] = D.cavity(16, 16, 16, 1e-3)
    out["cavity_odd"] = D.cavity(5, 7, 3, 1e-3, 2e-3, 0.5e-3)
    out["layered_pec"] = D.layered_device(70, 11, 9, n_layers=3, n_strips=2, n_ports=2, seed=7)
    out["layered_sigma"] = D.layered_device(20, 17, 13, n_layers=4, n_strips=3, n_ports=3,
                                            seed=8, strip_kind="sigma")
    rng = np.random.default_rng(9)
    mats = [D.Material(eps_r=float(rng.uniform(1, 12)), mu_r=float(rng.uniform(1, 3)),
                       sigma=float(rng.uniform(0, 3)), tan_delta=float(rng.uniform(0, 0.05)))
            for _ in range(3)] + [D.Material(is_pec=True)]
    cm = rng.integers(0, 4, (9, 10, 66)).astype(np.uint8)
    out["random_open"] = D.Device(dx=rng.uniform(1e-5, 2e-4, 66), dy=rng.uniform(1e-5, 2e-4, 10),
                                  dz=rng.uniform(1e-5, 2e-4, 9), cell_mat=cm, materials=mats,
                                  ports=[D.Port(3, 4, 1, 5, 37.0)], pec_walls=0b010110)
    return out


def plate_device(graded=True):
    """Parallel-plate case: electric walls at -z and +z only (the four side
    walls open), three z-layers of different lossy media, graded x/y/z
    spacings.  Driven by a uniform current density J along z."""
    rng = np.random.default_rng(17)
    ncx, ncy, ncz = 5, 4, 6
    h = (lambda n: rng.uniform(0.5e-3, 1.5e-3, n)) if graded else (lambda n: np.full(n, 1e-3))
    mats = [D.Material(eps_r=2.5, tan_delta=0.01), D.Material(eps_r=9.0, sigma=0.3),
            D.Material(eps_r=4.0, tan_delta=0.002, sigma=0.05)]
    cm = np.zeros((ncz, ncy, ncx), np.uint8)
    cm[2:4] = 1
    cm[4:] = 2
    return D.Device(dx=h(ncx), dy=h(ncy), dz=h(ncz), cell_mat=cm, materials=mats,
                    pec_walls=(1 << 4) | (1 << 5))


def plate_source(dev, jdens=1.0):
    """Impressed current per z-edge = J times the edge's dual-facet area
    (half cells at the open side walls), i.e. a uniform current density."""
    def dual(h):
        hp = np.concatenate([[0.0], h, [0.0]])
        return 0.5 * (hp[:-1] + hp[1:])
    nx, ny, nz = dev.nodes
    area = dual(dev.dy)[:, None] * dual(dev.dx)[None, :]
    j = np.zeros((nz, ny, nx, 3), np.complex128)
    j[: dev.ncz, :, :, 2] = jdens * area[None, :, :]
    return j.ravel()


def plate_closed_form(dev, omega, jdens=1.0):
    """A uniform field E_k along z in layer k is the gradient of a potential
    that depends on z alone, so the curl-curl term vanishes and eq. (e2)
    reduces per edge to (-omega^2 eps_k + j omega sigma_k) E_k (area) =
    -j omega J (area):  E_k = -j omega J / (-omega^2 eps_k + j omega sigma_k),
    eps_k = eps0 eps_r (1 - j tan delta); edge voltage E_k dz[k]."""
    nx, ny, nz = dev.nodes
    x = np.zeros((nz, ny, nx, 3), np.complex128)
    for k in range(dev.ncz):
        m = dev.materials[dev.cell_mat[k, 0, 0]]
        eps = EPS0 * m.eps_r * (1 - 1j * m.tan_delta)
        e = -1j * omega * jdens / (-omega ** 2 * eps + 1j * omega * m.sigma)
        x[k, :, :, 2] = e * dev.dz[k]
    return x.ravel()
