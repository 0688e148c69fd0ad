"""Seeded synthetic inputs: periodic boxes of point charges.

This module holds no u-series arithmetic; it only draws positions and charges.
Both the GPU library's tests/benchmarks and the FP64 oracle consume its
output.  Every generator returns float32 positions ``[n, 3]`` (Angstrom,
wrapped into [0, L)), float32 charges ``[n]`` (e) and the box ``(Lx, Ly, Lz)``.

Charges are exactly neutral in float32 arithmetic:
* random charges are quantised to multiples of 2^-20 and the last charge of
  each neutral group is minus the sum of the others (all such sums are exact);
* water uses q_O = -2 q_H, which is exact because doubling is exact.

The workloads stand in for the paper's DPPC membrane (Sec. IV: 72 lipids and
2189 waters), whose configurations are not available: a random-charge cube, a
3-site water box and a membrane-shaped slab of 10-site neutral groups in water.
"""
import math

import numpy as np

WATER_DENSITY = 0.0334            # molecules / A^3
OH_BOND = 0.9572                  # A
HOH_ANGLE = 104.52                # degrees
Q_H = np.float32(0.417)
Q_O = np.float32(-2.0) * Q_H      # = -0.834 exactly twice q_H
QUANTUM = 2.0 ** -20


def _quantise(x):
    return np.round(np.asarray(x, dtype=np.float64) / QUANTUM) * QUANTUM


def _random_rotations(rng, m):
    """m uniform random rotation matrices from normalised 4D Gaussian quaternions."""
    qv = rng.standard_normal((m, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    R = np.empty((m, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_sites():
    half = math.radians(HOH_ANGLE) / 2
    hx, hz = OH_BOND * math.sin(half), OH_BOND * math.cos(half)
    return np.array([[0.0, 0.0, 0.0], [hx, 0.0, hz], [-hx, 0.0, hz]])


def _wrap(xyz, box):
    box = np.asarray(box, dtype=np.float64)
    x = np.mod(np.asarray(xyz, dtype=np.float64), box)
    x32 = x.astype(np.float32)
    # float32 rounding can land exactly on L: fold those back to 0
    x32 = np.where(x32 >= box.astype(np.float32), np.float32(0), x32)
    return x32


def _place_waters(rng, centres, box):
    n_mol = centres.shape[0]
    R = _random_rotations(rng, n_mol)
    sites = np.einsum("mij,sj->msi", R, _water_sites()) + centres[:, None, :]
    xyz = sites.reshape(-1, 3)
    q = np.tile(np.array([Q_O, Q_H, Q_H], dtype=np.float32), n_mol)
    return _wrap(xyz, box), q


def random_cube(n=512, L=24.0, seed=1377):
    """n charges uniform in a cubic box of edge L, q ~ U[-1, 1] made neutral."""
    rng = np.random.default_rng(seed)
    xyz = rng.uniform(0.0, L, (n, 3))
    q = rng.uniform(-1.0, 1.0, n)
    q = _quantise(q - q.mean())
    if n > 0:
        q[-1] = -np.sum(q[:-1])
    return _wrap(xyz, (L, L, L)), q.astype(np.float32), (L, L, L)


def random_box(n, box, seed):
    """n charges uniform in an orthorhombic box, q ~ U[-1, 1] made neutral."""
    rng = np.random.default_rng(seed)
    box = tuple(float(v) for v in box)
    xyz = rng.uniform(0.0, 1.0, (n, 3)) * np.array(box)
    q = rng.uniform(-1.0, 1.0, n)
    q = _quantise(q - q.mean())
    if n > 0:
        q[-1] = -np.sum(q[:-1])
    return _wrap(xyz, box), q.astype(np.float32), box


def water_box(n_mol=None, L=64.0, seed=1378, jitter=0.3):
    """3-site water at 0.0334 molecules/A^3 in a cubic box: molecular centres
    are a random subset of a cubic lattice (jittered by U(+-jitter)), each
    molecule has a uniform random orientation."""
    rng = np.random.default_rng(seed)
    if n_mol is None:
        n_mol = int(round(WATER_DENSITY * L ** 3))
    m = int(math.ceil(n_mol ** (1.0 / 3.0) - 1e-9))
    h = L / m
    g = np.arange(m) * h + h / 2
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    pick = rng.choice(lat.shape[0], size=n_mol, replace=False)
    centres = lat[pick] + rng.uniform(-jitter, jitter, (n_mol, 3))
    xyz, q = _place_waters(rng, centres, (L, L, L))
    return xyz, q, (L, L, L)


class _SiteHash:
    """Spatial hash that rejects sites closer than dmin (periodic)."""

    def __init__(self, box, dmin):
        self.box = np.asarray(box, dtype=np.float64)
        self.dmin = dmin
        self.nc = np.maximum((self.box // dmin).astype(int), 1)
        self.cells = {}

    def _key(self, p):
        c = np.floor(np.mod(p, self.box) / self.box * self.nc).astype(int) % self.nc
        return tuple(c)

    def ok(self, pts):
        for p in pts:
            c = self._key(p)
            for dx in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dz in (-1, 0, 1):
                        k = ((c[0] + dx) % self.nc[0], (c[1] + dy) % self.nc[1],
                             (c[2] + dz) % self.nc[2])
                        for o in self.cells.get(k, ()):
                            d = p - o
                            d -= self.box * np.round(d / self.box)
                            if d @ d < self.dmin * self.dmin:
                                return False
        return True

    def add(self, pts):
        for p in pts:
            self.cells.setdefault(self._key(p), []).append(np.mod(p, self.box))


def membrane_slab(box=(100.0, 100.0, 90.0), half_thickness=20.0, n_groups=5210,
                  n_water=16700, seed=1379, dmin=0.8):
    """Membrane-shaped slab: n_groups neutral 10-site groups (sites uniform in
    a 2 A ball, q ~ N(0, 0.4^2) re-centred per group) centred on a jittered
    lattice inside |z - Lz/2| < half_thickness, and 3-site water filling the
    rest at 0.0334 molecules/A^3.  Sites of different molecules stay at least
    dmin apart."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    zc = box[2] / 2
    sh = _SiteHash(box, dmin)
    xyz_all, q_all = [], []
    # slab groups
    vol = box[0] * box[1] * 2 * (half_thickness - 2.0)
    h = (vol / n_groups) ** (1.0 / 3.0)
    nx, ny = int(math.ceil(box[0] / h)), int(math.ceil(box[1] / h))
    nz = int(math.ceil(n_groups / (nx * ny)))
    gz = zc - (half_thickness - 2.0) + (np.arange(nz) + 0.5) * 2 * (half_thickness - 2.0) / nz
    lat = np.stack(np.meshgrid((np.arange(nx) + 0.5) * box[0] / nx,
                               (np.arange(ny) + 0.5) * box[1] / ny, gz, indexing="ij"),
                   axis=-1).reshape(-1, 3)
    centres = lat[rng.choice(lat.shape[0], size=n_groups, replace=False)]
    centres += rng.uniform(-0.3, 0.3, centres.shape)
    for c in centres:
        sites = []
        while len(sites) < 10:
            v = rng.uniform(-2.0, 2.0, 3)
            if v @ v > 4.0:
                continue
            p = c + v
            if all(np.sum((p - s) ** 2) >= dmin * dmin for s in sites) and sh.ok([p]):
                sites.append(p)
        sh.add(sites)
        qg = _quantise(rng.normal(0.0, 0.4, 10))
        qg = qg - _quantise(np.mean(qg))
        qg[-1] = -np.sum(qg[:-1])
        xyz_all.append(np.array(sites))
        q_all.append(qg)
    # water outside the slab: a cubic-ish lattice over the water layer
    # zc + half_thickness + 1 <= z < zc - half_thickness - 1 + Lz (periodic),
    # 15% more points than molecules, a random subset of them used
    z0 = zc + half_thickness + 1.0
    tw = box[2] - 2.0 * (half_thickness + 1.0)
    hw = (box[0] * box[1] * tw / (1.15 * n_water)) ** (1.0 / 3.0)
    mx, my, mz = (int(math.ceil(box[0] / hw)), int(math.ceil(box[1] / hw)),
                  int(math.ceil(tw / hw)))
    lat = np.stack(np.meshgrid((np.arange(mx) + 0.5) * box[0] / mx,
                               (np.arange(my) + 0.5) * box[1] / my,
                               z0 + (np.arange(mz) + 0.5) * tw / mz, indexing="ij"),
                   axis=-1).reshape(-1, 3)
    order = rng.permutation(lat.shape[0])
    base = _water_sites()
    placed = 0
    for k in order:
        if placed == n_water:
            break
        for _ in range(20):
            c = lat[k] + rng.uniform(-0.3, 0.3, 3)
            R = _random_rotations(rng, 1)[0]
            sites = base @ R.T + c
            if sh.ok(sites):
                sh.add(sites)
                xyz_all.append(sites)
                q_all.append(np.array([Q_O, Q_H, Q_H], dtype=np.float64))
                placed += 1
                break
    if placed < n_water:
        raise RuntimeError("membrane_slab: lattice too small for %d waters" % n_water)
    xyz = np.concatenate(xyz_all)
    q = np.concatenate(q_all).astype(np.float32)
    return _wrap(xyz, box), q, tuple(float(v) for v in box)


def serving_request(k, seed=1381):
    """Request k of the serving stream: a water box with a log-uniform molecule
    count in [216, 16000] at 0.0334 molecules/A^3.  Returns (xyz, q, box)."""
    rng = np.random.default_rng([seed, k])
    n_mol = int(round(math.exp(rng.uniform(math.log(216), math.log(16000)))))
    L = (n_mol / WATER_DENSITY) ** (1.0 / 3.0)
    return water_box(n_mol=n_mol, L=L, seed=int(rng.integers(1 << 31)))


# the benchmark workloads, by name
WORKLOADS = {
    "random512": lambda: random_cube(512, 24.0, seed=1377),
    "water26k": lambda: water_box(None, 64.0, seed=1378),
    "slab100k": lambda: membrane_slab(seed=1379),
}
