"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module defines *inputs only*: geometries (which material occupies a point
of the unit cell), the permittivity tensors of those materials, Bloch wave
vectors along a Brillouin-zone path, and seeded random complex blocks.  It holds
none of the method's arithmetic (no difference operators, no DFT, no
permittivity discretisation, no penalty rule).

Conventions (Section 2.1, eqs (2.1)-(2.3); Section 3, eq (3.2)):

* grid division N, h = 1/N, 0-based cell indices (i, j, k) in [0, N)^3 taken
  modulo N, linear index p = i + N*j + N*N*k (x fastest), the same order as the
  Kronecker embeddings of Section 2.1, eq (2.6);
* the four point sets at which the inverse permittivity is sampled are the
  x-, y-, z-edge points and the volume (cell-centre) points of the Yee cell:

      x-edge ((i-1/2)h, j h, k h)     y-edge (i h, (j-1/2)h, k h)
      z-edge (i h, j h, (k-1/2)h)     volume ((i-1/2)h, (j-1/2)h, (k-1/2)h)

* a point is inside a shape iff it is strictly inside (distance < radius,
  |offset| < half-width); a slab covers z in [z0, z1);
* material id 0 is the background (air, inverse permittivity = identity); a
  later shape overrides an earlier one where they overlap.

The permittivity tables hold the INVERSE permittivity (the paper's eps_1 in
eq (1.5) is the inverse tensor, Assumption 3.1), complex Hermitian 3x3.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

POINT_SETS = ("ex", "ey", "ez", "vol")

# offsets (in units of h) of the four point sets relative to (i, j, k)
_OFFSETS = {
    "ex": (-0.5, 0.0, 0.0),
    "ey": (0.0, -0.5, 0.0),
    "ez": (0.0, 0.0, -0.5),
    "vol": (-0.5, -0.5, -0.5),
}


def point_coords(N: int, which: str) -> np.ndarray:
    """Coordinates in [0,1)^3 of one point set, shape (N^3, 3), index i + N j + N^2 k."""
    ox, oy, oz = _OFFSETS[which]
    i = np.arange(N, dtype=np.float64)
    # meshgrid in (z, y, x) order so that the flattened index is x fastest
    kk, jj, ii = np.meshgrid(i, i, i, indexing="ij")
    pts = np.stack([(ii.ravel() + ox) / N, (jj.ravel() + oy) / N, (kk.ravel() + oz) / N], axis=1)
    return np.mod(pts, 1.0)


def _min_image(d: np.ndarray) -> np.ndarray:
    return d - np.round(d)


@dataclasses.dataclass
class Sphere:
    center: Sequence[float]
    radius: float
    mat: int

    def contains(self, pts: np.ndarray) -> np.ndarray:
        d = _min_image(pts - np.asarray(self.center, dtype=np.float64))
        return np.einsum("ij,ij->i", d, d) < self.radius ** 2


@dataclasses.dataclass
class Rod:
    """Infinite circular rod along `axis` (0=x, 1=y, 2=z) through `center` (3-vector; the
    component along the axis is ignored)."""
    axis: int
    center: Sequence[float]
    radius: float
    mat: int

    def contains(self, pts: np.ndarray) -> np.ndarray:
        d = _min_image(pts - np.asarray(self.center, dtype=np.float64))
        d[:, self.axis] = 0.0
        return np.einsum("ij,ij->i", d, d) < self.radius ** 2


@dataclasses.dataclass
class SlabRod:
    """Rectangular rod along `axis` (0 or 1) inside the slab z in [z0, z1): the transverse
    in-plane coordinate must satisfy |c - offset| < half_width (minimal image)."""
    axis: int
    offset: float
    half_width: float
    z0: float
    z1: float
    mat: int

    def contains(self, pts: np.ndarray) -> np.ndarray:
        t = 1 - self.axis  # transverse in-plane axis
        d = np.abs(_min_image(pts[:, t] - self.offset))
        z = pts[:, 2]
        return (d < self.half_width) & (z >= self.z0) & (z < self.z1)


@dataclasses.dataclass
class Slab:
    """Layer lo <= coordinate < hi along `axis` (0=x, 1=y, 2=z), unbounded in the other two
    directions; lo and hi in [0, 1]."""
    axis: int
    lo: float
    hi: float
    mat: int

    def contains(self, pts: np.ndarray) -> np.ndarray:
        c = pts[:, self.axis]
        return (c >= self.lo) & (c < self.hi)


# Primitive lattice vectors as ROWS (lattice constant 1), Section 4, eq (4.1); a cell point with
# fractional coordinates xi (the unit-cube grid) sits at x = xi_1 a_1 + xi_2 a_2 + xi_3 a_3.
LATTICES = {
    "sc": np.eye(3),
    "fcc": np.array([[0.0, 0.5, 0.5], [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]]),
    "bcc": np.array([[-0.5, 0.5, 0.5], [0.5, -0.5, 0.5], [0.5, 0.5, -0.5]]),
    # a triclinic cell whose lattice matrix is not symmetric (catches transposed conventions)
    "tric": np.array([[1.0, 0.0, 0.0], [0.3, 0.9, 0.0], [0.2, 0.25, 0.8]]),
}

# Symmetry points of the Brillouin zones, Section 4, eq (4.2) (Cartesian, lattice constant 1)
BZ_POINTS = {
    "fcc": {"X": (0.0, 2 * math.pi, 0.0), "U": (math.pi / 2, 2 * math.pi, math.pi), "L": (math.pi,) * 3,
            "G": (0.0, 0.0, 0.0), "W": (math.pi, 2 * math.pi, 0.0), "K": (1.5 * math.pi, 1.5 * math.pi, 0.0)},
    "bcc": {"H'": (2 * math.pi, 0.0, 0.0), "G": (0.0, 0.0, 0.0), "P": (math.pi,) * 3, "N": (math.pi, 0.0, math.pi),
            "H": (0.0, 2 * math.pi, 0.0)},
}


@dataclasses.dataclass
class LatticeSphere:
    """Sphere of physical radius `radius` around the point with fractional coordinates `center`
    of a lattice (vectors as rows); periodic images through the 27 nearest lattice vectors."""
    lattice: np.ndarray
    center: Sequence[float]
    radius: float
    mat: int

    def contains(self, pts: np.ndarray) -> np.ndarray:
        L = np.asarray(self.lattice, dtype=np.float64)
        d = _min_image(pts - np.asarray(self.center, dtype=np.float64))
        best = np.full(pts.shape[0], np.inf)
        for n in np.array(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij")).reshape(3, -1).T:
            x = (d + n[None, :]) @ L
            best = np.minimum(best, np.einsum("ij,ij->i", x, x))
        return best < self.radius ** 2


def lattice_sphere(lattice: str, N: int, radius: float = 0.25, eps=13.0, k=(0.3, 0.5, 0.7), m: int = 8,
                   scheme: str = "crossdof") -> Workload:
    """A dielectric sphere at the lattice origin in air for the lattice `lattice` (LATTICES);
    eps a scalar or a 3x3 permittivity tensor."""
    L = LATTICES[lattice]
    ids = sample_ids(N, [LatticeSphere(L, (0.0, 0.0, 0.0), radius, 1)])
    e = eps * np.eye(3) if np.ndim(eps) == 0 else np.asarray(eps)
    return Workload("%s%d-sphere" % (lattice, N), N, ids, eps_table([e]), np.array([k], dtype=np.float64), m, scheme)


def sample_ids(N: int, shapes: Sequence) -> np.ndarray:
    """uint8 material ids, shape (4, N^3), rows in POINT_SETS order."""
    ids = np.zeros((4, N ** 3), dtype=np.uint8)
    for r, which in enumerate(POINT_SETS):
        pts = point_coords(N, which)
        for s in shapes:
            ids[r, s.contains(pts)] = s.mat
    return ids


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed rotation: Q of the QR of a 3x3 standard normal matrix, columns signed
    by diag(R), one column flipped if det < 0."""
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def inverse_tensor(eps: np.ndarray) -> np.ndarray:
    """Inverse of a Hermitian permittivity tensor, symmetrised to be exactly Hermitian."""
    inv = np.linalg.inv(np.asarray(eps, dtype=np.complex128))
    return 0.5 * (inv + inv.conj().T)


def eps_table(eps_list: Sequence[np.ndarray]) -> np.ndarray:
    """Inverse-permittivity table, complex (n_mat, 3, 3); entry 0 is air (identity) and entry
    i+1 is the inverse of eps_list[i]."""
    tab = [np.eye(3, dtype=np.complex128)]
    tab += [inverse_tensor(e) for e in eps_list]
    return np.stack(tab)


def gyrotropic_eps(e1: float, g: float, e3: float) -> np.ndarray:
    """[[e1, i g, 0], [-i g, e1, 0], [0, 0, e3]] (a Hermitian permittivity)."""
    return np.array([[e1, 1j * g, 0], [-1j * g, e1, 0], [0, 0, e3]], dtype=np.complex128)


def rotated_eps(rng: np.random.Generator, lo: float, hi: float) -> np.ndarray:
    """R diag(e) R^T with e_i ~ U[lo, hi] and R a random rotation (real symmetric eps)."""
    e = rng.uniform(lo, hi, size=3)
    R = random_rotation(rng)
    return (R * e[None, :]) @ R.T


# --- Brillouin-zone path of the simple cubic lattice (Section 4, eq (4.2)) ---------------
SC_POINTS = {
    "G": np.array([0.0, 0.0, 0.0]),
    "X": np.array([math.pi, 0.0, 0.0]),
    "M": np.array([math.pi, math.pi, 0.0]),
    "R": np.array([math.pi, math.pi, math.pi]),
}
SC_PATH = ("G", "X", "M", "G", "R")


def sc_kpath(nk: int) -> np.ndarray:
    """nk wave vectors on Gamma-X-M-Gamma-R, uniform in arc length, both ends included."""
    verts = [SC_POINTS[s] for s in SC_PATH]
    seg = [np.linalg.norm(verts[i + 1] - verts[i]) for i in range(len(verts) - 1)]
    L = float(sum(seg))
    out = np.zeros((nk, 3))
    cum = np.concatenate([[0.0], np.cumsum(seg)])
    for j in range(nk):
        s = L * j / (nk - 1) if nk > 1 else 0.0
        t = min(int(np.searchsorted(cum, s, side="right")) - 1, len(seg) - 1)
        f = (s - cum[t]) / seg[t]
        out[j] = verts[t] + f * (verts[t + 1] - verts[t])
    # snap tiny round-off so that the vertices are exact
    out[np.abs(out) < 1e-14] = 0.0
    return out


def random_block(seed: int, nvec: int, N: int) -> np.ndarray:
    """Seeded complex Gaussian block, shape (nvec, 3, N^3), complex128."""
    rng = np.random.default_rng(seed)
    n = 3 * N ** 3
    re = rng.standard_normal((nvec, n))
    im = rng.standard_normal((nvec, n))
    return (re + 1j * im).reshape(nvec, 3, N ** 3)


def random_complex(seed: int, shape) -> np.ndarray:
    """Seeded complex Gaussian array of any shape, complex128."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@dataclasses.dataclass
class Workload:
    name: str
    N: int
    ids: np.ndarray          # uint8 (4, N^3)
    table: np.ndarray        # complex (n_mat, 3, 3) inverse permittivity
    kpoints: np.ndarray      # (nk, 3)
    m: int                   # bands
    scheme: str              # "trivial" or "crossdof"

    @property
    def n(self) -> int:
        return 3 * self.N ** 3


def sphere_isotropic(N: int = 16, radius: float = 0.25, eps: float = 13.0,
                     k=(0.2 * math.pi, 0.4 * math.pi, 0.6 * math.pi), m: int = 10) -> Workload:
    """Simple-cubic, isotropic sphere eps=13, r=0.25a, centre (1/2,1/2,1/2), one k-point."""
    ids = sample_ids(N, [Sphere((0.5, 0.5, 0.5), radius, 1)])
    table = eps_table([eps * np.eye(3)])
    return Workload("sc%d-sphere-iso" % N, N, ids, table, np.array([k], dtype=np.float64), m, "crossdof")


def sphere_anisotropic(N: int = 64, nk: int = 40, m: int = 20, seed: int = 0,
                       radius: float = 0.3, scheme: str = "crossdof") -> Workload:
    """Simple-cubic, sphere r=0.3a with eps = R diag(e) R^T, e_i ~ U[4,14], R from `seed`."""
    rng = np.random.default_rng(seed)
    eps = rotated_eps(rng, 4.0, 14.0)
    ids = sample_ids(N, [Sphere((0.5, 0.5, 0.5), radius, 1)])
    return Workload("sc%d-sphere-aniso" % N, N, ids, eps_table([eps]), sc_kpath(nk), m, scheme)


def woodpile_gyrotropic(N: int = 128, nk: int = 60, m: int = 16, e1: float = 12.0,
                        g: float = 0.5, e3: float = 10.0, scheme: str = "crossdof") -> Workload:
    """Simple-cubic woodpile of four rod layers (rod width 0.25a) with gyrotropic eps."""
    shapes = [
        SlabRod(0, 0.25, 0.125, 0.00, 0.25, 1),
        SlabRod(1, 0.25, 0.125, 0.25, 0.50, 1),
        SlabRod(0, 0.75, 0.125, 0.50, 0.75, 1),
        SlabRod(1, 0.75, 0.125, 0.75, 1.00, 1),
    ]
    ids = sample_ids(N, shapes)
    return Workload("sc%d-woodpile-gyro" % N, N, ids, eps_table([gyrotropic_eps(e1, g, e3)]),
                    sc_kpath(nk), m, scheme)


def random_inclusions(N: int, seed: int, nk: int = 1, m: int = 16,
                      scheme: str = "crossdof") -> Workload:
    """1-4 spheres (r ~ U[0.1,0.3]) or rods (r ~ U[0.08,0.2]) with random anisotropic eps
    (eigenvalues ~ U[2,14]), each inclusion its own material."""
    rng = np.random.default_rng(seed)
    nincl = int(rng.integers(1, 5))
    shapes: List = []
    eps_list = []
    for t in range(nincl):
        c = rng.uniform(0.0, 1.0, size=3)
        if rng.uniform() < 0.5:
            shapes.append(Sphere(c, float(rng.uniform(0.1, 0.3)), t + 1))
        else:
            shapes.append(Rod(int(rng.integers(0, 3)), c, float(rng.uniform(0.08, 0.2)), t + 1))
        eps_list.append(rotated_eps(rng, 2.0, 14.0))
    ids = sample_ids(N, shapes)
    return Workload("sc%d-random-%d" % (N, seed), N, ids, eps_table(eps_list), sc_kpath(nk), m, scheme)


def random_unitary(rng: np.random.Generator) -> np.ndarray:
    """Haar-distributed 3x3 unitary: Q of the QR of a complex standard normal matrix, columns
    scaled by the phases of diag(R)."""
    g = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    d = np.diag(r)
    return q * (d / np.abs(d))[None, :]


def sphere_illconditioned(N: int, seed: int = 0, radius: float = 0.25, m: int = 10,
                          k=(math.pi / 7, 3 * math.pi / 5, 4 * math.pi / 13),
                          scheme: str = "crossdof") -> Workload:
    """Section 4, robustness under extreme cases: an inclusion whose inverse permittivity is
    U diag(1e-1, 1e-3, 1e-5) U^H with U a random unitary from `seed` (complex Hermitian, condition
    number 1e4), here a sphere of radius `radius` at the cell centre in air, at the paper's wave
    vector (1/7, 3/5, 4/13) pi."""
    rng = np.random.default_rng(seed)
    U = random_unitary(rng)
    einv = (U * np.array([1e-1, 1e-3, 1e-5])[None, :]) @ U.conj().T
    einv = 0.5 * (einv + einv.conj().T)
    ids = sample_ids(N, [Sphere((0.5, 0.5, 0.5), radius, 1)])
    table = np.stack([np.eye(3, dtype=np.complex128), einv])
    return Workload("sc%d-sphere-illcond" % N, N, ids, table, np.array([k], dtype=np.float64), m, scheme)


def smooth_isotropic(N: int, k=(math.pi, math.pi, math.pi), m: int = 8) -> Workload:
    """Simple-cubic cell with the smooth isotropic permittivity eps = 8.9 sin(2 pi (x+y+z)) + 13
    (Section 4, eq (4.7)).  Every sample point of the Yee cell has x + y + z = (t - 1/2) h mod 1
    for an integer t, so the field takes N values: material t (t < N <= 64) holds
    1/eps((t - 1/2) h) I, and each point gets the material of its own t."""
    if N > 64:
        raise ValueError("smooth_isotropic needs N <= 64 (one material per value of x+y+z)")
    ids = np.zeros((4, N ** 3), dtype=np.uint8)
    for r, which in enumerate(POINT_SETS):
        s = point_coords(N, which).sum(axis=1)
        t = np.round(s * N + 0.5).astype(np.int64) % N
        ids[r] = t.astype(np.uint8)
    tab = np.stack([np.eye(3, dtype=np.complex128) /
                    (8.9 * math.sin(2.0 * math.pi * (t - 0.5) / N) + 13.0) for t in range(N)])
    return Workload("sc%d-smooth-iso" % N, N, ids, tab, np.array([k], dtype=np.float64), m, "diagonal")
