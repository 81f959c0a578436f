"""Seeded synthetic inputs shared by the HIP path, the oracle and the benchmark.

This module generates structures, initial species, velocities and potential
parameter sets. It contains none of the method's arithmetic (no energies, no
acceptance tests, no random numbers that the sampler draws): the Monte Carlo
random numbers are Philox4x64-10 draws made on each side from the published
definition.

Workload shapes follow the paper's own runs:
  * a 10x10x10 bcc block of 2,000 sites (the per-processor size of the
    weak-scaling study, Sec. III.C, Fig. 9),
  * a 40x40x40 bcc block of 128,000 sites (Sec. III.C, Fig. 7),
  * a Voronoi nanocrystal of randomly oriented bcc grains (Sec. IV.B; scaled
    from 11 grains / 548,565 atoms to 16 grains / about 2M sites).
The tabulated Fe-Cu potentials of Sec. IV.B are not available; an analytic
Finnis-Sinclair form stands in for them (parameter sets below).

Units: Angstrom, eV, fs, atomic mass units, K.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, asdict

import numpy as np

A_LAT = 2.87                 # bcc lattice constant of the A (Fe-like) host, Angstrom
KB = 8.617333262e-5          # Boltzmann constant, eV/K
ACC_CONV = 9.648533212e-3    # (eV/Angstrom)/u -> Angstrom/fs^2
MASS_A = 55.845              # u (Fe)
MASS_B = 63.546              # u (Cu)


# --------------------------------------------------------------------------
# Potential parameter sets (analytic Finnis-Sinclair EAM)
#   pair      phi_XY(r) = eps_XY (rc - r)^2 (c0 + c1 r)
#   density   f_X(r)    = t_X (rc - r)^2
#   embedding F_X(rho)  = -A_X sqrt(rho)
# c0, c1 and A_A solve three conditions for pure A in bcc at a = 2.87 A:
# cohesive energy -4.28 eV/atom, zero pressure, bulk modulus 168 GPa.
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class EamFS:
    rc: float
    c0: float
    c1: float
    eps_aa: float
    eps_ab: float
    eps_bb: float
    t_a: float
    t_b: float
    a_a: float
    a_b: float

    def as_tuple(self):
        return (self.rc, self.c0, self.c1, self.eps_aa, self.eps_ab, self.eps_bb,
                self.t_a, self.t_b, self.a_a, self.a_b)

    def as_dict(self):
        return asdict(self)


_RC = 3.6
_C0 = 1.644349182320313
_C1 = -0.585659593910426
_AA = 1.423563309814

PARAM_SETS = {
    # performance set: distinct A-A / A-B / B-B pair terms, species-dependent density
    "FS-P1": EamFS(_RC, _C0, _C1, 1.0, 1.2, 0.85, 1.0, 1.25, _AA, 1.2),
    # identical species: every transmutation has Delta U = 0
    "IDEAL": EamFS(_RC, _C0, _C1, 1.0, 1.0, 1.0, 1.0, 1.0, _AA, _AA),
    # only the own embedding differs: sites are independent
    "INDEP": EamFS(_RC, _C0, _C1, 1.0, 1.0, 1.0, 1.0, 1.0, _AA, 1.2),
    # A <-> B symmetric
    "SYM": EamFS(_RC, _C0, _C1, 1.0, 1.2, 1.0, 1.0, 1.0, _AA, _AA),
    # species-independent density f_A = f_B (the neighbour-embedding term vanishes)
    "LITERAL": EamFS(_RC, _C0, _C1, 1.0, 1.2, 0.85, 1.0, 1.0, _AA, 1.2),
}


def params(name: str = "FS-P1") -> EamFS:
    return PARAM_SETS[name]


# --------------------------------------------------------------------------
# Tabulated potentials (a general two-species EAM given by tables, the form in
# which published EAM potentials are distributed): f_A, f_B, phi_AA, phi_AB, phi_BB at
# the radial knots r_k = k dr (k < nr), F_A, F_B at the density knots
# rho_k = k drho (k < nrho).  Pair and density terms vanish for r >= rc.
# The sets below tabulate closed forms on the knots; how the tables are
# interpolated is the consumer's business.
# --------------------------------------------------------------------------
@dataclass(eq=False)
class EamTable:
    rc: float
    dr: float
    drho: float
    f: np.ndarray     # (2, nr)
    phi: np.ndarray   # (3, nr): AA, AB, BB
    F: np.ndarray     # (2, nrho)

    @property
    def nr(self) -> int:
        return int(self.f.shape[1])

    @property
    def nrho(self) -> int:
        return int(self.F.shape[1])


def _tabulate(rc, dr, drho, rho_max, f, phi, F) -> EamTable:
    nr = int(math.ceil(rc / dr)) + 2
    nrho = int(math.ceil(rho_max / drho)) + 1
    r = dr * np.arange(nr, dtype=np.float64)
    rho = drho * np.arange(nrho, dtype=np.float64)
    inside = r < rc
    tf = np.stack([np.where(inside, f(x, r), 0.0) for x in (0, 1)])
    tphi = np.stack([np.where(inside, phi(k, r), 0.0) for k in (0, 1, 2)])
    tF = np.stack([F(x, rho) for x in (0, 1)])
    return EamTable(rc, dr, drho, np.ascontiguousarray(tf), np.ascontiguousarray(tphi),
                    np.ascontiguousarray(tF))


def table_fs(pot: EamFS, dr: float = 0.005, drho: float = 0.02,
             rho_max: float = 80.0) -> EamTable:
    """The Finnis-Sinclair functions of `pot` on the knots."""
    eps = (pot.eps_aa, pot.eps_ab, pot.eps_bb)
    t = (pot.t_a, pot.t_b)
    A = (pot.a_a, pot.a_b)
    return _tabulate(pot.rc, dr, drho, rho_max,
                     lambda x, r: t[x] * (pot.rc - r) ** 2,
                     lambda k, r: eps[k] * (pot.rc - r) ** 2 * (pot.c0 + pot.c1 * r),
                     lambda x, rho: -A[x] * np.sqrt(rho))


def table_x(dr: float = 0.01, drho: float = 0.05, rho_max: float = 80.0) -> EamTable:
    """A tabulated EAM unlike the Finnis-Sinclair form in every function: a
    cubic density tail, an extra cubic pair term and a linear embedding term
    (the FS-P1 parameters otherwise)."""
    p = PARAM_SETS["FS-P1"]
    eps = (p.eps_aa, p.eps_ab, p.eps_bb)
    t = (p.t_a, p.t_b)
    A = (p.a_a, p.a_b)
    return _tabulate(p.rc, dr, drho, rho_max,
                     lambda x, r: t[x] * (p.rc - r) ** 2 * (1.0 + 0.3 * (p.rc - r)),
                     lambda k, r: eps[k] * ((p.rc - r) ** 2 * (p.c0 + p.c1 * r)
                                            + 0.05 * (p.rc - r) ** 3),
                     lambda x, rho: -A[x] * np.sqrt(rho) + (0.002 + 0.001 * x) * rho)


def _plateau(r, lo, hi, w):
    """1 on [lo, hi], 0 farther than w outside it, a smooth cubic step between."""
    def step(t):
        t = np.clip(t, 0.0, 1.0)
        return t * t * (3.0 - 2.0 * t)
    return step((r - (lo - w)) / w) * step(((hi + w) - r) / w)


def table_ising(U: float = 0.1, dr: float = 0.01) -> EamTable:
    """The Ising-type bcc model of Sec. II.B as a tabulated pair model for
    the rigid lattice (a = 2.87 A): phi_XY equals eps_XY(1) on a plateau
    around the first-shell distance (2.49 A) and eps_XY(2) on one around the
    second (2.87 A), zero beyond 3.05 A; f = F = 0, so U = 1/2 sum_ij phi.
    eps_AA(1) = eps_BB(1) = -10 U, eps_AB(1) = -9.7 U, eps(2) = -2 U for
    every pair (U in eV).  Every knot within two spacings of a shell
    distance lies on its plateau, so the interpolant is exact there."""
    e1 = (-10.0 * U, -9.7 * U, -10.0 * U)  # AA, AB, BB
    e2 = -2.0 * U
    return _tabulate(3.6, dr, 0.5, 1.0,
                     lambda x, r: 0.0 * r,
                     lambda k, r: e1[k] * _plateau(r, 2.35, 2.62, 0.05)
                     + e2 * _plateau(r, 2.75, 3.0, 0.05),
                     lambda x, rho: 0.0 * rho)


TABLE_SETS = {"TAB-FS1": lambda: table_fs(PARAM_SETS["FS-P1"]), "TAB-X": table_x,
              "ISING": table_ising}


def table(name: str) -> EamTable:
    return TABLE_SETS[name]()


# --------------------------------------------------------------------------
# Structures
# --------------------------------------------------------------------------
def wrap(u: np.ndarray, L: float) -> np.ndarray:
    """Map coordinates into [0, L)."""
    u = np.mod(u, L)
    u[u >= L] -= L
    u[u < 0.0] = 0.0
    return u


def bcc(nx: int, ny: int, nz: int, a: float = A_LAT):
    """Perfect bcc block of nx*ny*nz conventional cells (2 sites each).

    Site index = 2*(ix + nx*(iy + ny*iz)) + basis.  Returns (x, y, z, box)."""
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ix = ix.ravel().astype(np.float64)
    iy = iy.ravel().astype(np.float64)
    iz = iz.ravel().astype(np.float64)
    n = ix.size
    x = np.empty(2 * n)
    y = np.empty(2 * n)
    z = np.empty(2 * n)
    x[0::2] = ix * a
    y[0::2] = iy * a
    z[0::2] = iz * a
    x[1::2] = (ix + 0.5) * a
    y[1::2] = (iy + 0.5) * a
    z[1::2] = (iz + 0.5) * a
    box = np.array([nx * a, ny * a, nz * a], dtype=np.float64)
    return x, y, z, box


def thermalize(x, y, z, box, sigma: float, seed: int):
    """I.i.d. Gaussian displacements (sigma per Cartesian component), wrapped."""
    rng = np.random.default_rng(seed)
    d = rng.normal(0.0, sigma, size=(3, x.size))
    return (wrap(x + d[0], box[0]), wrap(y + d[1], box[1]), wrap(z + d[2], box[2]))


def initial_species(n: int, c_init: float, seed: int) -> np.ndarray:
    """Exactly round(c_init*n) B sites (species 1), placed by a seeded permutation."""
    rng = np.random.default_rng(seed)
    nb = int(round(c_init * n))
    s = np.zeros(n, dtype=np.uint8)
    s[rng.permutation(n)[:nb]] = 1
    return s


def _quat_to_matrix(q):
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def _min_image(d, L):
    return d - L * np.round(d / L)


def voronoi_poly(ncell: int = 100, n_grains: int = 16, seed: int = 1003,
                 a: float = A_LAT, rmin: float = 2.0):
    """Periodic Voronoi polycrystal of randomly oriented bcc grains.

    The cubic box has edge ncell*a (so a single crystal would hold 2*ncell^3
    sites).  Grain seeds are uniform in the box; orientations are uniform unit
    quaternions.  Each grain's Voronoi cell (minimum-image distance to the
    seeds) is filled with its rotated bcc lattice centred on the seed.  For
    every cross-grain pair closer than rmin, the atom later in (grain, index)
    order is removed, pairs taken in ascending order.

    Returns (x, y, z, box, grain)."""
    from scipy.spatial import cKDTree

    L = ncell * a
    box = np.array([L, L, L])
    rng = np.random.default_rng(seed)
    seeds = rng.uniform(0.0, L, size=(n_grains, 3))
    q = rng.normal(size=(n_grains, 4))
    q /= np.linalg.norm(q, axis=1)[:, None]

    # Extent of each Voronoi cell, from a coarse probe grid (+ a margin).
    g = 48
    t = (np.arange(g) + 0.5) * (L / g)
    P = np.stack(np.meshgrid(t, t, t, indexing="ij"), axis=-1).reshape(-1, 3)
    d2 = np.zeros((P.shape[0], n_grains))
    for k in range(n_grains):
        d = _min_image(P - seeds[k], L)
        d2[:, k] = np.einsum("ij,ij->i", d, d)
    owner = np.argmin(d2, axis=1)
    rmax = np.zeros(n_grains)
    for k in range(n_grains):
        sel = owner == k
        rmax[k] = math.sqrt(d2[sel, k].max()) if sel.any() else 0.0
    rmax += math.sqrt(3.0) * (L / g) + 2.0 * a

    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])
    xs, grains = [], []
    for k in range(n_grains):
        R = _quat_to_matrix(q[k])
        m = int(math.ceil(rmax[k] / a)) + 1
        r1 = np.arange(-m, m + 1, dtype=np.float64)
        I = np.stack(np.meshgrid(r1, r1, r1, indexing="ij"), axis=-1).reshape(-1, 3)
        U = (I[:, None, :] + basis[None, :, :]).reshape(-1, 3) * a
        U = U[np.einsum("ij,ij->i", U, U) <= rmax[k] ** 2]
        U = U[np.all(np.abs(U) < 0.5 * L, axis=1)]
        p = seeds[k] + U @ R.T
        p = np.stack([wrap(p[:, 0].copy(), L), wrap(p[:, 1].copy(), L),
                      wrap(p[:, 2].copy(), L)], axis=1)
        best = np.full(p.shape[0], np.inf)
        arg = np.zeros(p.shape[0], dtype=np.int64)
        for kk in range(n_grains):
            d = _min_image(p - seeds[kk], L)
            dd = np.einsum("ij,ij->i", d, d)
            upd = dd < best
            best[upd] = dd[upd]
            arg[upd] = kk
        p = p[arg == k]
        xs.append(p)
        grains.append(np.full(p.shape[0], k, dtype=np.int32))
    pos = np.concatenate(xs)
    grain = np.concatenate(grains)

    tree = cKDTree(pos, boxsize=L)
    pairs = tree.query_pairs(rmin, output_type="ndarray")
    if pairs.size:
        pairs = np.sort(pairs, axis=1)
        pairs = pairs[grain[pairs[:, 0]] != grain[pairs[:, 1]]]
        order = np.lexsort((pairs[:, 1], pairs[:, 0]))
        pairs = pairs[order]
    removed = np.zeros(pos.shape[0], dtype=bool)
    for i, j in pairs:
        if not removed[i] and not removed[j]:
            removed[j] = True
    keep = ~removed
    pos = pos[keep]
    grain = grain[keep]
    return (np.ascontiguousarray(pos[:, 0]), np.ascontiguousarray(pos[:, 1]),
            np.ascontiguousarray(pos[:, 2]), box, grain)


def mb_velocities(species: np.ndarray, T: float, seed: int):
    """Maxwell-Boltzmann velocities (Angstrom/fs) at temperature T with the
    centre-of-mass momentum removed, rescaled to exactly T over 3N-3 degrees
    of freedom."""
    rng = np.random.default_rng(seed)
    m = np.where(species == 0, MASS_A, MASS_B)
    n = species.size
    sig = np.sqrt(KB * T / m * ACC_CONV)
    v = rng.normal(size=(3, n)) * sig[None, :]
    M = m.sum()
    for k in range(3):
        v[k] -= (m * v[k]).sum() / M
    ke = 0.5 * (m[None, :] * v * v).sum() / ACC_CONV
    t_now = 2.0 * ke / ((3 * n - 3) * KB)
    v *= math.sqrt(T / t_now)
    return (np.ascontiguousarray(v[0]), np.ascontiguousarray(v[1]),
            np.ascontiguousarray(v[2]))


def kinetic_temperature(vx, vy, vz, species):
    m = np.where(species == 0, MASS_A, MASS_B)
    ke = 0.5 * (m * (vx * vx + vy * vy + vz * vz)).sum() / ACC_CONV
    return 2.0 * ke / ((3 * species.size - 3) * KB), ke
