"""ctypes wrapper of the plain serial FP64 oracle (oracle/oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  The oracle
shares no code with the HIP library; both sides only share the seeded input
generators.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VCSGC_ORACLE_LIB points the tests at another build of oracle.c (used by
# tests/mutation_check.py to confirm that planted mistakes are caught).
LIB_PATH = os.environ.get("VCSGC_ORACLE_LIB", os.path.join(_HERE, "liboracle.so"))
SRC = os.path.join(_HERE, "oracle.c")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c11", "-fopenmp"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction into fused multiply-adds)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Pot(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("rc", "c0", "c1", "eps_aa", "eps_ab", "eps_bb", "t_a", "t_b", "a_a", "a_b")] + [
        ("tab", C.c_int32), ("nr", C.c_int32), ("nrho", C.c_int32), ("pad_", C.c_int32),
        ("inv_dr", C.c_double), ("inv_drho", C.c_double),
        ("cf", C.c_void_p * 2), ("cphi", C.c_void_p * 3), ("cF", C.c_void_p * 2)]


class SweepArgs(C.Structure):
    _fields_ = [("dmu0", C.c_double), ("kappa", C.c_double), ("cbar", C.c_double),
                ("temp", C.c_double), ("seed", C.c_uint64), ("replica", C.c_uint64),
                ("w0", C.c_int64), ("n_sweeps", C.c_int64), ("r_dep", C.c_double),
                ("one_cell", C.c_int32), ("mass_a", C.c_double), ("mass_b", C.c_double),
                ("local_steps", C.c_int32), ("colour_period", C.c_int32),
                ("grow_edge", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("trials", C.c_int64), ("local_accepts", C.c_int64), ("stages", C.c_int64),
                ("stage_accepts", C.c_int64), ("flips", C.c_int64), ("near_ties", C.c_int64),
                ("n_final", C.c_int64), ("sum_n", C.c_double), ("sum_n2", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Mlp(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("b1", C.c_void_p), ("w2", C.c_void_p), ("b2", C.c_void_p),
                ("w3", C.c_void_p), ("b3", C.c_void_p), ("mu", C.c_void_p), ("sd", C.c_void_p),
                ("out_mu", C.c_float), ("out_sd", C.c_float)]


class Da(C.Structure):
    _fields_ = [("mode", C.c_int), ("table", C.c_void_p), ("n_table", C.c_int64),
                ("mlp", C.c_void_p), ("dstart", C.c_void_p), ("dnj", C.c_void_p),
                ("dnr", C.c_void_p), ("stage1_pass", C.c_int64), ("dlog", C.c_void_p),
                ("dcap", C.c_int64), ("dn", C.c_int64)]


DA_MODES = {"off": 0, "table": 1, "perfect": 2, "zero": 3, "mlp": 4}
DESC_CUTOFF = 4.41
N_PARAMS = 4929

_P = C.c_void_p
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        L.or_philox4x64_10.argtypes = [_P, _P, _P]
        L.or_spline_coeffs.argtypes = [C.c_int32, _P, _P]
        L.or_spline_eval.restype = C.c_double
        L.or_spline_eval.argtypes = [_P, C.c_int32, C.c_double, C.c_double, _P]
        L.or_neighbors.restype = C.c_int64
        L.or_neighbors.argtypes = [C.c_int64, _P, _P, _P, _P, C.c_double, C.c_int, C.c_int64,
                                   _P, _P, _P, _P, _P, _P]
        L.or_density.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P]
        L.or_energy_atoms.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P]
        L.or_energy_total.restype = C.c_double
        L.or_energy_total.argtypes = [C.c_int64, _P]
        L.or_forces.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        L.or_delta_u.restype = C.c_double
        L.or_delta_u.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P]
        L.or_cell_grid.restype = C.c_int
        L.or_cell_grid.argtypes = [_P, C.c_double, _P]
        L.or_cell_grid_p.restype = C.c_int
        L.or_cell_grid_p.argtypes = [_P, C.c_double, C.c_int, _P]
        L.or_sweep.restype = C.c_int
        L.or_sweep.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                               _P, _P, _P, _P, C.c_int64, _P, _P, C.c_int64, _P, _P,
                               C.c_int64, _P]
        L.or_sweep_omp.restype = C.c_int
        L.or_sweep_omp.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                   _P, _P, _P, _P, C.c_int64, _P, C.c_int, _P]
        L.or_sweep_da.restype = C.c_int
        L.or_sweep_da.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                  _P, _P, C.c_int64, _P, _P, C.c_int64, _P, _P]
        L.or_descriptor.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, C.c_int, _P]
        L.or_bf16.restype = C.c_float
        L.or_bf16.argtypes = [C.c_float]
        L.or_mlp_forward.argtypes = [_P, C.c_int64, _P, C.c_int, _P, _P]
        L.or_mlp_grad.restype = C.c_double
        L.or_mlp_grad.argtypes = [_P, C.c_int64, _P, _P, C.c_int, _P]
        L.or_md.restype = C.c_int
        L.or_md.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double,
                            C.c_double, C.c_double, C.c_int64, _P, _P, _P, _P]
        L.or_md_omp.restype = C.c_int
        L.or_md_omp.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double,
                                C.c_double, C.c_double, C.c_int64, _P, _P, _P, _P, C.c_int]
        L.or_tree_sum.restype = C.c_double
        L.or_tree_sum.argtypes = [C.c_int64, _P]
        L.or_md_nvt.restype = C.c_int
        L.or_md_nvt.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double,
                                C.c_double, C.c_double, C.c_int64, C.c_double, C.c_double,
                                _P, _P, _P, _P, _P, _P]
        L.or_md_npt.restype = C.c_int
        L.or_md_npt.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_double,
                                C.c_double, C.c_double, C.c_int64, C.c_double, C.c_double,
                                C.c_double, C.c_double, _P, _P, _P, _P, _P, _P]
        L.or_cg.restype = C.c_int
        L.or_cg.argtypes = [C.c_int64, _P, _P, _P, _P, _P, _P, C.c_int64, C.c_int64,
                            C.c_double, C.c_double, C.c_double, C.c_int, _P, _P, _P, _P, _P,
                            _P, _P, _P, _P, _P, C.c_int64]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def spline_coeffs(y) -> np.ndarray:
    """The oracle's piecewise-cubic coefficients (4 per interval) through y."""
    y = _f64(y)
    c = np.zeros(4 * (y.size - 1))
    lib().or_spline_coeffs(int(y.size), _p(y), _p(c))
    return c


def spline_eval(c, n, x, inv_h):
    """(value, derivative) of the interpolant with coefficients c at x."""
    d = C.c_double()
    v = lib().or_spline_eval(_p(_f64(c)), int(n), float(x), float(inv_h), C.byref(d))
    return v, d.value


def pot_struct(pot) -> Pot:
    """The oracle's potential: analytic Finnis-Sinclair parameters, or a table
    (paper_1012_5082_amd.inputs.EamTable) with its coefficients computed here;
    they are kept on the table object as long as it lives."""
    if not hasattr(pot, "phi"):
        return Pot(*pot.as_tuple())
    co = getattr(pot, "_oracle_coeffs", None)
    if co is None:
        co = ([spline_coeffs(pot.f[x]) for x in (0, 1)],
              [spline_coeffs(pot.phi[k]) for k in (0, 1, 2)],
              [spline_coeffs(pot.F[x]) for x in (0, 1)])
        pot._oracle_coeffs = co
    P = Pot(pot.rc, *([0.0] * 9))
    P.tab, P.nr, P.nrho = 1, pot.nr, pot.nrho
    P.inv_dr, P.inv_drho = 1.0 / pot.dr, 1.0 / pot.drho
    for k in range(2):
        P.cf[k] = co[0][k].ctypes.data
        P.cF[k] = co[2][k].ctypes.data
    for k in range(3):
        P.cphi[k] = co[1][k].ctypes.data
    return P


def philox(key, ctr) -> np.ndarray:
    k = np.asarray(key, dtype=np.uint64)
    c = np.asarray(ctr, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_p(k), _p(c), _p(out))
    return out


class NeighborList:
    """CSR neighbour list: row i is entries start[i]:start[i+1] (j, r, dx, dy, dz)."""

    def __init__(self, start, j, r, dx, dy, dz):
        self.start, self.j, self.r, self.dx, self.dy, self.dz = start, j, r, dx, dy, dz

    @property
    def n(self):
        return self.start.size - 1

    def row(self, i):
        return self.j[self.start[i]:self.start[i + 1]]


def neighbors(x, y, z, box, cutoff, mode: int = 0, vectors: bool = True) -> NeighborList:
    """All pairs with r < cutoff; separation vectors only if vectors=True."""
    x, y, z, box = _f64(x), _f64(y), _f64(z), _f64(box)
    n = x.size
    cap = 16 * n + 64
    while True:
        start = np.empty(n + 1, dtype=np.int64)
        j = np.empty(cap, dtype=np.int32)
        r = np.empty(cap)
        dx, dy, dz = ((np.empty(cap) for _ in range(3)) if vectors else (None, None, None))
        tot = lib().or_neighbors(n, _p(x), _p(y), _p(z), _p(box), float(cutoff), int(mode), cap,
                                 _p(start), _p(j), _p(r), _p(dx), _p(dy), _p(dz))
        if tot < 0:
            raise ValueError("box too small for the requested neighbour mode")
        if tot <= cap:
            cut = (lambda a: None if a is None else a[:tot])  # noqa: E731
            return NeighborList(start, j[:tot], r[:tot], cut(dx), cut(dy), cut(dz))
        cap = int(tot)


def density(nl: NeighborList, species, pot) -> np.ndarray:
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    rho = np.zeros(nl.n)
    P = pot_struct(pot)
    lib().or_density(nl.n, _p(nl.start), _p(nl.j), _p(nl.r), _p(sp), C.byref(P), _p(rho))
    return rho


def energy_atoms(nl: NeighborList, species, pot, rho=None) -> np.ndarray:
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    if rho is None:
        rho = density(nl, sp, pot)
    e = np.zeros(nl.n)
    P = pot_struct(pot)
    lib().or_energy_atoms(nl.n, _p(nl.start), _p(nl.j), _p(nl.r), _p(sp), C.byref(P),
                          _p(_f64(rho)), _p(e))
    return e


def energy_total(e) -> float:
    e = _f64(e)
    return lib().or_energy_total(e.size, _p(e))


def forces(nl: NeighborList, species, pot, rho=None):
    if nl.dx is None:
        raise ValueError("forces need a neighbour list built with vectors=True")
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    if rho is None:
        rho = density(nl, sp, pot)
    fx, fy, fz = np.zeros(nl.n), np.zeros(nl.n), np.zeros(nl.n)
    P = pot_struct(pot)
    lib().or_forces(nl.n, _p(nl.start), _p(nl.j), _p(nl.r), _p(nl.dx), _p(nl.dy), _p(nl.dz),
                    _p(sp), C.byref(P), _p(_f64(rho)), _p(fx), _p(fy), _p(fz))
    return fx, fy, fz


def delta_u(nl: NeighborList, i, species, rho, pot) -> float:
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    P = pot_struct(pot)
    return lib().or_delta_u(int(i), _p(nl.start), _p(nl.j), _p(nl.r), _p(sp), _p(_f64(rho)),
                            C.byref(P))


def cell_grid(box, r_dep, period=2):
    box = _f64(box)
    nc = np.zeros(3, dtype=np.int32)
    if lib().or_cell_grid_p(_p(box), float(r_dep), int(period), _p(nc)):
        raise ValueError("box too small for two cells of edge r_dep")
    return nc


class SweepState:
    """Mutable chain state of the oracle (species, rho cache, n, sweep counter)."""

    def __init__(self, x, y, z, box, species, pot, nl: NeighborList | None = None,
                 vx=None, vy=None, vz=None):
        self.x, self.y, self.z, self.box = _f64(x), _f64(y), _f64(z), _f64(box)
        self.pot = pot
        self.species = np.array(species, dtype=np.uint8)
        self.nl = nl if nl is not None else neighbors(self.x, self.y, self.z, self.box, pot.rc,
                                                      vectors=False)
        self.rho = density(self.nl, self.species, pot)
        self.n_b = np.array([int(self.species.sum())], dtype=np.int64)
        self.w = 0
        self.vx = None if vx is None else _f64(vx).copy()
        self.vy = None if vy is None else _f64(vy).copy()
        self.vz = None if vz is None else _f64(vz).copy()

    @property
    def n(self):
        return self.x.size


def sweep(st: SweepState, dmu0, kappa, cbar, T, n_sweeps, seed, replica=0, r_dep=None,
          one_cell=False, log_trials=0, log_stages=0, overrides=None,
          mass_a=55.845, mass_b=63.546, local_steps=1, colour_period=2, grow_edge=0.0):
    """Run n_sweeps sweeps from the state's sweep counter; returns (stats, tlog, slog).
    local_steps = k: k trials per active cell per stage (exact local chains);
    colour_period 3: 27 colours on cells of edge >= r_dep / 2; grow_edge > 0:
    grown domains in cells of edge >= max(grow_edge, 2 r_dep)."""
    L = lib()
    if r_dep is None:
        r_dep = 2.0 * st.pot.rc
    a = SweepArgs(float(dmu0), float(kappa), float(cbar), float(T), int(seed), int(replica),
                  int(st.w), int(n_sweeps), float(r_dep), int(bool(one_cell)),
                  float(mass_a), float(mass_b), int(local_steps), int(colour_period),
                  float(grow_edge))
    tlog = np.zeros((max(log_trials, 0), 8)) if log_trials else None
    slog = np.zeros((max(log_stages, 0), 8)) if log_stages else None
    tn = np.zeros(1, dtype=np.int64)
    sn = np.zeros(1, dtype=np.int64)
    ov = None if overrides is None or len(overrides) == 0 else _f64(overrides)
    nov = 0 if ov is None else ov.shape[0]
    s = Stats()
    P = pot_struct(st.pot)
    rc = L.or_sweep(st.n, _p(st.x), _p(st.y), _p(st.z), _p(st.box), _p(st.nl.start),
                    _p(st.nl.j), _p(st.nl.r), _p(st.species), _p(st.rho), _p(st.n_b),
                    C.byref(P), C.byref(a), _p(st.vx), _p(st.vy), _p(st.vz),
                    _p(tlog), int(log_trials), _p(tn), _p(slog), int(log_stages), _p(sn),
                    _p(ov), int(nov), C.byref(s))
    if rc != 0:
        raise ValueError(f"or_sweep failed ({rc})")
    st.w += int(n_sweeps)
    if tlog is not None:
        tlog = tlog[:min(int(tn[0]), log_trials)]
    if slog is not None:
        slog = slog[:min(int(sn[0]), log_stages)]
    return s.as_dict(), tlog, slog


def sweep_omp(st: SweepState, dmu0, kappa, cbar, T, n_sweeps, seed, threads=None, replica=0,
              r_dep=None, log_stages=0, mass_a=55.845, mass_b=63.546, colour_period=2):
    """or_sweep's plain chain with the trials of each stage on several host
    threads (bitwise the serial chain); returns (stats, slog)."""
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    if r_dep is None:
        r_dep = 2.0 * st.pot.rc
    a = SweepArgs(float(dmu0), float(kappa), float(cbar), float(T), int(seed), int(replica),
                  int(st.w), int(n_sweeps), float(r_dep), 0, float(mass_a), float(mass_b), 1,
                  int(colour_period))
    slog = np.zeros((max(log_stages, 0), 8)) if log_stages else None
    sn = np.zeros(1, dtype=np.int64)
    s = Stats()
    P = pot_struct(st.pot)
    rc = lib().or_sweep_omp(st.n, _p(st.x), _p(st.y), _p(st.z), _p(st.box), _p(st.nl.start),
                            _p(st.nl.j), _p(st.nl.r), _p(st.species), _p(st.rho), _p(st.n_b),
                            C.byref(P), C.byref(a), _p(st.vx), _p(st.vy), _p(st.vz),
                            _p(slog), int(log_stages), _p(sn), int(threads), C.byref(s))
    if rc != 0:
        raise ValueError(f"or_sweep_omp failed ({rc})")
    st.w += int(n_sweeps)
    if slog is not None:
        slog = slog[:min(int(sn[0]), log_stages)]
    return s.as_dict(), slog


def md(x, y, z, vx, vy, vz, species, box, pot, dt, n_steps, mass_a=55.845, mass_b=63.546):
    """Velocity Verlet; returns new arrays (x, y, z, vx, vy, vz, fx, fy, fz, rho)."""
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    n = x.size
    fx, fy, fz, rho = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    P = pot_struct(pot)
    rc = lib().or_md(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(sp), _p(_f64(box)),
                     C.byref(P), float(mass_a), float(mass_b), float(dt), int(n_steps),
                     _p(fx), _p(fy), _p(fz), _p(rho))
    if rc != 0:
        raise ValueError("or_md failed")
    return x, y, z, vx, vy, vz, fx, fy, fz, rho


def md_omp(x, y, z, vx, vy, vz, species, box, pot, dt, n_steps, threads=None, mass_a=55.845,
           mass_b=63.546):
    """md() with every per-atom loop on several host threads (bitwise md())."""
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    n = x.size
    fx, fy, fz, rho = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    P = pot_struct(pot)
    rc = lib().or_md_omp(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(sp), _p(_f64(box)),
                         C.byref(P), float(mass_a), float(mass_b), float(dt), int(n_steps),
                         _p(fx), _p(fy), _p(fz), _p(rho), int(threads))
    if rc != 0:
        raise ValueError("or_md_omp failed")
    return x, y, z, vx, vy, vz, fx, fy, fz, rho


def tree_sum(v) -> float:
    v = _f64(v)
    return lib().or_tree_sum(v.size, _p(v))


def md_nvt(x, y, z, vx, vy, vz, species, box, pot, dt, n_steps, T, tau, xi=0.0, eta=0.0,
           mass_a=55.845, mass_b=63.546):
    """Nose-Hoover NVT velocity Verlet; returns new arrays
    (x, y, z, vx, vy, vz, fx, fy, fz, rho) and the thermostat state (xi, eta)."""
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    n = x.size
    fx, fy, fz, rho = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    th = np.array([xi, eta], dtype=np.float64)
    P = pot_struct(pot)
    rc = lib().or_md_nvt(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(sp), _p(_f64(box)),
                         C.byref(P), float(mass_a), float(mass_b), float(dt), int(n_steps),
                         float(T), float(tau), _p(th[0:1]), _p(th[1:2]), _p(fx), _p(fy), _p(fz),
                         _p(rho))
    if rc != 0:
        raise ValueError("or_md_nvt failed")
    return (x, y, z, vx, vy, vz, fx, fy, fz, rho), (float(th[0]), float(th[1]))


def md_npt(x, y, z, vx, vy, vz, species, box, pot, dt, n_steps, T, tau_t, p_ext, tau_p,
           xi=0.0, eta=0.0, pe=0.0, mass_a=55.845, mass_b=63.546):
    """Isotropic NPT (Nose-Hoover thermostat and barostat) velocity Verlet;
    returns (x, y, z, vx, vy, vz, fx, fy, fz, rho), the new box, the state
    (xi, eta, pe) and the virial of the last force evaluation.  p_ext in
    eV/A^3."""
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    vx, vy, vz = _f64(vx).copy(), _f64(vy).copy(), _f64(vz).copy()
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    n = x.size
    fx, fy, fz, rho = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    b = _f64(box).copy()
    st = np.array([xi, eta, pe], dtype=np.float64)
    vir = np.zeros(1)
    P = pot_struct(pot)
    rc = lib().or_md_npt(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(sp), _p(b),
                         C.byref(P), float(mass_a), float(mass_b), float(dt), int(n_steps),
                         float(T), float(tau_t), float(p_ext), float(tau_p), _p(st), _p(fx),
                         _p(fy), _p(fz), _p(rho), _p(vir))
    if rc != 0:
        raise ValueError("or_md_npt failed")
    return ((x, y, z, vx, vy, vz, fx, fy, fz, rho), b, (float(st[0]), float(st[1]), float(st[2])),
            float(vir[0]))


CG_REASONS = {1: "force", 2: "energy", 3: "iterations", 4: "evaluations", 5: "line search"}


def cg(x, y, z, species, box, pot, max_iter=1000, max_eval=100000, etol=0.0, ftol=1e-6,
       dmax=0.1, steepest=False, log_cap=0):
    """Conjugate-gradient relaxation (PR+ with a backtracking Armijo line
    search) at fixed species and box.  Returns (x, y, z, fx, fy, fz, rho),
    a dict (iterations, evaluations, energy, fnorm, reason) and the
    per-iteration log rows (E, E', a, sl, b, restart)."""
    x, y, z = _f64(x).copy(), _f64(y).copy(), _f64(z).copy()
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    n = x.size
    fx, fy, fz, rho = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)
    it, ev = np.zeros(1, np.int64), np.zeros(1, np.int64)
    e, fn = np.zeros(1), np.zeros(1)
    reason = np.zeros(1, np.int32)
    log = np.zeros((max(log_cap, 1), 6))
    P = pot_struct(pot)
    rc = lib().or_cg(n, _p(x), _p(y), _p(z), _p(sp), _p(_f64(box)), C.byref(P), int(max_iter),
                     int(max_eval), float(etol), float(ftol), float(dmax), int(bool(steepest)),
                     _p(fx), _p(fy), _p(fz), _p(rho), _p(it), _p(ev), _p(e), _p(fn),
                     _p(reason), _p(log) if log_cap > 0 else None, int(log_cap))
    if rc != 0:
        raise ValueError("or_cg failed")
    info = dict(iterations=int(it[0]), evaluations=int(ev[0]), energy=float(e[0]),
                fnorm=float(fn[0]), reason=int(reason[0]))
    return (x, y, z, fx, fy, fz, rho), info, log[:min(info["iterations"], log_cap)]


# ---------------------------------------------------------------------------
# surrogate
# ---------------------------------------------------------------------------
class MlpParams:
    """FP32 parameters of the 10-64-64-1 SiLU network plus the input and
    output normalization."""

    def __init__(self, w1, b1, w2, b2, w3, b3, mu, sd, out_mu, out_sd):
        f = lambda a, shape: np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(shape))  # noqa: E731
        self.w1, self.b1 = f(w1, (64, 10)), f(b1, (64,))
        self.w2, self.b2 = f(w2, (64, 64)), f(b2, (64,))
        self.w3, self.b3 = f(w3, (64,)), f(b3, (1,))
        self.mu, self.sd = f(mu, (10,)), f(sd, (10,))
        self.out_mu, self.out_sd = float(np.float32(out_mu)), float(np.float32(out_sd))

    @staticmethod
    def random(seed=0, mu=None, sd=None, out_mu=0.0, out_sd=1.0, scale=1.0):
        rng = np.random.default_rng(seed)
        w1 = rng.normal(0, scale / np.sqrt(10), (64, 10))
        w2 = rng.normal(0, scale / np.sqrt(64), (64, 64))
        w3 = rng.normal(0, scale / np.sqrt(64), 64)
        b1, b2, b3 = rng.normal(0, 0.1, 64), rng.normal(0, 0.1, 64), rng.normal(0, 0.1, 1)
        mu = np.zeros(10) if mu is None else mu
        sd = np.ones(10) if sd is None else sd
        return MlpParams(w1, b1, w2, b2, w3, b3, mu, sd, out_mu, out_sd)

    def flat(self):
        return np.concatenate([self.w1.ravel(), self.b1, self.w2.ravel(), self.b2, self.w3,
                               self.b3]).astype(np.float32)

    @staticmethod
    def from_flat(v, mu, sd, out_mu, out_sd):
        v = np.asarray(v, dtype=np.float32)
        return MlpParams(v[:640], v[640:704], v[704:4800], v[4800:4864], v[4864:4928],
                         v[4928:4929], mu, sd, out_mu, out_sd)

    def struct(self):
        m = Mlp(*(a.ctypes.data_as(C.c_void_p) for a in
                  (self.w1, self.b1, self.w2, self.b2, self.w3, self.b3, self.mu, self.sd)),
                self.out_mu, self.out_sd)
        m._keep = self
        return m


def bf16(v):
    return lib().or_bf16(float(v))


def descriptor(nl: NeighborList, i, species, rho, pot, flip=False):
    sp = np.ascontiguousarray(species, dtype=np.uint8)
    out = np.zeros(10)
    P = pot_struct(pot)
    lib().or_descriptor(int(i), _p(nl.start), _p(nl.j), _p(nl.r), _p(sp), _p(_f64(rho)),
                        C.byref(P), int(bool(flip)), _p(out))
    return out


def mlp_forward(m: MlpParams, d, bf16_emul=True):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1, 10))
    y, dE = np.zeros(d.shape[0]), np.zeros(d.shape[0])
    ms = m.struct()
    lib().or_mlp_forward(C.byref(ms), d.shape[0], _p(d), int(bool(bf16_emul)), _p(y), _p(dE))
    return y, dE


def mlp_grad(m: MlpParams, d, t, bf16_emul=False):
    d = np.ascontiguousarray(np.asarray(d, dtype=np.float64).reshape(-1, 10))
    t = _f64(t)
    g = np.zeros(N_PARAMS)
    ms = m.struct()
    loss = lib().or_mlp_grad(C.byref(ms), d.shape[0], _p(d), _p(t), int(bool(bf16_emul)), _p(g))
    return loss, g


def sweep_da(st: SweepState, dmu0, kappa, cbar, T, n_sweeps, seed, mode, replica=0, r_dep=None,
             one_cell=False, table=None, mlp: MlpParams | None = None,
             desc_nl: NeighborList | None = None, log_trials=0, log_stages=0, log_desc=0,
             colour_period=2, grow_edge=0.0):
    """Delayed-acceptance sweeps; returns (stats, stage-1 passes, tlog, slog),
    and with log_desc > 0 (table mode with desc_nl) also the descriptor log:
    rows (w, s, cell, current-state descriptor [10], flipped-state
    descriptor [10]) of every trial, at the trial's state."""
    L = lib()
    if r_dep is None:
        r_dep = 2.0 * st.pot.rc
    a = SweepArgs(float(dmu0), float(kappa), float(cbar), float(T), int(seed), int(replica),
                  int(st.w), int(n_sweeps), float(r_dep), int(bool(one_cell)), 55.845, 63.546, 1,
                  int(colour_period), float(grow_edge))
    da = Da()
    da.mode = DA_MODES[mode]
    keep = []
    if table is not None:
        tab = np.ascontiguousarray(np.asarray(table, dtype=np.float64).reshape(-1, 5))
        tab = tab[np.lexsort((tab[:, 2], tab[:, 1], tab[:, 0]))]
        keep.append(tab)
        da.table, da.n_table = tab.ctypes.data_as(C.c_void_p), tab.shape[0]
    if mlp is not None:
        ms = mlp.struct()
        keep.append(ms)
        da.mlp = C.cast(C.pointer(ms), C.c_void_p)
    if desc_nl is not None:
        da.dstart, da.dnj, da.dnr = _p(desc_nl.start), _p(desc_nl.j), _p(desc_nl.r)
    dlog = None
    if log_desc:
        dlog = np.zeros((log_desc, 23))
        da.dlog, da.dcap = _p(dlog), int(log_desc)
    tlog = np.zeros((max(log_trials, 0), 8)) if log_trials else None
    slog = np.zeros((max(log_stages, 0), 8)) if log_stages else None
    tn, sn = np.zeros(1, dtype=np.int64), np.zeros(1, dtype=np.int64)
    s = Stats()
    P = pot_struct(st.pot)
    rc = L.or_sweep_da(st.n, _p(st.x), _p(st.y), _p(st.z), _p(st.box), _p(st.nl.start),
                       _p(st.nl.j), _p(st.nl.r), _p(st.species), _p(st.rho), _p(st.n_b),
                       C.byref(P), C.byref(a), C.byref(da), _p(tlog), int(log_trials), _p(tn),
                       _p(slog), int(log_stages), _p(sn), C.byref(s))
    if rc != 0:
        raise ValueError(f"or_sweep_da failed ({rc})")
    st.w += int(n_sweeps)
    if tlog is not None:
        tlog = tlog[:min(int(tn[0]), log_trials)]
    if slog is not None:
        slog = slog[:min(int(sn[0]), log_stages)]
    if dlog is not None:
        return s.as_dict(), int(da.stage1_pass), tlog, slog, dlog[:min(int(da.dn), log_desc)]
    return s.as_dict(), int(da.stage1_pass), tlog, slog
