"""Workload definitions (synthetic, seeded), shaped like the paper's runs.

  c1   rigid 10x10x10 bcc, 2,000 sites (the per-processor block of the
       weak-scaling study, Sec. III.C), kappa = 1000, cbar = 0.05, 600 K
  c2   40x40x40 bcc, 128,000 sites, Gaussian displacements of 0.05 A
       (the 40^3 lattice of the parallel runs, Sec. III.C, Fig. 7),
       kappa = 1000, cbar in {0.02, 0.05, 0.10}, 600 K
  c3   16-grain Voronoi nanocrystal in a 100^3-cell box (about 1.96M sites
       after removing close cross-grain pairs), kappa = 1000, cbar = 0.03,
       700 K, 1 MC sweep per 20 velocity-Verlet steps of 1 fs (Sec. IV.B uses
       one MC cycle per 20 MD steps, 700 K, kappa = 1000)
  c4   64 rigid bcc replicas of uneven size (2,000 to 250,000 sites,
       log-uniform) on a T x kappa x cbar grid

dmu0 comes from dmu_table.json (written by oracle/calibrate_dmu.py); c3 takes
it from dmu_c3.json (oracle/calibrate_dmu_c3.py, calibrated on c3 itself).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def dmu_s(T: float, cbar: float) -> float:
    """Calibrated dmu_S(T, cbar) (eV), linear in cbar between table points."""
    tab = json.load(open(os.path.join(HERE, "dmu_table.json")))["entries"]
    Ts = sorted({e["T"] for e in tab})
    Tn = min(Ts, key=lambda t: abs(t - T))
    rows = sorted((e["cbar"], e["dmu"]) for e in tab if e["T"] == Tn)
    cs = np.array([r[0] for r in rows])
    ds = np.array([r[1] for r in rows])
    return float(np.interp(cbar, cs, ds))


def c1(c_init=0.05, seed=1001):
    x, y, z, box = I.bcc(10, 10, 10)
    sp = I.initial_species(x.size, c_init, seed)
    return dict(x=x, y=y, z=z, box=box, species=sp, T=600.0, kappa=1000.0, cbar=0.05,
                dmu0=dmu_s(600.0, 0.05), seed=2001, name="c1-bcc10")


def c2(cbar=0.05, seed=1002):
    x, y, z, box = I.bcc(40, 40, 40)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, cbar, seed + 10)
    return dict(x=x, y=y, z=z, box=box, species=sp, T=600.0, kappa=1000.0, cbar=cbar,
                dmu0=dmu_s(600.0, cbar), seed=2002, name="c2-bcc40-thermal")


def dmu_c3(T: float, cbar: float, kappa: float):
    """dmu0 calibrated on the polycrystal itself (dmu_c3.json, written by
    oracle/calibrate_dmu_c3.py), or None for another operating point."""
    path = os.path.join(HERE, "dmu_c3.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path))
    if e["T"] == T and e["cbar"] == cbar and e["kappa"] == kappa:
        return float(e["dmu0"])
    return None


def c3(seed=1003, cbar=0.03, T=700.0, with_velocities=True, calibrated=True):
    """calibrated: dmu0 from the calibration on this system when there is one
    for (T, cbar), else from the rigid-lattice table."""
    x, y, z, box, grain = I.voronoi_poly(100, 16, seed)
    sp = I.initial_species(x.size, cbar, seed + 10)
    dmu0 = dmu_c3(T, cbar, 1000.0) if calibrated else None
    if dmu0 is None:
        dmu0 = dmu_s(T, cbar)
    d = dict(x=x, y=y, z=z, box=box, species=sp, grain=grain, T=T, kappa=1000.0, cbar=cbar,
             dmu0=dmu0, seed=2003, dt=1.0, md_steps=20, name="c3-voronoi16")
    if with_velocities:
        d["vx"], d["vy"], d["vz"] = I.mb_velocities(sp, T, seed + 20)
    return d


def c4_replicas(n_rep=64, seed=1004):
    """Sizes log-uniform in [2,000, 250,000] as 2 nx ny nz with every n >= 6;
    T = {400,600,800}[r mod 3], kappa = {100,1000}[(r div 3) mod 2],
    cbar log-uniform in [0.01, 0.2]."""
    rng = np.random.default_rng(seed)
    reps = []
    for r in range(n_rep):
        target = math.exp(rng.uniform(math.log(2000), math.log(250000)))
        cells = target / 2.0
        base = max(6, int(round(cells ** (1.0 / 3.0))))
        nx = base
        ny = max(6, int(round(math.sqrt(cells / nx))))
        nz = max(6, int(round(cells / (nx * ny))))
        T = [400.0, 600.0, 800.0][r % 3]
        kappa = [100.0, 1000.0][(r // 3) % 2]
        cbar = math.exp(rng.uniform(math.log(0.01), math.log(0.2)))
        reps.append(dict(nx=nx, ny=ny, nz=nz, T=T, kappa=kappa, cbar=cbar,
                         dmu0=dmu_s(T, cbar), seed=3000 + r))
    return reps
