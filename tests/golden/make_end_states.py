"""Write the oracle's end states that the long GPU parity tests compare with
(tests/golden/end_states.json).  Calls only the oracle and the seeded input
generators (the serial oracle; on the polycrystal the sweeps use its
multi-threaded form, which is the serial chain bit for bit, as
tests/test_oracle_omp.py checks).

  c2_1000[cbar]  the 40^3 thermal system after 1,000 sweeps (kappa = 1000,
                 600 K, its calibrated dmu0) at cbar = 0.02, 0.05, 0.10
  c3_hybrid      the 1.96M-site polycrystal with Maxwell-Boltzmann velocities:
                 one sweep, 20 velocity-Verlet steps of 1 fs, one more sweep
  c3_production  the same polycrystal on the production schedule's path: 3
                 conjugate-gradient line searches, 4 Nose-Hoover NPT steps of
                 2.5 fs (700 K, zero pressure, 100 and 1000 fs coupling
                 times), one sweep

Each entry holds the sweep statistics and SHA-256 digests of the species,
density cache (and, for c3_hybrid, positions and velocities) as raw bytes.

    python tests/golden/make_end_states.py [c2] [c3] [c3p]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1012_5082_amd import inputs as I  # noqa: E402
from paper_1012_5082_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "end_states.json")
STAT_KEYS = ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final",
             "sum_n", "sum_n2")


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def add_stats(tot, s):
    if tot is None:
        return dict(s)
    out = {k: tot[k] + s[k] for k in tot}
    out["n_final"] = s["n_final"]
    return out


def c2_1000(cbar):
    pot = I.params("FS-P1")
    d = W.c2(cbar=cbar)
    st = O.SweepState(d["x"], d["y"], d["z"], d["box"], d["species"], pot)
    s, _, _ = O.sweep(st, d["dmu0"], d["kappa"], cbar, d["T"], 1000, d["seed"])
    return {"stats": {k: s[k] for k in STAT_KEYS}, "species": digest(st.species),
            "rho": digest(st.rho)}


def c3_hybrid():
    pot = I.params("FS-P1")
    d = W.c3()
    args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    st = O.SweepState(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"],
                      vy=d["vy"], vz=d["vz"])
    s1, _ = O.sweep_omp(st, *args, 1, d["seed"])
    x, y, z, vx, vy, vz, *_ = O.md(d["x"], d["y"], d["z"], st.vx, st.vy, st.vz, st.species,
                                   d["box"], pot, d["dt"], d["md_steps"])
    st2 = O.SweepState(x, y, z, d["box"], st.species, pot, vx=vx, vy=vy, vz=vz)
    st2.w = 1
    s2, _ = O.sweep_omp(st2, *args, 1, d["seed"])
    tot = add_stats(add_stats(None, s1), s2)
    return {"dmu0": d["dmu0"], "n_sites": int(d["x"].size),
            "stats_sweep1": {k: s1[k] for k in STAT_KEYS},
            "stats": {k: tot[k] for k in STAT_KEYS},
            "species": digest(st2.species), "rho": digest(st2.rho),
            "x": digest(x), "y": digest(y), "z": digest(z),
            "vx": digest(st2.vx), "vy": digest(st2.vy), "vz": digest(st2.vz)}


def c3_production():
    pot = I.params("FS-P1")
    d = W.c3()
    (x1, y1, z1, *_), relax, _ = O.cg(d["x"], d["y"], d["z"], d["species"], d["box"], pot,
                                      max_iter=3, ftol=1e-3, dmax=0.1)
    st, box, state, _ = O.md_npt(x1, y1, z1, d["vx"], d["vy"], d["vz"], d["species"], d["box"],
                                 pot, 2.5, 4, 700.0, 100.0, 0.0, 1000.0)
    ost = O.SweepState(*st[:3], box, d["species"], pot, vx=st[3], vy=st[4], vz=st[5])
    s1, _ = O.sweep_omp(ost, d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"])
    return {"dmu0": d["dmu0"], "n_sites": int(d["x"].size), "relax": relax,
            "box": [float(v) for v in box], "stats": {k: s1[k] for k in STAT_KEYS},
            "species": digest(ost.species), "rho": digest(ost.rho),
            "x": digest(st[0]), "y": digest(st[1]), "z": digest(st[2]),
            "vx": digest(ost.vx), "vy": digest(ost.vy), "vz": digest(ost.vz)}


def main():
    what = sys.argv[1:] or ["c2", "c3"]
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    t0 = time.time()
    if "c2" in what:
        res["c2_1000"] = {str(cb): c2_1000(cb) for cb in (0.02, 0.05, 0.10)}
        print(f"c2 done ({time.time() - t0:.0f} s)", flush=True)
    if "c3" in what:
        res["c3_hybrid"] = c3_hybrid()
        print(f"c3 done ({time.time() - t0:.0f} s)", flush=True)
    if "c3p" in what:
        res["c3_production"] = c3_production()
        print(f"c3p done ({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
