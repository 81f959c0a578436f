"""Calibrate dmu0 for the 16-grain polycrystal workload (1.96M sites, 700 K,
cbar = 0.03, kappa = 1000 eV) on that system itself, with the oracle only.

Parameter strategy of Sec. III.C: the acceptance of the parallel VC-SGC
sweep is largest when dmu0 equals the chemical driving force dmu of the
state being sampled, and Eq. gforce gives that driving force from a VC-SGC
run: dmu = phi + 2 kappa <c> = dmu0 + 2 kappa (<c> - cbar) (kappa per site).
The fixed point dmu0 <- dmu is iterated here.

The run is the workload's hybrid schedule from its initial state: WINDOW
cycles of one sweep and 20 velocity-Verlet steps of 1 fs (Maxwell-Boltzmann
velocities at 700 K, transmuted atoms' velocities rescaled), the window a
benchmark run covers, with <c> averaged over every stage of the window.
The alloy is supersaturated at this concentration and temperature, so the
driving force drifts as the lattice thermalizes and B atoms cluster; the
fixed point is that of the window.  On this non-stationary window the plain
update overshoots (successive estimates alternate about the fixed point at
about equal distance), so each step moves half way: dmu0 <- (dmu0 + dmu)/2.
The sweeps and MD steps run on the oracle's multi-threaded forms, which are
the serial oracle bit for bit (tests/test_oracle_omp.py).

Writes paper_1012_5082_amd/dmu_c3.json.  Calls only the oracle and the
seeded input generators.

    python oracle/calibrate_dmu_c3.py [start_dmu0]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1012_5082_amd import inputs as I  # noqa: E402
from paper_1012_5082_amd import workloads as W  # noqa: E402

OUT = os.path.join(ROOT, "paper_1012_5082_amd", "dmu_c3.json")
WINDOW = 25
MAX_ITERS = 5
TOL = 5e-4  # eV


def window_stats(d, pot, dmu0, threads, t0):
    """WINDOW hybrid cycles from the initial state: per-stage mean n, mean
    local drift dn_tot and stage acceptance."""
    x, y, z = d["x"], d["y"], d["z"]
    vx, vy, vz = d["vx"], d["vy"], d["vz"]
    sp = d["species"]
    ns, dns, accs = [], [], []
    for w in range(WINDOW):
        st = O.SweepState(x, y, z, d["box"], sp, pot, vx=vx, vy=vy, vz=vz)
        st.w = w
        n0 = int(st.n_b[0])
        _, sl = O.sweep_omp(st, dmu0, d["kappa"], d["cbar"], d["T"], 1, d["seed"],
                            threads=threads, log_stages=400)
        dn, acc = sl[:, 3], sl[:, 5]
        ns.append(n0 + np.cumsum(np.where(acc > 0, dn, 0)))
        dns.append(dn)
        accs.append(acc > 0)
        sp = st.species
        x, y, z, vx, vy, vz, *_ = O.md_omp(x, y, z, st.vx, st.vy, st.vz, sp, d["box"], pot,
                                           d["dt"], d["md_steps"], threads=threads)
        print(f"  cycle {w}: stage acceptance {np.mean(acc > 0):.3f}, mean dn_tot "
              f"{np.mean(dn):+.1f} ({time.time() - t0:.0f} s)", flush=True)
    return (float(np.mean(np.concatenate(ns))), float(np.mean(np.concatenate(dns))),
            float(np.mean(np.concatenate(accs))))


def main():
    threads = len(os.sched_getaffinity(0))
    pot = I.params("FS-P1")
    t0 = time.time()
    d = W.c3(calibrated=False)
    N = d["x"].size
    dmu0 = float(sys.argv[1]) if len(sys.argv) > 1 else d["dmu0"]
    print(f"c3: {N} sites, start dmu0 = {dmu0:+.5f}", flush=True)
    iters = []
    for it in range(MAX_ITERS):
        n_mean, drift, acc = window_stats(d, pot, dmu0, threads, t0)
        est = dmu0 + 2.0 * d["kappa"] * (n_mean / N - d["cbar"])
        iters.append({"dmu0": round(dmu0, 6), "mean_n_minus_Ncbar": round(n_mean - N * d["cbar"], 3),
                      "mean_local_dn_tot": round(drift, 3), "stage_acceptance": round(acc, 4),
                      "gforce_dmu": round(est, 6)})
        print(iters[-1], flush=True)
        done = abs(est - dmu0) < TOL
        dmu0 = 0.5 * (dmu0 + est)
        if done:
            break
    res = {"T": d["T"], "cbar": d["cbar"], "kappa": d["kappa"], "n_sites": N,
           "dmu0": round(dmu0, 5),
           "method": (f"Eq. gforce fixed point dmu0 <- dmu0 + kappa (<c> - cbar) (half steps), "
                      f"<c> over every stage of the first {WINDOW} hybrid cycles (1 sweep + 20 MD "
                      f"steps of 1 fs) from the initial state (seeds of the workload), FS-P1"),
           "iterations": iters}
    with open(OUT, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", OUT, f"({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
