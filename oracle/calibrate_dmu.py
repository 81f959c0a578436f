"""Calibrate the chemical-potential difference dmu_S(c, T) of the FS-P1 alloy
with the oracle, following the parameter strategy of Sec. III.C: a small
single-phase run gives the driving force at the target concentration.

Method (Eq. gforce / Eq. df1_vcsgc): run VC-SGC at target cbar with a
moderate kappa and measure dmu = phi + 2 kappa <c> = dmu0 + 2 kappa (<c> - cbar);
set dmu0 <- dmu and repeat.  At the fixed point <c> = cbar and dmu0 is the SGC
value at cbar.  System: rigid 10x10x10 bcc (2,000 sites).

Writes paper_1012_5082_amd/dmu_table.json.  Calls only the oracle and the
seeded input generators.

    python oracle/calibrate_dmu.py
"""
from __future__ import annotations

import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1012_5082_amd import inputs as I  # noqa: E402

OUT = os.path.join(ROOT, "paper_1012_5082_amd", "dmu_table.json")
KB = 8.617333262e-5
TEMPS = [400.0, 600.0, 700.0, 800.0]
CONCS = [0.01, 0.02, 0.03, 0.05, 0.075, 0.10, 0.15, 0.20]
KAPPA = 10.0


def calibrate(T, cbar, seed=7, sweeps=300, burn=50, iters=3):
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(10, 10, 10)
    N = x.size
    # dilute starting guess: isolated substitution energy 0.52 eV plus ideal mixing
    dmu0 = KB * T * math.log((1 - cbar) / cbar) - 0.52
    sp = I.initial_species(N, cbar, seed)
    st = O.SweepState(x, y, z, box, sp, pot)
    est = dmu0
    for it in range(iters):
        O.sweep(st, dmu0, KAPPA, cbar, T, burn, seed + 100 * it)
        ns = []
        for _ in range(sweeps):
            O.sweep(st, dmu0, KAPPA, cbar, T, 1, seed + 100 * it)
            ns.append(st.n_b[0])
        c = float(np.mean(ns)) / N
        est = dmu0 + 2.0 * KAPPA * (c - cbar)
        dmu0 = est
    return est, c


def main():
    table = {"method": "VC-SGC fixed point of dmu0 + 2 kappa (<c> - cbar), kappa = 10 eV, "
                       "rigid 10^3 bcc, FS-P1", "entries": []}
    for T in TEMPS:
        for c in CONCS:
            d, cm = calibrate(T, c)
            table["entries"].append({"T": T, "cbar": c, "dmu": round(d, 5), "c_measured": cm})
            print(f"T={T:5.0f} cbar={c:6.3f} dmu={d:+.5f} <c>={cm:.5f}", flush=True)
    with open(OUT, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
