"""The production schedule of the paper's precipitation runs (Sec. IV.B):
the polycrystal's grain boundaries relaxed by conjugate-gradient
minimization, an MD equilibration at the target temperature and pressure,
then VC-SGC MC/MD cycles, one sweep per 20 MD steps of 2.5 fs, with the
Nose-Hoover thermostat and barostat holding temperature and pressure.

Every step runs in the library's kernels (vcsgc_minimize, md_verlet_step
with the thermostat and barostat, vcsgc_sweep); this module only sequences
the calls and times the phases.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field


@dataclass
class Schedule:
    """Parameters of the schedule (defaults: the paper's Fe-Cu runs, with
    shorter phases)."""
    dmu0: float            # eV, Eq. trans_vcsgc_par1
    kappa: float = 1000.0  # eV per site, Eq. trans_vcsgc_par2
    cbar: float = 0.04     # target concentration
    T: float = 700.0       # K
    p_ext: float = 0.0     # eV/A^3
    dt: float = 2.5        # fs
    md_per_sweep: int = 20
    tau_t: float = 100.0   # fs, thermostat coupling time
    tau_p: float = 1000.0  # fs, barostat coupling time
    relax_iter: int = 200  # CG line searches
    relax_ftol: float = 1e-3
    relax_dmax: float = 0.1
    equil_steps: int = 400  # MD steps before the first sweep
    seed: int = 2003


@dataclass
class Phase:
    seconds: float = 0.0
    info: dict = field(default_factory=dict)


def relax_and_equilibrate(g, s: Schedule) -> dict:
    """CG relaxation, then NPT MD equilibration; g is a binding.VCSGC with
    velocities and forces."""
    import torch
    out = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out["relax"] = g.minimize(max_iter=s.relax_iter, ftol=s.relax_ftol, dmax=s.relax_dmax)
    torch.cuda.synchronize()
    out["relax_s"] = time.perf_counter() - t0
    g.set_thermostat(s.T, s.tau_t)
    g.set_barostat(s.p_ext, s.tau_p)
    t0 = time.perf_counter()
    g.md(s.dt, s.equil_steps)
    torch.cuda.synchronize()
    out["equil_s"] = time.perf_counter() - t0
    out["box"] = [float(v) for v in g.barostat()[1]]
    return out


def cycles(g, s: Schedule, n: int, stats: bool = True) -> dict:
    """n VC-SGC MC/MD cycles (one sweep, then md_per_sweep NPT steps), with
    the sweep and MD times taken separately (each ends with a device
    synchronization)."""
    import torch
    mc = md = 0.0
    agg = {"trials": 0, "flips": 0, "stages": 0, "stage_accepts": 0}
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.sweep(s.dmu0, s.kappa, s.cbar, s.T, 1, s.seed, stats=stats)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.md(s.dt, s.md_per_sweep)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        mc += t1 - t0
        md += t2 - t1
        if stats:
            for k in agg:
                agg[k] += st[k]
    agg["mc_s"], agg["md_s"] = mc, md
    return agg
