"""Benchmark: hybrid VC-SGC Monte Carlo / EAM MD on one MI355X.

One step = one hybrid cycle of the 1.96M-site Voronoi polycrystal: one
parallel VC-SGC sweep (N trials) followed by 20 velocity-Verlet steps
(dt = 1 fs), the 1:20 interleaving of the paper's production run.

The chain starts from the workload's initial state at the dmu0 calibrated
on this system (paper_1012_5082_amd/dmu_c3.json): W warmup cycles, then K
timed cycles.

Reported (one JSON line):
  value               MC trials/s of the sweeps in the timed region
                      (trials / summed sweep time, HIP events on the stream)
  accepted_flips_per_s, stage_acceptance
                      exact-accepted transmutations per second of sweep time
                      and the share of stages the global factor accepted
  md_atom_steps_per_s MD atom-steps/s of the MD parts of the same cycles
  ms_per_step         wall time per hybrid cycle
  roofline            the kernel class with the largest time in the timed
                      cycles: algorithmic bytes per launch / mean launch
                      duration (HIP events)
  roofline_sweep      the same for the sweep kernel
  cpu_baseline        the oracle on host cores: one serial sweep of the same
                      system, three sweeps on all cores, three serial MD steps

    python bench.py [--steps K] [--warmup W] [--no-cpu-baseline]
    python bench.py --copy-calib      (plain device copy, for counter scaling)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MC trials/s @2M atoms (plain vs surrogate-DA, same ⟨c⟩); MD atom-steps/s"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(kind, n, pairs_md, pairs_mc, trials, fused=0.0):
    """Compulsory HBM bytes of one launch (each array element counted once).

    forces    : (x,y,z,F') packed (32) + species (1) + row length (1) + neighbour
                indices (4 per r < rc + skin pair) + fx,fy,fz written (24); a
                launch that runs the next step's kick and drift instead of
                storing the forces reads v and the reference positions (48)
                and writes x,y,z, v and the packed positions (80) in place of
                the 24 bytes of forces; `fused` is the share of such launches
    density   : (x,y,z,species) packed (32) + species (1) + row length (1) +
                indices (4 per pair) + rho (8) and (x,y,z,F') (32) written
    kick_drift: x,y,z,v,F,species,reference positions read (105), x,y,z,v and the
                packed positions written (80)
    kick      : v, F, species read (49), v written (24)
    trial     : per trial, own species/rho/row length (10) + per r < rc pair the
                index, (rc-r)^2, c0+c1 r (20) and the neighbour's species and rho
                (9) + cell start/atom (8+4) + record (4)
    stage     : the trial bytes above with the site and ln u read from the site
                table (4+8 in place of the cell start/atom), plus per active cell
                the next sweep's draw: cell start/atom read (8+4), site and ln u
                written (4+8); `trials` is then (trials, active cells) per launch"""
    if kind == "forces":
        return (58 + fused * (48 + 80 - 24)) * n + 4 * pairs_md
    if kind == "density":
        return 74 * n + 4 * pairs_md
    if kind == "kick_drift":
        return 185 * n
    if kind == "kick":
        return 73 * n
    if kind == "trial":
        k = pairs_mc / n
        return trials * (26 + 21 * k)
    if kind == "stage":
        k = pairs_mc / n
        nt, ncells = trials
        return nt * (26 + 21 * k) + ncells * 24
    return None


HAS_BYTES = ("forces", "density", "kick_drift", "kick", "trial", "stage")
SAMPLE = 8  # sweep-kernel launches per timed launch

# kernel class -> (kernel symbol, source file, profile summary holding its
# FETCH_SIZE / WRITE_SIZE counters for the c3 hybrid cycle)
TRAFFIC = {
    "forces": ("k_forces", "paper_1012_5082_amd/csrc/md.hip", "profiles/k_forces_c3_traffic.md"),
    "density": ("k_density_md", "paper_1012_5082_amd/csrc/md.hip",
                "profiles/k_density_md_c3_traffic.md"),
    "stage": ("k_stage", "paper_1012_5082_amd/csrc/sweep.hip", "profiles/k_stage_c3_traffic.md"),
    "batch": ("k_stage_spec", "paper_1012_5082_amd/csrc/sweep.hip",
              "profiles/k_stage_spec_c3_traffic.md"),
}


def measured_traffic(cls, tiling=None):
    """HBM bytes per launch of the kernel from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the counter
    reads for a copy kernel of known size), or None when there is none, the
    kernel's source has changed since the counters were taken, or the
    summary names a sweep tiling other than this run's."""
    import hashlib
    import re
    ent = TRAFFIC.get(cls)
    if not ent:
        return None
    _, src, prof = ent
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        text = open(os.path.join(here, prof)).read()
        sha = hashlib.sha256(open(os.path.join(here, src), "rb").read()).hexdigest()
    except OSError:
        return None
    want = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch:\s*([0-9]+)", text)
    if not want or not val or want.group(1) != sha:
        return None
    til = re.search(r"tiling:\s*(\S+)", text)
    if til and tiling is not None and til.group(1) != tiling:
        return None
    return int(val.group(1))


def potential(name):
    """The analytic FS-P1 set, or a tabulated EAM (TAB-FS1 tabulates FS-P1)."""
    from paper_1012_5082_amd import inputs as I
    return I.params(name) if name == "FS-P1" else I.table(name)


def copy_calib():
    import torch
    n = 1 << 27  # 128 Mi doubles = 1 GiB
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copied {n * 8} bytes 5 times")
    print(json.dumps({"copy_bytes": n * 8, "launches": 5}))


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(d, pot):
    """The oracle as it stands, timed on this host on a bounded sample of the
    same workload: one serial sweep (the headline leg), three sweeps of the
    same chain with each stage's trials on all host cores of this process
    (bitwise the serial chain), and three serial velocity-Verlet steps of the
    same system (neighbour list rebuilt at every force evaluation)."""
    from oracle import oracle as O
    threads = min(16, len(os.sched_getaffinity(0)))
    t0 = time.perf_counter()
    st = O.SweepState(d["x"], d["y"], d["z"], d["box"], d["species"], pot)
    setup = time.perf_counter() - t0
    args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    t0 = time.perf_counter()
    s, _, _ = O.sweep(st, *args, 1, d["seed"])
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    s3, _ = O.sweep_omp(st, *args, 3, d["seed"], threads=threads)
    dt3 = time.perf_counter() - t0
    md_steps = 3
    t0 = time.perf_counter()
    O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["species"], d["box"], pot,
         d["dt"], md_steps)
    dtm = time.perf_counter() - t0
    n = d["x"].size
    return {"value": s["trials"] / dt, "unit": "trials/s", "cores": 1, "kind": "oracle",
            "sample": f"1 sweep ({s['trials']} trials) of the same {n}-site system, "
                      f"serial FP64 C oracle, {dt:.2f} s (neighbour list {setup:.1f} s untimed)",
            "openmp": {"value": round(s3["trials"] / dt3, 1), "unit": "trials/s",
                       "cores": threads, "kind": "oracle",
                       "sample": f"the next 3 sweeps ({s3['trials']} trials), each stage's "
                                 f"trials on {threads} threads, {dt3:.2f} s"},
            "md": {"value": round(n * md_steps / dtm, 1), "unit": "atom-steps/s", "cores": 1,
                   "kind": "oracle",
                   "sample": f"{md_steps} velocity-Verlet steps of the same system "
                             f"({md_steps + 1} force evaluations, each with its neighbour "
                             f"list), serial, {dtm:.2f} s"},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def _timed(fn):
    import torch
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    out = fn()
    b.record()
    torch.cuda.synchronize()
    return out, a.elapsed_time(b) / 1e3


def bench_production(args):
    """The paper's production schedule on the polycrystal (Sec. IV.B): CG
    relaxation of the grain boundaries, NPT equilibration at 700 K and zero
    pressure, then VC-SGC MC/MD cycles of one sweep and 20 NPT steps of
    2.5 fs; warmup cycles, then timed ones (sweep and MD timed apart)."""
    from paper_1012_5082_amd import production as PR
    from paper_1012_5082_amd import workloads as W
    from paper_1012_5082_amd.binding import VCSGC
    pot = potential(args.potential)
    d = W.c3()
    n = d["x"].size
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"], forces=True, skin=args.skin)
    st, k = args.tiling.split(":")
    g.set_tuning(st, int(k))
    s = PR.Schedule(dmu0=d["dmu0"], kappa=d["kappa"], cbar=d["cbar"], T=d["T"], seed=d["seed"])
    pre = PR.relax_and_equilibrate(g, s)
    log(f"production: relaxed ({pre['relax']['iterations']} line searches, {pre['relax_s']:.2f} s), "
        f"equilibrated ({s.equil_steps} steps, {pre['equil_s']:.2f} s)")
    PR.cycles(g, s, args.warmup, stats=False)
    r = PR.cycles(g, s, args.steps)
    out = {"metric": "MC trials/s and MD atom-steps/s on the production schedule",
           "value": round(r["trials"] / r["mc_s"], 1), "unit": "trials/s",
           "workload": f"c3-voronoi16 production schedule: {n} sites, CG relaxation, "
                       f"{s.equil_steps} NPT steps, then cycles of 1 sweep + {s.md_per_sweep} "
                       f"Nose-Hoover NPT steps of {s.dt} fs at {s.T} K, p = {s.p_ext} eV/A^3",
           "cycles": args.steps, "warmup": args.warmup, "potential": args.potential,
           "mc_ms_per_sweep": round(r["mc_s"] / args.steps * 1e3, 3),
           "md_ms_per_step": round(r["md_s"] / (args.steps * s.md_per_sweep) * 1e3, 4),
           "md_atom_steps_per_s": round(n * s.md_per_sweep * args.steps / r["md_s"], 1),
           "stage_acceptance": round(r["stage_accepts"] / max(r["stages"], 1), 4),
           "accepted_flips_per_s": round(r["flips"] / r["mc_s"], 1),
           "relax": pre["relax"], "relax_s": round(pre["relax_s"], 3),
           "equil_s": round(pre["equil_s"], 3), "box_after_equilibration": pre["box"],
           "sweep_tiling": args.tiling}
    g.close()
    return out


def bench_replicas(args):
    """64 rigid bcc replicas of uneven size on a T x kappa x cbar grid, all in
    one graph-captured persistent launch per call; tiling from the autotuner."""
    import numpy as np
    from paper_1012_5082_amd import autotune
    from paper_1012_5082_amd import inputs as I
    from paper_1012_5082_amd import workloads as W
    from paper_1012_5082_amd.binding import VCSGCBatch
    pot = potential(args.potential)
    reps = []
    for r in W.c4_replicas():
        x, y, z, box = I.bcc(r["nx"], r["ny"], r["nz"])
        reps.append(dict(x=x, y=y, z=z, box=box,
                         species=I.initial_species(x.size, r["cbar"], r["seed"]), **r))
    b = VCSGCBatch(reps, pot, colours=args.colours)
    par = [np.array([r[k] for r in reps]) for k in ("dmu0", "kappa", "cbar", "T")]
    seed = 4004
    tuned = autotune.tune(b, lambda k: b.sweep_batch(*par, k, seed, stats=False), use_cache=False)
    log(f"c4 autotune {tuned['choice']} {tuned['times_ms']}")
    n_sw = args.sweeps or 500
    stats, dt = _timed(lambda: b.sweep_batch(*par, n_sw, seed))
    trials = sum(s["trials"] for s in stats)
    flips = sum(s["flips"] for s in stats)
    sizes = [int(np.asarray(r["x"]).size) for r in reps]
    cmean = [s["sum_n"] / n_sw / n for s, n in zip(stats, sizes)]
    out = {"metric": "MC trials/s, 64 replicas in one launch", "value": round(trials / dt, 1),
           "unit": "trials/s", "workload": "c4-replicas64", "n_replicas": len(reps),
           "sites_total": int(sum(sizes)), "sites_min": min(sizes), "sites_max": max(sizes),
           "sweeps": n_sw, "seconds": round(dt, 4), "flips_per_s": round(flips / dt, 1),
           "tiling": list(tuned["choice"]), "workgroups": b.tuning()["workgroups"],
           "colours": args.colours, "potential": args.potential,
           "autotune_ms_per_sweep": {k: round(v, 3) for k, v in tuned["times_ms"].items()},
           "mean_c_first8": [round(c, 5) for c in cmean[:8]],
           "cbar_first8": [round(float(r["cbar"]), 5) for r in reps[:8]]}
    b.close()
    return out


def _blocked(series, nb=10):
    import numpy as np
    a = np.asarray(series, dtype=np.float64)
    m = a.size // nb
    bm = a[: m * nb].reshape(nb, m).mean(axis=1)
    return float(bm.mean()), float(bm.std(ddof=1) / np.sqrt(nb))


def bench_surrogate(args):
    """Surrogate delayed acceptance on the 1.96M-site polycrystal.

    1. the polycrystal (cells of edge >= 8.01 A, the descriptor's dependence
       range) is first relaxed by 100 plain sweeps; the (descriptor, exact
       dU) pair of every 128th trial of the last 80 of them is logged (10^6
       pairs) and two further sweeps give held-out pairs;
    2. hand-written training on the logged pairs (BF16 MFMA forward/backward,
       Adam);
    3. from the relaxed state a plain and a
       delayed-acceptance chain run with identical parameters: trials/s,
       exact-accepted moves/s, pre-rejection rate, and <c>, <E> (energy every
       10 sweeps, outside the timed sweeps) with blocked errors;
    4. step 3 twice: both chains on the stage pipeline (one stage per
       kernel), then each chain on its fastest tiling (stage pipeline or
       batches of 2..16 stages, from a few timed sweeps of each)."""
    import numpy as np
    import torch
    from paper_1012_5082_amd import inputs as I
    from paper_1012_5082_amd import workloads as W
    from paper_1012_5082_amd.binding import VCSGC, Mlp
    pot = I.params("FS-P1")
    d = W.c3(with_velocities=False)
    n = d["x"].size
    r_dep = 8.01
    sp = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    plain = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, descriptor=True,
                  r_dep=r_dep)
    plain.set_tuning("batch", 16)
    n_relax, n_unlogged = 100, 20
    t0 = time.perf_counter()
    plain.sweep(*sp, n_unlogged, d["seed"])
    plain.enable_sample_log(1_000_000, 128)
    plain.sweep(*sp, n_relax - n_unlogged, d["seed"])
    desc, dE = (t.clone() for t in plain.samples())
    t_log = time.perf_counter() - t0
    log(f"c5: {desc.shape[0]} training samples from the relaxation sweeps in {t_log:.1f} s")
    # held-out pairs from two further sweeps
    plain.enable_sample_log(200000, 97)
    plain.sweep(*sp, 2, d["seed"] + 1)
    hd, he = plain.samples()
    plain.disable_sample_log()
    net = Mlp(seed=7)
    net.fit_normalization(desc, dE)
    rep, t_train = _timed(lambda: net.train(desc, dE, epochs=10, batch=4096, lr=2e-3, seed=11))
    log(f"c5: trained {rep} in {t_train:.1f} s")
    pred = net.forward(hd.contiguous())
    rmse = float(torch.sqrt(torch.mean((pred - he) ** 2)))
    std_e = float(torch.std(he))
    relaxed = plain.species.cpu().numpy().copy()
    plain.close()

    def chain(name):
        g = VCSGC(d["x"], d["y"], d["z"], d["box"], relaxed, pot, descriptor=True, r_dep=r_dep)
        if name == "da":
            g.set_surrogate("mlp", net)
        return g

    # each chain's fastest tiling: a few timed sweeps per candidate
    def fastest(name):
        g = chain(name)
        times = {}
        for tl in ("stage:1", "batch:2", "batch:4", "batch:8", "batch:16"):
            st, k = tl.split(":")
            g.set_tuning(st, int(k))
            g.sweep(*sp, 1, 4242)
            _, dt = _timed(lambda: g.sweep(*sp, 5, 4243))
            times[tl] = round(dt / 5 * 1e3, 3)
        g.close()
        return min(times, key=times.get), times

    n_blocks = max(1, (args.sweeps or 400) // 10)
    choice = {nm: fastest(nm) for nm in ("plain", "da")}
    settings = (("per_stage", {"plain": "stage:1", "da": "stage:1"}),
                ("fastest", {nm: choice[nm][0] for nm in ("plain", "da")}))
    runs = {}
    for label, tilings in settings:
        res = {}
        for name in ("plain", "da"):
            g = chain(name)
            st, k = tilings[name].split(":")
            g.set_tuning(st, int(k))
            seed = 5005
            g.sweep(*sp, 2, seed + 999)  # warmup
            cs, es, trials, flips, pass1, secs = [], [], 0, 0, 0, 0.0
            for b in range(n_blocks):
                s, dt = _timed(lambda: g.sweep(*sp, 10, seed))
                secs += dt
                trials += s["trials"]
                flips += s["flips"]
                pass1 += s["stage1_pass"]
                cs.append(s["sum_n"] / 10 / n)
                es.append(g.energy() / n)
            g.close()
            cm, ce = _blocked(cs)
            em, ee = _blocked(es)
            res[name] = {"tiling": tilings[name], "trials_per_s": round(trials / secs, 1),
                         "exact_accepted_per_s": round(flips / secs, 1),
                         "ms_per_sweep": round(secs / (10 * n_blocks) * 1e3, 3),
                         "pre_rejection_rate": (round(1.0 - pass1 / trials, 5) if name == "da"
                                                else 0.0),
                         "mean_c": cm, "mean_c_err": ce, "mean_E_per_atom": em,
                         "mean_E_err": ee}
            log(f"c5 {label} {name}: {res[name]}")
        z = {}
        for key, err in (("mean_c", "mean_c_err"), ("mean_E_per_atom", "mean_E_err")):
            z[key] = abs(res["plain"][key] - res["da"][key]) / max(
                1e-30, float(np.hypot(res["plain"][err], res["da"][err])))
        res["da_over_plain_exact_accepted"] = round(
            res["da"]["exact_accepted_per_s"] / res["plain"]["exact_accepted_per_s"], 3)
        res["z_c"] = round(z["mean_c"], 3)
        res["z_E"] = round(z["mean_E_per_atom"], 3)
        runs[label] = res
    best = runs["fastest"]
    out = {"metric": "MC trials/s @2M atoms, plain vs surrogate-DA (same <c>, <E>)",
           "value": best["da"]["trials_per_s"], "unit": "trials/s", "workload": "c5-surrogate-da",
           "n_sites": n, "r_dep": r_dep, "relax_sweeps": n_relax, "sweeps_each": 10 * n_blocks,
           "tiling_ms_per_sweep": {nm: choice[nm][1] for nm in choice},
           "per_stage": runs["per_stage"], "fastest": best,
           "surrogate": {"train_samples": int(desc.shape[0]), "log_seconds": round(t_log, 2),
                         "train_seconds": round(t_train, 2),
                         "loss_first": rep["loss_first"], "loss_last": rep["loss_last"],
                         "steps": rep["steps"], "heldout_rmse_eV": rmse,
                         "heldout_dE_std_eV": std_e, "heldout_samples": int(hd.shape[0])}}
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calib", action="store_true")
    ap.add_argument("--workload", default="c3", choices=["c3", "c4", "c5", "production"],
                    help="c3: hybrid cycle (default line); c4: replica batch; c5: surrogate DA; "
                         "production: the paper's schedule (CG, NPT at 2.5 fs) on c3")
    ap.add_argument("--sweeps", type=int, default=0, help="c4/c5: timed sweeps")
    ap.add_argument("--local-steps", type=int, default=1,
                    help="c3: trials per active cell per stage (1 = the plain scheme)")
    ap.add_argument("--tiling", default="batch:3",
                    help="c3: sweep tiling strategy:k, or 'auto' for the autotuner")
    ap.add_argument("--colours", type=int, default=8, choices=[8, 27],
                    help="c3, c4: colours of the sweep (27: cells of edge >= r_dep / 2)")
    ap.add_argument("--grow-edge", type=float, default=0.0,
                    help="c3: grown overlapping domains in cells of edge >= max(this, 2 r_dep) "
                         "instead of the colouring (0: off)")
    ap.add_argument("--potential", default="FS-P1", choices=["FS-P1", "TAB-FS1", "TAB-X"],
                    help="c3, c4: the analytic Finnis-Sinclair set, or a tabulated EAM")
    ap.add_argument("--skin", type=float, default=0.3,
                    help="c3: MD neighbour-list skin (A)")
    ap.add_argument("--relax", type=int, default=0,
                    help="c3: untimed sweeps before the warmup cycles")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(replicas and spatial shards would be distributed per GPU; see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_calib:
        copy_calib()
        return

    if args.workload == "c4":
        print(json.dumps(bench_replicas(args)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(bench_surrogate(args)), flush=True)
        return
    if args.workload == "production":
        print(json.dumps(bench_production(args)), flush=True)
        return

    from paper_1012_5082_amd import inputs as I
    from paper_1012_5082_amd import workloads as W
    from paper_1012_5082_amd.binding import VCSGC

    pot = potential(args.potential)
    t0 = time.perf_counter()
    d = W.c3()
    n = d["x"].size
    log(f"workload {d['name']}: {n} sites generated in {time.perf_counter() - t0:.1f} s")
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"], skin=args.skin, colours=args.colours, grow_edge=args.grow_edge)
    if args.local_steps > 1:
        g.set_local_steps(args.local_steps)
    info = g.info()
    sweep_args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    md_steps, dt = d["md_steps"], d["dt"]

    # tiling: local chains always run stage by stage; otherwise the given one,
    # or the autotuner's (its timing sweeps are real sweeps of the chain)
    if args.local_steps > 1:
        g.set_tuning("stage", 1)
        tuned = {"choice": ("stage", 1), "times_ms": {}}
    elif args.tiling == "auto":
        from paper_1012_5082_amd import autotune
        tuned = autotune.tune(g, lambda k: g.sweep(*sweep_args, k, d["seed"], stats=False),
                              op=sweep_args,
                              use_cache=False)
    else:
        st, k = args.tiling.split(":")
        g.set_tuning(st, int(k))
        tuned = {"choice": (st, int(k)), "times_ms": {}}
    log(f"tiling: {tuned['choice']} {tuned['times_ms']}")
    # optional untimed sweeps before the warmup cycles (none by default: the
    # timed cycles follow the chain from its initial state)
    if args.relax > 0:
        g.sweep(*sweep_args, args.relax, d["seed"], stats=False)
    for k in range(args.warmup):
        g.sweep(*sweep_args, 1, d["seed"])
        g.md(dt, md_steps)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} cycles done")

    # timed region: K hybrid cycles.  Every kernel class is timed with HIP
    # events on the context's stream, one launch in SAMPLE of each (event
    # pairs at every launch would add host and stream work; the pipelines
    # time the span of each graph replay); the dominant class is the one with
    # the largest time over the timed cycles.
    g.kernel_timing(["trial", "commit", "stage", "density", "forces", "kick_drift", "kick",
                     "build", "persist"], every=SAMPLE)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
           torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    trials = 0
    flips = stages = stage_acc = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record()
        s = g.sweep(*sweep_args, 1, d["seed"])
        ev[k][1].record()
        g.md(dt, md_steps)
        ev[k][2].record()
        trials += s["trials"]
        flips += s["flips"]
        stages += s["stages"]
        stage_acc += s["stage_accepts"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mc_ms = sum(a.elapsed_time(b) for a, b, _ in ev)
    md_ms = sum(b.elapsed_time(c) for _, b, c in ev)
    kt = g.kernel_times()
    # per cycle: mean timed launch x all launches of the class
    breakdown = {k: (v[0] / v[1] * v[2] / args.steps, v[2] / args.steps) for k, v in kt.items()}
    top = max(breakdown, key=lambda k: breakdown[k][0])
    dominant = max((k for k in breakdown if k in HAS_BYTES), key=lambda k: breakdown[k][0])
    sweep_cls = "stage" if "stage" in breakdown else ("trial" if "trial" in breakdown else None)
    log("breakdown (ms per cycle, launches per cycle): " + ", ".join(
        f"{k}={v[0]:.3f}/{v[1]:.0f}" for k, v in sorted(breakdown.items(), key=lambda t: -t[1][0])))
    info2 = g.info()
    pairs_md = info2["md_pairs"]
    pairs_mc = info["mc_pairs"]
    nc = info["n_cells"]
    ncpc = nc[0] * nc[1] * nc[2] // 8

    def roof_entry(cls):
        """HBM roofline of one kernel class over the timed region: algorithmic
        bytes per launch / mean launch duration (HIP events)."""
        if cls not in kt:
            return None
        tot_ms, launches, all_launches = kt[cls]
        avg_s = tot_ms / launches / 1e3
        per_launch = 0
        if cls == "trial":
            per_launch = trials / max(1, all_launches)
        elif cls == "stage":
            per_launch = (trials / max(1, all_launches), stages * ncpc / max(1, all_launches))
        # every MD call of md_steps steps makes md_steps force passes with the
        # next step's kick and drift and one that stores the forces
        abytes = algorithmic_bytes(cls, n, pairs_md, pairs_mc, per_launch,
                                   fused=md_steps / (md_steps + 1))
        if not abytes:
            return None
        ach = abytes / avg_s / 1e9
        tcls = "batch" if cls == "stage" and tuned["choice"][0] == "batch" else cls
        return {"bound": "hbm", "kernel": TRAFFIC[tcls][0] if tcls in TRAFFIC else cls,
                "achieved": round(ach, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(tcls, "%s:%d" % tuple(tuned["choice"])),
                "bytes_per_launch": int(abytes),
                "avg_launch_us": round(avg_s * 1e6, 2), "timed_launches": launches,
                "launches": all_launches}

    roof = roof_entry(dominant)
    roof_sweep = roof_entry(sweep_cls) if sweep_cls else None

    value = trials / (mc_ms / 1e3)
    md_rate = n * md_steps * args.steps / (md_ms / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "trials/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{d['name']}: {n}-site 16-grain bcc Voronoi polycrystal "
                               f"(100^3-cell box), FS-P1 EAM, kappa=1000 eV, cbar=0.03, "
                               f"T=700 K, step = 1 VC-SGC sweep + 20 MD steps (dt=1 fs)",
                   "n_sites": n, "n_cells": info["n_cells"],
                   "stages_per_sweep": info["stages_per_sweep"], "colours": args.colours,
                   "grow_edge": args.grow_edge, "potential": args.potential,
                   "variant": ("plain" if args.local_steps == 1
                               else f"local chains of {args.local_steps} trials per cell"),
                   "sweep_tiling": list(tuned["choice"]),
                   "md_list_rebuilds": info2["md_rebuilds"]},
        "md_atom_steps_per_s": round(md_rate, 1),
        "mc_ms_per_sweep": round(mc_ms / args.steps, 3),
        "md_ms_per_step": round(md_ms / args.steps / md_steps, 4),
        "accepted_flips_per_s": round(flips / (mc_ms / 1e3), 1),
        "stage_acceptance": round(stage_acc / max(1, stages), 4),
        "kernel_breakdown_ms": {k: round(v[0], 4) for k, v in breakdown.items()},
        "top_kernel": top,
        "autotune_ms_per_sweep": {k: round(v, 3) for k, v in tuned["times_ms"].items()},
        "roofline": roof,
        "roofline_sweep": roof_sweep,
        "dmu0": d["dmu0"],
    }
    g.close()
    if not args.no_cpu_baseline:
        log("timing the oracle on host cores ...")
        out["cpu_baseline"] = cpu_baseline(d, pot)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
