"""Long and full-size GPU parity: what the benchmark runs, at its real
shape, against the oracle.

* the 40^3 thermal system after 1,000 sweeps on the batched stage pipeline
  (16 stages per batch, the benchmark's tiling), for cbar = 0.02, 0.05, 0.10;
* the 1.96M-site polycrystal with velocities on the same tiling: one sweep,
  20 MD steps, one more sweep (one hybrid cycle and the next sweep);
* the 64-replica batch of the replica workload (2,000 to 250,000 sites);
* checkpoint and resume through vcsgc_get_state / vcsgc_set_state;
* a bounded persistent-sweep wait forced to time out from the host.

The expected end states of the first two are the oracle's, stored as
digests by tests/golden/make_end_states.py (which calls only the oracle).
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W
from parity_utils import gpu_context, oracle_state

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "end_states.json")
STAT_KEYS = ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final",
             "sum_n", "sum_n2")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def golden():
    return json.load(open(GOLDEN))


def digest(t) -> str:
    a = t.cpu().numpy() if hasattr(t, "cpu") else t
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def add(tot, s):
    if tot is None:
        return dict(s)
    out = {k: tot[k] + s[k] for k in tot}
    out["n_final"] = s["n_final"]
    return out


@pytest.mark.parametrize("cbar", ["0.02", "0.05", "0.1"])
def test_c2_end_state_after_1000_sweeps(torch_cuda, golden, cbar):
    want = golden["c2_1000"][cbar]
    pot = I.params("FS-P1")
    d = W.c2(cbar=float(cbar))
    g = gpu_context(d, pot)
    g.set_tuning("batch", 16)
    tot = None
    for n_sw in (400, 600):
        tot = add(tot, g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], n_sw, d["seed"]))
    for k in STAT_KEYS:
        assert tot[k] == want["stats"][k], (k, tot[k], want["stats"][k], tot["near_ties"])
    assert digest(g.species) == want["species"]
    assert digest(g.rho()) == want["rho"]
    g.close()


@pytest.fixture(scope="module")
def c3_data():
    return W.c3()


def test_c3_bench_path_hybrid_cycle(torch_cuda, golden, c3_data):
    """The benchmark's path at its shape: batched pipeline (3 stages per
    batch) with velocities, [sweep; 20 MD steps] then a sweep on the list
    and density taken from the MD pass."""
    want = golden["c3_hybrid"]
    d = c3_data
    assert d["dmu0"] == want["dmu0"] and d["x"].size == want["n_sites"]
    pot = I.params("FS-P1")
    g = gpu_context(d, pot, velocities=True)
    g.set_tuning("batch", 3)
    args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    s1 = g.sweep(*args, 1, d["seed"])
    for k in STAT_KEYS:
        assert s1[k] == want["stats_sweep1"][k], (k, s1[k], want["stats_sweep1"][k])
    g.md(d["dt"], d["md_steps"])
    tot = add(s1, g.sweep(*args, 1, d["seed"]))
    for k in STAT_KEYS:
        assert tot[k] == want["stats"][k], (k, tot[k], want["stats"][k], tot["near_ties"])
    assert tot["stage_accepts"] > 0 and tot["flips"] > 0
    for nm in ("species", "x", "y", "z", "vx", "vy", "vz"):
        assert digest(getattr(g, nm)) == want[nm], nm
    assert digest(g.rho()) == want["rho"]
    g.close()


def test_c3_production_path(torch_cuda, golden, c3_data):
    """The production schedule's path at full size: 3 conjugate-gradient line
    searches, 4 Nose-Hoover NPT steps of 2.5 fs and a sweep on the batched
    pipeline, against the oracle's end state (relaxation result, box,
    statistics and digests of the state)."""
    want = golden["c3_production"]
    d = c3_data
    assert d["dmu0"] == want["dmu0"] and d["x"].size == want["n_sites"]
    pot = I.params("FS-P1")
    g = gpu_context(d, pot, velocities=True)
    assert g.minimize(max_iter=3, ftol=1e-3, dmax=0.1) == want["relax"]
    g.set_thermostat(700.0, 100.0)
    g.set_barostat(0.0, 1000.0)
    g.md(2.5, 4)
    assert [float(v) for v in g.barostat()[1]] == want["box"]
    g.set_tuning("batch", 3)
    s1 = g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"])
    for k in STAT_KEYS:
        assert s1[k] == want["stats"][k], (k, s1[k], want["stats"][k], s1["near_ties"])
    for nm in ("species", "x", "y", "z", "vx", "vy", "vz"):
        assert digest(getattr(g, nm)) == want[nm], nm
    assert digest(g.rho()) == want["rho"]
    g.close()


@pytest.mark.parametrize("colours,grow_edge", [(27, 0.0), (8, 15.1)])
def test_c3_finer_schemes_sweep(torch_cuda, oracle_mod, c3_data, colours, grow_edge):
    """27 colours and grown domains (cells of 15.9 A) at full size on the
    batched pipeline with velocities: two sweeps against the serial oracle."""
    from paper_1012_5082_amd.binding import VCSGC
    O = oracle_mod
    d = c3_data
    pot = I.params("FS-P1")
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"], colours=colours, grow_edge=grow_edge)
    g.set_tuning("batch", 3)
    args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    sg = g.sweep(*args, 2, d["seed"])
    st = oracle_state(O, d, pot, velocities=True)
    so, _, _ = O.sweep(st, *args, 2, d["seed"], colour_period=3 if colours == 27 else 2,
                       grow_edge=grow_edge)
    for k in STAT_KEYS:
        assert sg[k] == so[k], (k, sg[k], so[k], sg["near_ties"])
    assert sg["flips"] > 0
    for nm in ("species", "vx", "vy", "vz"):
        assert digest(getattr(g, nm)) == digest(getattr(st, nm)), nm
    assert digest(g.rho()) == digest(st.rho)
    g.close()


def test_c3_tabulated_hybrid(torch_cuda, oracle_mod, c3_data):
    """The tabulated form of the potential (TAB-FS1) at full size: a sweep
    on the batched pipeline, 2 MD steps and a sweep, against the oracle."""
    from paper_1012_5082_amd.binding import VCSGC
    O = oracle_mod
    d = c3_data
    pot = I.table("TAB-FS1")
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"])
    g.set_tuning("batch", 3)
    args = (d["dmu0"], d["kappa"], d["cbar"], d["T"])
    s1 = g.sweep(*args, 1, d["seed"])
    g.md(1.0, 2)
    tot = add(s1, g.sweep(*args, 1, d["seed"]))
    st = oracle_state(O, d, pot, velocities=True)
    o1, _, _ = O.sweep(st, *args, 1, d["seed"])
    x, y, z, vx, vy, vz, *_ = O.md(d["x"], d["y"], d["z"], st.vx, st.vy, st.vz, st.species,
                                   d["box"], pot, 1.0, 2)
    st2 = O.SweepState(x, y, z, d["box"], st.species, pot, vx=vx, vy=vy, vz=vz)
    st2.w = 1
    o2, _, _ = O.sweep(st2, *args, 1, d["seed"])
    want = add(o1, o2)
    for k in STAT_KEYS:
        assert tot[k] == want[k], (k, tot[k], want[k], tot["near_ties"])
    assert tot["flips"] > 0
    for nm, ref in (("species", st2.species), ("x", x), ("y", y), ("z", z), ("vx", st2.vx),
                    ("vy", st2.vy), ("vz", st2.vz)):
        assert digest(getattr(g, nm)) == digest(ref), nm
    assert digest(g.rho()) == digest(st2.rho)
    g.close()


def test_c3_local_chains(torch_cuda, oracle_mod, c3_data):
    """Local chains of 2 trials per cell and stage at full size (per-stage
    kernels, velocities; kappa = 100 eV, where some stages are accepted):
    two sweeps against the serial oracle."""
    from paper_1012_5082_amd.binding import VCSGC
    O = oracle_mod
    d = c3_data
    pot = I.params("FS-P1")
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"])
    g.set_local_steps(2)
    args = (d["dmu0"], 100.0, d["cbar"], d["T"])
    sg = g.sweep(*args, 2, d["seed"])
    st = oracle_state(O, d, pot, velocities=True)
    so, _, _ = O.sweep(st, *args, 2, d["seed"], local_steps=2)
    for k in STAT_KEYS:
        assert sg[k] == so[k], (k, sg[k], so[k], sg["near_ties"])
    assert sg["stage_accepts"] > 0 and sg["local_accepts"] > sg["flips"] > 0
    for nm in ("species", "vx", "vy", "vz"):
        assert digest(getattr(g, nm)) == digest(getattr(st, nm)), nm
    assert digest(g.rho()) == digest(st.rho)
    g.close()


def test_c4_replica_batch_matches_oracle(torch_cuda, oracle_mod):
    """All 64 replicas of the replica workload (sizes 2,000 to 250,000, one
    persistent launch per call, on two tilings): every replica equals its own
    oracle chain keyed (seed, replica)."""
    O = oracle_mod
    from paper_1012_5082_amd.binding import VCSGCBatch
    pot = I.params("FS-P1")
    reps = []
    for r in W.c4_replicas():
        x, y, z, box = I.bcc(r["nx"], r["ny"], r["nz"])
        reps.append(dict(x=x, y=y, z=z, box=box,
                         species=I.initial_species(x.size, r["cbar"], r["seed"]), **r))
    sizes = [r["x"].size for r in reps]
    assert len(reps) == 64 and max(sizes) >= 100000
    b = VCSGCBatch(reps, pot)
    par = [np.array([r[k] for r in reps]) for k in ("dmu0", "kappa", "cbar", "T")]
    seed = 4004
    b.set_tuning("graph", 4)
    s1 = b.sweep_batch(*par, 2, seed)
    b.set_tuning("graph", 1)
    s2 = b.sweep_batch(*par, 1, seed)
    for k, r in enumerate(reps):
        st = O.SweepState(r["x"], r["y"], r["z"], r["box"], r["species"], pot)
        so, _ = O.sweep_omp(st, r["dmu0"], r["kappa"], r["cbar"], r["T"], 3, seed, replica=k)
        assert s1[k]["trials"] + s2[k]["trials"] == so["trials"], k
        assert s1[k]["flips"] + s2[k]["flips"] == so["flips"], k
        assert s1[k]["sum_n"] + s2[k]["sum_n"] == so["sum_n"], k
        assert s2[k]["n_final"] == so["n_final"], k
        assert np.array_equal(b.replica_species(k), st.species), k
        assert np.array_equal(b.replica_rho(k), st.rho), k
    b.close()


@pytest.mark.parametrize("strategy", ["graph", "batch"])
def test_checkpoint_resume_is_bitwise(torch_cuda, oracle_mod, strategy):
    """get_state (counter, seed, density cache) after some sweeps, then a new
    context from the saved species with set_state: its continuation equals the
    first context's, bit for bit, and both equal the oracle's chain.  The
    restored density cache is the incrementally updated one; a fresh sum
    differs from it in the last bits."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    args = (d["dmu0"], 0.0, d["cbar"], d["T"])
    a = gpu_context(d, pot)
    a.set_tuning(strategy, 8 if strategy == "batch" else 1)
    a.sweep(*args, 4, d["seed"])
    ck = a.get_state(with_rho=True)
    assert ck["sweeps_done"] == 4 and ck["seed"] == d["seed"]
    sp = a.species.cpu().numpy().copy()
    d2 = dict(d, species=sp)
    b = gpu_context(d2, pot)
    b.set_tuning(strategy, 8 if strategy == "batch" else 1)
    fresh = b.rho().cpu().numpy()
    saved = ck["rho"].cpu().numpy()
    assert not np.array_equal(fresh, saved)  # incremental updates round differently
    b.set_state(ck["sweeps_done"], ck["seed"], ck["rho"])
    assert np.array_equal(b.rho().cpu().numpy(), saved)
    assert b.get_state()["n_b"] == ck["n_b"]
    sa = a.sweep(*args, 3, d["seed"])
    sb = b.sweep(*args, 3, d["seed"])
    for k in STAT_KEYS:
        assert sa[k] == sb[k], k
    assert np.array_equal(a.species.cpu().numpy(), b.species.cpu().numpy())
    assert np.array_equal(a.rho().cpu().numpy(), b.rho().cpu().numpy())
    st = oracle_state(O, d, pot)
    so, _, _ = O.sweep(st, *args, 7, d["seed"])
    assert so["n_final"] == sa["n_final"]
    assert np.array_equal(a.species.cpu().numpy(), st.species)
    assert np.array_equal(a.rho().cpu().numpy(), st.rho)
    a.close()
    b.close()


def test_persistent_wait_timeout_is_reported(torch_cuda):
    """A wait limit of one poll makes the persistent sweep's barrier waits
    time out (every wait is bounded, so every workgroup still exits): the
    call fails with VCSGC_E_BARRIER_TIMEOUT even without statistics, and the
    context stays in the error state."""
    from paper_1012_5082_amd.binding import VcsgcError
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    g = gpu_context(d, pot)
    g.set_tuning("persistent", 1)
    assert g.tuning()["workgroups"] > 1
    g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"], stats=False)
    g.set_wait_limit(1)
    with pytest.raises(VcsgcError) as e:
        g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 2, d["seed"], stats=False)
    assert e.value.code == -7
    with pytest.raises(VcsgcError) as e:
        g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"])
    assert e.value.code == -5
    g.close()
