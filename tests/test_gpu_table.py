"""Tabulated EAM (a general two-species embedded-atom potential given by
tables, Introduction and Sec. III) on the GPU against the oracle, bit for
bit: densities, energies and forces, every sweep kernel family, MD, the
hybrid cycle and a replica batch.

TAB-FS1 tabulates the Finnis-Sinclair set FS-P1; TAB-X differs from the
analytic form in every function.  Both sides build their own interpolation
coefficients from the same tables and evaluate them in the same order.
"""
import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W
from parity_utils import compare_logs, gpu_context, oracle_state, tie_overrides
from test_gpu_parity import _eam_parity, _md_system, _replica_set

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name", ["TAB-FS1", "TAB-X"])
def test_table_eam_parity(torch_cuda, oracle_mod, name):
    d = W.c1(c_init=0.3)
    d["x"], d["y"], d["z"] = I.thermalize(d["x"], d["y"], d["z"], d["box"], 0.05, 5)
    _eam_parity(oracle_mod, d, I.table(name))


@pytest.mark.parametrize("path", ["stage_logged", "batch", "graph", "chain3"])
def test_table_sweep_parity(torch_cuda, oracle_mod, path):
    """Three sweeps of the 40^3 thermal system with TAB-X on each kernel
    family: counters, species and density cache equal the oracle's (and the
    trial and stage logs on the logged path)."""
    O = oracle_mod
    tab = I.table("TAB-X")
    d = W.c2(cbar=0.05)
    k = 3 if path == "chain3" else 1
    args = (d["dmu0"], 10.0, d["cbar"], d["T"])
    g = gpu_context(d, tab)
    info = g.info()
    S = info["stages_per_sweep"]
    ncpc = int(np.prod(info["n_cells"])) // 8
    log = path == "stage_logged"
    if log:
        g.set_tuning("stage", 1)
        g.enable_log(3 * S * ncpc, 3 * S)
    elif path == "batch":
        g.set_tuning("batch", 4)
    elif path == "graph":
        g.set_tuning("graph", 1)
    else:
        g.set_local_steps(k)
    sg = g.sweep(*args, 3, d["seed"])
    st = oracle_state(O, d, tab)
    over = None
    if log:
        tl_g, sl_g, _, _ = g.logs()
        over = tie_overrides(tl_g, sl_g)
    so, tl_o, sl_o = O.sweep(st, *args, 3, d["seed"], log_trials=10 ** 8 if log else 0,
                             log_stages=10 ** 8 if log else 0, overrides=over, local_steps=k)
    if log:
        compare_logs(tl_g, sl_g, tl_o, sl_o)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert so["stage_accepts"] > 0 and so["flips"] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


def test_table_md_and_hybrid_cycle(torch_cuda, oracle_mod):
    """40 MD steps (with list rebuilds), then [sweep on the batched pipeline;
    20 MD steps] x 2 with TAB-X: positions, velocities, forces, species and
    density cache bit for bit."""
    O = oracle_mod
    tab = I.table("TAB-X")
    d = _md_system(n=12, c=0.1, seed=67)
    g = gpu_context(d, tab, velocities=True)
    g.md(1.0, 40)
    out = O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["species"], d["box"], tab,
               1.0, 40)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz"), out[:9]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    x, y, z, vx, vy, vz = out[:6]
    sp = d["species"]
    g.set_tuning("batch", 4)
    for cyc in range(2):
        g.sweep(d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        st = O.SweepState(x, y, z, d["box"], sp, tab, vx=vx, vy=vy, vz=vz)
        st.w = cyc
        O.sweep(st, d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        sp = st.species
        assert np.array_equal(g.species.cpu().numpy(), sp)
        assert np.array_equal(g.rho().cpu().numpy(), st.rho)
        g.md(1.0, 20)
        x, y, z, vx, vy, vz, *_ = O.md(x, y, z, st.vx, st.vy, st.vz, sp, d["box"], tab, 1.0, 20)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz"), (x, y, z, vx, vy, vz)):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    g.close()


def test_table_replica_batch(torch_cuda, oracle_mod):
    """A replica batch (persistent launch) with TAB-X equals independent
    oracle chains."""
    O = oracle_mod
    from paper_1012_5082_amd.binding import VCSGCBatch
    tab = I.table("TAB-X")
    reps = _replica_set(n_rep=4, seed=71)
    b = VCSGCBatch(reps, tab)
    args = [np.array([r[k] for r in reps]) for k in ("dmu0", "kappa", "cbar", "T")]
    s = b.sweep_batch(*args, 3, 991)
    for k, r in enumerate(reps):
        st = O.SweepState(r["x"], r["y"], r["z"], r["box"], r["species"], tab)
        so, _, _ = O.sweep(st, r["dmu0"], r["kappa"], r["cbar"], r["T"], 3, 991, replica=k)
        assert s[k]["flips"] == so["flips"] and s[k]["n_final"] == so["n_final"]
        assert np.array_equal(b.replica_species(k), st.species), k
        assert np.array_equal(b.replica_rho(k), st.rho), k
    b.close()


def test_table_rejects_bad_tables(torch_cuda):
    from paper_1012_5082_amd.binding import VCSGC, VcsgcError
    tab = I.table("TAB-X")
    x, y, z, box = I.bcc(10, 10, 10)
    sp = np.zeros(x.size, np.uint8)
    bad = I.EamTable(tab.dr * (tab.nr - 1) + 0.1, tab.dr, tab.drho, tab.f, tab.phi, tab.F)
    with pytest.raises(VcsgcError) as e:
        VCSGC(x, y, z, box, sp, bad)  # rc beyond the radial knots
    assert e.value.code == -1
    nan_f = tab.f.copy()
    nan_f[1, 5] = np.nan
    with pytest.raises(VcsgcError) as e:
        VCSGC(x, y, z, box, sp, I.EamTable(tab.rc, tab.dr, tab.drho, nan_f, tab.phi, tab.F))
    assert e.value.code == -1
