"""GPU (HIP, through the C ABI) against the oracle on identical seeded inputs.

Bar: integer state (species, n_B, site choices, decisions, counters) bit
for bit; FP64 dU within 1e-12 relative, forces within 1e-10 relative of the
sum of term magnitudes, energies/densities/positions bit for bit where the
arithmetic is the same (both sides evaluate the same expressions in the same
order without contraction); decisions may differ only at near ties
(|ln u + x| < 1e-9), where the oracle adopts the GPU's decision.
"""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W
from parity_utils import compare_logs, gpu_context, oracle_state, tie_overrides

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_device_sqrt_correctly_rounded(torch_cuda):
    torch = torch_cuda
    from paper_1012_5082_amd.binding import selftest_sqrt
    rng = np.random.default_rng(1)
    bits = rng.integers(0, 0x7FEFFFFFFFFFFFFF, size=4_000_000, dtype=np.int64)
    vals = np.concatenate([bits.view(np.float64),
                           rng.uniform(0.0, 40.0, 2_000_000),
                           rng.uniform(0.0, 1e-3, 500_000),
                           np.array([0.0, 1.0, 2.0, 4.0, 13.134408449586, 5e-324, 1e300])])
    x = torch.tensor(vals, dtype=torch.float64, device="cuda")
    got = selftest_sqrt(x).cpu().numpy()
    assert np.array_equal(got.view(np.int64), np.sqrt(vals).view(np.int64))


def _md_math_inputs(torch, gen, n):
    """n square-root arguments a and divisor pairs (a2, b) on the GPU: a third
    each of random bit patterns over [2^-767, 2^1023), uniform r^2 in
    (1e-6, 64) and arguments just above the squares of random numbers
    (where the rounding of the root is hardest); quotients of signed
    uniform and random-exponent numerators by uniform and random-exponent
    divisors."""
    k = n // 3
    dev = "cuda"
    lo, hi = 256, 2047  # biased exponents of 2^-767 and of the largest finite binade
    bits = (torch.randint(lo, hi, (k,), device=dev, generator=gen, dtype=torch.int64) << 52) | \
        torch.randint(0, 1 << 52, (k,), device=dev, generator=gen, dtype=torch.int64)
    a1 = bits.view(torch.float64)
    a2 = 1e-6 + 64.0 * torch.rand(k, device=dev, generator=gen, dtype=torch.float64)
    y = 1e-2 + 8.0 * torch.rand(n - 2 * k, device=dev, generator=gen, dtype=torch.float64)
    u = torch.nextafter(y, torch.full_like(y, float("inf"))) - y
    a3 = y * y + y * u
    a = torch.cat([a1, a2, a3])
    num = torch.cat([200.0 * torch.rand(n - k, device=dev, generator=gen, dtype=torch.float64) - 100.0,
                     torch.ldexp(torch.rand(k, device=dev, generator=gen, dtype=torch.float64) + 0.5,
                                 torch.randint(-900, 900, (k,), device=dev, generator=gen))])
    den = torch.cat([1e-3 + 10.0 * torch.rand(n - k, device=dev, generator=gen, dtype=torch.float64),
                     torch.ldexp(torch.rand(k, device=dev, generator=gen, dtype=torch.float64) + 0.5,
                                 torch.randint(-60, 60, (k,), device=dev, generator=gen))])
    return a, num, den


def test_md_math_correctly_rounded(torch_cuda):
    """The MD passes' square root and quotient are correctly rounded over the
    ranges they serve: 10^9 arguments of each against the library's sqrt and
    the device's IEEE division, and 2 x 10^7 of each against the host's."""
    torch = torch_cuda
    from paper_1012_5082_amd.binding import selftest_md_math, selftest_sqrt
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    for chunk in range(10):
        a, num, den = _md_math_inputs(torch, gen, 100_000_000)
        sq, _ = selftest_md_math(a, den)
        assert torch.equal(sq.view(torch.int64), selftest_sqrt(a).view(torch.int64)), chunk
        _, q = selftest_md_math(num, den)
        assert torch.equal(q.view(torch.int64), (num / den).view(torch.int64)), chunk
        if chunk < 2:  # host references on every tenth argument
            an, nn, dn = a[::10].cpu().numpy(), num[::10].cpu().numpy(), den[::10].cpu().numpy()
            assert np.array_equal(sq[::10].cpu().numpy().view(np.int64), np.sqrt(an).view(np.int64))
            assert np.array_equal(q[::10].cpu().numpy().view(np.int64), (nn / dn).view(np.int64))
        del a, num, den, sq, q


def test_create_rejects_bad_input(torch_cuda):
    from paper_1012_5082_amd.binding import VCSGC, VcsgcError
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(10, 10, 10)
    sp = np.zeros(x.size, np.uint8)
    xb = x.copy()
    xb[5] = box[0] + 1.0
    with pytest.raises(VcsgcError) as e:
        VCSGC(xb, y, z, box, sp, pot)
    assert e.value.code == -1
    sp2 = sp.copy()
    sp2[3] = 2
    with pytest.raises(VcsgcError) as e:
        VCSGC(x, y, z, box, sp2, pot)
    assert e.value.code == -1
    xs, ys, zs, bs = I.bcc(4, 4, 4)
    with pytest.raises(VcsgcError) as e:
        VCSGC(xs, ys, zs, bs, np.zeros(xs.size, np.uint8), pot)
    assert e.value.code == -2
    g = VCSGC(x, y, z, box, sp, pot)
    with pytest.raises(VcsgcError) as e:
        g.sweep(0.0, -1.0, 0.05, 600.0, 1, 1)
    assert e.value.code == -1
    with pytest.raises(VcsgcError):
        g.md(1.0, 1)   # MC-only context
    g.close()


def _eam_parity(O, d, pot):
    g = gpu_context(d, pot, forces=True)
    st = oracle_state(O, d, pot)
    rho_g = g.rho().cpu().numpy()
    assert np.array_equal(rho_g, st.rho)
    e_o = O.energy_atoms(st.nl, st.species, pot, st.rho)
    e_g = g.atom_energies().cpu().numpy()
    assert np.array_equal(e_g, e_o)
    U = g.energy(forces=True)
    assert abs(U - math.fsum(e_o)) <= 1e-12 * abs(U)
    nlv = O.neighbors(d["x"], d["y"], d["z"], d["box"], pot.rc)
    fo = O.forces(nlv, st.species, pot, st.rho)
    for a, b in zip((g.fx, g.fy, g.fz), fo):
        a = a.cpu().numpy()
        assert np.array_equal(a, b)
    g.close()


def test_eam_parity_c1_thermal(torch_cuda, oracle_mod):
    d = W.c1(c_init=0.3)
    d["x"], d["y"], d["z"] = I.thermalize(d["x"], d["y"], d["z"], d["box"], 0.05, 5)
    _eam_parity(oracle_mod, d, I.params("FS-P1"))


def test_eam_parity_c2(torch_cuda, oracle_mod):
    _eam_parity(oracle_mod, W.c2(cbar=0.10), I.params("FS-P1"))


def _dense_bins_system(kind):
    """Systems whose search bins need the larger bin capacity.  "cluster": a
    10^3 bcc block with a vacancy of radius 6 A holding a cluster of 20
    atoms within 0.4 A (20 atoms in one bin: more than its 16 slots).
    "clusters": 16 atoms within 0.05 A of every bin centre of a 7^3 grid of
    4.2 A bins (no bin over 16, but more staged atoms around a region than
    the 16-slot search stages; clusters 4.1 A apart, beyond rc + skin)."""
    rng = np.random.default_rng(61 if kind == "cluster" else 62)
    if kind == "cluster":
        x, y, z, box = I.bcc(10, 10, 10)
        c = 0.5 * box
        keep = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) > 6.0
        off = rng.uniform(-0.4, 0.4, size=(20, 3)) / np.sqrt(3.0)
        x = np.concatenate([x[keep], c[0] + off[:, 0]])
        y = np.concatenate([y[keep], c[1] + off[:, 1]])
        z = np.concatenate([z[keep], c[2] + off[:, 2]])
    else:
        b = 4.2
        box = np.full(3, 7 * b)
        g = (np.arange(7) + 0.5) * b
        cx, cy, cz = [a.ravel() for a in np.meshgrid(g, g, g, indexing="ij")]
        k = np.arange(16)
        grid = 0.025 * np.stack([k % 2, (k // 2) % 2, k // 4], axis=1) - [0.0125, 0.0125, 0.0375]
        off = grid[None] + rng.uniform(-0.003, 0.003, size=(cx.size, 16, 3))
        x = (cx[:, None] + off[..., 0]).ravel()
        y = (cy[:, None] + off[..., 1]).ravel()
        z = (cz[:, None] + off[..., 2]).ravel()
    sp = I.initial_species(x.size, 0.2, 63)
    return dict(x=x, y=y, z=z, box=np.asarray(box, dtype=np.float64), species=sp)


@pytest.mark.parametrize("kind", ["cluster", "clusters"])
def test_eam_parity_dense_bins(torch_cuda, oracle_mod, kind):
    """Bins grown on the way (the 32-slot search): densities, energies and
    forces still equal the oracle's bit for bit, and the MD list holds every
    pair within rc + skin."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _dense_bins_system(kind)
    _eam_parity(O, d, pot)
    g = gpu_context(d, pot, forces=True)
    g.energy(forces=True)
    nl = O.neighbors(d["x"], d["y"], d["z"], d["box"], pot.rc + 0.3, vectors=False)
    assert g.info()["md_pairs"] == nl.j.size
    g.close()


def _full_rows_system(cells=24):
    """A simple-cubic lattice of edge 1.7 A (0.005 A of noise): every atom
    has exactly 32 neighbours within rc + 0.1 A, all of them within rc
    (shells at 1.7, 2.40, 2.94 and 3.4 A; the next at 3.80 A)."""
    a = 1.7
    k = (np.arange(cells) + 0.5) * a
    x, y, z = [v.ravel().copy() for v in np.meshgrid(k, k, k, indexing="ij")]
    rng = np.random.default_rng(71 + cells)
    for v in (x, y, z):
        v += rng.uniform(-0.005, 0.005, v.size)
    box = np.full(3, cells * a)
    sp = I.initial_species(x.size, 0.2, 72)
    return dict(x=x, y=y, z=z, box=box, species=sp, dmu0=0.0, kappa=1000.0, cbar=0.2, T=600.0,
                seed=73)


def test_eam_parity_full_rows(torch_cuda, oracle_mod):
    """Every row of the MD list full (the lattice above with an MD-list skin
    of 0.1 A).  The lists come from the region search (eleven search bins
    per axis, grown to 32 slots).  A row holding the largest count must keep
    every neighbour: energies and forces equal the oracle's bit for bit."""
    O = oracle_mod
    pot = I.params("FS-P1")
    s = _full_rows_system()
    x, y, z, box, sp = s["x"], s["y"], s["z"], s["box"], s["species"]
    wide = O.neighbors(x, y, z, box, pot.rc + 0.1 + 1e-3, vectors=False)
    near = O.neighbors(x, y, z, box, pot.rc, vectors=False)
    assert np.all(np.diff(wide.start) == 32) and np.all(np.diff(near.start) == 32)
    zero = np.zeros(x.size)
    d = dict(x=x, y=y, z=z, vx=zero, vy=zero, vz=zero, box=box, species=sp)
    g = gpu_context(d, pot, velocities=True, skin=0.1)
    U = g.energy(forces=True)
    st = O.SweepState(x, y, z, box, sp, pot)
    e_o = O.energy_atoms(st.nl, st.species, pot, st.rho)
    assert np.array_equal(g.atom_energies().cpu().numpy(), e_o)
    assert abs(U - math.fsum(e_o)) <= 1e-12 * abs(U)
    fo = O.forces(O.neighbors(x, y, z, box, pot.rc), sp, pot, st.rho)
    for got, want in zip((g.fx, g.fy, g.fz), fo):
        assert np.array_equal(got.cpu().numpy(), want)
    info = g.info()
    assert info["md_pairs"] == 32 * x.size
    # two MD steps of 0.1 fs (no rebuild), then a sweep on the r < rc rows
    # filtered out of the full MD rows
    g.md(0.1, 2)
    out = O.md(x, y, z, zero, zero, zero, sp, box, pot, 0.1, 2)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz"), out[:6]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    s_g = g.sweep(0.0, 1000.0, 0.2, 600.0, 1, 73)
    st2 = O.SweepState(out[0], out[1], out[2], box, sp, pot, vx=out[3], vy=out[4], vz=out[5])
    s_o, _, _ = O.sweep(st2, 0.0, 1000.0, 0.2, 600.0, 1, 73)
    assert g.info()["mc_pairs"] == 32 * x.size
    for k in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert s_g[k] == s_o[k], k
    assert np.array_equal(g.species.cpu().numpy(), st2.species)
    assert np.array_equal(g.rho().cpu().numpy(), st2.rho)
    g.close()


@pytest.mark.parametrize("strategy,tpg", [("graph", 1), ("stage", 1), ("persistent", 1),
                                          ("batch", 3)])
def test_sweep_full_rows(torch_cuda, oracle_mod, strategy, tpg):
    """Every MC row full (32 neighbours within rc for every atom): each sweep
    strategy reproduces the oracle's chain over two sweeps."""
    r = _sweep_parity(oracle_mod, _full_rows_system(), I.params("FS-P1"), 2,
                      log=strategy != "batch", strategy=strategy, trials_per_group=tpg)
    assert r["flips"] > 0


def test_local_chain_full_rows(torch_cuda, oracle_mod):
    """Local chains of 2 trials per cell and stage on full MC rows: the chain
    (statistics, species and densities) equals the oracle's."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _full_rows_system()
    args = (d["dmu0"], 5.0, d["cbar"], d["T"])
    g = gpu_context(d, pot)
    g.set_local_steps(2)
    sg = g.sweep(*args, 2, d["seed"])
    st = oracle_state(O, d, pot)
    so, _, _ = O.sweep(st, *args, 2, d["seed"], local_steps=2)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert sg["flips"] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


def _sweep_parity(O, d, pot, n_sweeps, kappa=None, cbar=None, log=True, chunks=None,
                  strategy="graph", trials_per_group=1):
    kappa = d["kappa"] if kappa is None else kappa
    cbar = d["cbar"] if cbar is None else cbar
    args = (d["dmu0"], kappa, cbar, d["T"])
    g = gpu_context(d, pot)
    g.set_tuning(strategy, trials_per_group)
    info = g.info()
    S = info["stages_per_sweep"]
    ncpc = int(np.prod(info["n_cells"])) // 8
    st0 = oracle_state(O, d, pot)
    if log:
        g.enable_log(n_sweeps * S * ncpc, n_sweeps * S)
    chunks = chunks or [n_sweeps]
    gs = None
    for k in chunks:
        s = g.sweep(*args, k, d["seed"])
        gs = s if gs is None else {key: gs[key] + s[key] if key not in ("n_final",) else s[key]
                                   for key in s}
    sp_g = g.species.cpu().numpy()
    rho_g = g.rho().cpu().numpy()
    res = {}
    tl_g = sl_g = None
    if log:
        tl_g, sl_g, nt, ns = g.logs()
        assert nt == tl_g.shape[0] and ns == sl_g.shape[0]
    over = tie_overrides(tl_g, sl_g) if log else None
    so, tl_o, sl_o = O.sweep(st0, *args, n_sweeps, d["seed"], log_trials=10 ** 8 if log else 0,
                             log_stages=10 ** 8 if log else 0, overrides=over)
    if log:
        res = compare_logs(tl_g, sl_g, tl_o, sl_o)
    for k in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert gs[k] == so[k], (k, gs[k], so[k])
    assert gs["sum_n"] == so["sum_n"] and gs["sum_n2"] == so["sum_n2"]
    assert np.array_equal(sp_g, st0.species)
    assert np.array_equal(rho_g, st0.rho)
    g.close()
    res.update(gs)
    return res


@pytest.mark.parametrize("kappa", [1000.0, 10.0, 0.0])
def test_sweep_parity_c1(torch_cuda, oracle_mod, kappa):
    d = W.c1()
    r = _sweep_parity(oracle_mod, d, I.params("FS-P1"), 100, kappa=kappa)
    assert r["trials"] == 100 * 2000
    if kappa <= 10.0:
        assert r["flips"] > 0


@pytest.mark.parametrize("cbar", [0.02, 0.05, 0.10])
def test_sweep_parity_c2(torch_cuda, oracle_mod, cbar):
    d = W.c2(cbar=cbar)
    r = _sweep_parity(oracle_mod, d, I.params("FS-P1"), 10)
    assert r["flips"] > 0


@pytest.mark.parametrize("strategy,tpg", [("stage", 1), ("persistent", 1), ("graph", 3)])
def test_sweep_strategies_agree(torch_cuda, oracle_mod, strategy, tpg):
    """Per-stage launches, the direct persistent launch and other tilings of
    the graph-captured persistent launch all reproduce the oracle."""
    d = W.c2(cbar=0.05)
    r = _sweep_parity(oracle_mod, d, I.params("FS-P1"), 4, strategy=strategy,
                      trials_per_group=tpg)
    assert r["flips"] > 0
    r1 = _sweep_parity(oracle_mod, W.c1(), I.params("FS-P1"), 20, kappa=10.0,
                       strategy=strategy, trials_per_group=tpg)
    assert r1["trials"] == 20 * 2000


def _replica_set(n_rep=6, seed=55):
    """Uneven rigid bcc replicas on a T x kappa x cbar grid (small sizes)."""
    rng = np.random.default_rng(seed)
    reps = []
    for r in range(n_rep):
        nx, ny, nz = (int(v) for v in rng.integers(10, 19, size=3))
        x, y, z, box = I.bcc(nx, ny, nz)
        T = [400.0, 600.0, 800.0][r % 3]
        kappa = [100.0, 1000.0][(r // 3) % 2]
        cbar = float(np.exp(rng.uniform(np.log(0.01), np.log(0.2))))
        sp = I.initial_species(x.size, cbar, seed + r)
        reps.append(dict(x=x, y=y, z=z, box=box, species=sp, T=T, kappa=kappa, cbar=cbar,
                         dmu0=W.dmu_s(T, cbar)))
    return reps


def test_batch_replicas_match_oracle(torch_cuda, oracle_mod):
    """Each replica of a batch equals an independent oracle chain keyed
    (seed, replica index), with its own parameters and stage count."""
    O = oracle_mod
    from paper_1012_5082_amd.binding import VCSGCBatch
    pot = I.params("FS-P1")
    reps = _replica_set()
    b = VCSGCBatch(reps, pot)
    args = [np.array([r[k] for r in reps]) for k in ("dmu0", "kappa", "cbar", "T")]
    seed = 777
    s1 = b.sweep_batch(*args, 3, seed)
    s2 = b.sweep_batch(*args, 2, seed)
    for k, r in enumerate(reps):
        st = O.SweepState(r["x"], r["y"], r["z"], r["box"], r["species"], pot)
        so, _, _ = O.sweep(st, r["dmu0"], r["kappa"], r["cbar"], r["T"], 5, seed, replica=k)
        assert s1[k]["trials"] + s2[k]["trials"] == so["trials"]
        assert s1[k]["flips"] + s2[k]["flips"] == so["flips"]
        assert s2[k]["n_final"] == so["n_final"]
        assert np.array_equal(b.replica_species(k), st.species), k
        assert np.array_equal(b.replica_rho(k), st.rho), k
    b.close()


def test_sweep_chunking_and_determinism(torch_cuda, oracle_mod):
    d = W.c2(cbar=0.05)
    pot = I.params("FS-P1")
    _sweep_parity(oracle_mod, d, pot, 6, log=False, chunks=[2, 1, 3])
    a = gpu_context(d, pot)
    b = gpu_context(d, pot)
    a.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 5, 9)
    b.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 5, 9)
    assert np.array_equal(a.species.cpu().numpy(), b.species.cpu().numpy())
    assert np.array_equal(a.rho().cpu().numpy(), b.rho().cpu().numpy())
    a.close()
    b.close()


def test_stage_graph_replay(torch_cuda, oracle_mod):
    """Per-stage sweeps without logs run as a replayed graph of one sweep
    (sweep counter on the device, rebuilt when the parameters change): the
    chain equals the oracle's across calls, chunks and parameter changes."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    _sweep_parity(O, d, pot, 6, log=False, chunks=[2, 1, 3], strategy="stage")
    g = gpu_context(d, pot)
    g.set_tuning("stage", 1)
    st = oracle_state(O, d, pot)
    plan = [((d["dmu0"], d["kappa"], 0.05, d["T"]), 2), ((d["dmu0"] + 0.02, 10.0, 0.04, 650.0), 3),
            ((d["dmu0"], d["kappa"], 0.05, d["T"]), 1)]
    for args, k in plan:
        sg = g.sweep(*args, k, d["seed"])
        so, _, _ = O.sweep(st, *args, k, d["seed"])
        for key in ("trials", "local_accepts", "stage_accepts", "flips", "n_final"):
            assert sg[key] == so[key], key
        assert sg["sum_n"] == so["sum_n"]
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


@pytest.mark.parametrize("log", [True, False])
@pytest.mark.parametrize("kappa", [0.0, 10.0])
def test_stage_pipeline_accepting_stages(torch_cuda, oracle_mod, kappa, log):
    """The fused stage pipeline with many accepted stages (kappa = 0 accepts
    every stage with a local accept): the extra trial kernels after accepted
    stages, the host's top-up launches when its estimate falls short, direct
    launches (logs) and graph replays all give the oracle's chain."""
    d = W.c2(cbar=0.05)
    r = _sweep_parity(oracle_mod, d, I.params("FS-P1"), 3, kappa=kappa, log=log,
                      chunks=[1, 2], strategy="stage")
    assert r["stage_accepts"] > 0
    if kappa == 0.0:
        assert r["stage_accepts"] * 2 > r["stages"]


@pytest.mark.parametrize("D,kappa", [(1, 10.0), (4, 0.0), (8, 1000.0), (16, 10.0)])
def test_batched_pipeline_parity(torch_cuda, oracle_mod, D, kappa):
    """Batches of D stages tried on the state as it is and tested in order up
    to the first accepted stage (whose commit drops the trials after it): the
    chain equals the oracle's, across calls, with few and with most stages
    accepted (kappa = 0)."""
    d = W.c2(cbar=0.05)
    r = _sweep_parity(oracle_mod, d, I.params("FS-P1"), 3, kappa=kappa, log=False,
                      chunks=[1, 2], strategy="batch", trials_per_group=D)
    assert r["stage_accepts"] > 0


def test_batched_pipeline_timed_and_retuned(torch_cuda, oracle_mod):
    """The batched pipeline with per-kernel timing (event nodes in its graphs),
    a change of batch length between calls and a call of zero sweeps."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    g = gpu_context(d, pot)
    g.set_tuning("batch", 8)
    st = oracle_state(O, d, pot)
    args = (d["dmu0"], 10.0, d["cbar"], d["T"])
    g.kernel_timing(["stage"])
    s0 = g.sweep(*args, 0, d["seed"])
    assert s0["trials"] == 0 and s0["stages"] == 0
    for D, n_sw in ((8, 2), (3, 1)):
        g.set_tuning("batch", D)
        sg = g.sweep(*args, n_sw, d["seed"])
        so, _, _ = O.sweep(st, *args, n_sw, d["seed"])
        for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
            assert sg[key] == so[key], key
        assert sg["sum_n"] == so["sum_n"] and sg["sum_n2"] == so["sum_n2"]
    kt = g.kernel_times()
    assert kt["stage"][1] > 0 and kt["stage"][0] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


def test_stage_pipeline_timed_and_empty(torch_cuda, oracle_mod):
    """Per-kernel timing of the pipeline (event nodes in its graphs) and a
    call of zero sweeps leave the chain equal to the oracle's."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    g = gpu_context(d, pot)
    g.set_tuning("stage", 1)
    st = oracle_state(O, d, pot)
    args = (d["dmu0"], 10.0, d["cbar"], d["T"])
    g.kernel_timing(["stage"])
    s0 = g.sweep(*args, 0, d["seed"])
    assert s0["trials"] == 0 and s0["stages"] == 0
    sg = g.sweep(*args, 2, d["seed"])
    kt = g.kernel_times()
    assert kt["stage"][2] >= sg["stages"] and kt["stage"][1] > 0
    so, _, _ = O.sweep(st, *args, 2, d["seed"])
    for key in ("trials", "local_accepts", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


@pytest.mark.parametrize("k", [2, 5])
def test_local_chain_parity(torch_cuda, oracle_mod, k):
    """k trials per active cell per stage: every trial (its dU, decision and
    margin), every stage and the final state equal the oracle's."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    args = (d["dmu0"], 5.0, d["cbar"], d["T"])
    g = gpu_context(d, pot)
    g.set_local_steps(k)
    info = g.info()
    S = info["stages_per_sweep"]
    ncpc = int(np.prod(info["n_cells"])) // 8
    n_sw = 3
    g.enable_log(n_sw * S * ncpc * k, n_sw * S)
    sg = g.sweep(*args, n_sw, d["seed"])
    tl_g, sl_g, nt, ns = g.logs()
    st = oracle_state(O, d, pot)
    so, tl_o, sl_o = O.sweep(st, *args, n_sw, d["seed"], log_trials=10 ** 8, log_stages=10 ** 8,
                             overrides=tie_overrides(tl_g, sl_g), local_steps=k)
    compare_logs(tl_g, sl_g, tl_o, sl_o)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert 0 < sg["stage_accepts"] < sg["stages"]
    assert sg["local_accepts"] > sg["flips"]  # some stages were undone
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    # the same chain without logs (replayed graph), from a fresh context
    g2 = gpu_context(d, pot)
    g2.set_tuning("stage", 1)
    g2.set_local_steps(k)
    s2 = g2.sweep(*args, n_sw, d["seed"])
    assert s2["flips"] == so["flips"] and s2["n_final"] == so["n_final"]
    assert np.array_equal(g2.species.cpu().numpy(), st.species)
    g.close()
    g2.close()


def test_local_chain_undo_restores_velocities(torch_cuda, oracle_mod):
    """With velocities, trials of undone stages restore them exactly."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=16, c=0.1, seed=43)
    g = gpu_context(d, pot, velocities=True)
    g.set_local_steps(3)
    sg = g.sweep(d["dmu0"], 1.0, d["cbar"], d["T"], 2, d["seed"])
    st = O.SweepState(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
                      vz=d["vz"])
    so, _, _ = O.sweep(st, d["dmu0"], 1.0, d["cbar"], d["T"], 2, d["seed"], local_steps=3)
    assert sg["flips"] == so["flips"] and sg["stage_accepts"] < sg["stages"]
    for nm in ("vx", "vy", "vz"):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), getattr(st, nm)), nm
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    g.close()


def _md_system(n=10, T=700.0, seed=31, c=0.05):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return dict(x=x, y=y, z=z, box=box, species=sp, vx=vx, vy=vy, vz=vz, T=T, kappa=1000.0,
                cbar=c, dmu0=W.dmu_s(T, c), seed=4001)


def test_md_parity(torch_cuda, oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system()
    g = gpu_context(d, pot, velocities=True)
    g.md(1.0, 40)
    out = O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["species"], d["box"], pot,
               1.0, 40)
    names = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz")
    for nm, want in zip(names, out[:9]):
        got = getattr(g, nm).cpu().numpy()
        assert np.array_equal(got, want), nm
    g.close()


@pytest.mark.parametrize("n,skin", [(6, 0.75), (7, 0.3)])
def test_md_parity_build_paths(torch_cuda, oracle_mod, n, skin):
    """MD lists from both builders: a 6^3 box with a 0.75 A skin has three
    search bins per axis (one lane per atom), a 7^3 box with the default skin
    five (super-bins, odd count: the last super-bin is half empty).
    Device-decided rebuilds happen in the 60 steps at 1000 K; positions,
    velocities and forces stay bit for bit those of the oracle, and the
    list statistics equal a fresh build at the final positions."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=n, T=1000.0, seed=53 + n)
    g = gpu_context(d, pot, velocities=True, skin=skin)
    g.md(1.0, 60)
    out = O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"], d["species"], d["box"], pot,
               1.0, 60)
    names = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz")
    for nm, want in zip(names, out[:9]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    info = g.info()
    assert info["md_rebuilds"] >= 1
    x, y, z = out[0], out[1], out[2]
    nl = O.neighbors(x, y, z, d["box"], pot.rc, vectors=False)
    # the r < rc list filtered out of the MD list and the density cache from
    # the last MD density pass
    g.sweep(d["dmu0"], 0.0, d["cbar"], d["T"], 0, d["seed"])
    assert g.info()["mc_pairs"] == nl.j.size
    assert g.info()["mc_kmax_used"] == int(np.diff(nl.start).max())
    assert np.array_equal(g.rho().cpu().numpy(), O.density(nl, d["species"], pot))
    g.close()


@pytest.mark.parametrize("path", ["pipeline", "da_perfect", "chain3", "persistent", "batch",
                                  "da_batch"])
def test_sweep_paths_after_md(torch_cuda, oracle_mod, path):
    """Sweeps right after MD run on the r < rc list filtered out of the MD
    rows and on the last MD density pass: every sweep kernel family (fused
    pipeline, delayed acceptance with a perfect surrogate, local chains with
    their undo log, the persistent kernel) gives the oracle's chain bit for
    bit, velocities included."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=16, c=0.1, seed=47)
    kappa, n_sw, k = 1.0, 2, 3 if path == "chain3" else 1
    x, y, z, vx, vy, vz, *_ = O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                                   d["species"], d["box"], pot, 1.0, 20)
    g = gpu_context(d, pot, velocities=True)
    g.md(1.0, 20)
    if path in ("da_perfect", "da_batch"):
        g.set_surrogate("perfect")
    if path in ("batch", "da_batch"):
        g.set_tuning("batch", 4)
    elif path == "chain3":
        g.set_local_steps(k)
    elif path == "persistent":
        g.set_tuning("graph", 1)
    nl = O.neighbors(x, y, z, d["box"], pot.rc, vectors=False)
    assert np.array_equal(g.rho().cpu().numpy(), O.density(nl, d["species"], pot))
    info = g.info()
    S = info["stages_per_sweep"]
    ncpc = int(np.prod(info["n_cells"])) // 8
    assert info["mc_pairs"] == nl.j.size
    log = path in ("pipeline", "chain3")
    if log:
        g.enable_log(n_sw * S * ncpc * k, n_sw * S)
    sg = g.sweep(d["dmu0"], kappa, d["cbar"], d["T"], n_sw, d["seed"])
    st = O.SweepState(x, y, z, d["box"], d["species"], pot, vx=vx, vy=vy, vz=vz)
    over = None
    if log:
        tl_g, sl_g, _, _ = g.logs()
        over = tie_overrides(tl_g, sl_g)
    so, tl_o, sl_o = O.sweep(st, d["dmu0"], kappa, d["cbar"], d["T"], n_sw, d["seed"],
                             log_trials=10 ** 8 if log else 0, log_stages=10 ** 8 if log else 0,
                             overrides=over, local_steps=k)
    if log:
        compare_logs(tl_g, sl_g, tl_o, sl_o)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert sg["flips"] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    for nm in ("vx", "vy", "vz"):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), getattr(st, nm)), nm
    g.close()


def test_hybrid_cycle_parity(torch_cuda, oracle_mod):
    """[1 sweep; 20 MD steps] x 3 with velocity rescaling on transmutation."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=16, c=0.1, seed=41)
    g = gpu_context(d, pot, velocities=True)
    x, y, z = d["x"], d["y"], d["z"]
    vx, vy, vz = d["vx"], d["vy"], d["vz"]
    sp = d["species"]
    w = 0
    for cyc in range(3):
        g.sweep(d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        st = O.SweepState(x, y, z, d["box"], sp, pot, vx=vx, vy=vy, vz=vz)
        st.w = w
        O.sweep(st, d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        w += 1
        sp = st.species
        assert np.array_equal(g.rho().cpu().numpy(), st.rho)
        g.md(1.0, 20)
        x, y, z, vx, vy, vz, *_ = O.md(x, y, z, st.vx, st.vy, st.vz, sp, d["box"], pot, 1.0, 20)
        # the sweep's lists and density cache after MD come from the MD list and
        # the last MD density pass: equal to a fresh r < rc build at the new positions
        nl = O.neighbors(x, y, z, d["box"], pot.rc, vectors=False)
        assert np.array_equal(g.rho().cpu().numpy(), O.density(nl, sp, pot))
        assert g.info()["mc_pairs"] == nl.j.size
    assert np.array_equal(g.species.cpu().numpy(), sp)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz"), (x, y, z, vx, vy, vz)):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    g.close()


@pytest.fixture(scope="module")
def c3_data():
    return W.c3()


def test_full_size_c3_sweep_and_md(torch_cuda, oracle_mod, c3_data):
    """The 1.96M-site polycrystal: one full sweep (species and density cache
    bit for bit, every counter equal) and two MD steps (positions and
    velocities bit for bit)."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = c3_data
    g = gpu_context(d, pot, velocities=True)
    s = g.sweep(d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"])
    st = oracle_state(O, d, pot, velocities=True)
    so, _, _ = O.sweep(st, d["dmu0"], d["kappa"], d["cbar"], d["T"], 1, d["seed"])
    for k in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert s[k] == so[k], k
    assert s["trials"] >= 0.9 * x_size(d)
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.md(1.0, 2)
    out = O.md(d["x"], d["y"], d["z"], st.vx, st.vy, st.vz, st.species, d["box"], pot, 1.0, 2)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz"), out[:6]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    g.close()


def x_size(d):
    return d["x"].size


@pytest.mark.parametrize("path", ["stage_logged", "batch", "graph", "chain3", "da_perfect"])
def test_colours27_parity(torch_cuda, oracle_mod, path):
    """The 27-colour scheme (cells of edge >= r_dep / 2, colours by indices
    modulo 3) on every sweep kernel family: the chain equals the oracle's
    chain with the same colouring, bit for bit (trial and stage logs too on
    the logged path)."""
    O = oracle_mod
    from paper_1012_5082_amd.binding import VCSGC
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    k = 3 if path == "chain3" else 1
    args = (d["dmu0"], 10.0, d["cbar"], d["T"])
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, colours=27)
    info = g.info()
    nc = np.array(info["n_cells"])
    assert np.all(nc % 3 == 0) and np.array_equal(nc, O.cell_grid(d["box"], 2 * pot.rc, 3))
    ncells = int(np.prod(nc))
    assert info["stages_per_sweep"] == 27 * -(-d["x"].size // ncells)
    if path == "stage_logged":
        g.set_tuning("stage", 1)
        g.enable_log(3 * info["stages_per_sweep"] * (ncells // 27), 3 * info["stages_per_sweep"])
    elif path == "batch":
        g.set_tuning("batch", 4)
    elif path == "graph":
        g.set_tuning("graph", 1)
    elif path == "chain3":
        g.set_local_steps(k)
    elif path == "da_perfect":
        g.set_surrogate("perfect")
    sg = g.sweep(*args, 2, d["seed"])
    sg2 = g.sweep(*args, 1, d["seed"])
    st = oracle_state(O, d, pot)
    log = path == "stage_logged"
    over = None
    if log:
        tl_g, sl_g, _, _ = g.logs()
        over = tie_overrides(tl_g, sl_g)
    so, tl_o, sl_o = O.sweep(st, *args, 3, d["seed"], log_trials=10 ** 8 if log else 0,
                             log_stages=10 ** 8 if log else 0, overrides=over, local_steps=k,
                             colour_period=3)
    if log:
        compare_logs(tl_g, sl_g, tl_o, sl_o)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips"):
        assert sg[key] + sg2[key] == so[key], key
    assert sg2["n_final"] == so["n_final"]
    assert so["stage_accepts"] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


def test_colours27_after_md_and_replicas(torch_cuda, oracle_mod):
    """27 colours after MD with velocities (batched pipeline), and in a
    replica batch (persistent launch): both equal the oracle."""
    O = oracle_mod
    from paper_1012_5082_amd.binding import VCSGC, VCSGCBatch
    pot = I.params("FS-P1")
    d = _md_system(n=16, c=0.1, seed=49)
    x, y, z, vx, vy, vz, *_ = O.md(d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"],
                                   d["species"], d["box"], pot, 1.0, 20)
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"], colours=27)
    g.md(1.0, 20)
    g.set_tuning("batch", 4)
    sg = g.sweep(d["dmu0"], 1.0, d["cbar"], d["T"], 2, d["seed"])
    st = O.SweepState(x, y, z, d["box"], d["species"], pot, vx=vx, vy=vy, vz=vz)
    so, _, _ = O.sweep(st, d["dmu0"], 1.0, d["cbar"], d["T"], 2, d["seed"], colour_period=3)
    for key in ("trials", "local_accepts", "stages", "stage_accepts", "flips", "n_final"):
        assert sg[key] == so[key], key
    assert sg["flips"] > 0
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    for nm in ("vx", "vy", "vz"):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), getattr(st, nm)), nm
    g.close()
    reps = _replica_set(n_rep=4, seed=57)
    b = VCSGCBatch(reps, pot, colours=27)
    par = [np.array([r[k] for r in reps]) for k in ("dmu0", "kappa", "cbar", "T")]
    s1 = b.sweep_batch(*par, 2, 888)
    for k, r in enumerate(reps):
        stk = O.SweepState(r["x"], r["y"], r["z"], r["box"], r["species"], pot)
        sok, _, _ = O.sweep(stk, r["dmu0"], r["kappa"], r["cbar"], r["T"], 2, 888, replica=k,
                            colour_period=3)
        assert s1[k]["flips"] == sok["flips"] and s1[k]["n_final"] == sok["n_final"], k
        assert np.array_equal(b.replica_species(k), stk.species), k
    b.close()
