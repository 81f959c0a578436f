"""Pins of the oracle's surrogate pieces: bfloat16 rounding, MLP forward and
gradient, the local descriptor, and the exactness of delayed acceptance.

* bfloat16 rounding against torch's CPU float32 -> bfloat16 conversion;
* FP64 gradient against central finite differences of the FP64 loss;
* descriptor of a perfect pure-A bcc site against its shell counts, and the
  descriptor of the flipped state equal (bit for bit) to the descriptor
  computed after actually committing the flip (what makes the reverse-move
  surrogate value the true stage-1 value of the reverse move);
* delayed acceptance with a perfect surrogate equals the plain chain bit for
  bit; with a zero or an untrained random network it still samples the exact
  ensemble (16-site enumeration, identical-species closed form).
"""
import math

import numpy as np
import pytest

import exact_refs as X
from paper_1012_5082_amd import inputs as I


def test_bf16_rounding_matches_torch(oracle_mod):
    import torch
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.normal(0, 10, 4000), rng.uniform(-1e-3, 1e-3, 1000),
                           np.array([1.00390625, 1.01171875, -2.00781250, 0.0, 65504.0])])
    vals = vals.astype(np.float32)
    want = torch.tensor(vals).to(torch.bfloat16).float().numpy()
    got = np.array([oracle_mod.bf16(v) for v in vals], dtype=np.float32)
    assert np.array_equal(got, want)


def _samples(n=64, seed=1):
    rng = np.random.default_rng(seed)
    d = np.column_stack([rng.integers(0, 2, n), rng.integers(0, 4, (n, 3)),
                         rng.integers(6, 13, (n, 3)), rng.normal(13.0, 0.3, (n, 3))])
    t = rng.normal(0.4, 0.2, n)
    return d.astype(np.float64), t


def _params(seed=3):
    from oracle.oracle import MlpParams
    mu = np.array([0.5, 1, 1, 1, 8, 6, 12, 13, 13, 13], dtype=np.float64)
    sd = np.array([0.5, 1, 1, 1, 1, 1, 1, 0.5, 0.5, 0.5], dtype=np.float64)
    return MlpParams.random(seed, mu=mu, sd=sd, out_mu=0.4, out_sd=0.2)


def test_mlp_gradient_matches_finite_differences(oracle_mod):
    O = oracle_mod
    from oracle.oracle import MlpParams
    m = _params()
    d, t = _samples()
    loss, g = O.mlp_grad(m, d, t, bf16_emul=False)
    flat = m.flat().astype(np.float64)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(640, 8, replace=False), 640 + rng.choice(64, 4, replace=False),
                          704 + rng.choice(4096, 8, replace=False), 4800 + rng.choice(64, 4, replace=False),
                          4864 + rng.choice(64, 4, replace=False), [4928]])
    h = 1e-3

    def loss_at(v):
        mm = MlpParams.from_flat(v.astype(np.float32), m.mu, m.sd, m.out_mu, m.out_sd)
        y, _ = O.mlp_forward(mm, d, bf16_emul=False)
        tn = (t - m.out_mu) / m.out_sd
        return float(np.mean((y - tn) ** 2))

    # float32 parameters: perturb by exactly representable steps
    for k in idx:
        vp, vm = flat.copy(), flat.copy()
        vp[k] += h
        vm[k] -= h
        hp = float(np.float32(vp[k]) - np.float32(flat[k]))
        hm = float(np.float32(flat[k]) - np.float32(vm[k]))
        fd = (loss_at(vp) - loss_at(vm)) / (hp + hm)
        assert abs(fd - g[k]) <= 1e-5 * max(1e-3, abs(g[k])) + 1e-7, (k, fd, g[k])
    assert abs(loss - loss_at(flat)) < 1e-12


def test_mlp_bf16_emulation_close_to_fp64(oracle_mod):
    m = _params()
    d, t = _samples(256)
    y64, _ = oracle_mod.mlp_forward(m, d, bf16_emul=False)
    y16, _ = oracle_mod.mlp_forward(m, d, bf16_emul=True)
    assert np.max(np.abs(y64 - y16)) < 0.05 * np.max(np.abs(y64)) + 0.05
    _, g64 = oracle_mod.mlp_grad(m, d, t, bf16_emul=False)
    _, g16 = oracle_mod.mlp_grad(m, d, t, bf16_emul=True)
    assert np.linalg.norm(g64 - g16) < 0.05 * np.linalg.norm(g64)


def test_descriptor_perfect_lattice(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(6, 6, 6)
    sp = np.zeros(x.size, np.uint8)
    nl = O.neighbors(x, y, z, box, O.DESC_CUTOFF, vectors=False)
    rc_nl = O.neighbors(x, y, z, box, pot.rc, vectors=False)
    rho = O.density(rc_nl, sp, pot)
    d = O.descriptor(nl, 10, sp, rho, pot)
    assert np.array_equal(d[:7], [0, 0, 0, 0, 8, 6, 12])
    assert np.allclose(d[7:], rho[0], atol=1e-12)
    # flipped: s_i = 1; first- and second-shell densities move by (t_B - t_A)(rc - r)^2
    df = O.descriptor(nl, 10, sp, rho, pot, flip=True)
    assert df[0] == 1
    r1, r2 = I.A_LAT * math.sqrt(3) / 2, I.A_LAT
    assert abs(df[7] - (rho[0] + (pot.t_b - pot.t_a) * (pot.rc - r1) ** 2)) < 1e-12
    assert abs(df[8] - (rho[0] + (pot.t_b - pot.t_a) * (pot.rc - r2) ** 2)) < 1e-12
    assert abs(df[9] - rho[0]) < 1e-12


def test_flipped_descriptor_equals_committed_state(oracle_mod):
    """The descriptor of the proposed state, computed before the move, is
    bitwise the descriptor after the move is committed through the sweep."""
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(10, 10, 10)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 3)
    sp = I.initial_species(x.size, 0.2, 4)
    st = O.SweepState(x, y, z, box, sp, pot)
    dnl = O.neighbors(x, y, z, box, O.DESC_CUTOFF, vectors=False)
    # run sweeps and check at every committed flip of a sampled stage
    checked = 0
    for rep in range(6):
        before_sp, before_rho = st.species.copy(), st.rho.copy()
        s, tl, _ = O.sweep(st, -0.25, 0.5, 0.2, 600.0, 1, 31, log_trials=100000)
        changed = np.nonzero(st.species != before_sp)[0]
        # replay: pick sites that flipped and compare descriptors on a clone
        for i in changed[:5]:
            clone_sp, clone_rho = before_sp.copy(), before_rho.copy()
            pred = O.descriptor(dnl, i, clone_sp, clone_rho, pot, flip=True)
            # commit the single flip on the clone (the commit's density update)
            for e in range(st.nl.start[i], st.nl.start[i + 1]):
                j, r = st.nl.j[e], st.nl.r[e]
                t_new = pot.t_b if clone_sp[i] == 0 else pot.t_a
                t_old = pot.t_a if clone_sp[i] == 0 else pot.t_b
                clone_rho[j] = clone_rho[j] + (t_new * ((pot.rc - r) * (pot.rc - r))
                                               - t_old * ((pot.rc - r) * (pot.rc - r)))
            clone_sp[i] ^= 1
            after = O.descriptor(dnl, i, clone_sp, clone_rho, pot, flip=False)
            assert np.array_equal(pred, after)
            checked += 1
    assert checked > 5


def test_da_perfect_surrogate_equals_plain(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(10, 10, 10)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 9)
    sp = I.initial_species(x.size, 0.1, 10)
    a = O.SweepState(x, y, z, box, sp, pot)
    b = O.SweepState(x, y, z, box, sp, pot)
    args = (-0.22, 5.0, 0.1, 600.0)
    sa, _, _ = O.sweep(a, *args, 20, 5)
    sb, passes, _, _ = O.sweep_da(b, *args, 20, 5, "perfect")
    assert sa["flips"] > 50
    for k in ("trials", "local_accepts", "stage_accepts", "flips", "n_final"):
        assert sa[k] == sb[k], k
    assert passes == sa["local_accepts"]
    assert np.array_equal(a.species, b.species)
    assert np.array_equal(a.rho, b.rho)


E16 = dict(T=600.0, kappa=0.5, cbar=0.25, dmu0=-0.3)


@pytest.mark.parametrize("mode", ["zero", "mlp"])
def test_da_samples_exact_ensemble_16_sites(oracle_mod, mode):
    """Delayed acceptance with a poor surrogate (zero, or an untrained random
    network) in the serial chain of 16 sites still reproduces the exact
    enumeration averages: the second stage corrects any first stage."""
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(2, 2, 2)
    nl = O.neighbors(x, y, z, box, pot.rc)
    dnl = O.neighbors(x, y, z, box, O.DESC_CUTOFF, vectors=False)
    N = 16
    U = np.zeros(2 ** N)
    for s in range(2 ** N):
        sp = np.array([(s >> k) & 1 for k in range(N)], np.uint8)
        U[s] = O.energy_total(O.energy_atoms(nl, sp, pot))
    nb = np.array([bin(s).count("1") for s in range(2 ** N)])
    b = X.beta_of(E16["T"])
    phi = E16["dmu0"] - 2 * E16["kappa"] * E16["cbar"]
    lw = -b * (U + phi * nb + E16["kappa"] * nb * nb / N)
    pi = np.exp(lw - lw.max())
    pi /= pi.sum()
    c_ex = float((pi * nb).sum()) / N
    u_ex = float((pi * U).sum())
    m = None
    if mode == "mlp":
        m = _params(11)
        m.out_mu, m.out_sd = float(np.float32(0.3)), float(np.float32(0.5))
    st = O.SweepState(x, y, z, box, I.initial_species(16, 0.25, 3), pot, nl=nl)
    args = (E16["dmu0"], E16["kappa"], E16["cbar"], E16["T"])
    O.sweep_da(st, *args, 200, 404, mode, one_cell=True, mlp=m, desc_nl=dnl)
    cs, us = [], []
    passes = trials = 0
    for _ in range(12000):
        s, p1, _, _ = O.sweep_da(st, *args, 1, 404, mode, one_cell=True, mlp=m, desc_nl=dnl)
        passes += p1
        trials += s["trials"]
        cs.append(st.n_b[0] / N)
        us.append(O.energy_total(O.energy_atoms(nl, st.species, pot)))
    for series, want in ((cs, c_ex), (us, u_ex)):
        mean, err = X.batch_means(series, 40)
        assert abs(mean - want) < 3 * err, (mode, mean, want, err)
    assert 0 < passes < trials


def test_da_zero_surrogate_ideal_distribution(oracle_mod):
    O = oracle_mod
    x, y, z, box = I.bcc(10, 10, 10)
    T, kappa, cbar, dmu0 = 600.0, 2.0, 0.2, 0.0
    st = O.SweepState(x, y, z, box, I.initial_species(x.size, cbar, 2), I.params("IDEAL"))
    args = (dmu0, kappa, cbar, T)
    O.sweep_da(st, *args, 30, 88, "zero")
    ns = []
    for _ in range(600):
        O.sweep_da(st, *args, 1, 88, "zero")
        ns.append(st.n_b[0])
    p = X.normalize(X.vcsgc_logw_ideal(st.n, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
