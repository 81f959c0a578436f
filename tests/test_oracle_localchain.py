"""Pins of the oracle's k-step local chains (k trials per active cell per
stage, each on the state left by the previous one, the stage kept or undone
as a whole by the global factor on its net dn).

* k = 1 is the plain sweep, bit for bit;
* the stage kernel of a two-step local Metropolis chain followed by the
  global factor on the net change of n leaves the exact VC-SGC distribution
  of the 16-site cell invariant (transition matrix, to rounding), and a
  flipped sign of the global factor breaks it;
* the oracle's one-cell chain with k = 3 reproduces the 16-site enumeration
  averages;
* with identical A/B potentials and k = 4 over many cells, the distribution of
  n is the exact P(n) of the ideal VC-SGC ensemble.
"""
import numpy as np
import pytest
import scipy.sparse as sp_

import exact_refs as X
from paper_1012_5082_amd import inputs as I

E16 = dict(T=600.0, kappa=0.5, cbar=0.25, dmu0=-0.3)


def _pi16(e):
    b = X.beta_of(E16["T"])
    phi = E16["dmu0"] - 2 * E16["kappa"] * E16["cbar"]
    nb = e["nb"]
    lw = -b * (e["U"] + phi * nb + E16["kappa"] * nb * nb / e["N"])
    w = np.exp(lw - lw.max())
    return w / w.sum()


def test_one_step_is_the_plain_sweep(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(10, 10, 10)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 5)
    sp = I.initial_species(x.size, 0.1, 6)
    vx, vy, vz = I.mb_velocities(sp, 700.0, 7)
    a = O.SweepState(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz)
    b = O.SweepState(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz)
    args = (-0.22, 5.0, 0.1, 700.0, 6, 11)
    sa, ta, _ = O.sweep(a, *args, log_trials=10 ** 6)
    sb, tb, _ = O.sweep(b, *args, log_trials=10 ** 6, local_steps=1)
    assert sa == sb and sa["flips"] > 20
    assert np.array_equal(ta, tb)
    for k in ("species", "rho", "vx", "vy", "vz"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def _local_kernel(e):
    """One local Metropolis step of the one-cell chain: site uniform over the
    16, accepted with min{1, exp(-beta (dU + dmu0 dn))}."""
    N = e["N"]
    b = X.beta_of(E16["T"])
    s = np.arange(2 ** N)
    rows, cols, vals = [], [], []
    stay = np.ones(2 ** N)
    for i in range(N):
        t = s ^ (1 << i)
        dn = 1 - 2 * ((s >> i) & 1)
        p = np.minimum(1.0, np.exp(-b * (e["U"][t] - e["U"][s] + E16["dmu0"] * dn))) / N
        rows.append(s)
        cols.append(t)
        vals.append(p)
        stay -= p
    rows.append(s)
    cols.append(s)
    vals.append(stay)
    return sp_.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(2 ** N, 2 ** N))


def _stage_kernel(e, L2, sign=1.0):
    """Two local steps, then the global factor on the net change of n
    (endpoint-dependent), rejection back to the start."""
    N = e["N"]
    b = X.beta_of(E16["T"])
    c = L2.tocoo()
    n0, n1 = e["nb"][c.row], e["nb"][c.col]
    dn = (n1 - n0).astype(float)
    g = np.minimum(1.0, np.exp(-b * (E16["kappa"] / N) * dn *
                               (dn + sign * 2.0 * (n0 - N * E16["cbar"]))))
    moved = c.row != c.col
    P = sp_.csr_matrix((c.data[moved] * g[moved], (c.row[moved], c.col[moved])),
                       shape=L2.shape)
    stay = 1.0 - np.asarray(P.sum(axis=1)).ravel()
    return P + sp_.diags(stay)


def test_two_step_local_chain_is_exact(enum16):
    e = enum16
    pi = _pi16(e)
    L = _local_kernel(e)
    L2 = L @ L
    P = _stage_kernel(e, L2)
    assert np.max(np.abs(P.T @ pi - pi)) <= 1e-13 * pi.max()
    bad = _stage_kernel(e, L2, sign=-1.0)
    assert np.max(np.abs(bad.T @ pi - pi)) > 1e-4 * pi.max()


def test_local_chain_enumeration_16_sites(oracle_mod, enum16):
    O = oracle_mod
    e = enum16
    pi = _pi16(e)
    c_ex = float((pi * e["nb"]).sum()) / e["N"]
    u_ex = float((pi * e["U"]).sum())
    st = O.SweepState(e["x"], e["y"], e["z"], e["box"], I.initial_species(16, 0.25, 9), e["pot"],
                      nl=e["nl"])
    args = (E16["dmu0"], E16["kappa"], E16["cbar"], E16["T"])
    O.sweep(st, *args, 200, 505, one_cell=True, local_steps=3)
    cs, us = [], []
    for _ in range(15000):
        s, _, _ = O.sweep(st, *args, 1, 505, one_cell=True, local_steps=3)
        cs.append(st.n_b[0] / 16)
        us.append(O.energy_total(O.energy_atoms(e["nl"], st.species, e["pot"])))
    assert s["trials"] == 3 * 6  # ceil(16 / 3) stages of 3 trials
    for series, want in ((cs, c_ex), (us, u_ex)):
        mean, err = X.batch_means(series, 40)
        assert abs(mean - want) < 3 * err, (mean, want, err)


def test_local_chain_ideal_exact_distribution(oracle_mod):
    """Identical A/B potentials over 64 cells (8 active per stage), k = 4:
    P(n) is the exact ideal VC-SGC distribution.  The parameters keep the
    local acceptance below one (dmu0 > 0) and the composite moves small enough
    for the global factor to accept a good share of the stages."""
    O = oracle_mod
    x, y, z, box = I.bcc(14, 14, 14)
    T, kappa, cbar, dmu0 = 600.0, 0.3, 0.2, 0.05
    p = X.normalize(X.vcsgc_logw_ideal(x.size, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    st = O.SweepState(x, y, z, box, I.initial_species(x.size, m / x.size, 2), I.params("IDEAL"))
    args = (dmu0, kappa, cbar, T)
    s0, _, _ = O.sweep(st, *args, 20, 77, local_steps=4)
    # 5488 sites in 4^3 cells (8 per colour): 8 ceil(ceil(5488 / 64) / 4) = 176 stages
    # of 4 trials in each of the 8 active cells
    assert s0["trials"] == 20 * 176 * 8 * 4
    assert 0 < s0["stage_accepts"] < s0["stages"]
    ns = []
    for _ in range(500):
        O.sweep(st, *args, 1, 77, local_steps=4)
        ns.append(st.n_b[0])
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(np.var(ns) / v - 1.0) < 0.3
