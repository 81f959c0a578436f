"""Pins of the oracle's sampler against exact results of the ensemble.

* identical species, SGC: c = 1/(1 + exp(beta dmu))               (Sec. II.B)
* identical species, VC-SGC: P(n) ~ C(N,n) exp[-beta(phi n + kappa n^2/N)]
* independent sites (INDEP): Poisson-binomial DP tilted by the same factor
* 16-site bcc cell: exact enumeration of all 2^16 states vs the serial chain
* exact detailed balance of the decomposed acceptance (Eq. mod) on 16 sites
* A <-> B symmetry at dmu0 = 0, cbar = 1/2
* Eq. gforce (dmu = phi + 2 kappa <c>) and Eq. df2_vcsgc (variance)
Statistical checks use 3 sigma with batch-means errors on fixed seeds.
"""
import math

import numpy as np
import pytest

import exact_refs as X
from paper_1012_5082_amd import inputs as I


def _chain(O, st, n_sweeps, dmu0, kappa, cbar, T, seed, one_cell=False, energy=False, period=2):
    ns, us = [], []
    for _ in range(n_sweeps):
        O.sweep(st, dmu0, kappa, cbar, T, 1, seed, one_cell=one_cell, colour_period=period)
        ns.append(int(st.n_b[0]))
        if energy:
            us.append(O.energy_total(O.energy_atoms(st.nl, st.species, st.pot)))
    return np.array(ns, float), np.array(us, float)


def _c1_state(O, pot, seed=1, c_init=0.05, thermal=None):
    x, y, z, box = I.bcc(10, 10, 10)
    if thermal is not None:
        x, y, z = I.thermalize(x, y, z, box, 0.05, thermal)
    sp = I.initial_species(x.size, c_init, seed)
    return O.SweepState(x, y, z, box, sp, pot)


def test_ideal_sgc_closed_form(oracle_mod):
    O = oracle_mod
    st = _c1_state(O, I.params("IDEAL"))
    T, dmu = 600.0, 0.05
    ns, _ = _chain(O, st, 30, dmu, 0.0, 0.0, T, seed=101)       # burn-in
    ns, _ = _chain(O, st, 400, dmu, 0.0, 0.0, T, seed=101)
    mean, err = X.batch_means(ns)
    want = st.n * X.ideal_sgc_c(T, dmu)
    assert abs(mean - want) < 3 * err, (mean, want, err)
    # the binomial variance N c (1 - c)
    c = X.ideal_sgc_c(T, dmu)
    assert abs(ns.var() / (st.n * c * (1 - c)) - 1.0) < 0.2


@pytest.mark.parametrize("kappa,cbar,dmu0,period", [(2.0, 0.2, 0.0, 2), (10.0, 0.2, 0.0, 2),
                                                   (2.0, 0.2, 0.0, 3)])
def test_ideal_vcsgc_exact_distribution(oracle_mod, kappa, cbar, dmu0, period):
    """period 3: the 27-colour scheme (cells of edge >= r_dep / 2)."""
    O = oracle_mod
    st = _c1_state(O, I.params("IDEAL"), c_init=cbar)
    T = 600.0
    _chain(O, st, 30, dmu0, kappa, cbar, T, seed=202, period=period)
    ns, _ = _chain(O, st, 600, dmu0, kappa, cbar, T, seed=202, period=period)
    p = X.normalize(X.vcsgc_logw_ideal(st.n, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(ns.var() / v - 1.0) < 0.25, (ns.var(), v)


def test_ideal_vcsgc_wrong_sign_is_distinguishable():
    """The printed sign of the (c - c0) term (a repulsive constraint) gives a
    distribution whose mean differs from the exact one by many sigma, so the
    test above would catch it."""
    N, T, kappa, cbar, dmu0 = 2000, 600.0, 2.0, 0.2, 0.0
    p = X.normalize(X.vcsgc_logw_ideal(N, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    # with the constraint sign flipped, phi n + kappa n^2/N becomes phi' n - kappa n^2/N
    b = X.beta_of(T)
    phi = dmu0 + 2.0 * kappa * cbar
    n = np.arange(N + 1.0)
    from scipy.special import gammaln
    lw = gammaln(N + 1.0) - gammaln(n + 1) - gammaln(N - n + 1) - b * (phi * n - kappa * n * n / N)
    m2, _ = X.moments(X.normalize(lw))
    assert abs(m2 - m) > 20 * math.sqrt(v)


@pytest.mark.parametrize("period", [2, 3])
def test_indep_poisson_binomial(oracle_mod, period):
    O = oracle_mod
    pot = I.params("INDEP")
    st = _c1_state(O, pot, c_init=0.1, thermal=41)
    T, kappa, cbar, dmu0 = 600.0, 1.0, 0.1, -0.70
    # site energy of B relative to A: only the own embedding differs
    rho = st.rho
    de = (-pot.a_b + pot.a_a) * np.sqrt(rho)
    p = X.normalize(X.vcsgc_logw_indep(de, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    _chain(O, st, 30, dmu0, kappa, cbar, T, seed=303, period=period)
    ns, _ = _chain(O, st, 600, dmu0, kappa, cbar, T, seed=303, period=period)
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(ns.var() / v - 1.0) < 0.25


E16 = dict(T=600.0, kappa=0.5, cbar=0.25, dmu0=-0.3)


def _pi16(e):
    b = X.beta_of(E16["T"])
    phi = E16["dmu0"] - 2 * E16["kappa"] * E16["cbar"]
    nb = e["nb"]
    lw = -b * (e["U"] + phi * nb + E16["kappa"] * nb * nb / e["N"])
    w = np.exp(lw - lw.max())
    return w / w.sum()


def test_enumeration_16_sites(oracle_mod, enum16):
    O = oracle_mod
    e = enum16
    pi = _pi16(e)
    c_ex = float((pi * e["nb"]).sum()) / e["N"]
    u_ex = float((pi * e["U"]).sum())
    c2_ex = float((pi * e["nb"] ** 2).sum()) / e["N"] ** 2
    sp = I.initial_species(16, 0.25, 9)
    st = O.SweepState(e["x"], e["y"], e["z"], e["box"], sp, e["pot"], nl=e["nl"])
    args = (E16["dmu0"], E16["kappa"], E16["cbar"], E16["T"])
    _chain(O, st, 200, *args, seed=404, one_cell=True)
    ns, us = _chain(O, st, 20000, *args, seed=404, one_cell=True, energy=True)
    c = ns / 16
    for series, want in ((c, c_ex), (us, u_ex), (c * c, c2_ex)):
        mean, err = X.batch_means(series, 40)
        assert abs(mean - want) < 3 * err, (mean, want, err)


def _transitions(e, sign=+1.0, factor2=True):
    """Single-flip kernel of the serial decomposed test (Eq. mod): site chosen
    uniformly, local factor with dmu0, global factor with cbar."""
    N = e["N"]
    b = X.beta_of(E16["T"])
    kap, cbar, dmu0 = E16["kappa"], E16["cbar"], E16["dmu0"]
    s = np.arange(2 ** N)
    out = []
    for i in range(N):
        t = s ^ (1 << i)
        sig = (s >> i) & 1
        dn = 1 - 2 * sig
        du = e["U"][t] - e["U"][s]
        n = e["nb"]
        a_loc = np.minimum(1.0, np.exp(-b * (du + dmu0 * dn)))
        k2 = 2.0 if factor2 else 1.0
        a_glob = np.minimum(1.0, np.exp(-b * (kap / N) * dn * (dn + sign * k2 * (n - N * cbar))))
        out.append((t, a_loc * a_glob / N))
    return out


def test_decomposed_acceptance_is_exact(enum16):
    e = enum16
    pi = _pi16(e)
    # pi P = pi with P built from the single-flip kernel
    new = np.zeros_like(pi)
    stay = np.ones_like(pi)
    for t, p in _transitions(e):
        np.add.at(new, t, pi * p)
        stay -= p
    new += pi * stay
    assert np.max(np.abs(new - pi)) <= 1e-13 * pi.max()
    # the printed minus sign, or the missing factor 2 of Eq. mod, break it
    for kw in ({"sign": -1.0}, {"factor2": False}):
        new = np.zeros_like(pi)
        stay = np.ones_like(pi)
        for t, p in _transitions(e, **kw):
            np.add.at(new, t, pi * p)
            stay -= p
        new += pi * stay
        assert np.max(np.abs(new - pi)) > 1e-4 * pi.max()


def test_symmetric_point(oracle_mod):
    O = oracle_mod
    st = _c1_state(O, I.params("SYM"), c_init=0.5, thermal=51)
    T, kappa, cbar, dmu0 = 600.0, 1.0, 0.5, 0.0
    _chain(O, st, 30, dmu0, kappa, cbar, T, seed=505)
    ns, _ = _chain(O, st, 300, dmu0, kappa, cbar, T, seed=505)
    mean, err = X.batch_means(ns)
    assert abs(mean - 0.5 * st.n) < 3 * err, (mean, err)


def test_gforce_and_variance_relations(oracle_mod):
    """Eq. gforce: dmu = phi + 2 kappa <c> with dmu the SGC value at <c>;
    Eq. df2_vcsgc with the ideal-mixing F'' = N kT / (c(1-c)):
    var(c) = c(1-c) / (N (1 + 2 beta kappa c(1-c)))."""
    O = oracle_mod
    N, T, kappa, cbar, dmu0 = 2000, 600.0, 2.0, 0.3, 0.01
    b = X.beta_of(T)
    p = X.normalize(X.vcsgc_logw_ideal(N, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    c = m / N
    phi = dmu0 - 2 * kappa * cbar
    dmu_sgc = math.log((1 - c) / c) / b
    assert abs(phi + 2 * kappa * c - dmu_sgc) < 2e-3
    var_c = c * (1 - c) / (N * (1 + 2 * b * kappa * c * (1 - c)))
    assert abs(v / N ** 2 / var_c - 1) < 0.02
    # and the chain reproduces both
    st = _c1_state(O, I.params("IDEAL"), c_init=cbar)
    _chain(O, st, 30, dmu0, kappa, cbar, T, seed=606)
    ns, _ = _chain(O, st, 600, dmu0, kappa, cbar, T, seed=606)
    mean, err = X.batch_means(ns)
    cm = mean / N
    assert abs(phi + 2 * kappa * cm - math.log((1 - cm) / cm) / b) < 3 * err / N * (
        2 * kappa + 1 / (b * cm * (1 - cm))) + 2e-3
    assert abs(ns.var() / N ** 2 / var_c - 1) < 0.25


def test_chunking_invariance(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    a = _c1_state(O, pot, thermal=61)
    b = _c1_state(O, pot, thermal=61)
    args = (-0.37, 10.0, 0.05, 600.0)
    O.sweep(a, *args, 7, 77)
    O.sweep(b, *args, 3, 77)
    O.sweep(b, *args, 4, 77)
    assert np.array_equal(a.species, b.species)
    assert np.array_equal(a.rho, b.rho)
    assert a.n_b[0] == b.n_b[0]


def test_rho_cache_matches_fresh_density(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    st = _c1_state(O, pot, c_init=0.2, thermal=71)
    s, _, _ = O.sweep(st, -0.45, 5.0, 0.2, 600.0, 20, 88)
    assert s["flips"] > 100
    fresh = O.density(st.nl, st.species, pot)
    assert np.max(np.abs(fresh - st.rho)) < 1e-12


@pytest.mark.parametrize("period", [2, 3])
def test_same_stage_sites_are_independent(oracle_mod, period):
    """Within a stage every pair of trial sites is at least 2 rc apart (no
    site's energy change depends on another's species or density), for the
    eight-colour octant scheme and the 27-colour scheme on half-width cells;
    a stage's trials are the non-empty cells of one colour, C ceil(N / N_cells)
    stages per sweep."""
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(20, 20, 20)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 81)
    sp = I.initial_species(x.size, 0.05, 82)
    st = O.SweepState(x, y, z, box, sp, pot)
    _, tl, sl = O.sweep(st, -0.37, 1000.0, 0.05, 600.0, 1, 99, log_trials=300000,
                        log_stages=10000, colour_period=period)
    nc = O.cell_grid(box, 2 * pot.rc, period)
    ncells = int(np.prod(nc))
    assert np.all(nc % period == 0)
    assert np.all(box / nc >= 2 * pot.rc / (period - 1))
    ncol = period ** 3
    assert sl.shape[0] == ncol * -(-x.size // ncells)
    assert set(np.unique(sl[:, 2]).astype(int)) <= set(range(ncol))
    assert len(np.unique(sl[:, 2])) == ncol
    stages = tl[:, 1].astype(int)
    counts = np.bincount(stages, minlength=sl.shape[0])
    assert counts.max() <= ncells // ncol
    for s in np.unique(stages)[:40]:
        sites = tl[stages == s, 3].astype(int)
        P = np.stack([x[sites], y[sites], z[sites]], 1)
        d = P[:, None, :] - P[None, :, :]
        d -= box * np.round(d / box)
        r = np.sqrt((d * d).sum(-1))
        np.fill_diagonal(r, np.inf)
        assert r.min() >= 2 * pot.rc
