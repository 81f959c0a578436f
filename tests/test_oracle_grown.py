"""Pins of the oracle's grown domains (Sec. III.A, Fig. 6): cells of edge
e >= 2 r_dep, eight overlapping corner domains of edge e - r_dep per cell, a
stage's domain drawn at random and one trial in it per cell, the site drawn
with weight 8 / m (m: the cell's domains holding the atom).

* every logged trial site equals the one an independent reconstruction
  draws: numpy's Philox (a different implementation of the same generator),
  the domains from the geometry, the weighted draw by exact integer
  arithmetic;
* sites of one stage are at least r_dep apart, every cell whose drawn domain
  holds atoms makes one trial, and a sweep has ceil(N / N_cells) stages;
* the sampled ensemble is exact: identical species (closed-form P(n)) and
  independent sites (Poisson-binomial), as for the octant scheme.
"""
import numpy as np
import pytest

import exact_refs as X
from paper_1012_5082_amd import inputs as I

M64 = (1 << 64) - 1


def _philox_np(key, ctr):
    """Block at counter ctr from numpy's Philox (which increments first)."""
    c = [int(v) for v in ctr]
    for k in range(4):  # ctr - 1 over the 256-bit little-endian counter
        if c[k] > 0:
            c[k] -= 1
            break
        c[k] = M64
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


def _domains(x, y, z, box, r_dep, grow_edge):
    """(nc, lists): lists[(cell, k)] = (atoms ascending, weights 8 / m)."""
    emin = max(grow_edge, 2.0 * r_dep)
    nc = np.floor(box / emin).astype(int)
    pos = np.stack([x, y, z], 1)
    e = box / nc
    b = np.minimum(np.maximum((pos / e).astype(int), 0), nc - 1)
    u = pos - b * e
    ld = e - r_dep
    lo, hi = u < ld, u >= e - ld
    m = (lo.astype(int) + hi).prod(1)
    cell = b[:, 0] + nc[0] * (b[:, 1] + nc[1] * b[:, 2])
    lists = {}
    for k in range(8):
        kb = [(k >> d) & 1 for d in range(3)]
        inside = np.all([hi[:, d] if kb[d] else lo[:, d] for d in range(3)], axis=0)
        for c in range(int(nc.prod())):
            idx = np.nonzero(inside & (cell == c))[0]
            lists[(c, k)] = (idx, 8 // m[idx])
    return nc, lists


def _thermal(n=14, seed=5):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, 0.1, seed + 1)
    return x, y, z, box, sp


@pytest.mark.parametrize("n,grow_edge", [(14, 1e-9), (20, 28.0)])
def test_grown_draws_match_independent_reconstruction(oracle_mod, n, grow_edge):
    """cells of 20.1 A (domains 12.9 A) and of 28.7 A (domains 21.5 A)"""
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box, sp = _thermal(n=n)
    r_dep, seed = 2 * pot.rc, 4242
    st = O.SweepState(x, y, z, box, sp, pot)
    _, tl, sl = O.sweep(st, -0.3, 1000.0, 0.1, 600.0, 1, seed, log_trials=10 ** 6,
                        log_stages=10 ** 5, grow_edge=grow_edge)
    nc, lists = _domains(x, y, z, box, r_dep, grow_edge)
    ncells = int(nc.prod())
    assert ncells >= 8 and np.any([len(v[0]) != len(lists[(0, 0)][0]) for v in lists.values()])
    assert np.any([np.any(v[1] < 8) for v in lists.values()])  # domains overlap
    checked = 0
    for row in tl:
        w, s, c, site = int(row[0]), int(row[1]), int(row[2]), int(row[3])
        k = _philox_np((seed, 0), (w, s, 0, 0))[0] >> 61
        assert sl[s, 2] == k
        idx, wt = lists[(c, k)]
        cum = np.cumsum(wt)
        r = (_philox_np((seed, 0), (w, s, c, 1))[0] * int(cum[-1])) >> 64
        assert site == idx[np.searchsorted(cum, r, side="right")]
        checked += 1
    assert checked == tl.shape[0] > 1000


def test_grown_stages_and_independence(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box, sp = _thermal(n=16, seed=9)
    r_dep = 2 * pot.rc
    st = O.SweepState(x, y, z, box, sp, pot)
    _, tl, sl = O.sweep(st, -0.3, 1000.0, 0.1, 600.0, 1, 77, log_trials=10 ** 6,
                        log_stages=10 ** 5, grow_edge=16.0)
    nc, lists = _domains(x, y, z, box, r_dep, 16.0)
    ncells = int(nc.prod())
    assert sl.shape[0] == -(-x.size // ncells)
    stages = tl[:, 1].astype(int)
    for s in range(sl.shape[0]):
        k = int(sl[s, 2])
        sites = tl[stages == s, 3].astype(int)
        assert sites.size == sum(len(lists[(c, k)][0]) > 0 for c in range(ncells))
        if s < 40:
            P = np.stack([x[sites], y[sites], z[sites]], 1)
            d = P[:, None, :] - P[None, :, :]
            d -= box * np.round(d / box)
            r = np.sqrt((d * d).sum(-1))
            np.fill_diagonal(r, np.inf)
            assert r.min() >= r_dep


def _c1(O, pot, c_init, thermal=None):
    x, y, z, box = I.bcc(10, 10, 10)
    if thermal is not None:
        x, y, z = I.thermalize(x, y, z, box, 0.05, thermal)
    return O.SweepState(x, y, z, box, I.initial_species(x.size, c_init, 1), pot)


def _chain(O, st, n, args, seed):
    ns = []
    for _ in range(n):
        O.sweep(st, *args, 1, seed, grow_edge=1e-9)
        ns.append(int(st.n_b[0]))
    return np.array(ns, float)


def test_grown_ideal_vcsgc_exact_distribution(oracle_mod):
    O = oracle_mod
    st = _c1(O, I.params("IDEAL"), 0.2)
    args = (0.0, 2.0, 0.2, 600.0)
    _chain(O, st, 30, args, 505)
    ns = _chain(O, st, 600, args, 505)
    p = X.normalize(X.vcsgc_logw_ideal(st.n, 600.0, 0.0, 2.0, 0.2))
    m, v = X.moments(p)
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(ns.var() / v - 1.0) < 0.25


def test_grown_indep_poisson_binomial(oracle_mod):
    O = oracle_mod
    pot = I.params("INDEP")
    st = _c1(O, pot, 0.1, thermal=41)
    T, kappa, cbar, dmu0 = 600.0, 1.0, 0.1, -0.70
    de = (-pot.a_b + pot.a_a) * np.sqrt(st.rho)
    p = X.normalize(X.vcsgc_logw_indep(de, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    _chain(O, st, 30, (dmu0, kappa, cbar, T), 606)
    ns = _chain(O, st, 600, (dmu0, kappa, cbar, T), 606)
    mean, err = X.batch_means(ns)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(ns.var() / v - 1.0) < 0.25
