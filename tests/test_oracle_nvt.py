"""Pins of the oracle's Nose-Hoover NVT velocity Verlet (the thermostatted
MD of the paper's Fe-Cu application, Sec. IV.B) and of its fixed-shape sum:

* with an infinite coupling time the thermostat is inert and the steps are
  the NVE velocity-Verlet steps bit for bit;
* the extended energy K + U + Q xi^2/2 + g kB T eta is conserved;
* the integrator is time reversible (x, v, xi, eta return);
* the kinetic energy samples the canonical distribution: mean g kB T / 2 and
  variance g (kB T)^2 / 2 for g = 3N - 3 degrees of freedom;
* the fixed-shape sum is exact on integers and within rounding of an exact
  sum otherwise.
"""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I

KB = 8.617333262e-5


def _system(n=6, T=300.0, seed=5, c=0.1):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return x, y, z, vx, vy, vz, sp, box


def _kinetic(vx, vy, vz, sp):
    m = np.where(sp == 0, I.MASS_A, I.MASS_B)
    return 0.5 * math.fsum(m * (vx * vx + vy * vy + vz * vz)) / I.ACC_CONV


def _h_ext(O, out, th, sp, box, pot, T, tau):
    x, y, z, vx, vy, vz = out[:6]
    nl = O.neighbors(x, y, z, box, pot.rc)
    u = math.fsum(O.energy_atoms(nl, sp, pot))
    g = 3.0 * x.size - 3.0
    Q = g * KB * T * tau * tau
    xi, eta = th
    return _kinetic(vx, vy, vz, sp) + u + 0.5 * Q * xi * xi + g * KB * T * eta


def test_tree_sum(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(3)
    for n in (1, 255, 256, 257, 70000):
        ints = rng.integers(-1000, 1000, n).astype(np.float64)
        assert O.tree_sum(ints) == float(ints.sum())
        v = rng.uniform(0.0, 1.0, n)
        assert abs(O.tree_sum(v) - math.fsum(v)) <= 4 * n * 2.0 ** -53 * math.fsum(v)


def test_infinite_coupling_time_is_nve(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system()
    a = O.md(x, y, z, vx, vy, vz, sp, box, pot, 2.5, 30)
    b, th = O.md_nvt(x, y, z, vx, vy, vz, sp, box, pot, 2.5, 30, 700.0, math.inf)
    assert th == (0.0, 0.0)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)


def test_extended_energy_conserved(oracle_mod):
    """Over 1 ps the extended energy drifts by an amount that falls as dt^2
    (second-order splitting): halving dt divides the drift by about four,
    while the thermostat changes the kinetic energy by far more."""
    O = oracle_mod
    pot = I.params("FS-P1")
    T, tau = 700.0, 50.0
    x, y, z, vx, vy, vz, sp, box = _system(T=300.0)
    n = x.size
    h0 = _h_ext(O, (x, y, z, vx, vy, vz), (0.0, 0.0), sp, box, pot, T, tau)
    drift = {}
    for dt in (2.5, 1.25):
        out, th = O.md_nvt(x, y, z, vx, vy, vz, sp, box, pot, dt, int(1000 / dt), T, tau)
        drift[dt] = (_h_ext(O, out, th, sp, box, pot, T, tau) - h0) / n
        assert abs(_kinetic(*out[3:6], sp) - _kinetic(vx, vy, vz, sp)) / n > 2e-2
        assert abs(th[0]) > 0.0
    assert abs(drift[2.5]) < 3e-4, drift
    assert 3.0 < drift[2.5] / drift[1.25] < 5.0, drift


def test_time_reversal(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(T=500.0, seed=9)
    a, th = O.md_nvt(x, y, z, vx, vy, vz, sp, box, pot, 2.5, 60, 900.0, 40.0, xi=0.002)
    b, th2 = O.md_nvt(a[0], a[1], a[2], -a[3], -a[4], -a[5], sp, box, pot, 2.5, 60, 900.0, 40.0,
                      xi=-th[0], eta=th[1])
    for u, u0, L in ((b[0], x, box[0]), (b[1], y, box[1]), (b[2], z, box[2])):
        d = u - u0
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-9
    assert np.abs(b[3] + vx).max() < 1e-9
    assert abs(th2[0] + 0.002) < 1e-12 and abs(th2[1]) < 1e-9


@pytest.mark.slow
def test_canonical_kinetic_energy(oracle_mod):
    """128 atoms at 600 K: after equilibration the kinetic energy has the
    Gamma(g/2, kB T) mean and variance (blocked errors)."""
    O = oracle_mod
    pot = I.params("FS-P1")
    T, tau, dt = 600.0, 25.0, 2.5
    x, y, z, vx, vy, vz, sp, box = _system(n=4, T=T, seed=21, c=0.2)
    g = 3.0 * x.size - 3.0
    out, th = O.md_nvt(x, y, z, vx, vy, vz, sp, box, pot, dt, 2000, T, tau)
    ks = []
    for _ in range(600):
        out, th = O.md_nvt(*out[:6], sp, box, pot, dt, 10, T, tau, xi=th[0], eta=th[1])
        ks.append(_kinetic(*out[3:6], sp))
    ks = np.array(ks)
    kT = KB * T
    mean_ref, var_ref = 0.5 * g * kT, 0.5 * g * kT * kT
    blocks = ks.reshape(20, -1)
    err = blocks.mean(axis=1).std(ddof=1) / math.sqrt(20)
    assert abs(ks.mean() - mean_ref) < 4 * err + 0.01 * mean_ref, (ks.mean(), mean_ref, err)
    assert 0.7 < ks.var() / var_ref < 1.3, ks.var() / var_ref
