"""Pins of the oracle's tabulated EAM (a general two-species embedded-atom
potential given by tables: the class of short-range potentials named in the
Introduction and Sec. III, the class of the Fe-Cu potentials of Sec. IV.B).

The interpolant is checked against what it must reproduce by construction:
the knot values, exact quadratics (central-difference slopes are exact for
them), continuity of value and slope across knots.  The tabulated
Finnis-Sinclair set must reproduce the analytic potential (its density
function is a quadratic, so densities agree to rounding; energies and
forces to the interpolation error), and for a tabulated potential unlike
the analytic form the forces must be minus the gradient of the energy, the
transmutation energy must equal a local energy recompute, and MD must
conserve the total energy.
"""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I


def _thermal(n=6, seed=7, c=0.2):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.06, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    return x, y, z, box, sp


def test_spline_knots_quadratics_and_continuity(oracle_mod):
    O = oracle_mod
    rng = np.random.default_rng(2)
    h = 0.25  # a power of two: x / h is exact at the knots
    xk = h * np.arange(40)
    # knot values are reproduced exactly
    y = rng.normal(size=40)
    c = O.spline_coeffs(y)
    for k in range(39):
        v, _ = O.spline_eval(c, 40, xk[k], 1.0 / h)
        assert v == y[k]
    # value and slope are continuous across interior knots
    for k in range(1, 39):
        a = c[4 * (k - 1):4 * k]
        end_val = ((a[3] + a[2]) + a[1]) + a[0]
        end_der = (3.0 * a[3] + 2.0 * a[2]) + a[1]
        assert abs(end_val - y[k]) <= 1e-13
        assert abs(end_der - c[4 * k + 1]) <= 1e-13
    # a quadratic is reproduced on the interior intervals, slope included
    q = lambda t: 0.7 - 1.3 * t + 2.9 * t * t  # noqa: E731
    c = O.spline_coeffs(q(xk))
    for t in rng.uniform(xk[1], xk[38], 200):
        v, d = O.spline_eval(c, 40, t, 1.0 / h)
        assert abs(v - q(t)) <= 1e-12
        assert abs(d - (-1.3 + 5.8 * t)) <= 1e-12


def test_tabulated_fs_matches_analytic(oracle_mod):
    """TAB-FS1 tabulates FS-P1: the density function is a quadratic in r, so
    the densities agree to rounding; pair and embedding functions are
    interpolated (errors of order h^3 and below)."""
    O = oracle_mod
    fs, tab = I.params("FS-P1"), I.table("TAB-FS1")
    x, y, z, box, sp = _thermal()
    nl = O.neighbors(x, y, z, box, fs.rc)
    ra, rt = O.density(nl, sp, fs), O.density(nl, sp, tab)
    assert np.max(np.abs(ra - rt) / ra) <= 1e-14
    ea, et = O.energy_atoms(nl, sp, fs, ra), O.energy_atoms(nl, sp, tab, rt)
    assert np.max(np.abs(ea - et)) <= 1e-7
    fa, ft = O.forces(nl, sp, fs, ra), O.forces(nl, sp, tab, rt)
    for a, b in zip(fa, ft):
        assert np.max(np.abs(a - b)) <= 2e-4  # O(h^2) slope error of the cubic pair term
    for i in range(0, x.size, 17):
        assert abs(O.delta_u(nl, i, sp, ra, fs) - O.delta_u(nl, i, sp, rt, tab)) <= 1e-6


def test_tabulated_forces_are_minus_gradient(oracle_mod):
    O = oracle_mod
    tab = I.table("TAB-X")
    x, y, z, box, sp = _thermal(n=5, seed=19)
    nl = O.neighbors(x, y, z, box, tab.rc)
    fx, fy, fz = O.forces(nl, sp, tab)
    h = 1e-5
    rng = np.random.default_rng(3)
    for i in rng.choice(x.size, 6, replace=False):
        for comp, f in ((0, fx), (1, fy), (2, fz)):
            vals = []
            for sgn in (+1, -1):
                pos = [x.copy(), y.copy(), z.copy()]
                pos[comp][i] += sgn * h
                nl2 = O.neighbors(*pos, box, tab.rc)
                vals.append(math.fsum(O.energy_atoms(nl2, sp, tab)))
            g = -(vals[0] - vals[1]) / (2 * h)
            assert abs(g - f[i]) <= 1e-6 * max(1.0, abs(f[i]))


def test_tabulated_delta_u_equals_local_recompute(oracle_mod):
    O = oracle_mod
    tab = I.table("TAB-X")
    x, y, z, box, sp = _thermal(seed=29)
    nl = O.neighbors(x, y, z, box, tab.rc)
    rho = O.density(nl, sp, tab)
    e0 = O.energy_atoms(nl, sp, tab, rho)
    rng = np.random.default_rng(5)
    for i in rng.choice(x.size, 30, replace=False):
        du = O.delta_u(nl, i, sp, rho, tab)
        sp2 = sp.copy()
        sp2[i] ^= 1
        e1 = O.energy_atoms(nl, sp2, tab)
        idx = np.concatenate([[i], nl.row(i)])
        local = math.fsum(e1[idx]) - math.fsum(e0[idx])
        assert abs(du - local) <= 1e-12


@pytest.mark.parametrize("name", ["TAB-FS1", "TAB-X"])
def test_tabulated_nve_energy_conservation(oracle_mod, name):
    O = oracle_mod
    tab = I.table(name)
    x, y, z, box = I.bcc(6, 6, 6)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 5)
    sp = I.initial_species(x.size, 0.05, 6)
    vx, vy, vz = I.mb_velocities(sp, 700.0, 7)

    def etot(x, y, z, vx, vy, vz):
        nl = O.neighbors(x, y, z, box, tab.rc)
        u = math.fsum(O.energy_atoms(nl, sp, tab))
        m = np.where(sp == 0, I.MASS_A, I.MASS_B)
        return u + 0.5 * math.fsum(m * (vx * vx + vy * vy + vz * vz)) / I.ACC_CONV

    e0 = etot(x, y, z, vx, vy, vz)
    out = O.md(x, y, z, vx, vy, vz, sp, box, tab, 1.0, 100)
    e1 = etot(*out[:6])
    assert abs(e1 - e0) / x.size < 2e-5
