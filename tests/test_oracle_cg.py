"""Pins of the oracle's conjugate-gradient relaxation (Sec. IV.B relaxes the
nanocrystal's grain boundaries by conjugate-gradient minimization; the
oracle's variant is PR+ nonlinear CG with a backtracking Armijo line
search, Nocedal and Wright, Numerical Optimization, Secs. 3.1, 3.5, 5.2).

Pinned against what the method must satisfy whatever its internals:
  * a force-free structure is left as it is;
  * the minimum reached is the one an independent minimizer (scipy's
    L-BFGS-B on the same energy and forces) reaches from the same start;
  * every accepted step satisfies the sufficient-decrease condition, so the
    energy never rises;
  * the logged direction coefficient is the clipped Polak-Ribiere value of
    the iterates themselves, recomputed from the returned states with
    numpy dot products (a different summation order);
  * the stop reasons and limits.
"""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I

FORCE, ENERGY, ITER, EVAL, LINESEARCH = 1, 2, 3, 4, 5


def _defect_system(n=6, seed=11):
    """A bcc block with two vacancies, thermal displacements of 0.08 A and
    20% B sites."""
    x, y, z, box = I.bcc(n, n, n)
    keep = np.ones(x.size, bool)
    keep[[0, 5]] = False
    x, y, z = x[keep], y[keep], z[keep]
    x, y, z = I.thermalize(x, y, z, box, 0.08, seed)
    sp = I.initial_species(x.size, 0.2, seed + 1)
    return x, y, z, box, sp


def _energy_forces(O, pot, box, sp, x, y, z):
    nl = O.neighbors(x, y, z, box, pot.rc)
    fx, fy, fz = O.forces(nl, sp, pot)
    return math.fsum(O.energy_atoms(nl, sp, pot)), fx, fy, fz


def _min_image_diff(a, b, L):
    d = a - b
    return d - L * np.round(d / L)


def test_cg_leaves_a_force_free_lattice(oracle_mod):
    O = oracle_mod
    x, y, z, box = I.bcc(6, 6, 6)
    sp = np.zeros(x.size, np.uint8)
    pot = I.params("FS-P1")
    (xo, yo, zo, *_), info, _ = O.cg(x, y, z, sp, box, pot, ftol=1e-9)
    assert info["reason"] == FORCE and info["iterations"] == 0 and info["evaluations"] == 0
    assert np.array_equal(xo, x) and np.array_equal(yo, y) and np.array_equal(zo, z)


@pytest.mark.parametrize("name", ["FS-P1", "TAB-X"])
def test_cg_reaches_the_lbfgs_minimum(oracle_mod, name):
    from scipy.optimize import minimize
    O = oracle_mod
    pot = I.params(name) if name.startswith("FS") else I.table(name)
    x, y, z, box, sp = _defect_system()
    n = x.size
    (xo, yo, zo, fx, fy, fz, _), info, _ = O.cg(x, y, z, sp, box, pot, ftol=1e-7)
    # converged, or stopped where rounding defeats the decrease test
    assert info["reason"] in (FORCE, LINESEARCH)
    assert info["fnorm"] <= 1e-5

    def f(v):
        X, Y, Z = v[:n] % box[0], v[n:2 * n] % box[1], v[2 * n:] % box[2]
        e, gx, gy, gz = _energy_forces(O, pot, box, sp, X, Y, Z)
        return e, -np.concatenate([gx, gy, gz])

    r = minimize(f, np.concatenate([x, y, z]), jac=True, method="L-BFGS-B",
                 options=dict(gtol=1e-10, ftol=1e-15, maxiter=10000))
    e0 = _energy_forces(O, pot, box, sp, x, y, z)[0]
    assert e0 - info["energy"] > 10.0  # a real relaxation
    assert abs(r.fun - info["energy"]) <= 1e-9 * abs(r.fun)
    v = r.x
    for a, b, L in ((v[:n], xo, box[0]), (v[n:2 * n], yo, box[1]), (v[2 * n:], zo, box[2])):
        assert np.max(np.abs(_min_image_diff(a, b, L))) <= 1e-5
    # the returned forces are those at the returned positions
    e1, gx, gy, gz = _energy_forces(O, pot, box, sp, xo, yo, zo)
    assert abs(e1 - info["energy"]) <= 1e-10 * abs(e1)
    for a, b in ((fx, gx), (fy, gy), (fz, gz)):
        assert np.array_equal(a, b)


def test_cg_steps_satisfy_sufficient_decrease(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box, sp = _defect_system(seed=21)
    _, info, log = O.cg(x, y, z, sp, box, pot, ftol=1e-6, log_cap=10000)
    assert len(log) == info["iterations"] > 10
    E, Et, a, sl = log[:, 0], log[:, 1], log[:, 2], log[:, 3]
    assert np.all(sl > 0.0) and np.all(a > 0.0)
    assert np.all(Et <= E - 1e-4 * a * sl)
    assert np.all(Et < E)
    assert np.array_equal(E[1:], Et[:-1])  # each iteration starts where the last ended
    assert Et[-1] == info["energy"]


def test_cg_direction_coefficient_is_clipped_polak_ribiere(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box, sp = _defect_system(seed=31)
    _, info, log = O.cg(x, y, z, sp, box, pot, ftol=1e-6, log_cap=10000)
    assert info["iterations"] > 8
    forces = []
    for k in range(8):  # the state after k iterations, from a run stopped there
        (_, _, _, fx, fy, fz, _), ik, _ = O.cg(x, y, z, sp, box, pot, max_iter=k, ftol=1e-6)
        assert ik["iterations"] == k and ik["reason"] == ITER
        forces.append(np.concatenate([fx, fy, fz]))
    positive = 0
    for k in range(7):
        f0, f1 = forces[k], forces[k + 1]
        b = max(0.0, (np.dot(f1, f1) - np.dot(f1, f0)) / np.dot(f0, f0))
        assert abs(log[k, 4] - b) <= 1e-9 * max(1.0, b)
        positive += b > 0.0
    assert positive >= 2  # the coefficient is not always clipped here
    # the directions d_0 = F_0, d_{k+1} = F_{k+1} + b_k d_k (F after a
    # restart): the logged slope F_k . d_k of each line search
    d = forces[0]
    for k in range(8):
        if log[k, 5]:
            d = forces[k]
        sl = np.dot(forces[k], d)
        assert abs(log[k, 3] - sl) <= 1e-9 * abs(sl)
        if k < 7:
            d = forces[k + 1] + log[k, 4] * d


def test_cg_limits_and_reasons(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box, sp = _defect_system(n=5, seed=41)
    (xo, *_), info, _ = O.cg(x, y, z, sp, box, pot, max_iter=0)
    assert info["reason"] == ITER and np.array_equal(xo, x)
    _, info, _ = O.cg(x, y, z, sp, box, pot, max_eval=5, ftol=0.0)
    assert info["reason"] == EVAL and info["evaluations"] >= 5
    # no energy stop: the run ends when rounding defeats the decrease test
    (xo, yo, zo, *_), info, log = O.cg(x, y, z, sp, box, pot, etol=-1.0, ftol=0.0, log_cap=100000)
    assert info["reason"] == LINESEARCH
    (xp, yp, zp, *_), ip, _ = O.cg(x, y, z, sp, box, pot, etol=-1.0, ftol=0.0,
                                   max_iter=info["iterations"])
    assert ip["reason"] == ITER
    assert np.array_equal(xo, xp) and np.array_equal(yo, yp) and np.array_equal(zo, zp)
    assert info["fnorm"] <= 1e-5
