"""Pins of the oracle's isotropic NPT dynamics (the Nose-Hoover thermostat and
barostat of the paper's Fe-Cu runs, Sec. IV.B; Martyna-Tobias-Klein form):

  * the virial gives the configurational pressure -dU/dV (central
    differences of the energy under a uniform scaling of box and positions);
  * the extended energy H = K + U + pe^2/2W + P_ext V + Q xi^2/2 + (g+1) kT eta
    is conserved, its fluctuation falling as dt^2, at P_ext = 0 and P_ext > 0;
  * the dynamics is time reversible (x, v, xi, pe -> x, -v, -xi, -pe);
  * with an infinitely heavy barostat the box stays fixed and the run is the
    Nose-Hoover NVT run at the temperature with the same thermostat force;
  * a higher external pressure gives a smaller volume.
"""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I

KB, ACC = 8.617333262e-5, 9.648533212e-3


def _system(n=5, c=0.1, seed=5, T=700.0):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return x, y, z, vx, vy, vz, sp, box


def _extended_energy(O, pot, sp, st, box, state, T, tau_t, p_ext, tau_p):
    x, y, z, vx, vy, vz = st[:6]
    nl = O.neighbors(x, y, z, box, pot.rc)
    U = math.fsum(O.energy_atoms(nl, sp, pot))
    m = np.where(sp == 0, I.MASS_A, I.MASS_B)
    K = 0.5 * math.fsum(m * (vx * vx + vy * vy + vz * vz)) / ACC
    g1kT = (3.0 * x.size - 2.0) * KB * T
    Q, W = g1kT * tau_t ** 2, g1kT * tau_p ** 2
    xi, eta, pe = state
    return K + U + pe * pe / (2.0 * W) + p_ext * float(np.prod(box)) + 0.5 * Q * xi * xi + g1kT * eta


def test_virial_is_minus_volume_derivative_of_energy(oracle_mod):
    O = oracle_mod
    for pot in (I.params("FS-P1"), I.table("TAB-X")):
        x, y, z, vx, vy, vz, sp, box = _system(seed=9)
        zero = np.zeros_like(x)
        # no steps: the virial of the starting configuration
        _, _, _, vir = O.md_npt(x, y, z, zero, zero, zero, sp, box, pot, 1.0, 0, 700.0, 100.0,
                                0.0, 1000.0)
        V = float(np.prod(box))

        def U(lam):  # box and positions scaled by lam per edge
            b = box * lam
            nl = O.neighbors(x * lam, y * lam, z * lam, b, pot.rc)
            return math.fsum(O.energy_atoms(nl, sp, pot))

        d = 1e-5
        dUdV = (U(1.0 + d) - U(1.0 - d)) / (V * ((1.0 + d) ** 3 - (1.0 - d) ** 3))
        assert abs(vir / (3.0 * V) + dUdV) <= 1e-7 * max(1.0, abs(dUdV)) + 1e-9


@pytest.mark.parametrize("p_ext", [0.0, 0.01])
def test_npt_extended_energy_conserved(oracle_mod, p_ext):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(n=4)
    T, tt, tp = 700.0, 100.0, 150.0
    spread = []
    for dt in (2.0, 1.0):
        st, b, state = (x, y, z, vx, vy, vz), box.copy(), (0.0, 0.0, 0.0)
        h0 = _extended_energy(O, pot, sp, st, b, state, T, tt, p_ext, tp)
        dev = []
        steps = int(round(400 / dt))
        for _ in range(8):
            st, b, state, _ = O.md_npt(*st[:6], sp, b, pot, dt, steps // 8, T, tt, p_ext, tp,
                                       *state)
            dev.append(_extended_energy(O, pot, sp, st, b, state, T, tt, p_ext, tp) - h0)
        spread.append(np.max(np.abs(dev)))
        assert abs(float(np.prod(b)) / float(np.prod(box)) - 1.0) > 1e-3  # the box moved
    assert spread[0] / x.size < 5e-4
    assert 3.0 < spread[0] / spread[1] < 5.0  # second order in dt


def test_npt_time_reversible(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(seed=15)
    args = (700.0, 80.0, 0.005, 300.0)
    st, b, (xi, eta, pe), _ = O.md_npt(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 60, *args,
                                       0.01, 0.0, 3.0)
    x1, y1, z1, vx1, vy1, vz1 = st[:6]
    st2, b2, (xi2, _, pe2), _ = O.md_npt(x1, y1, z1, -vx1, -vy1, -vz1, sp, b, pot, 1.0, 60, *args,
                                         -xi, eta, -pe)
    for a, want, L in ((st2[0], x, box[0]), (st2[1], y, box[1]), (st2[2], z, box[2])):
        d = a - want
        assert np.max(np.abs(d - L * np.round(d / L))) <= 1e-8
    assert np.max(np.abs(st2[3] + vx)) <= 1e-10
    assert np.max(np.abs(b2 - box)) <= 1e-9
    assert abs(xi2 + 0.01) <= 1e-12 and abs(pe2 + 3.0) <= 1e-8


def test_npt_infinite_barostat_mass_is_nvt(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(seed=21)
    n, T, tt = x.size, 700.0, 100.0
    st, b, state, _ = O.md_npt(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 20, T, tt, 0.0, 1e30)
    assert np.array_equal(b, box)
    g = 3.0 * n - 3.0
    T2 = (g + 1.0) * T / g  # same g kB T and Q as the NPT thermostat
    tau2 = tt * math.sqrt((g + 1.0) * T / (g * T2))
    nv, (xi2, _) = O.md_nvt(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 20, T2, tau2)
    for a, w in zip(st[:6], nv[:6]):
        assert np.max(np.abs(a - w)) <= 1e-9
    assert abs(state[0] - xi2) <= 1e-12


def test_npt_pressure_orders_the_volume(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(seed=27)
    vols = []
    for p_ext in (-0.01, 0.0, 0.01):  # +-1.6 GPa
        st, b, state, v = (x, y, z, vx, vy, vz), box.copy(), (0.0, 0.0, 0.0), []
        for k in range(24):  # mean volume over the last 2 ps of 3 ps
            st, b, state, _ = O.md_npt(*st[:6], sp, b, pot, 2.5, 50, 700.0, 100.0, p_ext, 200.0,
                                       *state)
            if k >= 8:
                v.append(float(np.prod(b)))
        vols.append(np.mean(v))
    assert vols[0] > vols[1] > vols[2]
