"""Pins of the oracle's velocity-Verlet MD: energy conservation (NVE),
time reversibility, momentum conservation, and the transmutation rescaling
of velocities that keeps the kinetic energy unchanged."""
import math

import numpy as np

from paper_1012_5082_amd import inputs as I


def _system(n=8, T=700.0, seed=5, c=0.05):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return x, y, z, vx, vy, vz, sp, box


def _etot(O, x, y, z, vx, vy, vz, sp, box, pot):
    nl = O.neighbors(x, y, z, box, pot.rc)
    u = math.fsum(O.energy_atoms(nl, sp, pot))
    m = np.where(sp == 0, I.MASS_A, I.MASS_B)
    k = 0.5 * math.fsum(m * (vx * vx + vy * vy + vz * vz)) / I.ACC_CONV
    return u + k, u, k


def test_nve_energy_conservation(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system()
    e0, _, k0 = _etot(O, x, y, z, vx, vy, vz, sp, box, pot)
    out = O.md(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 200)
    e1, _, k1 = _etot(O, *out[:6], sp, box, pot)
    n = x.size
    # kinetic energy changes by a large fraction of itself (equipartition),
    # the total stays within 2e-5 eV/atom after 200 fs
    assert abs(k1 - k0) / n > 1e-3
    assert abs(e1 - e0) / n < 2e-5


def test_time_reversal(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(n=6, seed=9)
    a = O.md(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 50)
    b = O.md(a[0], a[1], a[2], -a[3], -a[4], -a[5], sp, box, pot, 1.0, 50)
    for u, u0, L in ((b[0], x, box[0]), (b[1], y, box[1]), (b[2], z, box[2])):
        d = u - u0
        d -= L * np.round(d / L)
        assert np.abs(d).max() < 1e-9
    assert np.abs(b[3] + vx).max() < 1e-9


def test_momentum_conserved(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(n=6, seed=13, c=0.3)
    out = O.md(x, y, z, vx, vy, vz, sp, box, pot, 1.0, 30)
    m = np.where(sp == 0, I.MASS_A, I.MASS_B)
    for v in out[3:6]:
        assert abs(math.fsum(m * v)) < 1e-9


def test_transmutation_keeps_kinetic_energy(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, vx, vy, vz, sp, box = _system(n=10, seed=17)
    st = O.SweepState(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz)
    m0 = np.where(st.species == 0, I.MASS_A, I.MASS_B)
    k0 = 0.5 * math.fsum(m0 * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2))
    s, _, _ = O.sweep(st, -0.45, 1.0, 0.1, 700.0, 5, 21)
    assert s["flips"] > 20
    m1 = np.where(st.species == 0, I.MASS_A, I.MASS_B)
    k1 = 0.5 * math.fsum(m1 * (st.vx ** 2 + st.vy ** 2 + st.vz ** 2))
    assert abs(k1 - k0) <= 1e-12 * k0
    # a site flipped back and forth ends with its velocity up to rounding
    same = st.species == sp
    assert np.all(np.abs(st.vx[same] - vx[same]) <= 1e-15 * np.abs(vx[same]))
    ratio = st.vx[~same] / vx[~same]
    want = np.where(sp[~same] == 0, math.sqrt(I.MASS_A / I.MASS_B), math.sqrt(I.MASS_B / I.MASS_A))
    assert np.allclose(ratio, want, rtol=1e-15, atol=0)
