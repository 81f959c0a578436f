"""Pins of the oracle's EAM energy, density, forces and transmutation energy.

Each check compares against something the oracle does not compute itself:
perfect-lattice shell sums in closed form, the conditions the FS-P1 constants
were solved for (cohesive energy, zero pressure, bulk modulus), Newton's third
law, central differences of the energy, a local energy recompute, and
parameter sets where the transmutation energy has a closed form.
"""
import math

import numpy as np
import pytest

from exact_refs import lattice_shells
from paper_1012_5082_amd import inputs as I

EV_A3_TO_GPA = 160.21766208


def _shell_energy(p, a, species_all=0):
    """Per-atom energy of a pure bcc crystal from its two shells (closed form)."""
    t = p.t_a if species_all == 0 else p.t_b
    A = p.a_a if species_all == 0 else p.a_b
    eps = p.eps_aa if species_all == 0 else p.eps_bb
    rho = sum(n * t * (p.rc - r) ** 2 for n, r in lattice_shells(a))
    pair = sum(n * eps * (p.rc - r) ** 2 * (p.c0 + p.c1 * r) for n, r in lattice_shells(a))
    return -A * math.sqrt(rho) + 0.5 * pair, rho


@pytest.fixture(scope="module")
def fs():
    return I.params("FS-P1")


def test_perfect_lattice_closed_forms(oracle_mod, fs):
    O = oracle_mod
    x, y, z, box = I.bcc(6, 6, 6)
    nl = O.neighbors(x, y, z, box, fs.rc)
    assert np.all(np.diff(nl.start) == 14)
    sp = np.zeros(x.size, np.uint8)
    rho = O.density(nl, sp, fs)
    e = O.energy_atoms(nl, sp, fs, rho)
    e_ref, rho_ref = _shell_energy(fs, I.A_LAT)
    assert np.allclose(rho, rho_ref, rtol=0, atol=1e-12)
    assert np.allclose(e, e_ref, rtol=0, atol=1e-12)
    # the conditions FS-P1 was solved for
    assert abs(e_ref - (-4.28)) < 1e-9
    assert abs(rho_ref - 13.134408449586) < 1e-9
    fx, fy, fz = O.forces(nl, sp, fs, rho)
    assert max(np.abs(fx).max(), np.abs(fy).max(), np.abs(fz).max()) < 1e-12


def test_equilibrium_and_bulk_modulus(oracle_mod, fs):
    """dE/da = 0 and B = 168 GPa at a0, from central differences of the oracle energy."""
    O = oracle_mod

    def e_at(a):
        x, y, z, box = I.bcc(5, 5, 5, a=a)
        nl = O.neighbors(x, y, z, box, fs.rc)
        sp = np.zeros(x.size, np.uint8)
        return O.energy_total(O.energy_atoms(nl, sp, fs)) / x.size

    a0, h = I.A_LAT, 1e-4
    em, e0, ep = e_at(a0 - h), e_at(a0), e_at(a0 + h)
    dE = (ep - em) / (2 * h)
    d2E = (ep - 2 * e0 + em) / (h * h)
    assert abs(dE) < 1e-6
    # Omega = a^3 / 2 per atom: B = Omega d2E/dOmega2 = d2E/da2 / (4.5 a) at equilibrium
    B = d2E / (4.5 * a0) * EV_A3_TO_GPA
    assert abs(B - 168.0) < 0.05


def test_substitution_energy_closed_form(oracle_mod, fs):
    """A -> B at one site of perfect pure-A bcc, against the shell sums."""
    O = oracle_mod
    x, y, z, box = I.bcc(6, 6, 6)
    nl = O.neighbors(x, y, z, box, fs.rc)
    sp = np.zeros(x.size, np.uint8)
    rho = O.density(nl, sp, fs)
    du = O.delta_u(nl, 37, sp, rho, fs)
    rb = rho[0]
    own = -fs.a_b * math.sqrt(rb) + fs.a_a * math.sqrt(rb)
    pair = 0.0
    emb = 0.0
    for n, r in lattice_shells(I.A_LAT):
        d2 = (fs.rc - r) ** 2
        pair += n * (fs.eps_ab - fs.eps_aa) * d2 * (fs.c0 + fs.c1 * r)
        emb += n * (-fs.a_a * math.sqrt(rb + (fs.t_b - fs.t_a) * d2) + fs.a_a * math.sqrt(rb))
    assert abs(du - (own + pair + emb)) < 1e-12
    assert 0.45 < du < 0.6   # about +0.52 eV for an isolated B in A


def _thermal(seed=7, c=0.3, n=6):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    return x, y, z, box, sp


def test_delta_u_equals_local_recompute(oracle_mod, fs):
    O = oracle_mod
    x, y, z, box, sp = _thermal()
    nl = O.neighbors(x, y, z, box, fs.rc)
    rho = O.density(nl, sp, fs)
    e0 = O.energy_atoms(nl, sp, fs, rho)
    rng = np.random.default_rng(5)
    for i in rng.choice(x.size, 40, replace=False):
        du = O.delta_u(nl, i, sp, rho, fs)
        sp2 = sp.copy()
        sp2[i] ^= 1
        e1 = O.energy_atoms(nl, sp2, fs)
        near = np.zeros(x.size, bool)
        near[i] = True
        near[nl.row(i)] = True
        # energies outside {i} + neighbours of i are bitwise unchanged
        assert np.array_equal(e1[~near], e0[~near])
        idx = np.nonzero(near)[0]
        local = math.fsum(e1[idx]) - math.fsum(e0[idx])
        assert abs(du - local) <= 1e-13


def test_ideal_and_indep_closed_forms(oracle_mod):
    O = oracle_mod
    x, y, z, box, sp = _thermal(seed=11)
    ideal, indep = I.params("IDEAL"), I.params("INDEP")
    nl = O.neighbors(x, y, z, box, ideal.rc)
    rho_i = O.density(nl, sp, ideal)
    rho_d = O.density(nl, sp, indep)
    for i in range(0, x.size, 13):
        assert O.delta_u(nl, i, sp, rho_i, ideal) == 0.0
        s = int(sp[i])
        A_new = indep.a_b if s == 0 else indep.a_a
        A_old = indep.a_a if s == 0 else indep.a_b
        want = -A_new * math.sqrt(rho_d[i]) + A_old * math.sqrt(rho_d[i])
        assert abs(O.delta_u(nl, i, sp, rho_d, indep) - want) <= 1e-14


def test_literal_has_no_neighbour_embedding_term(oracle_mod):
    """With f_A = f_B a transmutation leaves every rho_j unchanged (checked
    bitwise), and dU still equals the local energy recompute."""
    O = oracle_mod
    lit = I.params("LITERAL")
    x, y, z, box, sp = _thermal(seed=13)
    nl = O.neighbors(x, y, z, box, lit.rc)
    rho = O.density(nl, sp, lit)
    for i in range(0, x.size, 29):
        du = O.delta_u(nl, i, sp, rho, lit)
        sp2 = sp.copy()
        sp2[i] ^= 1
        assert np.array_equal(O.density(nl, sp2, lit), rho)
        e0 = O.energy_atoms(nl, sp, lit, rho)
        e1 = O.energy_atoms(nl, sp2, lit, rho)
        idx = np.concatenate([[i], nl.row(i)])
        assert abs(du - (math.fsum(e1[idx]) - math.fsum(e0[idx]))) <= 1e-13


def test_newton_third_law(oracle_mod, fs):
    O = oracle_mod
    x, y, z, box, sp = _thermal(seed=17)
    nl = O.neighbors(x, y, z, box, fs.rc)
    fx, fy, fz = O.forces(nl, sp, fs)
    scale = np.abs(fx).sum()
    for f in (fx, fy, fz):
        assert abs(math.fsum(f)) <= 1e-13 * scale


def test_forces_are_minus_gradient(oracle_mod, fs):
    O = oracle_mod
    x, y, z, box, sp = _thermal(seed=19, n=5)
    nl = O.neighbors(x, y, z, box, fs.rc)
    fx, fy, fz = O.forces(nl, sp, fs)
    h = 1e-5
    rng = np.random.default_rng(3)
    for i in rng.choice(x.size, 6, replace=False):
        for comp, f in ((0, fx), (1, fy), (2, fz)):
            vals = []
            for sgn in (+1, -1):
                pos = [x.copy(), y.copy(), z.copy()]
                pos[comp][i] += sgn * h
                nl2 = O.neighbors(*pos, box, fs.rc)
                vals.append(math.fsum(O.energy_atoms(nl2, sp, fs)))
            g = -(vals[0] - vals[1]) / (2 * h)
            assert abs(g - f[i]) <= 1e-6 * max(1.0, abs(f[i]))


def test_neighbor_modes_agree(oracle_mod, fs):
    """Binned search, brute-force minimum image and brute-force image sums
    give identical lists on boxes where all three apply."""
    O = oracle_mod
    x, y, z, box, sp = _thermal(seed=23, n=6)
    a = O.neighbors(x, y, z, box, fs.rc, mode=3)
    b = O.neighbors(x, y, z, box, fs.rc, mode=1)
    c = O.neighbors(x, y, z, box, fs.rc, mode=2)
    for u, v in ((a, b), (a, c)):
        assert np.array_equal(u.start, v.start)
        assert np.array_equal(u.j, v.j)
        assert np.array_equal(u.r, v.r)
        assert np.array_equal(u.dx, v.dx)
    # every pair is symmetric
    pairs = set()
    for i in range(a.n):
        for j in a.row(i):
            pairs.add((i, int(j)))
    assert all((j, i) in pairs for i, j in pairs)


def test_small_box_image_sums(oracle_mod, fs):
    """16-site bcc (box 5.74 A < 2 rc): the second shell of each site holds
    three atoms seen through two images each; rho and E still equal the
    perfect-lattice closed forms."""
    O = oracle_mod
    x, y, z, box = I.bcc(2, 2, 2)
    nl = O.neighbors(x, y, z, box, fs.rc)
    assert np.all(np.diff(nl.start) == 14)
    assert len(set(nl.row(0).tolist())) == 8 + 3
    sp = np.zeros(16, np.uint8)
    e_ref, rho_ref = _shell_energy(fs, I.A_LAT)
    rho = O.density(nl, sp, fs)
    assert np.allclose(rho, rho_ref, atol=1e-12, rtol=0)
    assert np.allclose(O.energy_atoms(nl, sp, fs, rho), e_ref, atol=1e-12, rtol=0)
