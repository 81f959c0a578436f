"""The paper's own quantitative results for its Ising-type model (Sec. II.B:
bcc, eps_AA(1) = eps_BB(1) = -10 U, eps_AB(1) = -9.7 U, eps(2) = -2 U,
k_B T = 0.8617 U, 2,000 sites, starting from a 50% solid solution),
reproduced by the oracle:

* serial VC-SGC-MC at c0 = 50% reaches an acceptance of about 47%
  (Sec. III.C, closing remarks on Fig. 10; the optimal dmu0 is 0 by the
  model's A <-> B symmetry);
* the SGC method cannot hold a concentration inside the miscibility gap
  (Sec. II.B): at dmu = 0 from the 50% solution the chain runs off to one of
  the coexisting phases.

The model is the tabulated pair model inputs.table("ISING") on the rigid
lattice (f = F = 0); one active cell per stage (r_dep = 14.3 A: two cells per
axis) makes the sweep the serial chain with the global factor applied to
every single move.
"""
import numpy as np

from paper_1012_5082_amd import inputs as I

U = 0.1
T = 0.8617 * U / I.KB


def _state(O):
    x, y, z, box = I.bcc(10, 10, 10)
    return O.SweepState(x, y, z, box, I.initial_species(x.size, 0.5, 7), I.table("ISING"))


def test_serial_vcsgc_acceptance_is_the_papers(oracle_mod):
    O = oracle_mod
    st = _state(O)
    args = (0.0, 1.0 * U, 0.5, T)
    O.sweep(st, *args, 150, 11, r_dep=14.3)
    s, _, _ = O.sweep(st, *args, 150, 11, r_dep=14.3)
    acc = s["flips"] / s["trials"]
    assert abs(acc - 0.47) <= 0.015, acc
    assert abs(s["sum_n"] / 150 / st.n - 0.5) <= 0.01


def test_sgc_cannot_hold_the_miscibility_gap(oracle_mod):
    O = oracle_mod
    st = _state(O)
    O.sweep(st, 0.0, 0.0, 0.5, T, 150, 11, r_dep=14.3)
    c = int(st.n_b[0]) / st.n
    assert abs(c - 0.5) > 0.2, c
