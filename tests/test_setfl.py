"""setfl reading and writing (paper_1012_5082_amd.setfl): a table written
and read back is the same table (pair values to the rounding of r phi / r),
the header fields land where the format puts them, and the potential read
back gives the oracle's energies and forces of the original to rounding."""
import math

import numpy as np

from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import setfl


def test_setfl_round_trip(tmp_path):
    tab = I.table("TAB-X")
    p = tmp_path / "x.setfl"
    setfl.write(str(p), tab, elements=("Fe", "Cu"), masses=(55.845, 63.546))
    back, el, masses = setfl.read(str(p))
    assert el == ["Fe", "Cu"] and masses == [55.845, 63.546]
    assert (back.nr, back.nrho, back.dr, back.drho, back.rc) == (tab.nr, tab.nrho, tab.dr,
                                                                  tab.drho, tab.rc)
    assert np.array_equal(back.f, tab.f) and np.array_equal(back.F, tab.F)
    assert np.allclose(back.phi[:, 1:], tab.phi[:, 1:], rtol=4e-16, atol=1e-300)
    assert np.array_equal(back.phi[:, 0], back.phi[:, 1])


def test_setfl_layout(tmp_path):
    """A hand-written file: F columns first, then f, then r phi for
    (1,1), (2,1), (2,2)."""
    nr, nrho, dr, drho = 5, 3, 1.0, 0.5
    lines = ["c1", "c2", "c3", "2 Fe Cu", f"{nrho} {drho} {nr} {dr} 3.5",
             "26 55.845 2.87 bcc", "0 -1 -2", "5 4 3 2 1",
             "29 63.546 3.61 fcc", "0 -3", "-4", "6 5 4 3 2",
             "0 2 4 6 8", "0 3 6 9 12", "0 4 8 12 16"]
    p = tmp_path / "h.setfl"
    p.write_text("\n".join(lines) + "\n")
    t, el, m = setfl.read(str(p))
    assert el == ["Fe", "Cu"] and m == [55.845, 63.546] and t.rc == 3.5
    assert np.array_equal(t.F, [[0, -1, -2], [0, -3, -4]])
    assert np.array_equal(t.f, [[5, 4, 3, 2, 1], [6, 5, 4, 3, 2]])
    assert np.array_equal(t.phi, [[2, 2, 2, 2, 2], [3, 3, 3, 3, 3], [4, 4, 4, 4, 4]])


def test_setfl_potential_matches_original(oracle_mod, tmp_path):
    O = oracle_mod
    tab = I.table("TAB-X")
    p = tmp_path / "x.setfl"
    setfl.write(str(p), tab)
    back, _, _ = setfl.read(str(p))
    x, y, z, box = I.bcc(6, 6, 6)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 3)
    sp = I.initial_species(x.size, 0.3, 4)
    nl = O.neighbors(x, y, z, box, tab.rc)
    e0, e1 = math.fsum(O.energy_atoms(nl, sp, tab)), math.fsum(O.energy_atoms(nl, sp, back))
    assert abs(e0 - e1) <= 1e-12 * abs(e0)
    for a, b in zip(O.forces(nl, sp, tab), O.forces(nl, sp, back)):
        assert np.max(np.abs(a - b)) <= 1e-12
