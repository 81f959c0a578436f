"""Nose-Hoover NPT on the GPU (vcsgc_set_barostat + md_verlet_step) against
the oracle's or_md_npt, bit for bit: positions, velocities, forces, box,
barostat momentum, thermostat state and virial; the hybrid cycle on a
changing box; the sweep's check of its cell grid.
"""
import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from parity_utils import gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _system(n=10, c=0.1, seed=31, T=700.0):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, box=box, species=sp)


def _run_both(O, d, pot, dt, steps, T, tau_t, p_ext, tau_p, skin=0.3, blocks=1):
    g = gpu_context(d, pot, velocities=True, forces=True, skin=skin)
    g.set_thermostat(T, tau_t)
    g.set_barostat(p_ext, tau_p)
    st = (d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"])
    box, state, vir = d["box"].copy(), (0.0, 0.0, 0.0), 0.0
    for b in range(blocks):
        print(f"[npt] n={d['x'].size} block {b} p_ext={p_ext} skin={skin}", flush=True)
        g.md(dt, steps)
        st, box, state, vir = O.md_npt(*st[:6], d["species"], box, pot, dt, steps, T, tau_t, p_ext,
                                       tau_p, *state)
        pe, gbox, gvir = g.barostat()
        xi, eta = g.thermostat()
        assert np.array_equal(gbox, box)
        assert (pe, xi, eta, gvir) == (state[2], state[0], state[1], vir)
        for nm, want in zip(("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz"), st[:9]):
            assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    return g, st, box, state


def test_npt_parity_expanding_box(torch_cuda, oracle_mod):
    """-3.2 GPa at 700 K: the box expands (after a first contraction)."""
    d = _system()
    g, _, box, _ = _run_both(oracle_mod, d, I.params("FS-P1"), 2.5, 20, 700.0, 100.0, -0.02,
                             200.0, blocks=3)
    assert np.prod(box) > 1.001 * np.prod(d["box"])
    g.close()


def test_npt_parity_compressed_tabulated(torch_cuda, oracle_mod):
    """+3.2 GPa with TAB-X: the box shrinks (lists rebuilt against the
    scaled build positions)."""
    d = _system(seed=41)
    g, _, box, _ = _run_both(oracle_mod, d, I.table("TAB-X"), 2.5, 30, 700.0, 100.0, 0.02, 150.0,
                             blocks=2)
    assert np.prod(box) < 0.997 * np.prod(d["box"])
    g.close()


def test_npt_parity_thin_skin(torch_cuda, oracle_mod):
    """MD-list skin 0.05 A: rebuilds nearly every step."""
    d = _system(n=8, seed=51)
    g, _, _, _ = _run_both(oracle_mod, d, I.params("FS-P1"), 2.0, 25, 900.0, 50.0, -0.01, 100.0,
                           skin=0.05)
    g.close()


def test_npt_hybrid_cycle(torch_cuda, oracle_mod):
    """[20 NPT steps; one sweep on the batched pipeline] x 2: the sweep's cells,
    lists and density cache follow the box."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _system(n=12, c=0.05, seed=61)
    g = gpu_context(d, pot, velocities=True, forces=True)
    g.set_thermostat(700.0, 100.0)
    g.set_barostat(0.0, 200.0)
    g.set_tuning("batch", 3)
    st = (d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"])
    box, state, sp = d["box"].copy(), (0.0, 0.0, 0.0), d["species"]
    args = (-0.2, 1000.0, 0.05, 700.0)
    for cyc in range(2):
        g.md(2.5, 20)
        st, box, state, _ = O.md_npt(*st[:6], sp, box, pot, 2.5, 20, 700.0, 100.0, 0.0, 200.0,
                                     *state)
        g.sweep(*args, 1, 77)
        ost = O.SweepState(*st[:3], box, sp, pot, vx=st[3], vy=st[4], vz=st[5])
        ost.w = cyc
        O.sweep(ost, *args, 1, 77)
        sp = ost.species
        st = (*st[:3], ost.vx, ost.vy, ost.vz)
        assert np.array_equal(g.species.cpu().numpy(), sp)
        assert np.array_equal(g.rho().cpu().numpy(), ost.rho)
        for nm, want in zip(("x", "vx"), (st[0], st[3])):
            assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    g.close()


def test_sweep_rejects_a_box_below_its_cell_grid(torch_cuda):
    """r_dep = 14.3 A on a 28.7 A box: two cells of 14.35 A per axis; at
    +8 GPa the box shrinks below them and the sweep refuses to run."""
    from paper_1012_5082_amd.binding import VCSGC, VcsgcError
    d = _system(seed=71)
    pot = I.params("FS-P1")
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, vx=d["vx"], vy=d["vy"],
              vz=d["vz"], forces=True, r_dep=14.3)
    g.sweep(-0.2, 1000.0, 0.1, 700.0, 1, 5)
    g.set_thermostat(700.0, 100.0)
    g.set_barostat(0.05, 100.0)
    g.md(2.5, 60)
    assert g.barostat()[1][0] / 2 < 14.3
    with pytest.raises(VcsgcError) as e:
        g.sweep(-0.2, 1000.0, 0.1, 700.0, 1, 5)
    assert e.value.code == -2
    g.close()


def test_barostat_arguments(torch_cuda):
    from paper_1012_5082_amd.binding import VcsgcError
    d = _system(n=8)
    g = gpu_context(d, I.params("FS-P1"), velocities=True, forces=True)
    for a in ((float("nan"), 100.0), (0.0, -1.0), (0.0, float("inf"))):
        with pytest.raises(VcsgcError):
            g.set_barostat(*a)
    g.set_barostat(0.0, 100.0)
    with pytest.raises(VcsgcError):  # no thermostat
        g.md(1.0, 1)
    g.close()
