"""The production schedule (paper_1012_5082_amd.production: CG relaxation,
NPT equilibration, VC-SGC MC/MD cycles with NPT steps of 2.5 fs) on a small
Voronoi polycrystal, against the same sequence of oracle calls, bit for bit.
"""
import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("colours,grow_edge,potential", [(8, 0.0, "FS-P1"), (27, 0.0, "FS-P1"),
                                                       (8, 15.0, "FS-P1"), (8, 0.0, "setfl")])
def test_production_schedule_matches_oracle(torch_cuda, oracle_mod, tmp_path, colours, grow_edge,
                                            potential):
    """With the octant scheme, 27 colours and grown domains (cells of 17.2 A),
    and with a tabulated potential read from a setfl file (TAB-X written as
    setfl and read back)."""
    O = oracle_mod
    from paper_1012_5082_amd import production as PR
    from paper_1012_5082_amd.binding import VCSGC
    if potential == "setfl":
        from paper_1012_5082_amd import setfl
        path = str(tmp_path / "tab_x.eam.alloy")
        setfl.write(path, I.table("TAB-X"))
        pot = setfl.read(path)[0]
    else:
        pot = I.params(potential)
    x, y, z, box, _ = I.voronoi_poly(12, 4, 23)
    sp = I.initial_species(x.size, 0.04, 24)
    vx, vy, vz = I.mb_velocities(sp, 700.0, 25)
    # skin 0.1 A: before relaxation some boundary sites have 33 neighbours
    # within rc + 0.3 A, more than a list row holds
    g = VCSGC(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz, forces=True, skin=0.1,
              colours=colours, grow_edge=grow_edge)
    g.set_tuning("batch", 3)
    s = PR.Schedule(dmu0=-0.25, cbar=0.04, relax_iter=30, equil_steps=40, tau_p=300.0, seed=99)
    print(f"[production] n={x.size} colours={colours} grow_edge={grow_edge}", flush=True)
    pre = PR.relax_and_equilibrate(g, s)
    agg = PR.cycles(g, s, 3)

    (x1, y1, z1, *_), ro, _ = O.cg(x, y, z, sp, box, pot, max_iter=s.relax_iter,
                                    ftol=s.relax_ftol, dmax=s.relax_dmax)
    assert pre["relax"] == ro
    st, b, state, _ = O.md_npt(x1, y1, z1, vx, vy, vz, sp, box, pot, s.dt, s.equil_steps, s.T,
                               s.tau_t, s.p_ext, s.tau_p)
    assert pre["box"] == list(b)
    spc, trials, flips = sp, 0, 0
    for cyc in range(3):
        ost = O.SweepState(*st[:3], b, spc, pot, vx=st[3], vy=st[4], vz=st[5])
        ost.w = cyc
        so, _, _ = O.sweep(ost, s.dmu0, s.kappa, s.cbar, s.T, 1, s.seed,
                           colour_period=3 if colours == 27 else 2, grow_edge=grow_edge)
        trials += so["trials"]
        flips += so["flips"]
        spc = ost.species
        st, b, state, _ = O.md_npt(*st[:3], ost.vx, ost.vy, ost.vz, spc, b, pot, s.dt,
                                   s.md_per_sweep, s.T, s.tau_t, s.p_ext, s.tau_p, *state)
    assert (agg["trials"], agg["flips"]) == (trials, flips) and flips > 0
    assert np.array_equal(g.species.cpu().numpy(), spc)
    for nm, want in zip(("x", "y", "z", "vx", "vy", "vz"), st[:6]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    assert np.array_equal(g.barostat()[1], b)
    g.close()


def test_production_resume_from_checkpoint(torch_cuda):
    """A production run checkpointed after two cycles (positions,
    velocities, species, box, the thermostat's xi and eta, the barostat's
    momentum, the sweep counter and seed) and resumed in a fresh context
    ends bit for bit where the uninterrupted run ends two cycles later."""
    from paper_1012_5082_amd import production as PR
    from paper_1012_5082_amd.binding import VCSGC
    pot = I.params("FS-P1")
    x, y, z, box, _ = I.voronoi_poly(12, 4, 23)
    sp = I.initial_species(x.size, 0.04, 24)
    vx, vy, vz = I.mb_velocities(sp, 700.0, 25)
    s = PR.Schedule(dmu0=-0.25, cbar=0.04, relax_iter=30, equil_steps=40, tau_p=300.0, seed=99)
    g = VCSGC(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz, forces=True, skin=0.1)
    g.set_tuning("batch", 3)
    PR.relax_and_equilibrate(g, s)
    PR.cycles(g, s, 2)
    ck = {nm: getattr(g, nm).cpu().numpy().copy() for nm in ("x", "y", "z", "vx", "vy", "vz")}
    ck["species"] = g.species.cpu().numpy().copy()
    pe, bx, _ = g.barostat()
    xi, eta = g.thermostat()
    state = g.get_state()
    a = PR.cycles(g, s, 2)
    g2 = VCSGC(ck["x"], ck["y"], ck["z"], np.asarray(bx), ck["species"], pot, vx=ck["vx"],
               vy=ck["vy"], vz=ck["vz"], forces=True, skin=0.1)
    g2.set_tuning("batch", 3)
    g2.set_thermostat(s.T, s.tau_t, xi, eta)
    g2.set_barostat(s.p_ext, s.tau_p, pe)
    g2.set_state(state["sweeps_done"], state["seed"])
    b = PR.cycles(g2, s, 2)
    assert (a["trials"], a["flips"]) == (b["trials"], b["flips"]) and a["flips"] > 0
    for nm in ("x", "y", "z", "vx", "vy", "vz", "species"):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), getattr(g2, nm).cpu().numpy()), nm
    assert np.array_equal(g.barostat()[1], g2.barostat()[1])
    assert g.thermostat() == g2.thermostat()
    g.close()
    g2.close()
