"""Nose-Hoover NVT MD on the GPU against the oracle (or_md_nvt): positions,
velocities, forces and the thermostat state (xi, eta) bit for bit, on both
MD-list rebuild paths, across calls, and inside the hybrid MC/MD cycle at
the paper's production time step of 2.5 fs (Sec. IV.B)."""
import math

import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W
from parity_utils import gpu_context

pytestmark = pytest.mark.gpu

NAMES = ("x", "y", "z", "vx", "vy", "vz", "fx", "fy", "fz")


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _md_system(n=10, T=700.0, seed=31, c=0.05):
    x, y, z, box = I.bcc(n, n, n)
    x, y, z = I.thermalize(x, y, z, box, 0.05, seed)
    sp = I.initial_species(x.size, c, seed + 1)
    vx, vy, vz = I.mb_velocities(sp, T, seed + 2)
    return dict(x=x, y=y, z=z, box=box, species=sp, vx=vx, vy=vy, vz=vz, T=T, kappa=1000.0,
                cbar=c, dmu0=W.dmu_s(T, c), seed=4001)


@pytest.mark.parametrize("n,T", [(10, 700.0), (16, 1200.0)])
def test_nvt_parity(torch_cuda, oracle_mod, n, T):
    """Two calls of 30 steps of 2.5 fs, heating the system towards T + 300 K
    (so the thermostat works and the MD list is rebuilt)."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=n, T=T, seed=40 + n)
    g = gpu_context(d, pot, velocities=True)
    g.set_thermostat(T + 300.0, 40.0, xi=0.001)
    g.md(2.5, 30)
    g.md(2.5, 30)
    state = (d["x"], d["y"], d["z"], d["vx"], d["vy"], d["vz"])
    th = (0.001, 0.0)
    for _ in range(2):
        out, th = O.md_nvt(*state, d["species"], d["box"], pot, 2.5, 30, T + 300.0, 40.0,
                           xi=th[0], eta=th[1])
        state = out[:6]
    for nm, want in zip(NAMES, out[:9]):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    xi, eta = g.thermostat()
    assert xi == th[0] and eta == th[1], ((xi, eta), th)
    assert g.info()["md_rebuilds"] >= 1
    g.close()


def test_nvt_infinite_coupling_time_is_nve(torch_cuda):
    """tau = infinity: the thermostat's kernels leave the NVE trajectory of
    the fused NVE passes unchanged, bit for bit."""
    pot = I.params("FS-P1")
    d = _md_system(n=16, T=900.0, seed=61)
    a = gpu_context(d, pot, velocities=True)
    b = gpu_context(d, pot, velocities=True)
    b.set_thermostat(900.0, math.inf)
    a.md(2.5, 25)
    b.md(2.5, 25)
    for nm in NAMES[:6]:
        assert np.array_equal(getattr(a, nm).cpu().numpy(), getattr(b, nm).cpu().numpy()), nm
    assert b.thermostat() == (0.0, 0.0)
    a.close()
    b.close()


def test_nvt_hybrid_cycle_parity(torch_cuda, oracle_mod):
    """[1 sweep; 20 NVT steps of 2.5 fs] x 3 with velocity rescaling on
    transmutation: species, density cache, positions, velocities and the
    thermostat state equal the oracle's."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _md_system(n=16, c=0.1, seed=41)
    g = gpu_context(d, pot, velocities=True)
    g.set_thermostat(700.0, 100.0)
    x, y, z = d["x"], d["y"], d["z"]
    vx, vy, vz = d["vx"], d["vy"], d["vz"]
    sp = d["species"]
    th = (0.0, 0.0)
    for cyc in range(3):
        g.sweep(d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        st = O.SweepState(x, y, z, d["box"], sp, pot, vx=vx, vy=vy, vz=vz)
        st.w = cyc
        O.sweep(st, d["dmu0"], 1.0, d["cbar"], d["T"], 1, d["seed"])
        sp = st.species
        assert np.array_equal(g.rho().cpu().numpy(), st.rho)
        g.md(2.5, 20)
        out, th = O.md_nvt(x, y, z, st.vx, st.vy, st.vz, sp, d["box"], pot, 2.5, 20, 700.0,
                           100.0, xi=th[0], eta=th[1])
        x, y, z, vx, vy, vz = out[:6]
    assert np.array_equal(g.species.cpu().numpy(), sp)
    for nm, want in zip(NAMES[:6], (x, y, z, vx, vy, vz)):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    assert g.thermostat() == th
    g.close()
