"""Conjugate-gradient relaxation on the GPU (vcsgc_minimize) against the
oracle's or_cg, bit for bit: iteration and evaluation counts, stop reason,
energy, |F|, positions and forces; then the sweep from the relaxed state.
"""
import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I
from parity_utils import gpu_context

pytestmark = pytest.mark.gpu

FORCE, ENERGY, ITER, EVAL, LINESEARCH = 1, 2, 3, 4, 5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _defect(n=10, seed=7, holes=(0, 5, 333, 1201)):
    x, y, z, box = I.bcc(n, n, n)
    keep = np.ones(x.size, bool)
    keep[list(holes)] = False
    x, y, z = x[keep], y[keep], z[keep]
    x, y, z = I.thermalize(x, y, z, box, 0.08, seed)
    sp = I.initial_species(x.size, 0.2, seed + 1)
    return dict(x=x, y=y, z=z, box=box, species=sp)


def _poly(ncell=12, grains=4, seed=5):
    x, y, z, box, _ = I.voronoi_poly(ncell, grains, seed)
    sp = I.initial_species(x.size, 0.04, seed + 1)
    return dict(x=x, y=y, z=z, box=box, species=sp)


def _compare(O, d, pot, skin=0.3, **kw):
    g = gpu_context(d, pot, forces=True, skin=skin)
    print(f"[cg] n={d['x'].size} {kw}", flush=True)
    rg = g.minimize(**kw)
    (x, y, z, fx, fy, fz, _), ro, _ = O.cg(d["x"], d["y"], d["z"], d["species"], d["box"], pot,
                                            **kw)
    for k in ("iterations", "evaluations", "reason", "energy", "fnorm"):
        assert rg[k] == ro[k], (k, rg[k], ro[k])
    for nm, want in zip(("x", "y", "z", "fx", "fy", "fz"), (x, y, z, fx, fy, fz)):
        assert np.array_equal(getattr(g, nm).cpu().numpy(), want), nm
    return g, ro, (x, y, z)


@pytest.mark.parametrize("name", ["FS-P1", "TAB-X"])
def test_cg_parity_defect_lattice(torch_cuda, oracle_mod, name):
    pot = I.params(name) if name.startswith("FS") else I.table(name)
    g, ro, _ = _compare(oracle_mod, _defect(), pot, max_iter=300, ftol=1e-6, dmax=0.1)
    assert ro["reason"] in (FORCE, LINESEARCH) and ro["iterations"] > 20
    g.close()


def test_cg_parity_polycrystal(torch_cuda, oracle_mod):
    """Grain-boundary relaxation of a 4-grain Voronoi polycrystal, 60 line
    searches (MD-list skin 0.1 A: before relaxation some boundary sites have
    33 neighbours within rc + 0.3 A, more than a list row holds)."""
    d = _poly()
    g, ro, _ = _compare(oracle_mod, d, I.params("FS-P1"), skin=0.1, max_iter=60, ftol=1e-6,
                        dmax=0.1)
    assert ro["reason"] == ITER
    g.close()


def test_cg_parity_every_trial_rebuilds(torch_cuda, oracle_mod):
    """skin = 0: every trial position rebuilds the MD list."""
    g, _, _ = _compare(oracle_mod, _defect(n=8, seed=9, holes=(3,)), I.params("FS-P1"), skin=0.0,
                       max_iter=40, ftol=1e-6, dmax=0.2)
    g.close()


def test_cg_limits_and_line_search_end(torch_cuda, oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _defect(n=8, seed=13, holes=(1, 77))
    g, ro, _ = _compare(O, d, pot, etol=-1.0, ftol=0.0, max_iter=100000, dmax=0.1)
    assert ro["reason"] == LINESEARCH
    g.close()
    g, ro, _ = _compare(O, d, pot, max_eval=7, ftol=0.0)
    assert ro["reason"] == EVAL
    g.close()
    g, ro, _ = _compare(O, d, pot, max_iter=0)
    assert ro["reason"] == ITER
    g.close()


def test_cg_then_sweep(torch_cuda, oracle_mod):
    """Two sweeps (batched pipeline) from the relaxed polycrystal: the
    sweep's lists and density cache are rebuilt from the new positions."""
    O = oracle_mod
    pot = I.params("FS-P1")
    d = _poly(seed=17)
    g, _, (x, y, z) = _compare(O, d, pot, skin=0.1, max_iter=25, ftol=1e-6, dmax=0.1)
    g.set_tuning("batch", 3)
    args = (-0.2, 1000.0, 0.04, 700.0)
    sg = g.sweep(*args, 2, 91)
    st = O.SweepState(x, y, z, d["box"], d["species"], pot)
    so, _, _ = O.sweep(st, *args, 2, 91)
    for k in ("trials", "stage_accepts", "flips", "n_final"):
        assert sg[k] == so[k], k
    assert np.array_equal(g.species.cpu().numpy(), st.species)
    assert np.array_equal(g.rho().cpu().numpy(), st.rho)
    g.close()


def test_cg_rejects_bad_parameters(torch_cuda):
    from paper_1012_5082_amd.binding import VcsgcError
    d = _defect(n=6, holes=(0,))
    g = gpu_context(d, I.params("FS-P1"), forces=True)
    for kw in (dict(max_iter=-1), dict(ftol=-1.0), dict(dmax=0.0), dict(dmax=1e3),
               dict(etol=float("nan"))):
        with pytest.raises(VcsgcError) as e:
            g.minimize(**kw)
        assert e.value.code == -1
    g.close()
    g = gpu_context(d, I.params("FS-P1"))  # no force arrays
    with pytest.raises(VcsgcError):
        g.minimize()
    g.close()
