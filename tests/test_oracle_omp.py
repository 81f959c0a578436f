"""The all-core CPU baselines are the serial oracle bit for bit: or_sweep_omp
gives the same species, density cache, velocities, counters and stage
records after several calls, at a kappa that accepts most stages and at one
that rejects most of them; or_md_omp gives the same positions, velocities,
forces and densities as or_md."""
import numpy as np
import pytest

from paper_1012_5082_amd import inputs as I


@pytest.mark.parametrize("kappa,dmu0", [(0.0, -0.30), (1000.0, -0.23), (10.0, -0.26)])
def test_omp_sweep_is_the_serial_chain(oracle_mod, kappa, dmu0):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(16, 16, 16)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 31)
    sp = I.initial_species(x.size, 0.05, 32)
    vx, vy, vz = I.mb_velocities(sp, 600.0, 33)
    a = O.SweepState(x, y, z, box, sp, pot, vx=vx, vy=vy, vz=vz)
    b = O.SweepState(x, y, z, box, sp, pot, nl=a.nl, vx=vx, vy=vy, vz=vz)
    for call, ns in enumerate((3, 2)):
        sa, _, la = O.sweep(a, dmu0, kappa, 0.05, 600.0, ns, 91, log_stages=10000)
        sb, lb = O.sweep_omp(b, dmu0, kappa, 0.05, 600.0, ns, 91, threads=4, log_stages=10000)
        assert sa == sb, (call, sa, sb)
        assert np.array_equal(la, lb)
        assert np.array_equal(a.species, b.species)
        assert np.array_equal(a.rho.view(np.uint64), b.rho.view(np.uint64))
        for u, v in ((a.vx, b.vx), (a.vy, b.vy), (a.vz, b.vz)):
            assert np.array_equal(u.view(np.uint64), v.view(np.uint64))
        assert a.n_b[0] == b.n_b[0] and a.w == b.w
    assert sa["stage_accepts"] > 0


def test_omp_md_is_the_serial_md(oracle_mod):
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(12, 12, 12)
    x, y, z = I.thermalize(x, y, z, box, 0.05, 41)
    sp = I.initial_species(x.size, 0.1, 42)
    vx, vy, vz = I.mb_velocities(sp, 1200.0, 43)
    a = O.md(x, y, z, vx, vy, vz, sp, box, pot, 2.0, 15)
    b = O.md_omp(x, y, z, vx, vy, vz, sp, box, pot, 2.0, 15, threads=4)
    for u, v in zip(a, b):
        assert np.array_equal(u.view(np.uint64), v.view(np.uint64))
