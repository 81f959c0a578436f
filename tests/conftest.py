import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    if not os.path.exists(O.LIB_PATH):
        O.build(force=False)
    return O


@pytest.fixture(scope="session")
def enum16(oracle_mod):
    """16-site bcc cell (2 x 2 x 2 conventional cells, periodic image sums):
    the FS-P1 energy of all 2^16 species assignments."""
    import numpy as np
    from paper_1012_5082_amd import inputs as I
    O = oracle_mod
    pot = I.params("FS-P1")
    x, y, z, box = I.bcc(2, 2, 2)
    nl = O.neighbors(x, y, z, box, pot.rc)
    N = 16
    U = np.zeros(2 ** N)
    for s in range(2 ** N):
        sp = np.array([(s >> k) & 1 for k in range(N)], np.uint8)
        U[s] = O.energy_total(O.energy_atoms(nl, sp, pot))
    nb = np.array([bin(s).count("1") for s in range(2 ** N)])
    return dict(x=x, y=y, z=z, box=box, nl=nl, U=U, nb=nb, pot=pot, N=N)
