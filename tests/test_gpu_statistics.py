"""Statistical checks of the GPU chain at sizes the oracle cannot sample:
with identical A/B potentials the VC-SGC distribution of n is known in closed
form, P(n) ~ C(N, n) exp[-beta (phi n + (kappa/N) n^2)], for any geometry.
The mean and variance of n over GPU sweeps are compared with it at 128,000
sites (40^3 thermal bcc) and at the 1.96M-site polycrystal, for the plain
scheme and for local chains of 4 trials per cell."""
import numpy as np
import pytest

import exact_refs as X
from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W
from parity_utils import gpu_context

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(d, T, kappa, cbar, dmu0, n_warm, n_meas, k=1, seed=606):
    N = d["x"].size
    p = X.normalize(X.vcsgc_logw_ideal(N, T, dmu0, kappa, cbar))
    m, v = X.moments(p)
    dd = dict(d)
    dd["species"] = I.initial_species(N, m / N, 12)
    g = gpu_context(dd, I.params("IDEAL"))
    if k > 1:
        g.set_local_steps(k)
    args = (dmu0, kappa, cbar, T)
    g.sweep(*args, n_warm, seed, stats=False)
    ns = []
    for _ in range(n_meas):
        ns.append(g.sweep(*args, 1, seed)["n_final"])
    g.close()
    return np.array(ns, dtype=np.float64), m, v


def _balanced_dmu0(T, c):
    """dmu0 at which plain SGC of the ideal mixture has concentration c, so
    that composite moves carry no net drift (kT ln((1 - c) / c))."""
    return X.KB * T * np.log((1.0 - c) / c)


def _check_moments(ns, m, v):
    """Mean and variance of n within 3 standard errors (batches) of the
    exact values; the variance's error bar must itself be below 7% of v, so
    that a wrong factor in the global term (a kappa off by 2 changes v by
    about 40% here) fails."""
    mean, err = X.batch_means(ns)
    var, verr = X.batch_variance(ns)
    assert verr < 0.07 * v, (var, verr, v)
    assert abs(mean - m) < 3 * err, (mean, m, err)
    assert abs(var - v) < 3 * verr, (var, v, verr)


@pytest.mark.parametrize("k", [1, 4])
def test_ideal_distribution_128k(torch_cuda, k):
    d = W.c2(cbar=0.1)
    ns, m, v = _run(d, 600.0, 0.5, 0.1, _balanced_dmu0(600.0, 0.1), 30, 1600, k=k)
    _check_moments(ns, m, v)


def test_ideal_distribution_polycrystal(torch_cuda):
    d = W.c3(with_velocities=False)
    ns, m, v = _run(d, 700.0, 0.5, 0.03, _balanced_dmu0(700.0, 0.03), 20, 1200)
    _check_moments(ns, m, v)
