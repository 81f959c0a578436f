"""What the trained surrogate gains, at an unchanged ensemble.

The network is trained by the library's own kernels on (descriptor, exact dU)
pairs logged from plain sweeps of the 40^3 thermal system.  From one state,
a plain chain and a delayed-acceptance chain with that network run the same
number of sweeps: their mean concentration and mean energy per atom agree
within three standard errors (batch means), while the network's first stage
rejects most trials before any exact energy change is evaluated.  The exact
FP64 dU still decides every accepted move (stage 2, Christen and Fox), so
the two chains sample one ensemble; what the network buys is the exact
evaluations it avoids."""
import numpy as np
import pytest

import exact_refs as X
from paper_1012_5082_amd import inputs as I
from paper_1012_5082_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _trained_network(torch, d, pot, args):
    from paper_1012_5082_amd.binding import VCSGC, Mlp
    g = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, descriptor=True)
    g.sweep(*args, 10, 31)
    g.enable_sample_log(300000, 17)
    g.sweep(*args, 40, 32)
    desc, dE = g.samples()
    # the log fills through an atomic counter: a fixed order makes the
    # trained network (and so this test) deterministic
    a = torch.cat([dE.view(-1, 1), desc], dim=1).cpu().numpy()
    a = a[np.lexsort(a.T[::-1])]
    dE = torch.tensor(a[:, 0].copy(), device="cuda")
    desc = torch.tensor(a[:, 1:].copy(), device="cuda")
    g.close()
    net = Mlp(seed=3)
    net.fit_normalization(desc, dE)
    net.train(desc, dE, epochs=6, batch=4096, lr=2e-3, seed=4)
    pred = net.forward(desc)
    rmse = float(torch.sqrt(torch.mean((pred - dE) ** 2)))
    return net, rmse, float(torch.std(dE)), desc.shape[0]


def test_trained_surrogate_same_ensemble_fewer_exact_evaluations(torch_cuda):
    torch = torch_cuda
    from paper_1012_5082_amd.binding import VCSGC
    pot = I.params("FS-P1")
    d = W.c2(cbar=0.05)
    kappa = 10.0
    args = (d["dmu0"], kappa, d["cbar"], d["T"])
    net, rmse, sd, n_samples = _trained_network(torch, d, pot, args)
    assert rmse < 0.5 * sd, (rmse, sd)
    # a common starting state, relaxed by plain sweeps
    g0 = VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, descriptor=True,
               r_dep=8.01)
    g0.sweep(*args, 40, 33)
    start = g0.species.cpu().numpy().copy()
    g0.close()
    N = d["x"].size
    res = {}
    for name in ("plain", "da"):
        g = VCSGC(d["x"], d["y"], d["z"], d["box"], start, pot, descriptor=True, r_dep=8.01)
        if name == "da":
            g.set_surrogate("mlp", net)
        cs, es = [], []
        trials = flips = pass1 = 0
        t = 0.0
        for blk in range(60):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            s = g.sweep(*args, 5, 34)
            ev[1].record()
            torch.cuda.synchronize()
            t += ev[0].elapsed_time(ev[1]) / 1e3
            trials += s["trials"]
            flips += s["flips"]
            pass1 += s["stage1_pass"]
            cs.append(s["sum_n"] / 5 / N)
            es.append(g.energy() / N)
        g.close()
        mc, ec = X.batch_means(cs, 10)
        me, ee = X.batch_means(es, 10)
        res[name] = dict(c=mc, c_err=ec, E=me, E_err=ee, pre_rejected=1.0 - pass1 / trials,
                         flips_per_s=flips / t, trials_per_s=trials / t, flips=flips)
    p, q = res["plain"], res["da"]
    print(f"surrogate: {n_samples} samples, RMSE {rmse:.4f} eV (dE spread {sd:.4f} eV); "
          f"plain {p}; da {q}")
    assert abs(p["c"] - q["c"]) < 3 * np.hypot(p["c_err"], q["c_err"]) + 1e-6, (p, q)
    assert abs(p["E"] - q["E"]) < 3 * np.hypot(p["E_err"], q["E_err"]) + 1e-6, (p, q)
    # the gain: most trials are settled without an exact energy change
    assert q["pre_rejected"] > 0.8, q
    assert p["pre_rejected"] == 0.0
    assert q["flips"] > 0 and p["flips"] > 0
    net.close()
