"""Helpers for GPU-vs-oracle parity tests."""
from __future__ import annotations

import numpy as np

TIE = 1e-9


def gpu_context(d, pot, velocities=False, forces=False, skin=0.3):
    from paper_1012_5082_amd.binding import VCSGC
    kw = {}
    if velocities:
        kw = dict(vx=d["vx"], vy=d["vy"], vz=d["vz"])
    return VCSGC(d["x"], d["y"], d["z"], d["box"], d["species"], pot, forces=forces, skin=skin,
                 **kw)


def oracle_state(O, d, pot, velocities=False):
    kw = {}
    if velocities:
        kw = dict(vx=d["vx"], vy=d["vy"], vz=d["vz"])
    return O.SweepState(d["x"], d["y"], d["z"], d["box"], d["species"], pot, **kw)


def tie_overrides(tl, sl):
    """GPU decisions at near ties, in the oracle's override format
    (w, s, cell or -1 for the global test, decision)."""
    rows = []
    for r in tl:
        if abs(r[7]) < TIE:
            rows.append((r[0], r[1], r[2], r[5]))
    for r in sl:
        if r[4] > 0 and abs(r[7]) < TIE:
            rows.append((r[0], r[1], -1.0, r[5]))
    return np.array(rows, dtype=np.float64).reshape(-1, 4)


def compare_logs(tl_g, sl_g, tl_o, sl_o, du_rtol=1e-12):
    """Trial logs: identical (w, s, cell, site, dn) everywhere, identical
    decisions away from near ties, dU within du_rtol relative.  Stage logs:
    identical colour, dn_tot, record counts and decisions."""
    assert tl_g.shape == tl_o.shape, (tl_g.shape, tl_o.shape)
    assert np.array_equal(tl_g[:, :5], tl_o[:, :5])
    away = (np.abs(tl_g[:, 7]) >= TIE) & (np.abs(tl_o[:, 7]) >= TIE)
    assert np.array_equal(tl_g[away, 5], tl_o[away, 5])
    du_g, du_o = tl_g[:, 6], tl_o[:, 6]
    scale = np.maximum(np.abs(du_o), 1e-300)
    rel = np.abs(du_g - du_o) / scale
    assert np.all((rel <= du_rtol) | (du_g == du_o)), float(rel.max())
    assert sl_g.shape == sl_o.shape, (sl_g.shape, sl_o.shape)
    assert np.array_equal(sl_g[:, :5], sl_o[:, :5])
    g_away = (np.abs(sl_g[:, 7]) >= TIE) | (sl_g[:, 4] == 0)
    assert np.array_equal(sl_g[g_away, 5], sl_o[g_away, 5])
    return {"max_du_rel": float(rel.max()) if rel.size else 0.0,
            "du_bitwise": bool(np.array_equal(du_g, du_o)),
            "trials": int(tl_g.shape[0]), "stages": int(sl_g.shape[0])}
