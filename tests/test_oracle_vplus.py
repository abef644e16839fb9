"""Pins of the oracle's VEGAS+ adaptive stratification (Lepage 2021) on top of the Vegas map."""
import math

import numpy as np
import pytest

import pins_analytic as pa
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _vplus(w, on=1):
    for p in w.processes:
        p.vegas_plus = on
    return w


def test_strata_count():
    assert ob.lib().orc_vplus_strata(1 << 18, 9) == 3   # 3^9 = 19683 <= 2^17 < 4^9
    assert ob.lib().orc_vplus_strata(10_000, 6) == 4    # 4^6 = 4096 <= 5000 < 5^6
    assert ob.lib().orc_vplus_strata(100, 6) == 1


def test_one_stratum_is_plain_vegas():
    """With N < 2 * 2^D there is a single hypercube: the same samples, estimate, variance and adapted map as plain
    Vegas (up to the order of the sums)."""
    w1, w2 = wl.w22_mb(n_grid=32), _vplus(wl.w22_mb(n_grid=32))
    out = []
    for w in (w1, w2):
        ow = ob.OracleWorld(w)
        items, n = ow.items()
        sel = [items[i] for i in range(n) if items[i].eval_idx in (10, 20)]
        arr = (ob.Item * len(sel))(*sel)
        rc, r = ow.run_items(arr, len(sel), 100, 3)
        assert rc == 0
        out.append(r)
    np.testing.assert_allclose(out[1]["I_it"], out[0]["I_it"], rtol=1e-13)
    np.testing.assert_allclose(out[1]["V_it"], out[0]["V_it"], rtol=1e-11)
    np.testing.assert_allclose(out[1]["maps"], out[0]["maps"], rtol=1e-13)


def test_vplus_mb_loss_matches_closed_form():
    m, sig = 1.0, 0.02
    w = _vplus(wl.w22_mb(n_grid=64, sigma_E=sig))
    ow = ob.OracleWorld(w)
    rc, fit = ow.fit(0)
    ff = lambda p: float(ow.f_batch(0, fit, np.array([p]), np.array([math.hypot(p, m)]))[0])
    items, n = ow.items()
    sel = [items[i] for i in range(n) if items[i].term == 1 and items[i].eval_idx in (20, 30, 40)]
    arr = (ob.Item * len(sel))(*sel)
    rc, r = ow.run_items(arr, len(sel), 1 << 16, 6)
    assert rc == 0
    q = ow.grid_q(0)
    for k, it in enumerate(sel):
        L = pa.mb_loss_closed_form(q[it.eval_idx], w.species[0].f[it.eval_idx], ff, m)
        assert abs(r["Ibar"][k] - L) <= 4 * r["sigma"][k] + 0.15 * sig * L, (it.eval_idx, r["Ibar"][k], L)


def test_vplus_error_estimate_matches_the_scatter():
    """Over 24 seeds (fresh maps each), the reported sigma of an adapted VEGAS+ iteration (the stratified variance
    sum_h V_h^2 var_h / n_h) matches the spread of the estimates.  (Plain Vegas is reported beside it: on this
    thin-shell integrand, with ~5 samples per hypercube, the adaptive allocation does not beat it.)"""
    w = wl.w22_mb(n_grid=32, sigma_E=0.02)
    ests, sig, sig_plain = [], [], []
    for seed in range(24):
        for on in (1, 0):
            ow = ob.OracleWorld(_vplus(wl.w22_mb(n_grid=32, sigma_E=0.02), on))
            items, n = ow.items()
            sel = [items[i] for i in range(n) if items[i].eval_idx == 16 and items[i].term == 0]
            arr = (ob.Item * 1)(*sel)
            rc, r = ow.run_items(arr, 1, 20_000, 4, seed=seed)
            assert rc == 0
            if on:
                ests.append(r["I_it"][0, -1])
                sig.append(math.sqrt(r["V_it"][0, -1]))
            else:
                sig_plain.append(math.sqrt(r["V_it"][0, -1]))
    spread = float(np.std(ests, ddof=1))
    assert 0.6 < spread / float(np.mean(sig)) < 1.6, (spread, np.mean(sig), np.mean(sig_plain))
