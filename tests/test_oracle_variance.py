"""Pin of the oracle's plain-Vegas error estimate against the scatter of its own estimates over independent seeds.

Per iteration the estimate is I = S1/N with variance V = (S2/N - I^2)/(N - 1); iterations combine by inverse variance,
sigma = (sum 1/V)^(-1/2) (Sec. II.D; Lepage's Vegas).  If these are right, the reported sigma matches the standard
deviation of the estimates over seeds (32 seeds: the sample standard deviation is good to about 13 %, so the ratio is
asserted in [0.6, 1.6]).  Mistakes this catches: V without the 1/(N - 1) (sigma about sqrt(N) too large), the
combined sigma taken as the root of the mean V, or of the summed V (2x too large at four iterations), a variance of
S2/N alone, and any other error in sigma by a factor outside [0.6, 1.6].
"""
import numpy as np
import pytest

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl

SEEDS = range(100, 132)


def _items():
    w = wl.w22_mb(n_grid=32, sigma_E=0.05)
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    sel = [i for i in range(n) if items[i].eval_idx == 14]  # gain and loss at q ~ 0.6
    arr = (ob.Item * len(sel))(*[items[i] for i in sel])
    return ow, arr, len(sel)


@pytest.mark.parametrize("adapt,nitn", [(False, 1), (True, 4)])
def test_sigma_matches_scatter_over_seeds(adapt, nitn):
    ow, items, n = _items()
    est, sig = [], []
    for seed in SEEDS:
        rc, r = ow.run_items(items, n, 4096, nitn, seed=seed, adapt=adapt)
        assert rc == 0
        est.append(r["Ibar"])
        sig.append(r["sigma"])
    est, sig = np.array(est), np.array(sig)
    for i in range(n):
        scatter = np.std(est[:, i], ddof=1)
        reported = np.sqrt(np.mean(sig[:, i] ** 2))
        assert 0.6 < scatter / reported < 1.6, (i, scatter, reported)
        if not adapt:  # one iteration: sigma is sqrt(V) itself
            rc, r = ow.run_items(items, n, 4096, 1, seed=SEEDS[0], adapt=False)
            assert r["sigma"][i] == pytest.approx(np.sqrt(r["V_it"][i, 0]), rel=1e-15)


def test_two_sample_identity():
    """With N = 2 samples on the uniform map, I = (W_1 + W_2)/2 and V = (W_1 - W_2)^2 / 4 (the two-sample variance of
    the mean).  W_n is the integrand at x = lo + y (hi - lo) times the map's Jacobian prod(hi - lo), from the sample's
    uniforms.  This catches a dropped -I^2 or N - 1, which the scatter test cannot resolve on a thin-shell
    integrand whose second moment dwarfs I^2."""
    w = wl.w22_mb(n_grid=32, sigma_E=0.5)
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    nb = w.processes[0].n_bins
    checked = 0
    for i in range(n):
        it = items[i]
        if it.eval_idx % 5:
            continue
        D = 6
        m = ow.map_uniform(it, nb).reshape(12, nb + 1)[:D]
        lo, hi = m[:, 0], m[:, nb]
        W = []
        for s in range(2):
            y = ob.uniforms(7, it.uid, 0, 0, s, D)
            W.append(np.prod(hi - lo) * ow.integrand_at(it, lo + y * (hi - lo)))
        one = (ob.Item * 1)(it)
        rc, r = ow.run_items(one, 1, 2, 1, seed=7, adapt=False)
        assert rc == 0
        I, V = r["I_it"][0, 0], r["V_it"][0, 0]
        assert I == pytest.approx(0.5 * (W[0] + W[1]), rel=1e-9, abs=1e-300)
        assert V == pytest.approx(0.25 * (W[0] - W[1]) ** 2, rel=1e-8, abs=1e-300)
        checked += W[0] != W[1]
    assert checked >= 4
