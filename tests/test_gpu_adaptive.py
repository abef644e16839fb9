"""Adaptive Vegas parity at the benchmark's dimension (2<->3, D = 9) and at D = 12 (2->4), where the map adaptation
kernel gives some waves a second dimension (8 waves over 9 or 12 dimensions).

Stepwise: for each iteration k both sides start from the oracle's map before k; the GPU's I_k, V_k and adapted map
must equal the oracle's (the FP64 contract per item: 1e-12 relative plus the rounding term of the energies, see
gpu_util; edges to 1e-12 of each dimension's range).  Free-running: ten adaptive iterations on both sides from the
uniform map agree in the first iteration to the same contract and statistically thereafter (adaptation amplifies
rounding differences, so the two runs are two different Monte Carlo histories).
"""
import numpy as np
import pytest

from gpu_util import check_fp64_items, gpu_available, oracle_items_matching, say
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl

pytestmark = pytest.mark.gpu

NB = 50


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bm():
    from paper_2603_28848_amd import boltzmc
    return boltzmc


def _ranges(w, items, n):
    """Per item and map row, the width of the dimension's range (r: the particle's grid range; theta: pi;
    phi: 2 pi), as an (n, 12 (nb + 1)) array matching the map layout (unused rows 1)."""
    ow = ob.OracleWorld(w)
    out = np.ones((n, 12 * (NB + 1)))
    for i in range(n):
        m = ow.map_uniform(items[i], NB).reshape(12, NB + 1)
        D = ow.item_dims(items[i])
        for d in range(D):
            out[i, d * (NB + 1):(d + 1) * (NB + 1)] = m[d, NB] - m[d, 0]
    return out


def _stepwise(w, N, n_iter, tag, edge_tol=1e-12):
    bm = _bm()
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    uids = [items[i].uid for i in range(n)]
    rng = _ranges(w, items, n)
    ctx = bm.from_workload(w)
    maps = np.stack([ow.map_uniform(items[i], NB) for i in range(n)])
    worst = {"bound": 0.0, "edge": 0.0}
    for k in range(n_iter):
        say("%s stepwise iteration %d (%d items, N=%d)" % (tag, k, n, N))
        rc, r = ow.run_items(items, n, N, 1, maps=maps.copy(), first_iter=k)
        assert rc == 0
        ctx.maps_set(uids, maps)
        ctx.collision(-1, -1, bm.default_opts(seed=0, epoch=0, precision=0, n_iter=1, n_samples=N, first_iter=k))
        res = ctx.item_results(1)
        assert [int(u) for u in res["uid"]] == uids
        _, _, frac = check_fp64_items(ow, items, n, res, r, N, 1, maps=maps, first_iter=k)
        worst["bound"] = max(worst["bound"], frac)
        gm = ctx.maps_get(uids, NB)
        om = r["maps"]
        e = float(np.max(np.abs(gm - om) / rng))
        say("%s map %d: max edge err / range %.3e" % (tag, k, e))
        worst["edge"] = max(worst["edge"], e)
        assert e < edge_tol
        assert not np.array_equal(om, maps)  # the map did move
        maps = om
    say("%s stepwise worst: %s" % (tag, worst))


def test_stepwise_adaptation_2to3_D9():
    """2<->3 BE (the benchmark's process and dimension) on 24 nodes of [0.01, 30], 2^14 samples, three iterations."""
    _stepwise(wl.w23_be(n_grid=24, N=1 << 14, nitn=3), 1 << 14, 3, "2to3")


def test_stepwise_adaptation_2to4_D12():
    """2->4 FD with m(t) = 1 + 0.1 sin t on 10 nodes of [0.005, 40], 2^14 samples, three iterations.  At
    sigma_E = 0.002 single shell samples carry whole bins of the training histograms, and their W differs between the
    two sides by up to 2e-10 relative (the rounding of the energies amplified by the Gaussian, the FP64 contract's
    rounding term).  An edge placed inside a sparse bin moves by that relative error times the bin's share of the
    whole histogram's weight, so the adapted edges differ by up to 1.4e-11 of the range (measured, iteration 2; the
    amount depends on how the compiler contracts the kinematics into fused multiply-adds), and the edges are held to
    5e-11 of the range here."""
    _stepwise(wl.w24_fd(n_grid=10, N=1 << 14, nitn=3), 1 << 14, 3, "2to4", edge_tol=5e-11)


def test_free_running_2to3_first_iteration_and_statistics():
    """Ten adaptive iterations of 2^14 samples on 24 nodes: iteration 0 (the common uniform map) to the FP64 contract
    per item, the final C within 6 sigma of the oracle's."""
    bm = _bm()
    N, nitn = 1 << 14, 10
    w = wl.w23_be(n_grid=24, N=N, nitn=nitn)
    ctx = bm.from_workload(w)
    C, S = ctx.collision(-1, -1, bm.default_opts(seed=5, epoch=1, precision=0))
    res = ctx.item_results(nitn)
    ow = ob.OracleWorld(w)
    items, n = oracle_items_matching(ow, res["uid"])
    rc, r = ow.run_items(items, n, N, nitn, seed=5, epoch=1)
    assert rc == 0
    check_fp64_items(ow, items, n, res, r, N, 1, seed=5, epoch=1)
    Co, So = ow.combine(items, n, r["Ibar"], r["sigma"], 0)
    z = (C - Co) / np.sqrt(S ** 2 + So ** 2)
    gross = np.zeros(24)
    for i in range(n):
        gross[items[i].eval_idx] += items[i].mult * abs(r["Ibar"][i])
    say("free-running 2to3: max |dC|/sigma %.2f, max |dC| / gross rate %.2e" %
        (np.max(np.abs(z)), np.max(np.abs(C - Co) / gross)))
    assert np.max(np.abs(z)) < 6.0
