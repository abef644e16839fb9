"""GPU parity of VEGAS+ adaptive stratified sampling against the oracle, through the C-ABI."""
import numpy as np
import pytest

from gpu_util import TOL, assert_items_close, gpu_available, item_scale, say
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bm():
    from paper_2603_28848_amd import boltzmc
    return boltzmc


def _vplus(w):
    for p in w.processes:
        p.vegas_plus = 1
    return w


def _oracle_items(ow, uids):
    items, n = ow.items()
    by = {items[i].uid: items[i] for i in range(n)}
    sel = [by[int(u)] for u in uids]
    return (ob.Item * len(sel))(*sel), len(sel)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["2to2", "2to3", "multi", "multi_spline"])
def test_vplus_frozen_parity(which, precision):
    """Frozen runs keep the uniform allocation N / M: every item and iteration against the oracle.  "multi*": the
    two-species set AA->BB, AA->AAA, AA->AABB in one launch (one, two and three integrated particles: the kernel
    instance for several particle counts)."""
    bm = _bm()
    if which == "2to2":
        w, N, nitn = _vplus(wl.w22_mb()), 10_000, 3
    elif which == "2to3":
        w, N, nitn = _vplus(wl.w23_be(n_grid=24, N=1 << 13)), 1 << 13, 2
    else:
        w, N, nitn = _vplus(wl.w_multi(n_grid=16, N=(1 << 12, 1 << 12, 1 << 12), nitn=2, sigma_E=0.05)), 1 << 12, 2
        for p in w.processes:
            p.eval_stride = 1
        if which == "multi_spline":  # the instance with the alternative rules' tables
            for sp in w.species:
                sp.interp = wl.INTERP_SPLINE
    say("vegas+ frozen %s precision=%d" % (which, precision))
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=9, epoch=1, precision=precision, freeze_maps=1, n_iter=nitn, n_samples=N)
    C, S = ctx.collision(-1, -1, opts)
    res = ctx.item_results(nitn)
    ow = ob.OracleWorld(w)
    items, n = _oracle_items(ow, res["uid"])
    rc, r = ow.run_items(items, n, N, nitn, seed=9, epoch=1, adapt=False)
    assert rc == 0
    tol = TOL[precision]
    if which != "2to2" and precision == 0:
        tol = 1e-10  # few in-shell samples per item on the uniform map (the few-sample tolerance)
    sc = item_scale(items, n, r["Ibar"])
    assert_items_close(res["I_it"], r["I_it"], tol, "I_it", scale=sc)
    assert_items_close(res["V_it"], r["V_it"], 10 * tol, "V_it", scale=sc * sc / N)


def test_vplus_adaptive_iterations_follow_the_oracle():
    """Adaptive FP64 run: iteration 0 (uniform allocation, uniform map) to the FP64 tolerance; the map after it and the
    next iteration, which samples with the adapted map and the reallocated hypercubes, to 1e-9 (the map's adaptation
    amplifies ulp-level differences ~100x per iteration)."""
    bm = _bm()
    w = _vplus(wl.w22_mb())
    N, nitn = 10_000, 2
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=4, epoch=0, precision=0, n_iter=nitn, n_samples=N)
    ctx.collision(-1, -1, opts)
    res = ctx.item_results(nitn)
    ow = ob.OracleWorld(w)
    items, n = _oracle_items(ow, res["uid"])
    rc, r = ow.run_items(items, n, N, nitn, seed=4, epoch=0, adapt=True)
    assert rc == 0
    sc = item_scale(items, n, r["Ibar"])
    assert_items_close(res["I_it"][:, 0], r["I_it"][:, 0], TOL[0], "I_0", scale=sc)
    assert_items_close(res["I_it"][:, 1], r["I_it"][:, 1], 1e-9, "I_1", scale=sc)
    nb = w.processes[0].n_bins
    maps = ctx.maps_get(res["uid"], nb)
    used = 6 * (nb + 1)  # D = 6 rows of edges; the rest of each map slot is unused
    err = np.max(np.abs(maps[:, :used] - r["maps"][:, :used]))
    say("map edges max abs diff %.3e" % err)
    assert err <= 1e-9 * 20.0  # edges in [0, 20]


def test_vplus_refused_by_the_adjoint():
    bm = _bm()
    ctx = bm.from_workload(_vplus(wl.w22_mb()))
    opts = bm.default_opts(seed=3, epoch=2, n_iter=1, freeze_maps=1, eval_stride=1, n_samples=1000)
    ni, no = ctx.plan_size(-1, -1, opts)
    with pytest.raises(bm.BmcError):
        ctx.vjp(np.ones(no), -1, -1, opts)
