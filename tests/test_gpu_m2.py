"""GPU parity of the polynomial matrix element |M|^2 = lambda^2 P(s, t) against the oracle, through the C-ABI."""
import numpy as np
import pytest

from gpu_util import (TOL, assert_items_close, check_fp64_items, fp64_point_bound, gpu_available, item_scale,
                      oracle_items_matching, point_scale, say)
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl

pytestmark = pytest.mark.gpu

COEF = (0.4, 0.15, -0.08, 0.01, 0.004, 0.02)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _bm():
    from paper_2603_28848_amd import boltzmc
    return boltzmc


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["2to2", "2to3", "ab_unequal"])
def test_poly_m2_frozen_maps_parity(which, precision):
    bm = _bm()
    if which == "2to2":
        w, N, nitn = wl.w22_mb(), 10_000, 3
    elif which == "2to3":
        w, N, nitn = wl.w23_be(n_grid=32, N=1 << 14), 1 << 14, 2
    else:  # A B -> A B with unequal masses: s and t of distinct positions matter
        n, q_min, q_max = 32, 0.02, 20.0
        q = wl.log_nodes(q_min, q_max, n)
        sp = [wl.Species("A", wl.BOSE, n, q_min, q_max, wl.f_equilibrium(q, 1.0, 1.3, wl.BOSE), m0=1.0),
              wl.Species("B", wl.MB, n, q_min, q_max, wl.f_equilibrium(q, 0.3, 0.9, wl.MB), m0=0.3)]
        w = wl.Workload("ab", sp, [wl.Process([0, 1], [1, 0], n_samples=10_000, n_iter=3)])
        N, nitn = 10_000, 3
    for p in w.processes:
        p.m2_kind, p.m2_coef = wl.M2_POLY, COEF
    say("poly |M|^2 %s precision=%d" % (which, precision))
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=8, epoch=3, precision=precision, freeze_maps=1, n_iter=nitn, n_samples=N)
    C, S = ctx.collision(-1, -1, opts)
    res = ctx.item_results(nitn)
    ow = ob.OracleWorld(w)
    items, n_all = ow.items()
    by = {items[i].uid: items[i] for i in range(n_all)}
    sel = [by[int(u)] for u in res["uid"]]
    arr = (ob.Item * len(sel))(*sel)
    rc, r = ow.run_items(arr, len(sel), N, nitn, seed=8, epoch=3, adapt=False)
    assert rc == 0
    tol = TOL[precision]
    if precision == 0:
        B1, B2, _ = check_fp64_items(ow, arr, len(sel), res, r, N, nitn, seed=8, epoch=3)
    else:
        assert_items_close(res["I_it"], r["I_it"], tol, "I_it", scale=item_scale(arr, len(sel), r["Ibar"]))
    off = 0
    for a, s in enumerate(w.species):
        Co, So = ow.combine(arr, len(sel), r["Ibar"], r["sigma"], a)
        if precision == 0:
            bound = fp64_point_bound(arr, len(sel), r, B1, B2, a, s.n_grid)
        else:
            bound = tol * np.maximum(point_scale(arr, len(sel), r["Ibar"], a, s.n_grid), 1e-300)
        assert np.all(np.abs(C[off:off + s.n_grid] - Co) <= bound)
        off += s.n_grid


def test_poly_m2_is_refused_by_the_adjoint_and_the_exact_path():
    bm = _bm()
    w = wl.w22_mb()
    w.processes[0].m2_kind, w.processes[0].m2_coef = wl.M2_POLY, COEF
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=3, epoch=2, n_iter=1, freeze_maps=1, eval_stride=1, n_samples=1000)
    ni, no = ctx.plan_size(-1, -1, opts)
    with pytest.raises(bm.BmcError):
        ctx.vjp(np.ones(no), -1, -1, opts)
    with pytest.raises(bm.BmcError):
        ctx.collision_exact22(-1, -1, opts)


@pytest.mark.parametrize("precision", [0, 1])
def test_unit_polynomial_through_the_general_instance_matches_constant_m2(precision):
    """A polynomial |M|^2 with P = 1 runs the second pass's general instance (full tables: q_j, M_j or E_j, y_j, and
    f_j per node, three blocks per CU); the constant |M|^2 runs the linear-rule instance (tables of f_j alone, the
    compact layout, four blocks per CU for the FP32 integrand).  Both against the oracle on the same frozen maps and
    samples (FP64: the rounding contract; FP32 integrand: 1e-5), and against each other: the two instances contract
    the FP64 kinematics into fused multiply-adds differently, so they agree to rounding, not bitwise."""
    bm = _bm()
    N, nitn = 1 << 14, 2
    w = wl.w23_be(n_grid=32, N=N, nitn=nitn)
    ow = ob.OracleWorld(w)
    out = []
    for kind in (wl.M2_CONST, wl.M2_POLY):
        for p in w.processes:
            p.m2_kind, p.m2_coef = kind, (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
        ctx = bm.from_workload(w)
        ctx.collision(-1, -1, bm.default_opts(seed=4, epoch=1, precision=precision, freeze_maps=1, n_iter=nitn,
                                              n_samples=N))
        out.append(ctx.item_results(nitn))
    assert np.array_equal(out[0]["uid"], out[1]["uid"])
    items, n = oracle_items_matching(ow, out[0]["uid"])
    rc, r = ow.run_items(items, n, N, nitn, seed=4, epoch=1, adapt=False)
    assert rc == 0
    for k, res in enumerate(out):
        say("%s |M|^2, precision %d" % (("constant", "unit polynomial")[k], precision))
        if precision == 0:
            check_fp64_items(ow, items, n, res, r, N, nitn, seed=4, epoch=1)
        else:
            assert_items_close(res["I_it"], r["I_it"], TOL[1], "I_it", scale=item_scale(items, n, r["Ibar"]))
    d = np.abs(out[0]["I_it"] - out[1]["I_it"])
    say("instances differ by max |dI| / |I| %.3e" % float(np.max(d / np.maximum(np.abs(r["I_it"]), 1e-300))))
