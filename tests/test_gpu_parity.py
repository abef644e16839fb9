"""GPU parity of the HIP path (through the C-ABI) against the CPU oracle on the same seeded inputs.

Vegas adaptation with a narrow Gaussian delta amplifies 1-ulp differences by ~30-100x per iteration, so
parity is checked (i) on frozen maps across all iterations, (ii) one adaptive iteration at a time from a
common map produced by the oracle, and (iii) for free-running runs on the first iteration (common uniform
map) plus a statistical check of the final values.
"""
import numpy as np
import pytest

from gpu_util import (TOL, assert_items_close, check_fp64_items, fp64_point_bound, gpu_available, item_scale,
                      oracle_items_matching, point_scale, say)
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


def _run_gpu(w, opts, process=-1, species=-1):
    bm = _bm()
    ctx = bm.from_workload(w)
    C, S = ctx.collision(process, species, opts)
    n_iter = opts.n_iter if opts.n_iter > 0 else w.processes[0].n_iter
    res = ctx.item_results(n_iter)
    return ctx, C, S, res


# --------------------------------------------------------------------------------------- frozen maps
@pytest.mark.parametrize("precision", [0, 1])
def test_frozen_maps_2to2_all_items(precision):
    """2->2 MB, 32-point grid, 4 iterations x 1e4 samples on the uniform map: every item and every C."""
    bm = _bm()
    w = wl.w22_mb()
    say("frozen 2to2 precision=%d" % precision)
    opts = bm.default_opts(seed=0, epoch=0, precision=precision, freeze_maps=1, n_iter=4, n_samples=10_000)
    ctx, C, S, res = _run_gpu(w, opts)
    ow = ob.OracleWorld(w)
    items, n = oracle_items_matching(ow, res["uid"])
    rc, r = ow.run_items(items, n, 10_000, 4, adapt=False)
    assert rc == 0
    tol = TOL[precision]
    assert_items_close(res["I_it"], r["I_it"], tol, "I_it")
    assert_items_close(res["Ibar"], r["Ibar"], tol, "Ibar")
    assert_items_close(res["sigma"], r["sigma"], 10 * tol, "sigma")
    Co, So = ow.combine(items, n, r["Ibar"], r["sigma"], 0)
    scale = point_scale(items, n, r["Ibar"], 0, 32)
    err = np.abs(C - Co)
    say("C max err / scale %.3e" % np.max(err / scale))
    assert np.all(err <= tol * scale)
    np.testing.assert_allclose(S, So, rtol=10 * tol, atol=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_frozen_maps_2to3_full_size_sampled_items(precision):
    """2<->3 BE on the 128-point grid at the full 2^18 samples per item: GPU evaluates all 512 items in one
    batched launch; the oracle recomputes a sample of items (first, interior, last nodes; both sides, both
    terms) and they must match item by item (results depend only on each item's counters and map)."""
    bm = _bm()
    w = wl.w23_be()
    say("frozen 2to3 full-size precision=%d" % precision)
    opts = bm.default_opts(seed=0, epoch=0, precision=precision, freeze_maps=1, n_iter=2)
    ctx, C, S, res = _run_gpu(w, opts)
    assert len(res["uid"]) == 512
    pick = [i for i, u in enumerate(res["uid"]) if (int(u) & 0x3FFFF) in (0, 47, 127)]
    ow = ob.OracleWorld(w)
    items, n = oracle_items_matching(ow, res["uid"][pick])
    rc, r = ow.run_items(items, n, 1 << 18, 2, adapt=False)
    assert rc == 0
    if precision == 0:
        check_fp64_items(ow, items, n, res, r, 1 << 18, 2, sel=pick)
    else:
        scale = item_scale(items, n, r["Ibar"])
        assert_items_close(res["I_it"][pick], r["I_it"], TOL[1], "I_it", scale=scale)
        assert_items_close(res["sigma"][pick], r["sigma"], 10 * TOL[1], "sigma", scale=scale)


def test_headline_full_size_adaptive_in_the_bench_launch_configuration():
    """The benchmark's own call: 2<->3 BE, 512 items x 10 adaptive iterations x 2^18 samples, FP32 integrand, the
    launch shape picked by the autotuner.  Sampled items (first, interior, last nodes; both sides, both terms)
    against the oracle's free-running run of the same items: iteration 0 (the common uniform map) to the FP32-integrand
    tolerance, the combined estimate after ten adaptive iterations within 6 sigma (adaptation amplifies rounding
    differences, so later iterations are two different Monte Carlo histories)."""
    bm = _bm()
    w = wl.w23_be()
    ctx = bm.from_workload(w)
    opts = bm.default_opts(seed=0, epoch=0, precision=bm.FP32I)
    b, ch, ms = ctx.autotune(-1, -1, opts)
    say("headline full size, adaptive, autotuned to %d blocks/CU, chunk %d" % (b, ch))
    C, S = ctx.collision(-1, -1, opts)
    res = ctx.item_results(10)
    assert len(res["uid"]) == 512
    pick = [i for i, u in enumerate(res["uid"]) if (int(u) & 0x3FFFF) in (0, 47, 127)]
    ow = ob.OracleWorld(w)
    items, n = oracle_items_matching(ow, res["uid"][pick])
    rc, r = ow.run_items(items, n, 1 << 18, 10, seed=0, epoch=0)
    assert rc == 0
    scale = item_scale(items, n, r["Ibar"])
    assert_items_close(res["I_it"][pick, 0], r["I_it"][:, 0], TOL[1], "I_it[0]", scale=scale)
    z = (res["Ibar"][pick] - r["Ibar"]) / np.sqrt(res["sigma"][pick] ** 2 + r["sigma"] ** 2)
    say("headline adaptive: max |dIbar|/sigma over %d sampled items = %.2f" % (n, float(np.max(np.abs(z)))))
    assert np.max(np.abs(z)) < 6.0


# -------------------------------------------------------------------------------- stepwise adaptation
def test_stepwise_adaptation_2to2():
    """From the oracle's map before iteration k, one GPU iteration (Philox iteration index k) reproduces the
    oracle's I_k, V_k and adapted map."""
    bm = _bm()
    w = wl.w22_mb()
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    nb = 50
    maps = np.full((n, 12 * (nb + 1)), np.nan)
    ctx = bm.from_workload(w)
    uids = [items[i].uid for i in range(n)]
    for k in range(4):
        say("stepwise iteration %d" % k)
        if k == 0:
            maps_k = np.stack([ow.map_uniform(items[i], nb) for i in range(n)])
        else:
            maps_k = maps.copy()
        rc, r = ow.run_items(items, n, 10_000, 1, maps=maps_k.copy(), first_iter=k)
        assert rc == 0
        ctx.maps_set(uids, maps_k)
        opts = bm.default_opts(seed=0, epoch=0, precision=0, n_iter=1, n_samples=10_000, first_iter=k)
        ctx.collision(-1, -1, opts)
        res = ctx.item_results(1)
        assert list(res["uid"]) == uids
        assert_items_close(res["I_it"][:, 0], r["I_it"][:, 0], 1e-12, "I_%d" % k)
        assert_items_close(res["V_it"][:, 0], r["V_it"][:, 0], 1e-11, "V_%d" % k)
        gm = ctx.maps_get(uids, nb)
        om = r["maps"]
        # edges relative to each dimension's range
        rng = np.repeat(np.array([20.0, np.pi, 2 * np.pi] * 4), nb + 1)
        d_err = np.max(np.abs(gm - om)[:, : 6 * (nb + 1)] / rng[: 6 * (nb + 1)])
        say("map %d max edge err / range %.3e" % (k, d_err))
        assert d_err < 1e-12
        maps = om


# ------------------------------------------------------------------------------------ free running
def test_free_running_2to2_first_iteration_and_statistics():
    bm = _bm()
    w = wl.w22_mb()
    opts = bm.default_opts(seed=0, epoch=0, precision=0)
    ctx, C, S, res = _run_gpu(w, opts)
    ow = ob.OracleWorld(w)
    items, n = oracle_items_matching(ow, res["uid"])
    rc, r = ow.run_items(items, n, 10_000, 4)
    assert_items_close(res["I_it"][:, 0], r["I_it"][:, 0], 1e-12, "I_0")
    Co, So = ow.combine(items, n, r["Ibar"], r["sigma"], 0)
    z = (C - Co) / np.sqrt(S ** 2 + So ** 2)
    say("free-running 2to2: max |dC|/sigma = %.2f, rel err vs oracle max %.2e" %
        (np.max(np.abs(z)), np.max(np.abs(C - Co) / point_scale(items, n, r["Ibar"], 0, 32))))
    assert np.max(np.abs(z)) < 6.0


# -------------------------------------------------------------------------------------------- modes
@pytest.mark.parametrize("precision", [0, 1])
def test_plain_equals_batched_bitwise_and_run_to_run(precision):
    bm = _bm()
    w = wl.w23_be(n_grid=24, N=3000, nitn=3)
    outs = []
    for launch in (0, 1, 0):
        ctx = bm.from_workload(w)
        C, S = ctx.collision(-1, -1, bm.default_opts(seed=7, epoch=3, launch=launch, precision=precision))
        outs.append((C, S, ctx.item_results(3)))
    for C, S, res in outs[1:]:
        assert np.array_equal(C, outs[0][0]) and np.array_equal(S, outs[0][1])
        assert np.array_equal(res["I_it"], outs[0][2]["I_it"])


@pytest.mark.parametrize("precision", [0, 1])
def test_plain_and_batched_groupings_agree_to_rounding(precision):
    """At 2^17 samples an item has 32 units: a batched launch sums its second pass in 4 records of 8 units, a
    per-grid-point launch in 32 records of one unit.  On frozen maps the two differ only in the order of the FP64
    sums, and each launch mode repeats itself bitwise."""
    bm = _bm()
    w = wl.w23_be(n_grid=16, N=1 << 17, nitn=2)
    outs = {0: [], 1: []}
    for launch in (0, 1, 0, 1):
        ctx = bm.from_workload(w)
        C, S = ctx.collision(-1, -1, bm.default_opts(seed=7, epoch=3, launch=launch, precision=precision,
                                                     freeze_maps=1))
        outs[launch].append((C, S))
    for launch in (0, 1):
        (C0, S0), (C1, S1) = outs[launch]
        assert np.array_equal(C0, C1) and np.array_equal(S0, S1), launch
    (Cb, Sb), (Cp, Sp) = outs[0][0], outs[1][0]
    assert np.all(Sb > 0)
    dC = np.max(np.abs(Cb - Cp) / Sb)
    dS = np.max(np.abs(Sb - Sp) / Sb)
    say("groupings: max |C_batched - C_plain| / sigma = %.2e, max rel dsigma = %.2e" % (dC, dS))
    assert dC < 1e-9 and dS < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_launch_tuning_and_autotuner_do_not_change_results(precision):
    bm = _bm()
    w = wl.w23_be(n_grid=24, N=5000, nitn=3)
    res = []
    for tuning in ((1, 1), (4, 8), (2, 16), None):
        ctx = bm.from_workload(w)
        o = bm.default_opts(seed=4, epoch=1, precision=precision)
        if tuning is None:
            b, ch, ms = ctx.autotune(-1, -1, o)
            say("autotune: %d blocks/CU, chunk %d, %.3f ms" % (b, ch, ms))
        else:
            ctx.set_launch_tuning(*tuning)
        C, S = ctx.collision(-1, -1, o)
        res.append((C, S, ctx.item_results(3)["I_it"]))
    for C, S, I in res[1:]:
        assert np.array_equal(C, res[0][0]) and np.array_equal(S, res[0][1]) and np.array_equal(I, res[0][2])


def test_frozen_and_adjoint_calls_leave_no_bin_counts_behind():
    """The screening pass adds every sample to its item's bin counts and each iteration's reduction reads and clears
    them. A frozen-map collision (which adapts nothing) or an adjoint call (whose screening keeps no counts) must
    leave them clear: the adapting collision after either equals, bitwise, the same collision on a fresh context."""
    bm = _bm()
    w = wl.w23_be(n_grid=16, N=1 << 14, nitn=3)
    o = bm.default_opts(seed=5, epoch=2)
    ref = bm.from_workload(w)
    C0, S0 = ref.collision(-1, -1, o)
    a = bm.from_workload(w)
    a.collision(-1, -1, bm.default_opts(seed=9, epoch=7, freeze_maps=1))
    C1, S1 = a.collision(-1, -1, o)
    assert np.array_equal(C1, C0) and np.array_equal(S1, S0)
    b = bm.from_workload(w)
    ni, no = b.plan_size(-1, -1, o)
    b.collision(-1, -1, bm.default_opts(seed=9, epoch=7, freeze_maps=1))  # the plan and the adjoint's screening lists
    b.vjp(np.ones(no), -1, -1, bm.default_opts(seed=9, epoch=7, precision=0))
    C2, S2 = b.collision(-1, -1, o)
    assert np.array_equal(C2, C0) and np.array_equal(S2, S0)


def test_selection_invariance():
    """An item's results do not depend on which other items share the launch."""
    bm = _bm()
    w = wl.w23_be(n_grid=24, N=3000, nitn=2)
    ctx = bm.from_workload(w)
    ctx.collision(-1, -1, bm.default_opts(seed=1, freeze_maps=1))
    all_res = ctx.item_results(2)
    ctx2 = bm.from_workload(w)
    ctx2.collision(-1, 0, bm.default_opts(seed=1, freeze_maps=1, eval_stride=5))
    sub = ctx2.item_results(2)
    idx = {int(u): i for i, u in enumerate(all_res["uid"])}
    for j, u in enumerate(sub["uid"]):
        assert np.array_equal(sub["I_it"][j], all_res["I_it"][idx[int(u)]])


# ----------------------------------------------------------------------------------- edge cases
def test_ragged_units_and_small_sizes():
    """Sample counts that are not multiples of the block (ragged last unit), the minimum of 2 samples,
    2 Vegas bins and a 10-node grid."""
    bm = _bm()
    # With only a handful of samples an item's estimate can come from one sample far off the energy shell, where an
    # ulp of dE (the energies of the conserved particle differ by an ulp between the two sine/cosine libraries)
    # becomes a relative error of |dE|/sigma_E^2 times it: the FP64 contract's rounding term covers it.
    for N, nb, ng in ((4097 + 255, 50, 16), (2, 2, 10), (777, 3, 12)):
        w = wl.w22_mb(n_grid=ng, N=N, nitn=2)
        w.processes[0].n_bins = nb
        say("ragged N=%d nb=%d grid=%d" % (N, nb, ng))
        opts = bm.default_opts(seed=5, precision=0, freeze_maps=1)
        ctx, C, S, res = _run_gpu(w, opts)
        ow = ob.OracleWorld(w)
        items, n = oracle_items_matching(ow, res["uid"])
        rc, r = ow.run_items(items, n, N, 2, seed=5, adapt=False)
        assert rc == 0
        check_fp64_items(ow, items, n, res, r, N, 2, seed=5)


def test_error_paths():
    bm = _bm()
    w = wl.w22_mb(n_grid=16)
    ctx = bm.from_workload(w)
    with pytest.raises(bm.BmcError) as e:
        ctx.collision(5, -1, bm.default_opts())
    assert e.value.code == bm.EINVAL
    with pytest.raises(bm.BmcError) as e:
        ctx.set_f(0, -np.ones(16))
    assert e.value.code == bm.ERANGE
    with pytest.raises(bm.BmcError) as e:
        ctx.collision(-1, -1, bm.default_opts(precision=7))
    assert e.value.code == bm.EINVAL
    fd = wl.w24_fd(n_grid=16, N=64, nitn=1)
    ctx2 = bm.from_workload(fd)
    with pytest.raises(bm.BmcError) as e:
        ctx2.set_f(0, np.full(16, 1.5))
    assert e.value.code == bm.ERANGE


# ------------------------------------------------------------------------------- points off the grid
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("which", ["2to2", "2to3"])
def test_points_off_the_grid(precision, which):
    """Collision integral at momenta between grid nodes, below the grid and above it (observed f interpolated
    inside the grid, from the fit outside), frozen maps: every item and every point against the oracle."""
    bm = _bm()
    if which == "2to2":
        w, N, nitn = wl.w22_mb(), 10_000, 3
    else:
        w, N, nitn = wl.w23_be(n_grid=32, N=1 << 13), 1 << 13, 2
    sp = w.species[0]
    qg = wl.log_nodes(sp.q_min, sp.q_max, sp.n_grid)
    q = np.array([0.5 * sp.q_min, np.sqrt(qg[3] * qg[4]), 0.3 * qg[10] + 0.7 * qg[11], qg[17], 1.3 * sp.q_max])
    say("off-grid %s precision=%d" % (which, precision))
    opts = bm.default_opts(seed=3, epoch=0, precision=precision, freeze_maps=1, n_iter=nitn, n_samples=N)
    ctx = bm.from_workload(w)
    C, S = ctx.collision(-1, 0, opts, eval_q=q)
    assert C.shape == (len(q),)
    res = ctx.item_results(nitn)
    ow = ob.OracleWorld(w)
    items, n = ow.items_at(q, species=0)
    by = {items[i].uid: items[i] for i in range(n)}
    assert sorted(by) == sorted(int(u) for u in res["uid"])
    sel = [by[int(u)] for u in res["uid"]]
    items = (ob.Item * len(sel))(*sel)
    rc, r = ow.run_items(items, n, N, nitn, seed=3, adapt=False)
    assert rc == 0
    tol = TOL[precision]
    Co, So = ow.combine_at(items, n, r["Ibar"], r["sigma"], len(q))
    err = np.abs(C - Co)
    if precision == 0:
        B1, B2, _ = check_fp64_items(ow, items, n, res, r, N, nitn, seed=3)
        bound = fp64_point_bound(items, n, r, B1, B2, 0, len(q))
        say("C max err / bound %.3f" % np.max(err / bound))
        assert np.all(err <= bound)
    else:
        assert_items_close(res["I_it"], r["I_it"], tol, "I_it", scale=item_scale(items, n, r["Ibar"]))
        scale = point_scale(items, n, r["Ibar"], 0, len(q))
        say("C max err / scale %.3e" % np.max(err / scale))
        assert np.all(err <= tol * scale)
        np.testing.assert_allclose(S, So, rtol=10 * tol, atol=1e-300)
    # the same context still evaluates its grid afterwards, with the grid's own items
    Cg, _ = ctx.collision(-1, 0, opts)
    assert Cg.shape == (sp.n_grid,)
    for bad_q, bad_species in ((np.ones(257), 0), (np.array([1.0, -1.0]), 0), (np.array([1.0]), -1)):
        with pytest.raises(bm.BmcError):
            ctx.collision(-1, bad_species, opts, eval_q=bad_q)
