"""Helpers of the GPU parity tests: the same seeded workload on the HIP path (through the C-ABI binding) and
on the oracle, and the tolerance forms.

Tolerances (FP64 1e-12, FP32-integrand 1e-5, relative):
  * per item:  |I_gpu - I_oracle| <= tol |I_oracle|
  * per point: |C_gpu - C_oracle| <= tol * sum over the point's items of mult |I_oracle|  (C can cross zero)
  * sigma:     10 tol relative
FP64 per item, with the rounding term (assert_fp64_items): |I_gpu - I_oracle| <= 1e-12 |I_oracle| + 4 eps B1 and
|V_gpu - V_oracle| <= 1e-12 |V_oracle| + 4 eps B2, where B1 = (1/N) sum_n |W_n| s_n, B2 = (2/(N(N-1))) sum_n W_n^2 s_n
and s_n = (|dE_n| / sigma_E)(sum_i E_i / sigma_E) (OracleWorld.sensitivity).  The two sides compute the same
formulas in FP64 but take sine and cosine from different libraries (each within an ulp), so the momentum components,
and through them the conserved particle's energy and dE, may differ by about 2 eps sum_i E_i; the Gaussian factor
moves by |dE|/sigma_E^2 times that (Eq. 15).  On an item carried by one or two shell samples this reaches 1e-10 for
sigma_E = 0.002, far above 1e-12.  The factor 4 is twice the first-order estimate; measured errors stay below 0.7 eps B.
"""
import sys

import numpy as np
import pytest

TOL = {0: 1e-12, 1: 1e-5}
EPS = 2.0 ** -52
ROUND_C = 4.0


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def say(msg):
    sys.stdout.write("[gpu-test] %s\n" % msg)
    sys.stdout.flush()


def oracle_items_matching(ow, uids):
    items, n = ow.items()
    by = {items[i].uid: items[i] for i in range(n)}
    from oracle import binding as ob
    sel = [by[int(u)] for u in uids]
    return (ob.Item * len(sel))(*sel), len(sel)


def item_scale(items, n, I):
    """Per item: the gross rate sum mult |I| over all items at the same (process set, species, node) -- the
    scale the collision integral at that node is compared on.  Items far smaller than it (pure off-shell
    estimates) are compared against it instead of their own value."""
    acc = {}
    for i in range(n):
        key = (items[i].species, items[i].eval_idx)
        acc[key] = acc.get(key, 0.0) + items[i].mult * abs(I[i])
    return np.array([acc[(items[i].species, items[i].eval_idx)] for i in range(n)])


def assert_items_close(got, want, tol, what="I", scale=None):
    """|got - want| <= tol * max(|want|, scale) elementwise (scale: per item, e.g. item_scale)."""
    got, want = np.asarray(got), np.asarray(want)
    err = np.abs(got - want)
    ref = np.abs(want)
    if scale is not None:
        sc = np.asarray(scale)
        if ref.ndim == 2 and sc.ndim == 1:
            sc = sc[:, None]
        ref = np.maximum(ref, sc)
    bound = tol * ref
    bad = np.nonzero(err > bound)[0]
    rel = np.where(ref != 0, err / np.where(ref != 0, ref, 1), err)
    msg = "%s: max rel err %.3e (tol %.1e), %d / %d outside" % (what, rel.max() if rel.size else 0, tol, bad.size,
                                                               got.size)
    say(msg)
    assert bad.size == 0, msg + " first: %s" % (list(zip(got[bad[:5]], want[bad[:5]])),)
    return float(rel.max()) if rel.size else 0.0


def point_scale(items, n, Ibar, species, n_grid):
    s = np.zeros(n_grid)
    for i in range(n):
        if items[i].species == species:
            s[items[i].eval_idx] += items[i].mult * abs(Ibar[i])
    return s


def assert_fp64_items(got, want, B, what="I"):
    """FP64 contract per item (and iteration): |got - want| <= 1e-12 |want| + 4 eps B (B = B1 for estimates, B2 for
    variances, same shape as want).  Reports the largest error relative to |want| and to the bound."""
    got, want, B = np.asarray(got), np.asarray(want), np.asarray(B)
    assert got.shape == want.shape == B.shape, (got.shape, want.shape, B.shape)
    err = np.abs(got - want)
    bound = TOL[0] * np.abs(want) + ROUND_C * EPS * B
    bad = np.argwhere(err > bound)
    with np.errstate(divide="ignore", invalid="ignore"):
        own = np.where(want != 0, err / np.abs(want), np.where(err > 0, np.inf, 0.0))
        frac = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    msg = "%s: max err / |value| %.3e, max err / bound %.3f, %d / %d outside" % (
        what, float(np.max(own)) if own.size else 0.0, float(np.max(frac)) if frac.size else 0.0, len(bad), got.size)
    say(msg)
    assert len(bad) == 0, msg + " first: %s" % ([(got[tuple(i)], want[tuple(i)], bound[tuple(i)]) for i in bad[:5]],)
    return float(np.max(frac)) if frac.size else 0.0


def fp64_bounds(ow, items, n, N, nitn, seed=0, epoch=0, maps=None, first_iter=0):
    """(B1, B2) of the oracle's items for the iterations compared (frozen maps; uniform if None)."""
    return ow.sensitivity(items, n, N, nitn, seed=seed, epoch=epoch, maps=maps, first_iter=first_iter)


def check_fp64_items(ow, items, n, res, r, N, nitn, seed=0, epoch=0, maps=None, first_iter=0, sel=None):
    """FP64 contract for the per-iteration estimates and variances of the compared items (res: GPU item results,
    r: oracle results of the same items; sel: rows of res matching r)."""
    B1, B2 = fp64_bounds(ow, items, n, N, nitn, seed, epoch, maps, first_iter)
    gI = res["I_it"] if sel is None else res["I_it"][sel]
    gV = res["V_it"] if sel is None else res["V_it"][sel]
    fI = assert_fp64_items(gI[:, :nitn], r["I_it"][:, :nitn], B1, "I_it")
    fV = assert_fp64_items(gV[:, :nitn], r["V_it"][:, :nitn], B2, "V_it")
    return B1, B2, max(fI, fV)


def fp64_point_bound(items, n, r, B1, B2, species, n_points):
    """Bound on |C_gpu - C_oracle| per point implied by the per-item FP64 contract: for each item the bound of its
    inverse-variance combination (the largest per-iteration bound of I, plus the weights' relative bound times the
    spread of the iterations' estimates), summed with the multiplicities over the point's items."""
    I, V, Ib = r["I_it"], r["V_it"], r["Ibar"]
    out = np.zeros(n_points)
    for i in range(n):
        if items[i].species != species:
            continue
        bI = TOL[0] * np.abs(I[i]) + ROUND_C * EPS * B1[i]
        with np.errstate(divide="ignore", invalid="ignore"):
            bV = np.where(V[i] > 0, (TOL[0] * V[i] + ROUND_C * EPS * B2[i]) / V[i], 0.0)
        out[items[i].eval_idx] += items[i].mult * (np.max(bI) + 2 * np.max(bV) * np.max(np.abs(I[i] - Ib[i])))
    return out
