"""Helpers of the GPU parity tests: the same seeded workload on the HIP path (through the C-ABI binding) and
on the oracle, and the tolerance forms.

Tolerances (FP64 1e-12, FP32-integrand 1e-5, relative):
  * per item:  |I_gpu - I_oracle| <= tol |I_oracle|
  * per point: |C_gpu - C_oracle| <= tol * sum over the point's items of mult |I_oracle|  (C can cross zero)
  * sigma:     10 tol relative
"""
import sys

import numpy as np
import pytest

TOL = {0: 1e-12, 1: 1e-5}


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
