"""Pins of the oracle's non-constant matrix element: |M|^2 = lambda^2 P(s, t) with P quadratic in the Mandelstam
invariants."""
import math

import numpy as np
import pytest

import pins_analytic as pa
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def test_poly_reduces_to_constant_bitwise():
    w1 = wl.w22_mb(n_grid=32)
    w2 = wl.w22_mb(n_grid=32)
    w2.processes[0].m2_kind, w2.processes[0].m2_coef = wl.M2_POLY, (1.0, 0, 0, 0, 0, 0)
    r = []
    for w in (w1, w2):
        ow = ob.OracleWorld(w)
        items, n = ow.items()
        sel = [items[i] for i in range(n) if items[i].eval_idx in (8, 20)]
        arr = (ob.Item * len(sel))(*sel)
        rc, res = ow.run_items(arr, len(sel), 4096, 2, adapt=False)
        assert rc == 0
        r.append(res["I_it"])
    assert np.array_equal(r[0], r[1])


@pytest.mark.parametrize("coef", [(0.5, 0.2, 0.0, 0.0, 0.0, 0.0), (1.0, 0.0, -0.3, 0.0, 0.0, 0.0),
                                  (0.0, 0.0, 0.0, 0.05, 0.02, 0.04)])
def test_poly_mb_loss_matches_two_body_closed_form(coef):
    """Loss items of MB 2->2 with an s- and t-dependent |M|^2 against the two-body closed form with the centre-of-mass
    average of t (a sign error in s or t fails one of the three polynomials; for identical final particles t and u
    are interchangeable, as they are physically)."""
    m, sig = 1.0, 0.02
    w = wl.w22_mb(n_grid=64, sigma_E=sig)
    w.processes[0].m2_kind, w.processes[0].m2_coef = wl.M2_POLY, coef
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
        L = pa.mb_loss_poly_closed_form(q[it.eval_idx], w.species[0].f[it.eval_idx], ff, m, coef=coef, p2_max=20.0)
        assert abs(r["Ibar"][k] - L) <= 4 * r["sigma"][k] + 0.15 * sig * abs(L), (it.eval_idx, r["Ibar"][k], L)


def test_poly_equilibrium_is_stationary_and_adjoint_refuses():
    """Detailed balance does not depend on |M|^2 (the same P(s, t) at each point for gain and loss): C[f_eq] ~ 0 with
    the equilibrium-exact rule; the adjoint and the exact-delta path refuse a non-constant |M|^2."""
    n, q_min, q_max = 48, 0.05, 14.0
    q = wl.log_nodes(q_min, q_max, n)
    sp = wl.Species("phi", wl.BOSE, n, q_min, q_max, wl.f_equilibrium(q, 1.0, 1.0, wl.BOSE), m0=1.0,
                    interp=wl.INTERP_EQEXACT)
    out = {}
    for tm in (wl.TERMS_NET, wl.TERMS_SPLIT):
        pr = wl.Process([0, 0], [0, 0], sigma_E=0.01, term_mode=tm, m2_kind=wl.M2_POLY,
                        m2_coef=(0.3, 0.1, -0.05, 0.0, 0.0, 0.01))
        ow = ob.OracleWorld(wl.Workload("eq", [sp], [pr]))
        items, ni = ow.items()
        sel = [items[i] for i in range(ni) if items[i].eval_idx in (16, 24, 32) and items[i].term == 0]
        arr = (ob.Item * len(sel))(*sel)
        rc, r = ow.run_items(arr, len(sel), 1 << 15, 4)
        assert rc == 0
        out[tm] = r
    for k in range(3):
        G = out[wl.TERMS_SPLIT]["Ibar"][k]
        assert G > 0
        assert abs(out[wl.TERMS_NET]["Ibar"][k]) <= 4 * out[wl.TERMS_NET]["sigma"][k] + 2e-4 * G
    rc, *_ = ow.vjp(arr, len(sel), np.ones(len(sel)), 256, 0)
    assert rc == -1
    rc, _ = ow.exact22(arr, len(sel))
    assert rc == -1
