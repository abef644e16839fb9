"""Pins of the oracle's exact-delta 2->2 path (Sec. IV semi-analytic reduction; Appendix B)."""
import math

import numpy as np
import pytest
from scipy import integrate

import pins_analytic as pa
from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _paper_F_numeric(p1, p3, px, E1, E3, Ex, m1, m2, m3, mx, M2=1.0):
    """F = int dcos(theta) |M|^2 pi / sqrt(-a) Theta(b^2 - 4 a c) with a, b, c exactly as printed in Appendix B
    (backward term: px = p4), integrated numerically (the discontinuity located by a fine scan)."""
    Q = m1 ** 2 - m2 ** 2 + m3 ** 2 + mx ** 2
    gam = E3 * Ex - E1 * E3 - E1 * Ex
    kappa = p1 * p1 + p3 * p3

    def parts(c):
        eps = p1 * p3 * c
        a = px ** 2 * (-4 * kappa + 8 * eps)
        b = px * (-p1 + eps / p1) * (8 * gam + 4 * Q + 8 * eps)
        cc = 4 * p3 ** 2 * px ** 2 * (1 - c * c) - (2 * (gam + eps) + Q) ** 2
        return a, b, cc

    def g(c):
        a, b, cc = parts(c)
        if b * b - 4 * a * cc < 0 or a >= 0:
            return 0.0
        return M2 * math.pi / math.sqrt(-a)

    grid = np.linspace(-1, 1, 20001)
    inside = np.array([g(c) > 0 for c in grid])
    if not inside.any():
        return 0.0
    edges = grid[np.flatnonzero(np.diff(inside.astype(int)) != 0)]
    pts = sorted(set([-1.0, 1.0] + list(edges)))
    total = 0.0
    for lo, hi in zip(pts[:-1], pts[1:]):
        val, _ = integrate.quad(g, lo, hi, limit=200, epsabs=0, epsrel=1e-12)
        total += val
    return total


def test_kinematic_function_matches_the_printed_integrand():
    """Closed-form F against numerical integration of the printed a, b, c, unequal masses, random momenta (the
    discontinuity is bracketed to the 1e-4 scan, so agreement is at that level where the window is cut)."""
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(60):
        m1, m2, m3, m4 = rng.uniform(0.2, 2.0, 4)
        p1, p3, p4 = rng.uniform(0.1, 4.0, 3)
        E1, E3, E4 = math.hypot(p1, m1), math.hypot(p3, m3), math.hypot(p4, m4)
        E2 = E3 + E4 - E1
        if E2 < m2:
            continue
        G = m1 ** 2 - m2 ** 2 + m3 ** 2 + m4 ** 2 + 2 * (E3 * E4 - E1 * E3 - E1 * E4)
        Fc = ob.lib().orc_kinematic_F(p1, p3, p4, G, 1.0)
        Fn = _paper_F_numeric(p1, p3, p4, E1, E3, E4, m1, m2, m3, m4)
        assert Fc == pytest.approx(Fn, rel=2e-3, abs=1e-6 * max(Fn, 1e-12)), (m1, m2, m3, m4, p1, p3, p4)
        checked += Fn > 0
    assert checked >= 10


def _w22(stat, n, q_min, q_max, f_fn, m=1.0, term=wl.TERMS_SPLIT):
    q = wl.log_nodes(q_min, q_max, n)
    sp = wl.Species("phi", stat, n, q_min, q_max, f_fn(q), m0=m)
    return wl.Workload("x", [sp], [wl.Process([0, 0], [0, 0], term_mode=term)])


def _exact_at(w, pred):
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    sel = [items[i] for i in range(n) if pred(items[i])]
    arr = (ob.Item * len(sel))(*sel)
    rc, I = ow.exact22(arr, len(sel))
    assert rc == 0
    return sel, I


@pytest.mark.parametrize("term", [0, 1])
def test_exact22_converges_to_independent_references(term):
    """Gain (BE) against the independent Gauss-Legendre evaluation of the same reduction, loss (MB) against the
    textbook two-body closed form: the trapezoid in ln q converges to the reference at order 1.5 to 2 (the kinematic
    function has square-root edges), so the error falls by 2^1.5 to 4 from 256 to 512 nodes, and stays within 1e-3
    at 512 nodes."""
    errs = {}
    for n in (256, 512):
        if term == 0:
            q_min, q_max = 0.01, 30.0
            w = _w22(wl.BOSE, n, q_min, q_max, lambda q: 0.8 / np.expm1(np.sqrt(q * q + 1.0) / 1.5))
        else:
            q_min, q_max = 1e-3, 40.0
            w = _w22(wl.MB, n, q_min, q_max, lambda q: np.exp(-np.sqrt(q * q + 1.0)))
        q = wl.log_nodes(q_min, q_max, n)
        # momenta where the energy-conserving band of the integrand (width ~ 2 p1 in p3) spans many grid spacings;
        # at p1 -> 0 the band narrows below the spacing and the rule degrades to first order
        nodes = [int(np.argmin(np.abs(q - x))) for x in (0.5, 1.5, 4.0)]
        sel, I = _exact_at(w, lambda it: it.term == term and it.eval_idx in nodes)
        for k, it in enumerate(sel):
            p1 = q[it.eval_idx]
            if term == 0:
                ref = pa.semi_analytic_gain(p1, lambda qq, E: 0.8 / np.expm1(np.asarray(E) / 1.5), 1.0, 1.0,
                                            q_lo=q_min, q_hi=q_max)
            else:
                ref = pa.mb_loss_closed_form(p1, math.exp(-math.hypot(p1, 1.0)),
                                             lambda p: math.exp(-math.hypot(p, 1.0)), 1.0, p2_max=q_max)
            errs.setdefault(nodes.index(it.eval_idx), []).append(abs(I[k] / ref - 1.0))
    for k, (e256, e512) in errs.items():
        assert e512 < 1e-3, (k, e256, e512)
        assert e256 / e512 > 2.5, (k, e256, e512)


@pytest.mark.parametrize("masses", [(1.0, 1.0), (1.0, 0.3)])
def test_exact22_detailed_balance_with_unequal_masses(masses):
    """A B -> A B style process written as two species (masses mA, mB) at a common equilibrium: the gain and loss
    terms agree to the quadrature error; a non-equilibrium f (negative control) breaks the balance."""
    mA, mB = masses
    n, q_min, q_max = 192, 0.01, 30.0
    q = wl.log_nodes(q_min, q_max, n)
    out = {}
    for eq in (True, False):
        fA = wl.f_equilibrium(q, mA, 1.0, wl.BOSE) * (1.0 if eq else (1.0 + 0.5 * np.exp(-q)))
        fB = wl.f_equilibrium(q, mB, 1.0, wl.BOSE)
        sp = [wl.Species("A", wl.BOSE, n, q_min, q_max, fA, m0=mA), wl.Species("B", wl.BOSE, n, q_min, q_max, fB, m0=mB)]
        w = wl.Workload("ab", sp, [wl.Process([0, 1], [0, 1])])
        ow = ob.OracleWorld(w)
        items, ni = ow.items()
        nodes = [int(np.argmin(np.abs(q - x))) for x in (0.5, 1.5, 4.0)]
        sel = [items[i] for i in range(ni) if items[i].species == 0 and items[i].side == 0
               and items[i].eval_idx in nodes]
        arr = (ob.Item * len(sel))(*sel)
        rc, I = ow.exact22(arr, len(sel))
        assert rc == 0
        by = {}
        for k, it in enumerate(sel):
            by.setdefault(it.eval_idx, {})[it.term] = I[k]
        out[eq] = by
    for j, gl in out[True].items():
        assert abs(gl[0] - gl[1]) <= 2e-3 * gl[1], (j, gl)
    assert max(abs(gl[0] - gl[1]) / gl[1] for gl in out[False].values()) > 0.05


def test_exact22_agrees_with_monte_carlo_at_narrow_width():
    """The Monte Carlo estimator converges to the exact-delta value as sigma_E -> 0 (within 4 sigma + the
    smearing bias + the trapezoid error)."""
    fbe = lambda q: 0.8 / np.expm1(np.sqrt(q * q + 1.0) / 1.5)
    w = _w22(wl.BOSE, 128, 0.01, 20.0, fbe)
    w.processes[0].sigma_E = 0.005
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    sel = [items[i] for i in range(n) if items[i].eval_idx in (50, 80)]
    arr = (ob.Item * len(sel))(*sel)
    rc, I = ow.exact22(arr, len(sel))
    assert rc == 0
    rc, r = ow.run_items(arr, len(sel), 1 << 17, 6)
    assert rc == 0
    for k in range(len(sel)):
        assert abs(r["Ibar"][k] - I[k]) <= 4 * r["sigma"][k] + 5e-3 * I[k], (k, r["Ibar"][k], I[k], r["sigma"][k])


def test_exact22_h_theorem_and_conservation():
    """Noise-free H theorem: for the non-thermal initial condition of Sec. V.A on a grid wide enough that
    collisions do not carry energy past its end, the exact-delta 2->2 operator's entropy production
    sum_j w_j C_j ln((1 + f_j) / f_j) is positive (14 % of its absolute scale), while its number and energy moments
    vanish to the quadrature error (trapezoid weights q^2 dq)."""
    n, q_min, q_max = 96, 0.02, 40.0
    q = wl.log_nodes(q_min, q_max, n)
    f0 = wl.f_fermi_step(q)
    w = wl.Workload("h", [wl.Species("phi", wl.BOSE, n, q_min, q_max, f0, m0=1.0)],
                    [wl.Process([0, 0], [0, 0], term_mode=wl.TERMS_NET)])
    ow = ob.OracleWorld(w)
    items, ni = ow.items()
    rc, I = ow.exact22(items, ni)
    assert rc == 0
    C, _ = ow.combine(items, ni, I, np.zeros(ni), 0)
    E = np.sqrt(q * q + 1.0)
    dq = np.zeros_like(q)
    dq[1:] += 0.5 * np.diff(q)
    dq[:-1] += 0.5 * np.diff(q)
    wq = q * q * dq
    rel = lambda v: (wq @ v) / (wq @ np.abs(v))
    assert rel(C * np.log1p(1.0 / f0)) > 0.1
    assert abs(rel(C)) < 1e-6
    assert abs(rel(E * C)) < 2e-2


def test_exact22_rejects_other_processes():
    w = wl.w23_be(n_grid=16, N=256, nitn=1)
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    rc, _ = ow.exact22(items, 1)
    assert rc == -1
