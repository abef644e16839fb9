"""Pins of the oracle's species tables, roles and statistical factor against what the paper fixes:
the extrapolation form is exact for equilibrium distributions (Sec. III.B), the interpolation rule is
exact for functions linear in ln q, the particle-role rules (Appendix A), the multiplicities
C_phi = 2 C_2 + 3 C_3 and 2 C_2 for phi phi <-> phi phi (Sec. II.C), and the gain / loss products
the paper prints for phi phi <-> phi phi phi (Sec. II.C, the C_2 and C_3 lists)."""
import math

import numpy as np
import pytest

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _world(species, processes, **kw):
    return ob.OracleWorld(wl.Workload("t", species, processes, **kw))


def _sp(stat, f_fn, n=64, q_min=0.01, q_max=30.0, m=1.0, **kw):
    q = wl.log_nodes(q_min, q_max, n)
    return wl.Species("s", stat, n, q_min, q_max, f_fn(q), m0=m, **kw)


# ------------------------------------------------------------------------------------------------ tables
def test_grid_nodes_logarithmic():
    ow = _world([_sp(wl.MB, lambda q: np.exp(-q), n=33, q_min=0.02, q_max=40.0)], [])
    q = ow.grid_q(0)
    assert q[0] == pytest.approx(0.02, rel=1e-15) and q[-1] == pytest.approx(40.0, rel=1e-14)
    r = q[1:] / q[:-1]
    assert np.allclose(r, (40.0 / 0.02) ** (1 / 32), rtol=1e-13)


def test_interpolation_exact_for_linear_in_log_q():
    c0, c1 = 2.0, -0.25
    ow = _world([_sp(wl.MB, lambda q: c0 + c1 * np.log(q), n=40, q_min=0.01, q_max=1.0)], [])
    rc, fit = ow.fit(0)
    rng = np.random.default_rng(0)
    for q in np.exp(rng.uniform(math.log(0.01), math.log(1.0), 200)):
        assert ow.f_at(0, fit, q, 1.0) == pytest.approx(c0 + c1 * math.log(q), rel=1e-13, abs=1e-13)


def test_interpolation_hits_nodes():
    ow = _world([_sp(wl.BOSE, lambda q: 0.3 / (1 + q * q), n=50)], [])
    rc, fit = ow.fit(0)
    q = ow.grid_q(0)
    f = ow.w.species[0].f
    for j in range(1, 49):
        assert ow.f_at(0, fit, q[j], 1.0) == pytest.approx(f[j], rel=1e-12)


@pytest.mark.parametrize("stat", [wl.BOSE, wl.FERMI, wl.MB])
@pytest.mark.parametrize("a,m,T,mu", [(1.0, 1.0, 1.0, 0.0), (1.7, 0.5, 0.8, 0.0), (1.0, 2.0, 1.3, -0.4),
                                      (1.0, 1.0, 2.0, 0.6)])
def test_extrapolation_exact_for_equilibrium(stat, a, m, T, mu):
    """log(1/f + eta) = (E - mu)/T exactly for f_eq, so the fit reproduces f_eq outside the grid."""
    if stat == wl.BOSE and mu >= m:
        pytest.skip("BE needs mu < m")
    n, q_min, q_max = 48, 0.05, 20.0
    q = wl.log_nodes(q_min, q_max, n)
    f = wl.f_equilibrium(q / a, m, T, stat, mu)
    t = 100.0 * a * a  # radiation domination with t0 = 100, a0 = 1 gives a(t) = a
    sp = wl.Species("s", stat, n, q_min, q_max, f, m0=m)
    ow = ob.OracleWorld(wl.Workload("t", [sp], [], t=t, expansion=wl.EXP_RADIATION, a0=1.0, t0=100.0))
    rc, fit = ow.fit(0)
    assert rc == 0
    assert fit[1] == pytest.approx(1.0 / T, rel=1e-9) and fit[3] == pytest.approx(1.0 / T, rel=1e-9)
    for qq in [1e-4, 0.01, 0.049, 20.5, 35.0, 60.0]:
        p = qq / a
        E = math.sqrt(p * p + m * m)
        want = wl.f_equilibrium(np.array([p]), m, T, stat, mu)[0]
        assert ow.f_at(0, fit, qq, E) == pytest.approx(want, rel=1e-12)


def test_fit_rejects_bad_tables():
    ok = _world([_sp(wl.FERMI, lambda q: 0.5 / (1 + np.exp(q - 3)))], [])
    assert ok.fit(0)[0] == 0
    fd_ge1 = _world([_sp(wl.FERMI, lambda q: np.where(q < 0.02, 1.0, 0.5 / (1 + np.exp(q - 3))))], [])
    assert fd_ge1.fit(0)[0] == -3
    nonpos = _world([_sp(wl.MB, lambda q: np.where(q > 25, 0.0, np.exp(-q)))], [])
    assert nonpos.fit(0)[0] == -3
    rising = _world([_sp(wl.MB, lambda q: np.exp(0.1 * q))], [])
    assert rising.fit(0)[0] == -3


# ------------------------------------------------------------------------------------------------ roles
def _proc(ins, outs, **kw):
    return wl.Process(list(ins), list(outs), **kw)


@pytest.mark.parametrize("ins,outs,a,side,want", [
    # 2->2 identical, symmetric: conserved on the observed side
    ((0, 0), (0, 0), 0, 0, (0, 1, [2, 3])),
    ((0, 0), (0, 0), 0, 1, (2, 3, [0, 1])),
    # 2->3: conserved on the fewer-particle (initial) side
    ((0, 0), (0, 0, 0), 0, 0, (0, 1, [2, 3, 4])),
    ((0, 0), (0, 0, 0), 0, 1, (2, 0, [1, 3, 4])),
    # 3->2: fewer-particle side is the final state
    ((0, 0, 0), (0, 0), 0, 0, (0, 3, [1, 2, 4])),
    ((0, 0, 0), (0, 0), 0, 1, (3, 4, [0, 1, 2])),
    # 2->4
    ((0, 0), (0, 0, 0, 0), 0, 1, (2, 0, [1, 3, 4, 5])),
    # 1->2 decay observed in the initial state: the only fewer-side slot is taken -> opposite side
    ((0,), (1, 1), 0, 0, (0, 1, [2])),
    ((0,), (1, 1), 1, 1, (1, 0, [2])),
    # mixed species: AA -> BB
    ((0, 0), (1, 1), 1, 1, (2, 3, [0, 1])),
    ((0, 0), (0, 0, 1, 1), 1, 1, (4, 0, [1, 2, 3, 5])),
])
def test_roles(ins, outs, a, side, want):
    sp = [_sp(wl.MB, lambda q: np.exp(-q)), _sp(wl.MB, lambda q: np.exp(-q))]
    ow = _world(sp, [_proc(ins, outs)])
    rc, io, ic, integ = ow.roles(0, a, side)
    assert rc == 0
    assert (io, ic, integ) == want


@pytest.mark.parametrize("ins,outs,mask,a,want", [
    ((0, 0), (0, 0), wl.SIDES_AUTO, 0, (2, 0)),       # phi phi <-> phi phi: 2 C_2 (one side)
    ((0, 0), (0, 0, 0), wl.SIDES_AUTO, 0, (2, 3)),    # phi phi <-> phi phi phi: 2 C_2 + 3 C_3
    ((0, 0), (0, 0, 0), wl.SIDES_OUT, 0, (0, 3)),     # C_3 only (the paper's incorrect variant)
    ((0, 0), (0, 0), wl.SIDES_BOTH, 0, (2, 2)),
    ((0, 0), (1, 1), wl.SIDES_AUTO, 0, (2, 0)),
    ((0, 0), (1, 1), wl.SIDES_AUTO, 1, (0, 2)),
    ((0, 1), (1, 0), wl.SIDES_AUTO, 1, (1, 0)),       # self-reverse with distinct species
    ((0, 0), (0, 0, 1, 1), wl.SIDES_AUTO, 0, (2, 2)),
])
def test_multiplicities(ins, outs, mask, a, want):
    sp = [_sp(wl.MB, lambda q: np.exp(-q)), _sp(wl.MB, lambda q: np.exp(-q))]
    ow = _world(sp, [_proc(ins, outs, side_mask=mask)])
    assert (ow.multiplicity(0, a, 0), ow.multiplicity(0, a, 1)) == want


def test_item_enumeration_and_uids():
    sp = [_sp(wl.MB, lambda q: np.exp(-q), n=20)]
    ow = _world(sp, [_proc((0, 0), (0, 0, 0), eval_stride=3)])
    items, n = ow.items()
    pts = list(range(0, 20, 3))
    assert n == 2 * 2 * len(pts)
    uids = [items[i].uid for i in range(n)]
    assert uids == sorted(uids)
    it = items[len(pts) * 3 + 1]  # side 1, term 1, second point
    assert (it.side, it.term, it.eval_idx, it.mult) == (1, 1, 3, 3)
    assert it.uid == (1 << 19) | (1 << 18) | 3


# -------------------------------------------------------------------------------- statistical factor
def test_stat_factor_matches_paper_lists_2to3():
    """phi phi <-> phi phi phi, positions 0..4 = (p, 2 | 3, 4, 5) in the paper's labels.  C_2: observed on
    the 2-particle side; C_3: observed on the 3-particle side (with the observed leg at position 2)."""
    f = np.array([0.31, 0.17, 0.23, 0.41, 0.07])
    eta = np.ones(5)
    fp, f2, f3, f4, f5 = f
    # C_2 (observed p at position 0, other initial particle f2)
    assert ob.stat_factor(2, 5, 0, wl.TERMS_SPLIT, 0, f, eta) == pytest.approx(f3 * f4 * f5 * (1 + fp) * (1 + f2), rel=1e-15)
    assert ob.stat_factor(2, 5, 0, wl.TERMS_SPLIT, 1, f, eta) == pytest.approx(fp * f2 * (1 + f3) * (1 + f4) * (1 + f5), rel=1e-15)
    # C_3 (observed at position 2; f1 f2 are positions 0, 1; f4 f5 are positions 3, 4)
    g = np.array([0.11, 0.29, 0.37, 0.05, 0.19])
    f1, f2b, fpb, f4b, f5b = g
    assert ob.stat_factor(2, 5, 1, wl.TERMS_SPLIT, 0, g, eta) == pytest.approx(f1 * f2b * (1 + fpb) * (1 + f4b) * (1 + f5b), rel=1e-15)
    assert ob.stat_factor(2, 5, 1, wl.TERMS_SPLIT, 1, g, eta) == pytest.approx(fpb * f4b * f5b * (1 + f1) * (1 + f2b), rel=1e-15)
    # NET is gain - loss
    net = ob.stat_factor(2, 5, 1, wl.TERMS_NET, 0, g, eta)
    assert net == pytest.approx(f1 * f2b * (1 + fpb) * (1 + f4b) * (1 + f5b) - fpb * f4b * f5b * (1 + f1) * (1 + f2b), rel=1e-14)


def test_stat_factor_fermi_and_mb():
    f = np.array([0.3, 0.2, 0.6, 0.1])
    assert ob.stat_factor(2, 4, 0, wl.TERMS_SPLIT, 0, f, -np.ones(4)) == pytest.approx(0.6 * 0.1 * 0.7 * 0.8)
    assert ob.stat_factor(2, 4, 0, wl.TERMS_SPLIT, 1, f, np.zeros(4)) == pytest.approx(0.3 * 0.2)


def test_equilibrium_detailed_balance_of_factor():
    """For f = 1/(e^{E/T} - eta) the ratio gain/loss = exp((sum_obs E - sum_opp E)/T) (per-leg
    f/(1 + eta f) = e^{-E/T}); with energy conservation gain = loss."""
    T = 1.3
    E = np.array([1.2, 2.5, 1.9, 1.8])  # E0 + E1 = E2 + E3
    for eta in (1.0, -1.0, 0.0):
        f = 1.0 / (np.exp(E / T) - eta)
        g = ob.stat_factor(2, 4, 0, wl.TERMS_SPLIT, 0, f, eta * np.ones(4))
        l = ob.stat_factor(2, 4, 0, wl.TERMS_SPLIT, 1, f, eta * np.ones(4))
        assert g == pytest.approx(l, rel=1e-13)
