"""Pins of the oracle's interpolation variants (Sec. III.B): the cubic spline in linear q against the library
not-a-knot spline, and the equilibrium-exact rule (log(1/f + eta) linear in E) against equilibrium closed forms."""
import numpy as np
import pytest
from scipy.interpolate import CubicSpline

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _world(interp, f_fn, n=40, q_min=0.05, q_max=12.0, m=1.0, stat=wl.BOSE, expansion=False):
    q = wl.log_nodes(q_min, q_max, n)
    sp = wl.Species("phi", stat, n, q_min, q_max, f_fn(q), m0=m, interp=interp)
    w = wl.Workload("interp", [sp], [wl.Process([0, 0], [0, 0])])
    if expansion:
        w.expansion, w.a0, w.t0, w.t = wl.EXP_RADIATION, 1.0, 1.0, 2.25  # a = 1.5
    return ob.OracleWorld(w), q


def _inside(q, k=400, seed=0):
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(q[0]), np.log(q[-1]), k))


def test_spline_matches_library_not_a_knot_spline():
    f_fn = lambda q: 0.8 / np.expm1(np.sqrt(q * q + 1.0) / 1.5) * (1 + 0.3 * np.sin(q))
    ow, q = _world(wl.INTERP_SPLINE, f_fn)
    rc, fit = ow.fit(0)
    assert rc == 0
    x = _inside(q)
    got = ow.f_batch(0, fit, x, np.sqrt(x * x + 1.0))
    want = CubicSpline(q, f_fn(q))(x)  # not-a-knot is the library default
    np.testing.assert_allclose(got, want, rtol=1e-11, atol=1e-13 * np.max(np.abs(want)))
    # the second derivatives themselves
    M = np.zeros(len(q))
    ob.lib().orc_spline_second_derivatives(len(q), ob._dp(np.ascontiguousarray(q)), ob._dp(f_fn(q)), ob._dp(M))
    np.testing.assert_allclose(M, CubicSpline(q, f_fn(q))(q, 2), rtol=1e-9, atol=1e-11 * np.max(np.abs(M)))


@pytest.mark.parametrize("interp", [wl.INTERP_LINLOG, wl.INTERP_SPLINE, wl.INTERP_EQEXACT])
def test_every_rule_passes_through_the_nodes(interp):
    f_fn = lambda q: np.exp(-np.sqrt(q * q + 1.0)) * (1.0 + 0.3 * np.exp(-q))
    ow, q = _world(interp, f_fn, stat=wl.MB)
    rc, fit = ow.fit(0)
    got = ow.f_batch(0, fit, q, np.sqrt(q * q + 1.0))
    np.testing.assert_allclose(got, f_fn(q), rtol=1e-13)


@pytest.mark.parametrize("stat,mu,expansion", [(wl.BOSE, -0.2, False), (wl.FERMI, 0.7, True), (wl.MB, 0.3, False)])
def test_eqexact_is_exact_for_equilibrium(stat, mu, expansion):
    """log(1/f + eta) = (E - mu) / T is linear in E, so the rule reproduces any equilibrium between the nodes
    (also with a = 1.5, where E_j = sqrt((q_j/a)^2 + m^2)); the linear-in-ln q rule does not (negative control)."""
    T, m = 0.8, 1.0
    a = 1.5 if expansion else 1.0
    f_fn = lambda q: wl.f_equilibrium(q / a, m, T, stat, mu)
    x = _inside(wl.log_nodes(0.05, 12.0, 40), seed=1)
    E = np.sqrt((x / a) ** 2 + m * m)
    exact = f_fn(x)
    for interp in (wl.INTERP_EQEXACT, wl.INTERP_LINLOG):
        ow, q = _world(interp, f_fn, stat=stat, expansion=expansion)
        rc, fit = ow.fit(0)
        assert rc == 0
        got = ow.f_batch(0, fit, x, E)
        err = np.max(np.abs(got / exact - 1.0))
        if interp == wl.INTERP_EQEXACT:
            assert err < 1e-12, err
        else:
            assert err > 1e-4, err


def test_eqexact_equilibrium_is_stationary_on_a_coarse_grid():
    """P1 with the equilibrium-exact rule on 24 nodes: BE 2->2 at equilibrium gives C within 4 sigma (+ 2e-4 of the
    gain term for the smearing bias) of zero, while the linear-in-ln q rule leaves an interpolation bias that the
    same run resolves at more than 5 sigma (negative control)."""
    n, q_min, q_max = 24, 0.05, 14.0
    q = wl.log_nodes(q_min, q_max, n)
    pts = (8, 12, 16)

    def run(interp, term_mode):
        sp = wl.Species("phi", wl.BOSE, n, q_min, q_max, wl.f_equilibrium(q, 1.0, 1.0, wl.BOSE), m0=1.0,
                        interp=interp)
        w = wl.Workload("eq", [sp], [wl.Process([0, 0], [0, 0], sigma_E=0.01, term_mode=term_mode)])
        ow = ob.OracleWorld(w)
        items, ni = ow.items()
        keep = [items[i] for i in range(ni) if items[i].eval_idx in pts and items[i].term == 0]
        arr = (ob.Item * len(keep))(*keep)
        rc, r = ow.run_items(arr, len(keep), 1 << 15, 4)
        assert rc == 0
        return r

    G = run(wl.INTERP_EQEXACT, wl.TERMS_SPLIT)["Ibar"]
    eq = run(wl.INTERP_EQEXACT, wl.TERMS_NET)
    lin = run(wl.INTERP_LINLOG, wl.TERMS_NET)
    for i in range(len(pts)):
        assert abs(eq["Ibar"][i]) <= 4 * eq["sigma"][i] + 2e-4 * G[i], (pts[i], eq["Ibar"][i], eq["sigma"][i])
        assert abs(lin["Ibar"][i]) > 5 * lin["sigma"][i], (pts[i], lin["Ibar"][i], lin["sigma"][i])

