"""Pins of the oracle's Euler and Heun combinations (Sec. III.C, Eqs. 18-19) through their order of convergence.

With the deterministic exact-delta 2->2 operator (Sec. IV) in place of the Monte Carlo one, d log f/dt = C[f]/f is
an ordinary differential equation; with radiation-dominated expansion (Sec. III.E) it depends on t explicitly.  (The
expanding case uses massless particles: then energy conservation between comoving grid momenta does not depend on
a, the set of node pairs of the reduction stays fixed and C scales as a power of a, so the right-hand side stays
smooth in t, apart from rounding-level switches between the fit and the table at the grid's ends: node pairs
such as q_3 = q_1 put the dependent momentum on a node up to rounding, and at an end node the fit and the table
differ.  Those switches, of relative size 1e-8 here, leave the finest Heun runs a noise floor of a few 1e-6, so the
expanding case checks Heun's order on coarser steps.)
Integrated to a fixed time with n, 2n and 4n steps, the global error against a much finer Heun solution falls by
about 2 per halving of dt for Euler (first order) and about 4 for Heun (second order).

Mistakes this catches: the Heun average with dt in place of dt/2 (the scheme is then not consistent: no
convergence), k2 divided by f instead of the predictor f* or evaluated at t instead of t + dt (Heun drops to first
order), and an Euler step with the wrong sign or factor (no convergence to the Heun limit).  (A predictor taken
linearly, f + dt k1, in place of the log-space Euler step keeps second order and is not told apart here.)
"""
import numpy as np
import pytest

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _world(t0=None):
    """2->2 Bose-Einstein scalar, m = 1, 24 nodes on [0.05, 12]; with t0, massless on 32 nodes of [0.005, 40] (f at
    both ends far below its bulk) and radiation-dominated from t = t0 (a = 1)."""
    if t0 is None:
        n, lo, hi, m0 = 24, 0.05, 12.0, 1.0
    else:
        n, lo, hi, m0 = 32, 0.005, 40.0, 0.0
    f0 = wl.f_fermi_step(wl.log_nodes(lo, hi, n))
    w = wl.Workload("order", [wl.Species("phi", wl.BOSE, n, lo, hi, f0, m0=m0)],
                    [wl.Process([0, 0], [0, 0], sigma_E=0.02)])
    if t0 is not None:
        w.expansion, w.a0, w.t0, w.t = wl.EXP_RADIATION, 1.0, t0, t0
    return w


def _run(t0, method, n, T):
    ow = ob.OracleWorld(_world(t0))
    for _ in range(n):
        rc, dt = ow.step_exact22(method, T / n)
        assert rc == 0 and dt == T / n
    return np.log(ow.f[0])


@pytest.mark.parametrize("expansion", [False, True])
def test_euler_first_and_heun_second_order(expansion):
    ow = ob.OracleWorld(_world(1.0 if expansion else None))  # C at a = 1 does not depend on t0
    rc, C0 = ow.collision_exact22_all()
    assert rc == 0
    T = 0.5 / np.max(np.abs(C0 / ow.f[0]))  # log f moves by about 0.5 over the run
    t0 = T if expansion else None  # with expansion a grows from 1 to sqrt(2) over the run
    ref = _run(t0, 1, 512, T)
    steps = (8, 16, 32)
    err = {}
    for method in (0, 1):
        err[method] = [np.max(np.abs(_run(t0, method, n, T) - ref)) for n in steps]
    e_eu, e_he = err[0], err[1]
    assert e_eu[0] > 1e-3  # the run is long enough to resolve the schemes' errors
    r_eu = [e_eu[0] / e_eu[1], e_eu[1] / e_eu[2]]
    r_he = [e_he[0] / e_he[1], e_he[1] / e_he[2]]
    assert all(1.7 < r < 2.3 for r in r_eu), (e_eu, r_eu)
    if expansion:
        assert 3.4 < r_he[0] < 5.0 and r_he[1] > 2.5, (e_he, r_he)
    else:
        assert all(3.4 < r < 4.6 for r in r_he), (e_he, r_he)
    assert e_he[1] < 0.05 * e_eu[1]


def test_heun_step_size_from_k1_bounds_euler_change():
    """The adaptive dt of a Heun step is eps / max|k1/f| (Eq. 20): the Euler predictor moves log f by eps exactly
    at the fastest node, whatever k2 then does."""
    ow = ob.OracleWorld(_world())
    rc, C0 = ow.collision_exact22_all()
    f0 = ow.f[0].copy()
    rc, dt = ow.step_exact22(1, -1.0, eps=0.2)
    assert rc == 0
    assert dt == pytest.approx(0.2 / np.max(np.abs(C0 / f0)), rel=1e-15)
    assert ow.t == dt
