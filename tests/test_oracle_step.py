"""Pins of the oracle's log-space time stepping (Sec. III.C): the adaptive step bounds the fractional
change of f by epsilon (Eq. 20); a 2->2 step conserves particle number and energy up to the Monte Carlo noise and
the grid's truncation, for Euler and Heun steps alike.  (The sign of the entropy change of one Monte Carlo step is
decided by the noise at these sample counts; the H theorem is pinned on the noise-free exact-delta operator.)"""
import numpy as np
import pytest

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _moments(w, f):
    sp = w.species[0]
    q = wl.log_nodes(sp.q_min, sp.q_max, sp.n_grid)
    E = np.sqrt(q * q + sp.m0 ** 2)
    dq = np.zeros_like(q)
    dq[1:] += 0.5 * np.diff(q)
    dq[:-1] += 0.5 * np.diff(q)
    s = (1 + f) * np.log1p(f) - f * np.log(f)
    return (q * q * dq) @ s, (q * q * dq) @ f, (E * q * q * dq) @ f


def _world():
    q = wl.log_nodes(0.02, 14.0, 48)
    f0 = wl.f_fermi_step(q)
    return wl.Workload("st", [wl.Species("phi", wl.BOSE, 48, 0.02, 14.0, f0, m0=1.0)],
                       [wl.Process([0, 0], [0, 0], sigma_E=0.02)])


@pytest.mark.parametrize("method", [0, 1])
def test_step_conserves_number_and_energy(method):
    """|dN/N| and |dE/E| stay below 3 % of the largest fractional change of f (over seeds 0..7 at 2^16 samples the
    largest ratio is 0.017; a C off by a factor E, or with a term dropped, gives ratios of order 0.4)."""
    w = _world()
    ow = ob.OracleWorld(w)
    f0 = ow.f[0].copy()
    S0, N0, E0 = _moments(w, f0)
    rc, dt = ow.step(method, -1.0, 0.1, 1e3, 1 << 16, 3)
    assert rc == 0 and dt > 0 and ow.t == pytest.approx(dt)
    S1, N1, E1 = _moments(w, ow.f[0])
    change = np.max(np.abs(np.log(ow.f[0] / f0)))
    assert change > 0.05
    assert abs(N1 / N0 - 1) < 0.03 * change and abs(E1 / E0 - 1) < 0.03 * change


def test_adaptive_step_bounds_fractional_change():
    w = _world()
    ow = ob.OracleWorld(w)
    f0 = ow.f[0].copy()
    rc, dt = ow.step(0, -1.0, 0.2, 1e3, 1 << 12, 2)
    assert rc == 0
    assert np.max(np.abs(np.log(ow.f[0]) - np.log(f0))) == pytest.approx(0.2, rel=1e-12)


def test_step_dt_max_and_fixed_dt():
    ow = ob.OracleWorld(_world())
    rc, dt = ow.step(1, -1.0, 0.3, 0.5, 1 << 11, 2)
    assert rc == 0 and dt == 0.5
    ow2 = ob.OracleWorld(_world())
    rc, dt = ow2.step(1, 0.25, 0.3, 100.0, 1 << 11, 2)
    assert rc == 0 and dt == 0.25 and ow2.t == 0.25


def test_heun_uses_same_dt_as_euler():
    """Both methods take dt from k1 = C[f(t)] (same counters, same maps), so the steps agree."""
    oe, oh = ob.OracleWorld(_world()), ob.OracleWorld(_world())
    f0 = oe.f[0].copy()
    rc, dte = oe.step(0, -1.0, 0.02, 1e3, 1 << 12, 2)
    rc2, dth = oh.step(1, -1.0, 0.02, 1e3, 1 << 12, 2)
    assert rc == 0 and rc2 == 0 and dte == dth
    assert not np.array_equal(oe.f[0], oh.f[0])


def test_step_rejects_invalid_state_and_keeps_f():
    w = _world()
    w.species[0].stat = wl.FERMI
    w.species[0].f = w.species[0].f * 0 + 1.2  # Fermi-Dirac occupation above 1
    ow = ob.OracleWorld(w)
    f0 = ow.f[0].copy()
    rc, dt = ow.step(1, -1.0, 0.3, 1.0, 1 << 10, 1)
    assert rc == -3
    assert np.array_equal(ow.f[0], f0) and ow.t == 0.0
