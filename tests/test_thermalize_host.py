"""Host logic of the thermalisation runner: the moments, the equilibrium fixed by them, and the Bose-Einstein fit."""
import numpy as np
import pytest

from paper_2603_28848_amd import thermalize as th
from paper_2603_28848_amd import workloads as wl


@pytest.mark.parametrize("T,mu", [(2.0, 0.5), (1.2, -0.3), (2.7, 0.0)])
def test_equilibrium_recovered_from_its_moments(T, mu):
    q = wl.log_nodes(0.1, 50.0, 272)
    f = wl.f_equilibrium(q, 1.0, T, wl.BOSE, mu)
    N, E = th.moments(q, f, 1.0)
    T2, mu2 = th.equilibrium_for(q, N, E, 1.0)
    assert T2 == pytest.approx(T, rel=1e-7) and mu2 == pytest.approx(mu, abs=1e-7)
    Tf, muf = th.fit_T_mu(q, f, 1.0)
    assert Tf == pytest.approx(T, rel=1e-10) and muf == pytest.approx(mu, abs=1e-9)
    if mu == 0.0:
        T3, mu3 = th.equilibrium_for(q, N, E, 1.0, mu_zero=True)
        assert T3 == pytest.approx(T, rel=1e-9) and mu3 == 0.0


def test_moments_match_quadrature_of_the_closed_forms():
    """MB with m = 0 on a wide grid: int p^2 e^{-p} dp = 2, int p^3 e^{-p} dp = 6."""
    q = wl.log_nodes(1e-4, 80.0, 2000)
    N, E = th.moments(q, np.exp(-q), 0.0)
    assert N == pytest.approx(2.0, rel=1e-5) and E == pytest.approx(6.0, rel=1e-5)
