"""Pins of the oracle's vector-Jacobian product against central finite differences of the oracle's own
frozen-map estimator with common random numbers (same counters, same maps): the estimator is smooth in the
f table values, the masses and the coupling, so the difference quotient with h = 1e-6 (relative) agrees
with the analytic adjoint to ~1e-7."""
import numpy as np
import pytest

from oracle import binding as ob
from paper_2603_28848_amd import workloads as wl


def _loss(ow, items, n, coef, N, seed=3, epoch=2):
    rc, r = ow.run_items(items, n, N, 1, seed=seed, epoch=epoch, adapt=False, first_iter=0)
    assert rc == 0
    return float(np.dot(coef, r["I_it"][:, 0]))


def _setup(w, N):
    ow = ob.OracleWorld(w)
    items, n = ow.items()
    rng = np.random.default_rng(0)
    coef = rng.normal(size=n)
    rc, gf, gm, gl = ow.vjp(items, n, coef, N, 0, seed=3, epoch=2)
    assert rc == 0
    return ow, items, n, coef, gf, gm, gl


def _fd_f(ow, items, n, coef, N, s, j, h=1e-6):
    f = ow.f[s]
    f0 = f[j]
    f[j] = f0 * (1 + h)
    lp = _loss(ow, items, n, coef, N)
    f[j] = f0 * (1 - h)
    lm = _loss(ow, items, n, coef, N)
    f[j] = f0
    return (lp - lm) / (2 * h * f0)


def _world(shape, N):
    if shape.startswith("23be"):
        w = wl.w23_be(n_grid=20, q_min=0.05, q_max=8.0, sigma_E=0.05, N=N, nitn=1)
    elif shape.startswith("22mb_tail"):  # small q_max: the conserved momentum often leaves the grid (extrapolation)
        w = wl.w22_mb(n_grid=16, q_min=0.1, q_max=3.0, sigma_E=0.05, N=N, nitn=1)
    else:  # 2->4 FD with m(t) = 1 + 0.1 sin t
        w = wl.w24_fd(n_grid=16, q_min=0.05, q_max=6.0, sigma_E=0.05, N=N, nitn=1)
    rule = {"spline": wl.INTERP_SPLINE, "eqexact": wl.INTERP_EQEXACT}.get(shape.split("_")[-1], wl.INTERP_LINLOG)
    for s in w.species:
        s.interp = rule
    return w


@pytest.mark.parametrize("shape", ["23be", "22mb_tail", "23be_spline", "23be_eqexact", "22mb_tail_spline",
                                   "22mb_tail_eqexact"])
def test_vjp_f_matches_finite_differences(shape):
    """Through every interpolation rule of Sec. III.B: the spline's second derivatives tie each node to all others
    (the adjoint solves the transposed spline system), the equilibrium-exact rule interpolates log(1/f + eta)."""
    N = 1 << 11
    w = _world(shape, N)
    ow, items, n, coef, gf, gm, gl = _setup(w, N)
    ng = w.species[0].n_grid
    for j in (0, 2, 4, ng // 2, ng - 5, ng - 2, ng - 1):
        fd = _fd_f(ow, items, n, coef, N, 0, j)
        assert gf[j] == pytest.approx(fd, rel=2e-6, abs=1e-9 * np.max(np.abs(gf))), (j, gf[j], fd)


def test_vjp_mass_and_coupling_match_finite_differences():
    w = wl.w23_be(n_grid=20, q_min=0.05, q_max=8.0, sigma_E=0.05, N=1 << 11, nitn=1)
    N = 1 << 11
    ow, items, n, coef, gf, gm, gl = _setup(w, N)
    h = 1e-6
    sp = ow.sp[0]
    m0 = sp.m0
    sp.m0 = m0 + h
    lp = _loss(ow, items, n, coef, N)
    sp.m0 = m0 - h
    lm = _loss(ow, items, n, coef, N)
    sp.m0 = m0
    assert gm[0] == pytest.approx((lp - lm) / (2 * h), rel=1e-6)
    pr = ow.pr[0]
    lam = pr.coupling
    pr.coupling = lam + h
    lp = _loss(ow, items, n, coef, N)
    pr.coupling = lam - h
    lm = _loss(ow, items, n, coef, N)
    pr.coupling = lam
    assert gl[0] == pytest.approx((lp - lm) / (2 * h), rel=1e-7)
    # |M|^2 = lambda^2: dL/dlambda = 2 L / lambda exactly
    assert gl[0] == pytest.approx(2 * _loss(ow, items, n, coef, N) / lam, rel=1e-12)


def test_vjp_time_dependent_mass_fd():
    w = wl.w24_fd(n_grid=16, q_min=0.05, q_max=6.0, sigma_E=0.05, N=1 << 10, nitn=1)
    N = 1 << 10
    ow, items, n, coef, gf, gm, gl = _setup(w, N)
    h = 1e-6
    sp = ow.sp[0]
    m0 = sp.m0
    sp.m0 = m0 + h
    lp = _loss(ow, items, n, coef, N)
    sp.m0 = m0 - h
    lm = _loss(ow, items, n, coef, N)
    sp.m0 = m0
    assert gm[0] == pytest.approx((lp - lm) / (2 * h), rel=1e-6)


@pytest.mark.parametrize("shape", ["23be_eqexact", "24fd_eqexact", "23be_spline"])
def test_vjp_mass_matches_finite_differences_through_interpolation_rules(shape):
    """The equilibrium-exact rule interpolates in E between node energies sqrt((q_j/a)^2 + m^2), so m moves the
    nodes as well as the particle's own energy; the spline is in q and m does not enter it."""
    N = 1 << 10
    w = _world(shape, N)
    ow, items, n, coef, gf, gm, gl = _setup(w, N)
    h = 1e-6
    sp = ow.sp[0]
    m0 = sp.m0
    sp.m0 = m0 + h
    lp = _loss(ow, items, n, coef, N)
    sp.m0 = m0 - h
    lm = _loss(ow, items, n, coef, N)
    sp.m0 = m0
    assert gm[0] == pytest.approx((lp - lm) / (2 * h), rel=1e-6)


def test_spline_adjoint_is_the_transpose_of_the_spline_map():
    """The spline's second derivatives are linear in f: with the columns dM/df_j from the oracle's own spline solve
    of unit vectors, the adjoint of g equals (dM/df)^T g (to rounding), on the nonuniform logarithmic grid."""
    import ctypes as C
    L = ob.lib()
    n = 12
    q = np.exp(np.log(0.05) + np.arange(n) * (np.log(8.0) - np.log(0.05)) / (n - 1))
    dp = C.POINTER(C.c_double)
    L.orc_spline_second_derivatives.argtypes = [C.c_int, dp, dp, dp]
    L.orc_spline_adjoint.argtypes = [C.c_int, dp, dp, dp]
    J = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M = np.zeros(n)
        assert L.orc_spline_second_derivatives(n, q.ctypes.data_as(dp), e.ctypes.data_as(dp), M.ctypes.data_as(dp)) == 0
        J[:, j] = M
    g = np.random.default_rng(4).normal(size=n)
    out = np.zeros(n)
    assert L.orc_spline_adjoint(n, q.ctypes.data_as(dp), g.ctypes.data_as(dp), out.ctypes.data_as(dp)) == 0
    np.testing.assert_allclose(out, J.T @ g, rtol=1e-10, atol=1e-12 * np.max(np.abs(J.T @ g)))
