"""Independent reference values for the collision integral of 2->2 contact scattering.

These are *not* Monte-Carlo estimators and share no code with either implementation.  They pin the
normalisation and the gain/loss structure of the estimator:

* ``mb_loss_closed_form`` -- the loss term with the observed particle on the initial side for
  Maxwell-Boltzmann statistics (no 1 +- f factors on the final side) written with the textbook
  two-body phase space Phi_2(s) = sqrt(lambda(s, m^2, m^2)) / (8 pi s) = sqrt(1 - 4 m^2/s) / (8 pi):
      L(p1) = f1 lam^2 / (128 pi^3 E1) Int_0^inf dp2 (p2^2/E2) f2 Int_{-1}^{1} dc sqrt(1 - 4 m^2 / s),
      s = 2 m^2 + 2 (E1 E2 - p1 p2 c).
  The c integral is done in closed form with the antiderivative of sqrt(1 - a/s) in s.
* ``semi_analytic_gain`` -- the paper's semi-analytic backward (gain) term (Sec. IV Eq. 22 and
  Appendix B): exact energy conservation, E2 = E3 + E4 - E1, and the angular kinematic function
      F = Int dcos(theta) |M|^2 pi / sqrt(-a) Theta(b^2 - 4 a c),
  which for constant |M|^2 integrates in closed form.  With eps = p1 p3 c and kappa = p1^2 + p3^2,
  sqrt(-a) = 2 p4 sqrt(kappa - 2 eps) and b^2 - 4ac >= 0 reduces to
  (Q + 2 gamma + 2 eps)^2 <= 4 p4^2 (kappa - 2 eps), an interval [c_lo, c_hi] of c, so
      F = |M|^2 pi [sqrt(kappa - 2 p1 p3 c_lo) - sqrt(kappa - 2 p1 p3 c_hi)] / (2 p1 p3 p4).
  The remaining (p3, p4) integral is done by Gauss-Legendre panels on a logarithmic partition.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import integrate


def _c_integral_sqrt(p1, p2, E1, E2, m):
    """Int_{-1}^{1} dc sqrt(1 - 4 m^2 / s(c)), s = 2 m^2 + 2 (E1 E2 - p1 p2 c)."""
    a = 4.0 * m * m
    A = 2.0 * m * m + 2.0 * E1 * E2
    B = 2.0 * p1 * p2

    def G(s):
        s = max(s, a)
        return math.sqrt(s * (s - a)) - a * math.log(math.sqrt(s) + math.sqrt(s - a))

    s_hi, s_lo = A + B, A - B
    if B == 0.0:
        return 2.0 * math.sqrt(max(0.0, 1.0 - a / A))
    return (G(s_hi) - G(s_lo)) / B


def mb_loss_closed_form(p1, f1, f2_fn, m=1.0, lam=1.0, p2_max=60.0):
    E1 = math.hypot(p1, m)

    def integrand(p2):
        E2 = math.hypot(p2, m)
        return p2 * p2 / E2 * f2_fn(p2) * _c_integral_sqrt(p1, p2, E1, E2, m)

    val, _ = integrate.quad(integrand, 0.0, p2_max, limit=400, epsabs=0.0, epsrel=1e-10)
    return f1 * lam * lam / (128.0 * math.pi ** 3 * E1) * val


def kinematic_F(p1, p3, p4, E1, E3, E4, m, lam=1.0):
    """Closed-form angular kinematic function of the backward term for equal masses (vectorised in p3, p4)."""
    Q = 2.0 * m * m  # m1^2 - m2^2 + m3^2 + m4^2 with all masses equal
    gamma = E3 * E4 - E1 * E3 - E1 * E4
    kappa = p1 * p1 + p3 * p3
    u = p1 * p3
    K0 = Q + 2.0 * gamma
    disc = K0 + p4 * p4 + kappa
    ok = disc > 0.0
    sq = np.sqrt(np.where(ok, disc, 0.0))
    c_minus = (-(K0 + 2.0 * p4 * p4) - 2.0 * p4 * sq) / (2.0 * u)
    c_plus = (-(K0 + 2.0 * p4 * p4) + 2.0 * p4 * sq) / (2.0 * u)
    c_lo = np.maximum(-1.0, c_minus)
    c_hi = np.minimum(1.0, c_plus)
    ok = ok & (c_hi > c_lo)
    r_lo = np.sqrt(np.maximum(kappa - 2.0 * u * c_lo, 0.0))
    r_hi = np.sqrt(np.maximum(kappa - 2.0 * u * c_hi, 0.0))
    F = lam * lam * math.pi * (r_lo - r_hi) / (2.0 * p1 * p3 * p4)
    return np.where(ok, F, 0.0)


def _gl_log_panels(lo, hi, n_panels, order):
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.exp(np.linspace(math.log(lo), math.log(hi), n_panels + 1))
    pts, wts = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        pts.append(0.5 * (b - a) * x + 0.5 * (b + a))
        wts.append(0.5 * (b - a) * w)
    return np.concatenate(pts), np.concatenate(wts)


def semi_analytic_gain(p1, f_fn, eta, m=1.0, lam=1.0, q_lo=0.01, q_hi=20.0, n_panels=120, order=8):
    """Backward (gain) term of 2->2 at observed momentum p1 with integrated p3, p4 in [q_lo, q_hi]:
        C_BW = 2/(2 pi)^4 * 1/(2 E1) Int dp3 p3^2/(2 E3) Int dp4 p4^2/(2 E4) F f3 f4 (1 + eta f1)(1 + eta f2).
    f_fn(q, E) must accept arrays (E is the physical energy)."""
    E1 = math.hypot(p1, m)
    x, w = _gl_log_panels(q_lo, q_hi, n_panels, order)
    p3 = x[:, None]
    p4 = x[None, :]
    W = w[:, None] * w[None, :]
    E3 = np.sqrt(p3 * p3 + m * m)
    E4 = np.sqrt(p4 * p4 + m * m)
    E2 = E3 + E4 - E1
    allowed = E2 >= m
    p2 = np.sqrt(np.maximum(E2 * E2 - m * m, 0.0))
    F = kinematic_F(p1, p3, p4, E1, E3, E4, m, lam) * allowed
    f3 = f_fn(p3 * np.ones_like(p4), E3 * np.ones_like(p4))
    f4 = f_fn(p4 * np.ones_like(p3), E4 * np.ones_like(p3))
    f1 = f_fn(np.array([p1]), np.array([E1]))[0]
    f2 = f_fn(p2, np.where(allowed, E2, m))
    integrand = p3 * p3 / (2 * E3) * p4 * p4 / (2 * E4) * F * f3 * f4 * (1 + eta * f1) * (1 + eta * f2)
    return 2.0 / (2.0 * math.pi) ** 4 / (2.0 * E1) * float(np.sum(W * integrand))


def mb_loss_poly_closed_form(p1, f1, f2_fn, m=1.0, lam=1.0, coef=(1.0, 0, 0, 0, 0, 0), p2_max=60.0):
    """The MB loss term with |M|^2 = lam^2 P(s, t), P = c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2, equal masses.
    The final-state phase space is the two-body one, Phi_2(s) = sqrt(1 - 4 m^2 / s) / (8 pi), over which t is
    uniform in the centre-of-mass angle: t = A + B cos(theta*), A = 2 m^2 - s/2, B = s/2 - 2 m^2, so
    <t> = A and <t^2> = A^2 + B^2 / 3.  The (p2, c) integral is done numerically."""
    c0, c1, c2, c3, c4, c5 = coef
    E1 = math.hypot(p1, m)

    def G(s):
        A, B = 2 * m * m - 0.5 * s, 0.5 * s - 2 * m * m
        return c0 + c1 * s + c2 * A + c3 * s * s + c4 * s * A + c5 * (A * A + B * B / 3.0)

    def inner(p2):
        E2 = math.hypot(p2, m)

        def h(c):
            s = 2 * m * m + 2 * (E1 * E2 - p1 * p2 * c)
            return math.sqrt(max(0.0, 1.0 - 4 * m * m / s)) * G(s)

        v, _ = integrate.quad(h, -1.0, 1.0, epsabs=0.0, epsrel=1e-11)
        return p2 * p2 / E2 * f2_fn(p2) * v

    val, _ = integrate.quad(inner, 0.0, p2_max, limit=400, epsabs=0.0, epsrel=1e-9)
    return f1 * lam * lam / (128.0 * math.pi ** 3 * E1) * val
