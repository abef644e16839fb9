"""Seeded synthetic workloads (inputs only).

This module builds the *inputs* of a collision-integral evaluation -- species definitions, the values
of f on each species' grid, process definitions and Monte-Carlo settings -- for the workload shapes
used in tests and benchmarks.  It holds none of the estimator's arithmetic; both the HIP path and the
CPU reference receive the same plain numbers from here.

The shapes follow the paper's own workloads: logarithmic comoving grids, m = 1 scalars with constant
|M|^2 = lambda^2 = 1, non-thermal or near-equilibrium f (paper Sec. V.A), 2->2 / 2<->3 / 2->4 contact
processes, Gaussian delta widths of a few 1e-3 and Vegas with 50 bins per dimension and alpha = 0.5
(Appendix C).  There is no public dataset behind any of them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

BOSE, FERMI, MB = 1, -1, 0
MASS_CONST, MASS_SIN = 0, 1
EXP_NONE, EXP_RADIATION = 0, 1
TERMS_SPLIT, TERMS_NET = 0, 1
SIDES_AUTO, SIDES_IN, SIDES_OUT, SIDES_BOTH = 0, 1, 2, 3
WIDTH_ABS, WIDTH_REL = 0, 1
INTERP_LINLOG, INTERP_SPLINE, INTERP_EQEXACT = 0, 1, 2
M2_CONST, M2_POLY = 0, 1


@dataclasses.dataclass
class Species:
    name: str
    stat: int
    n_grid: int
    q_min: float
    q_max: float
    f: np.ndarray
    mass_kind: int = MASS_CONST
    m0: float = 1.0
    mA: float = 0.0
    mw: float = 0.0
    interp: int = INTERP_LINLOG


@dataclasses.dataclass
class Process:
    ins: List[int]
    outs: List[int]
    coupling: float = 1.0
    sigma_E: float = 0.01
    alpha: float = 0.5
    e_cut: float = 0.0
    n_bins: int = 50
    term_mode: int = TERMS_SPLIT
    side_mask: int = SIDES_AUTO
    eval_stride: int = 1
    n_samples: int = 10_000
    n_iter: int = 4
    width_mode: int = WIDTH_ABS  # WIDTH_REL: sigma_E is the fraction w of (E_in + E_out) / 2
    width_adapt: int = 0
    width_lo: float = 1e-3
    width_hi: float = 1e-2
    width_factor: float = 1.25
    width_min: float = 1e-4
    width_max: float = 0.2
    vegas_plus: int = 0          # 1: adaptive stratified sampling (VEGAS+) on top of the map
    beta: float = 0.75           # VEGAS+ allocation exponent
    m2_kind: int = M2_CONST      # M2_POLY: |M|^2 = coupling^2 P(s, t) with the coefficients below
    m2_coef: Tuple[float, ...] = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)  # c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2


@dataclasses.dataclass
class Workload:
    name: str
    species: List[Species]
    processes: List[Process]
    t: float = 0.0
    expansion: int = EXP_NONE
    a0: float = 1.0
    t0: float = 1.0
    seed: int = 0
    epoch: int = 0

    def copy(self) -> "Workload":
        return Workload(
            name=self.name,
            species=[dataclasses.replace(s, f=np.array(s.f, dtype=np.float64)) for s in self.species],
            processes=[dataclasses.replace(p, ins=list(p.ins), outs=list(p.outs)) for p in self.processes],
            t=self.t, expansion=self.expansion, a0=self.a0, t0=self.t0, seed=self.seed, epoch=self.epoch)


def log_nodes(q_min: float, q_max: float, n: int) -> np.ndarray:
    """Node positions used only to tabulate input functions of q."""
    return np.exp(np.log(q_min) + (np.log(q_max) - np.log(q_min)) / (n - 1) * np.arange(n))


def _energy(q, m):
    return np.sqrt(q * q + m * m)


def f_equilibrium(q, m, T, stat, mu=0.0):
    x = (_energy(q, m) - mu) / T
    if stat == BOSE:
        return 1.0 / np.expm1(x)
    if stat == FERMI:
        return 1.0 / (np.exp(x) + 1.0)
    return np.exp(-x)


def f_fermi_step(q, p0=3.0, w=2.0):
    """The paper's non-thermal initial condition 1 / (1 + exp((q - p0)/w)), p0 = 3, w = 2 (Sec. V.A)."""
    return 1.0 / (1.0 + np.exp((q - p0) / w))


def smoothed_noise(n: int, rng: np.random.Generator, width: float = 3.0, half: int = 9) -> np.ndarray:
    """iid N(0,1) per node, smoothed by a Gaussian kernel (sigma = `width` nodes, +-`half` nodes,
    reflecting ends) and rescaled to unit variance."""
    z = rng.standard_normal(n)
    k = np.exp(-0.5 * (np.arange(-half, half + 1) / width) ** 2)
    k /= k.sum()
    zp = np.pad(z, half, mode="reflect")
    s = np.convolve(zp, k, mode="valid")
    return s / s.std()


# --------------------------------------------------------------------------------------------------
# Workload shapes
# --------------------------------------------------------------------------------------------------

def w22_mb(n_grid=32, q_min=0.01, q_max=20.0, sigma_E=0.01, N=10_000, nitn=4) -> Workload:
    """2->2 single real scalar, m = 1, MB statistics, |M|^2 = 1, f = e^{-E}(1 + 0.3 e^{-q}) on a 32-point
    log grid in [0.01, 20], sigma_E = 0.01, 4 x 1e4 Vegas samples, 50 bins (6-dim)."""
    q = log_nodes(q_min, q_max, n_grid)
    f = np.exp(-_energy(q, 1.0)) * (1.0 + 0.3 * np.exp(-q))
    sp = Species("phi", MB, n_grid, q_min, q_max, f, m0=1.0)
    pr = Process([0, 0], [0, 0], coupling=1.0, sigma_E=sigma_E, n_samples=N, n_iter=nitn)
    return Workload("2to2_mb_m1_grid%d" % n_grid, [sp], [pr])


def w23_be(n_grid=128, q_min=0.01, q_max=30.0, sigma_E=0.005, N=1 << 18, nitn=10) -> Workload:
    """2<->3 single scalar, m = 1, BE statistics, |M|^2 = 1, f = 0.8 f_BE(T = 1.5) on a 128-point log grid
    in [0.01, 30], sigma_E = 0.005, 10 x 2^18 samples per point per side and term (9-dim)."""
    q = log_nodes(q_min, q_max, n_grid)
    f = 0.8 * f_equilibrium(q, 1.0, 1.5, BOSE)
    sp = Species("phi", BOSE, n_grid, q_min, q_max, f, m0=1.0)
    pr = Process([0, 0], [0, 0, 0], coupling=1.0, sigma_E=sigma_E, n_samples=N, n_iter=nitn)
    return Workload("2to3_be_m1_grid%d" % n_grid, [sp], [pr])


def w_multi(n_grid=256, q_min=0.01, q_max=30.0, sigma_E=0.005, N=(1 << 16, 1 << 18, 1 << 20), nitn=2,
            strides=(4, 2, 1), seed_noise=3) -> Workload:
    """Two coupled species (A: BE m = 1; B: FD m = 0.5), processes AA->BB (2->2), AA->AAA (2->3) and
    AA->AABB (2->4) with uneven sample counts and evaluation strides, radiation-dominated expansion
    (t0 = 100, a0 = 1), f = f_eq(T = 1) * clip(1 + 0.5 z, 0.1, 1.9) with z smoothed unit-variance noise."""
    q = log_nodes(q_min, q_max, n_grid)
    rng = np.random.default_rng(seed_noise)
    zA = smoothed_noise(n_grid, rng)
    zB = smoothed_noise(n_grid, rng)
    fA = f_equilibrium(q, 1.0, 1.0, BOSE) * np.clip(1.0 + 0.5 * zA, 0.1, 1.9)
    fB = f_equilibrium(q, 0.5, 1.0, FERMI) * np.clip(1.0 + 0.5 * zB, 0.1, 1.9)
    A = Species("A", BOSE, n_grid, q_min, q_max, fA, m0=1.0)
    B = Species("B", FERMI, n_grid, q_min, q_max, fB, m0=0.5)
    P1 = Process([0, 0], [1, 1], sigma_E=sigma_E, eval_stride=strides[0], n_samples=N[0], n_iter=nitn)
    P2 = Process([0, 0], [0, 0, 0], sigma_E=sigma_E, eval_stride=strides[1], n_samples=N[1], n_iter=nitn)
    P3 = Process([0, 0], [0, 0, 1, 1], sigma_E=sigma_E, eval_stride=strides[2], n_samples=N[2], n_iter=nitn)
    return Workload("multi_AB_22_23_24_grid%d" % n_grid, [A, B], [P1, P2, P3], t=100.0,
                    expansion=EXP_RADIATION, a0=1.0, t0=100.0)


def w23_adjoint(n_grid=256, q_min=0.1, q_max=50.0, sigma_E=0.005, N=1 << 20, nitn=1) -> Workload:
    """2<->3, BE, m = 1, lambda = 1 on the paper's 256-node log grid in [0.1, 50] with its non-thermal
    initial condition 1/(1 + e^{(q-3)/2})."""
    q = log_nodes(q_min, q_max, n_grid)
    f = f_fermi_step(q)
    sp = Species("phi", BOSE, n_grid, q_min, q_max, f, m0=1.0)
    pr = Process([0, 0], [0, 0, 0], coupling=1.0, sigma_E=sigma_E, n_samples=N, n_iter=nitn)
    return Workload("2to3_be_adjoint_grid%d" % n_grid, [sp], [pr])


def w24_fd(n_grid=512, q_min=0.005, q_max=40.0, sigma_E=0.002, N=1 << 22, nitn=8) -> Workload:
    """2->4 single FD scalar with m(t) = 1 + 0.1 sin t evaluated at t = 1, 512-node log grid in
    [0.005, 40], f = 1/(1 + e^{(q-3)/2}), sigma_E = 0.002, 8 x 2^22 samples (12-dim)."""
    q = log_nodes(q_min, q_max, n_grid)
    f = f_fermi_step(q)
    sp = Species("phi", FERMI, n_grid, q_min, q_max, f, mass_kind=MASS_SIN, m0=1.0, mA=0.1, mw=1.0)
    pr = Process([0, 0], [0, 0, 0, 0], coupling=1.0, sigma_E=sigma_E, n_samples=N, n_iter=nitn)
    return Workload("2to4_fd_msin_grid%d" % n_grid, [sp], [pr], t=1.0)


def total_samples(w: Workload, n_items_per_proc: List[int]) -> int:
    return int(sum(n * p.n_samples * p.n_iter for n, p in zip(n_items_per_proc, w.processes)))
