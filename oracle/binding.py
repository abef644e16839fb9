"""ctypes binding of the CPU FP64 reference (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark import this module.
It marshals a workload description into the plain C structures of oracle.h and calls liboracle.so.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

MAXD = 12


def build(force: bool = True) -> str:
    """Compiles oracle.c with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-fopenmp", "-fPIC", "-shared",
               os.path.join(_HERE, "oracle.c"), "-o", LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class Species(C.Structure):
    _fields_ = [("stat", C.c_int), ("n_grid", C.c_int), ("q_min", C.c_double), ("q_max", C.c_double),
                ("mass_kind", C.c_int), ("m0", C.c_double), ("mA", C.c_double), ("mw", C.c_double),
                ("f", C.POINTER(C.c_double)), ("interp", C.c_int), ("aux", C.POINTER(C.c_double))]


class Process(C.Structure):
    _fields_ = [("n_in", C.c_int), ("n_out", C.c_int), ("sp", C.c_int * 6), ("coupling", C.c_double),
                ("sigma_E", C.c_double), ("alpha", C.c_double), ("e_cut", C.c_double), ("n_bins", C.c_int),
                ("term_mode", C.c_int), ("side_mask", C.c_int), ("eval_stride", C.c_int), ("width_mode", C.c_int),
                ("width_adapt", C.c_int), ("width_lo", C.c_double), ("width_hi", C.c_double),
                ("width_factor", C.c_double), ("width_min", C.c_double), ("width_max", C.c_double),
                ("vegas_plus", C.c_int), ("beta", C.c_double), ("m2_kind", C.c_int), ("m2_c", C.c_double * 6)]


class World(C.Structure):
    _fields_ = [("n_species", C.c_int), ("species", C.POINTER(Species)), ("n_proc", C.c_int),
                ("procs", C.POINTER(Process)), ("t", C.c_double), ("expansion", C.c_int), ("a0", C.c_double),
                ("t0", C.c_double)]


class Item(C.Structure):
    _fields_ = [("proc", C.c_int), ("species", C.c_int), ("side", C.c_int), ("term", C.c_int),
                ("eval_idx", C.c_int), ("mult", C.c_int), ("uid", C.c_uint32), ("q_obs", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_sample_uniforms.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, C.c_int64, C.c_int, dp]
        L.orc_grid_q.argtypes = [C.POINTER(Species), C.c_int]
        L.orc_grid_q.restype = C.c_double
        L.orc_mass.argtypes = [C.POINTER(Species), C.c_double]
        L.orc_mass.restype = C.c_double
        L.orc_scale_factor.argtypes = [C.POINTER(World), C.c_double]
        L.orc_scale_factor.restype = C.c_double
        L.orc_fit.argtypes = [C.POINTER(Species), C.c_double, C.c_double, dp]
        L.orc_f_at.argtypes = [C.POINTER(Species), dp, C.c_double, C.c_double]
        L.orc_f_at.restype = C.c_double
        L.orc_f_batch.argtypes = [C.POINTER(Species), dp, C.c_int64, dp, dp, dp]
        L.orc_f_batch.restype = None
        L.orc_spline_second_derivatives.argtypes = [C.c_int, dp, dp, dp]
        L.orc_stat_factor.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, dp, dp]
        L.orc_stat_factor.restype = C.c_double
        L.orc_integrand_batch.argtypes = [C.POINTER(World), C.POINTER(Item), C.c_int64, dp, dp]
        L.orc_kinematic_F.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_kinematic_F.restype = C.c_double
        L.orc_exact22.argtypes = [C.POINTER(World), C.c_int, C.POINTER(Item), dp]
        L.orc_vplus_strata.argtypes = [C.c_int64, C.c_int]
        L.orc_point_width.argtypes = [C.POINTER(Process), C.c_int, dp]
        L.orc_point_width.restype = C.c_double
        L.orc_width_control.argtypes = [C.POINTER(Process), C.c_int, dp, dp, C.c_double]
        L.orc_width_control.restype = C.c_double
        L.orc_side_multiplicity.argtypes = [C.POINTER(Process), C.c_int, C.c_int]
        L.orc_roles.argtypes = [C.POINTER(Process), C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int)]
        L.orc_list_items.argtypes = [C.POINTER(World), C.c_int, C.c_int, C.c_int, C.POINTER(Item), C.c_int]
        L.orc_list_items_at.argtypes = [C.POINTER(World), C.c_int, C.c_int, C.POINTER(C.c_double), C.c_int,
                                        C.POINTER(Item), C.c_int]
        L.orc_map_uniform.argtypes = [C.POINTER(World), C.POINTER(Item), dp]
        L.orc_integrand_at.argtypes = [C.POINTER(World), C.POINTER(Item), dp, dp]
        L.orc_run_items.argtypes = [C.POINTER(World), C.c_int, C.POINTER(Item), C.c_int64, C.c_int, C.c_int,
                                    C.c_uint64, C.c_uint32, C.c_int, dp, dp, dp, dp, dp, C.c_int]
        L.orc_combine.argtypes = [C.POINTER(World), C.c_int, C.POINTER(Item), dp, dp, C.c_int, dp, dp]
        L.orc_combine.restype = None
        L.orc_collision_all.argtypes = [C.POINTER(World), C.c_int64, C.c_int, C.c_uint64, C.c_uint32, C.c_int, dp,
                                        dp, dp, C.c_int]
        L.orc_vjp.argtypes = [C.POINTER(World), C.c_int, C.POINTER(Item), dp, C.c_int64, C.c_int, C.c_uint64,
                              C.c_uint32, dp, dp, dp, dp, C.c_int]
        L.orc_step.argtypes = [C.POINTER(World), C.c_int, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int,
                               C.c_uint64, C.c_uint32, C.c_int, dp, dp, C.c_int]
        L.orc_item_dims.argtypes = [C.POINTER(World), C.POINTER(Item)]
        L.orc_items_sensitivity.argtypes = [C.c_void_p, C.c_int, C.POINTER(Item), C.c_int64, C.c_int, C.c_int,
                                            C.c_uint64, C.c_uint32, dp, dp, dp, C.c_int]
        L.orc_adapt_dim.argtypes = [dp, C.c_int, dp, dp, C.c_double]
        L.orc_adapt_dim.restype = None
        L.orc_collision_exact22_all.argtypes = [C.POINTER(World), dp, dp]
        L.orc_step_exact22.argtypes = [C.POINTER(World), C.c_int, C.c_double, C.c_double, C.c_double, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return list(o)


def stat_factor(n_in, n, obs_side, term_mode, term, f, eta):
    f = np.ascontiguousarray(f, dtype=np.float64)
    eta = np.ascontiguousarray(eta, dtype=np.float64)
    return lib().orc_stat_factor(n_in, n, obs_side, term_mode, term, _dp(f), _dp(eta))


def adapt_dim(edges, h, cnt, alpha):
    """The oracle's Vegas adaptation of one dimension: new edges from old edges (nb + 1), per-bin training sums h
    and counts cnt (nb each)."""
    e = np.ascontiguousarray(edges, dtype=np.float64).copy()
    h = np.ascontiguousarray(h, dtype=np.float64)
    c = np.ascontiguousarray(cnt, dtype=np.float64)
    assert e.size == h.size + 1 == c.size + 1
    lib().orc_adapt_dim(_dp(e), h.size, _dp(h), _dp(c), alpha)
    return e


def uniforms(seed, uid, epoch, it, n, D):
    y = np.zeros(D)
    lib().orc_sample_uniforms(seed, uid, epoch, it, n, D, _dp(y))
    return y


class OracleWorld:
    """A workload (paper_2603_28848_amd.workloads.Workload) held as oracle structures."""

    def __init__(self, w):
        self.w = w
        self.f = [np.ascontiguousarray(s.f, dtype=np.float64).copy() for s in w.species]
        self.aux = [np.zeros(s.n_grid) for s in w.species]  # spline second derivatives / node energies
        self.sp = (Species * len(w.species))()
        for i, s in enumerate(w.species):
            self.sp[i] = Species(s.stat, s.n_grid, s.q_min, s.q_max, s.mass_kind, s.m0, s.mA, s.mw, _dp(self.f[i]),
                                 s.interp, _dp(self.aux[i]))
        self.pr = (Process * max(1, len(w.processes)))()
        for i, p in enumerate(w.processes):
            sp = (C.c_int * 6)(*(list(p.ins) + list(p.outs) + [0] * (6 - len(p.ins) - len(p.outs))))
            self.pr[i] = Process(len(p.ins), len(p.outs), sp, p.coupling, p.sigma_E, p.alpha, p.e_cut, p.n_bins,
                                 p.term_mode, p.side_mask, p.eval_stride, p.width_mode, p.width_adapt, p.width_lo,
                                 p.width_hi, p.width_factor, p.width_min, p.width_max, p.vegas_plus, p.beta,
                                 p.m2_kind,
                                 (C.c_double * 6)(*p.m2_coef))
        self.world = World(len(w.species), self.sp, len(w.processes), self.pr, w.t, w.expansion, w.a0, w.t0)
        self._maps = None

    # ---- basic pieces ---------------------------------------------------------------------------
    @property
    def t(self):
        return self.world.t

    def fit(self, species, t=None):
        t = self.world.t if t is None else t
        a = lib().orc_scale_factor(C.byref(self.world), t)
        out = np.zeros(4)
        rc = lib().orc_fit(C.byref(self.sp[species]), a, t, _dp(out))
        return rc, out

    def f_at(self, species, fit, q, E):
        fit = np.ascontiguousarray(fit, dtype=np.float64)
        return lib().orc_f_at(C.byref(self.sp[species]), _dp(fit), q, E)

    def f_batch(self, species, fit, q, E):
        q = np.ascontiguousarray(q, dtype=np.float64)
        E = np.ascontiguousarray(E, dtype=np.float64)
        fit = np.ascontiguousarray(fit, dtype=np.float64)
        out = np.zeros_like(q)
        lib().orc_f_batch(C.byref(self.sp[species]), _dp(fit), q.size, _dp(q), _dp(E), _dp(out))
        return out

    def integrand_batch(self, item, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        n = x.shape[0]
        out = np.zeros(n)
        rc = lib().orc_integrand_batch(C.byref(self.world), C.byref(item), n, _dp(x), _dp(out))
        assert rc == 0, rc
        return out

    def grid_q(self, species):
        return np.array([lib().orc_grid_q(C.byref(self.sp[species]), j) for j in range(self.sp[species].n_grid)])

    def roles(self, proc, species, side):
        io, ic = C.c_int(), C.c_int()
        integ = (C.c_int * 6)()
        rc = lib().orc_roles(C.byref(self.pr[proc]), species, side, C.byref(io), C.byref(ic), integ)
        n = self.pr[proc].n_in + self.pr[proc].n_out
        return rc, io.value, ic.value, list(integ)[: n - 2]

    def multiplicity(self, proc, species, side):
        return lib().orc_side_multiplicity(C.byref(self.pr[proc]), species, side)

    def items(self, proc=-1, species=-1, stride=0):
        n = lib().orc_list_items(C.byref(self.world), proc, species, stride, None, 0)
        arr = (Item * max(1, n))()
        lib().orc_list_items(C.byref(self.world), proc, species, stride, arr, n)
        return arr, n

    def items_at(self, q, proc=-1, species=0):
        """Work items at evaluation momenta q (off the grid) of one species."""
        q = np.ascontiguousarray(q, dtype=np.float64)
        n = lib().orc_list_items_at(C.byref(self.world), proc, species, _dp(q), len(q), None, 0)
        arr = (Item * max(1, n))()
        lib().orc_list_items_at(C.byref(self.world), proc, species, _dp(q), len(q), arr, n)
        return arr, n

    def width_control(self, items, n_items, Ibar, sigma, proc):
        """The width of process proc after an evaluation with these item results (Appendix C controller); the
        oracle's process record is updated and the new width returned."""
        sel = [i for i in range(n_items) if items[i].proc == proc]
        Ib = np.ascontiguousarray(np.asarray(Ibar, dtype=np.float64)[sel])
        sg = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64)[sel])
        w = lib().orc_width_control(C.byref(self.pr[proc]), len(sel), _dp(Ib), _dp(sg), self.pr[proc].sigma_E)
        self.pr[proc].sigma_E = w
        return w

    def exact22(self, items, n_items):
        """Exact-delta estimates of 2->2 items (the semi-analytic reduction); (rc, I)."""
        I = np.zeros(max(1, n_items))
        rc = lib().orc_exact22(C.byref(self.world), n_items, items, _dp(I))
        return rc, I[:n_items]

    def point_width(self, proc, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        return lib().orc_point_width(C.byref(self.pr[proc]), len(E), _dp(E))

    def combine_at(self, items, n_items, Ibar, sigma, n_q):
        """C and sigma at the evaluation points of items_at: C = sum mult sign Ibar, sigma^2 = sum mult^2 sigma^2
        (Eq. 7; the loss term enters with a minus sign), item by item in order."""
        Cv, S = np.zeros(n_q), np.zeros(n_q)
        for i in range(n_items):
            it = items[i]
            sgn = -1.0 if (self.pr[it.proc].term_mode == 0 and it.term == 1) else 1.0
            Cv[it.eval_idx] += it.mult * sgn * Ibar[i]
            S[it.eval_idx] += it.mult * it.mult * sigma[i] * sigma[i]
        return Cv, np.sqrt(S)

    def integrand_at(self, item, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.zeros(1)
        rc = lib().orc_integrand_at(C.byref(self.world), C.byref(item), _dp(x), _dp(v))
        assert rc == 0, rc
        return v[0]

    def item_dims(self, item):
        return lib().orc_item_dims(C.byref(self.world), C.byref(item))

    def map_uniform(self, item, nb):
        m = np.zeros(MAXD * (nb + 1))
        lib().orc_map_uniform(C.byref(self.world), C.byref(item), _dp(m))
        return m

    # ---- Monte Carlo -----------------------------------------------------------------------------
    def run_items(self, items, n_items, N, nitn, seed=0, epoch=0, maps=None, threads=0, first_iter=0, adapt=True):
        nb = self.pr[items[0].proc].n_bins if n_items else 50
        stride = MAXD * (nb + 1)
        if maps is None:
            maps = np.full((n_items, stride), np.nan)
        I_it = np.zeros((n_items, nitn))
        V_it = np.zeros((n_items, nitn))
        Ib = np.zeros(n_items)
        sg = np.zeros(n_items)
        rc = lib().orc_run_items(C.byref(self.world), n_items, items, N, first_iter, nitn, seed, epoch, int(adapt),
                                 _dp(maps), _dp(I_it), _dp(V_it), _dp(Ib), _dp(sg), threads)
        return rc, dict(I_it=I_it, V_it=V_it, Ibar=Ib, sigma=sg, maps=maps)

    def sensitivity(self, items, n_items, N, nitn, seed=0, epoch=0, maps=None, first_iter=0, threads=0):
        """Per item and iteration on fixed maps (uniform if None): (B1, B2), the first-order bounds of another correct
        FP64 evaluation's difference in I and V per unit of relative rounding of the energies."""
        if maps is None:
            maps = np.stack([self.map_uniform(items[i], self.pr[items[i].proc].n_bins) for i in range(n_items)])
        maps = np.ascontiguousarray(maps, dtype=np.float64)
        B1 = np.zeros((n_items, nitn))
        B2 = np.zeros((n_items, nitn))
        rc = lib().orc_items_sensitivity(C.byref(self.world), n_items, items, N, first_iter, nitn, seed, epoch,
                                         _dp(maps), _dp(B1), _dp(B2), threads)
        assert rc == 0, rc
        return B1, B2

    def combine(self, items, n_items, Ibar, sigma, species):
        n = self.sp[species].n_grid
        Cv, S = np.zeros(n), np.zeros(n)
        lib().orc_combine(C.byref(self.world), n_items, items, _dp(np.ascontiguousarray(Ibar)),
                          _dp(np.ascontiguousarray(sigma)), species, _dp(Cv), _dp(S))
        return Cv, S

    def _all_maps(self, nb):
        n = lib().orc_list_items(C.byref(self.world), -1, -1, 0, None, 0)
        if self._maps is None or self._maps.shape[0] != n:
            self._maps = np.full((max(1, n), MAXD * (nb + 1)), np.nan)
        return self._maps

    def collision_all(self, N, nitn, seed=0, epoch=0, threads=0, adapt=True):
        nb = self.pr[0].n_bins
        maps = self._all_maps(nb)
        tot = sum(s.n_grid for s in self.w.species)
        Cv, S = np.zeros(tot), np.zeros(tot)
        rc = lib().orc_collision_all(C.byref(self.world), N, nitn, seed, epoch, int(adapt), _dp(maps), _dp(Cv), _dp(S),
                                     threads)
        return rc, Cv, S

    def vjp(self, items, n_items, coef, N, iter_=0, seed=0, epoch=0, maps=None, threads=0):
        """Gradients of sum_i coef_i I_i (frozen maps, one iteration): grad_f (all grids), grad_m, grad_lambda."""
        nb = self.pr[items[0].proc].n_bins
        stride = MAXD * (nb + 1)
        if maps is None:
            maps = np.full((n_items, stride), np.nan)
        maps = np.ascontiguousarray(maps, dtype=np.float64)
        coef = np.ascontiguousarray(coef, dtype=np.float64)
        tot = sum(s.n_grid for s in self.w.species)
        gf = np.zeros(tot)
        gm = np.zeros(len(self.w.species))
        gl = np.zeros(max(1, len(self.w.processes)))
        rc = lib().orc_vjp(C.byref(self.world), n_items, items, _dp(coef), N, iter_, seed, epoch, _dp(maps), _dp(gf),
                           _dp(gm), _dp(gl), threads)
        return rc, gf, gm, gl[: len(self.w.processes)]

    def collision_exact22_all(self):
        """(rc, C) of every species' grid by the exact-delta 2->2 operator."""
        tot = sum(s.n_grid for s in self.w.species)
        Cv, S = np.zeros(tot), np.zeros(tot)
        rc = lib().orc_collision_exact22_all(C.byref(self.world), _dp(Cv), _dp(S))
        return rc, Cv

    def step_exact22(self, method, dt, eps=0.3, dt_max=1e30):
        """One Euler (0) or Heun (1) step with the exact-delta 2->2 operator; (rc, dt used)."""
        dtu = np.zeros(1)
        rc = lib().orc_step_exact22(C.byref(self.world), method, dt, eps, dt_max, _dp(dtu))
        return rc, dtu[0]

    def step(self, method, dt, eps, dt_max, N, nitn, seed=0, epoch=0, threads=0, adapt=True):
        nb = self.pr[0].n_bins
        maps = self._all_maps(nb)
        dtu = np.zeros(1)
        rc = lib().orc_step(C.byref(self.world), method, dt, eps, dt_max, N, nitn, seed, epoch, int(adapt), _dp(maps),
                            _dp(dtu), threads)
        return rc, dtu[0]
