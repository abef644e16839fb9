"""Thermalisation runs on the GPU path (Sec. V): a single scalar (m = 1, |M|^2 = lambda^2, H = 0) starts from the
non-thermal f0 = 1 / (1 + e^{(q - p0)/w}) on a logarithmic grid and evolves under phi phi -> phi phi or
phi phi <-> phi phi phi with log-space Heun steps of adaptive size; particle number and energy are recorded along
the way, and the end state is compared with the Bose-Einstein distribution fixed by the conserved quantities.

The moments are diagnostics on the host: N ~ int q^2 f dq and E ~ int q^2 E f dq by the trapezoidal rule in ln q
on the grid (their common factor 4 pi / (2 pi)^3 cancels in N/N0 and E/E0).

    python -m paper_2603_28848_amd.thermalize --process 2to2 --steps 400
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import Dict, List

import numpy as np

from . import workloads as wl


def moments(q: np.ndarray, f: np.ndarray, m: float, a: float = 1.0):
    """(N, E) ~ (int p^2 f dp, int p^2 E f dp) by the trapezoidal rule in ln q, p = q / a."""
    lq = np.log(q)
    h = lq[1] - lq[0]
    wt = np.full(len(q), h)
    wt[0] = wt[-1] = 0.5 * h
    p = q / a
    E = np.sqrt(p * p + m * m)
    w = wt * p ** 3  # dp = p dln q
    return float(np.sum(w * f)), float(np.sum(w * E * f))


def equilibrium_for(q: np.ndarray, N: float, E: float, m: float, mu_zero: bool = False):
    """(T, mu) of the Bose-Einstein distribution with the same N and E on the same grid and rule (mu = 0 fixes T by
    E alone: the number-changing process drives mu to 0)."""
    from scipy import optimize

    def mom(T, mu):
        return moments(q, wl.f_equilibrium(q, m, T, wl.BOSE, mu), m)

    if mu_zero:
        T = optimize.brentq(lambda T: mom(T, 0.0)[1] - E, 0.05, 50.0)
        return T, 0.0

    def res(x):
        T, mu = x[0], min(x[1], m - 1e-9)
        n, e = mom(T, mu)
        return [math.log(n / N), math.log(e / E)]

    sol = optimize.fsolve(res, [1.5, 0.0], full_output=True)
    T, mu = float(sol[0][0]), float(min(sol[0][1], m - 1e-9))
    return T, mu


def fit_T_mu(q: np.ndarray, f: np.ndarray, m: float, lo: float = 0.5, hi: float = 8.0):
    """Least-squares line log(1/f + 1) = (E - mu) / T over lo <= q <= hi (Bose-Einstein form)."""
    sel = (q >= lo) & (q <= hi)
    E = np.sqrt(q[sel] ** 2 + m * m)
    y = np.log(1.0 / f[sel] + 1.0)
    b, a0 = np.polyfit(E, y, 1)
    T = 1.0 / b
    return T, -a0 * T


def run(process: str = "2to2", n_grid: int = 272, q_min: float = 0.1, q_max: float = 50.0, m: float = 1.0,
        coupling: float = 1.0, sigma_E: float = 0.01, n_samples: int = 1 << 16, n_iter: int = 2, steps: int = 200,
        eps: float = 0.3, dt_max: float = 1e6, t_end: float = math.inf, side_mask: int = wl.SIDES_AUTO,
        precision: int = 1, seed: int = 0, record_every: int = 10, width_mode: int = wl.WIDTH_ABS,
        interp: int = wl.INTERP_LINLOG, term_mode: int = wl.TERMS_SPLIT, log=None) -> Dict:
    """Heun steps (adaptive dt = min(dt_max, eps / max|C/f|)) until `steps` or t_end; histories of t, N/N0, E/E0."""
    from . import boltzmc as bm

    q = wl.log_nodes(q_min, q_max, n_grid)
    f0 = wl.f_fermi_step(q)
    outs = [0, 0] if process == "2to2" else [0, 0, 0]
    sp = wl.Species("phi", wl.BOSE, n_grid, q_min, q_max, f0, m0=m, interp=interp)
    pr = wl.Process([0, 0], outs, coupling=coupling, sigma_E=sigma_E, n_samples=n_samples, n_iter=n_iter,
                    side_mask=side_mask, width_mode=width_mode, width_adapt=int(width_mode == wl.WIDTH_REL),
                    term_mode=term_mode)
    ctx = bm.from_workload(wl.Workload("thermalize_" + process, [sp], [pr]))
    N0, E0 = moments(q, f0, m)
    mid = (q >= 0.3) & (q <= 10.0)
    mu_zero = process != "2to2"

    def deviation(f):
        """max |log(f / f_eq)| over 0.3 <= q <= 10, f_eq fixed by the current N and E (mu = 0 for 2<->3)."""
        Nn, En = moments(q, f, m)
        T, mu = equilibrium_for(q, Nn, En, m, mu_zero=mu_zero)
        return float(np.max(np.abs(np.log(f[mid] / wl.f_equilibrium(q[mid], m, T, wl.BOSE, mu)))))

    hist: Dict[str, List[float]] = {"step": [0], "t": [0.0], "N": [1.0], "E": [1.0], "dt": [0.0],
                                    "dev": [deviation(f0)], "width": [ctx.get_width(0)]}
    t0 = time.perf_counter()
    t = 0.0
    stopped = ""
    retries = 0
    last_dt = 0.0
    for s in range(1, steps + 1):
        opts = bm.default_opts(seed=seed, epoch=2 * s, precision=precision)
        try:
            dt = ctx.step(bm.HEUN, -1.0, eps, dt_max, opts)
        except bm.BmcError as e:
            # the library restored f and t: the corrector left the valid range (a Monte Carlo outlier of k2 / f* in
            # the tail, which the k1-based step bound does not see); retry with fixed steps of half the last size
            dt, tries = 0.5 * last_dt, 0
            while dt > 0.0 and tries < 4:
                try:
                    ctx.step(bm.HEUN, dt, eps, dt_max, opts)
                    break
                except bm.BmcError:
                    dt, tries = 0.5 * dt, tries + 1
            else:
                stopped = "step %d: %s" % (s, e)
                if log:
                    log("stopped at " + stopped)
                break
            retries += 1
        last_dt = dt
        t += dt
        if s % record_every == 0 or s == steps or t >= t_end:
            f = ctx.get_f(0, n_grid)
            Nn, En = moments(q, f, m)
            dev = deviation(f)
            wd = ctx.get_width(0)
            for k, v in (("step", s), ("t", t), ("N", Nn / N0), ("E", En / E0), ("dt", dt), ("dev", dev),
                         ("width", wd)):
                hist[k].append(v)
            if log:
                log("step %d t %.4g dt %.3g N/N0 %.5f E/E0 %.5f dev %.4f width %.4g" % (
                    s, t, dt, Nn / N0, En / E0, dev, wd))
        if t >= t_end:
            break
    f = ctx.get_f(0, n_grid)
    Nn, En = moments(q, f, m)
    T_eq, mu_eq = equilibrium_for(q, Nn, En, m, mu_zero=mu_zero)
    T_fit, mu_fit = fit_T_mu(q, f, m)
    return {
        "process": process, "stopped": stopped, "retried_steps": retries, "side_mask": side_mask, "term_mode": term_mode, "interp": interp, "n_grid": n_grid, "n_samples": n_samples,
        "n_iter": n_iter,
        "sigma_E": sigma_E, "eps": eps, "steps": hist["step"][-1], "t": t, "wall_s": time.perf_counter() - t0,
        "N_over_N0": Nn / N0, "E_over_E0": En / E0, "T_eq": T_eq, "mu_eq": mu_eq, "T_fit": T_fit, "mu_fit": mu_fit,
        "max_log_dev_from_eq": deviation(f), "initial_max_log_dev": hist["dev"][0], "width_end": ctx.get_width(0),
        "max_abs_E_drift": float(np.max(np.abs(np.array(hist["E"]) - 1.0))),
        "max_abs_N_drift": float(np.max(np.abs(np.array(hist["N"]) - 1.0))),
        "history": hist, "f": f.tolist(), "q": q.tolist(),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--process", choices=["2to2", "2to3"], default="2to2")
    ap.add_argument("--n-grid", type=int, default=272)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--samples", type=int, default=1 << 16)
    ap.add_argument("--iters", type=int, default=2)
    ap.add_argument("--eps", type=float, default=0.3)
    ap.add_argument("--t-end", type=float, default=math.inf)
    ap.add_argument("--dt-max", type=float, default=1e6)
    ap.add_argument("--net", action="store_true", help="gain - loss with one integrator per point (TERMS_NET)")
    ap.add_argument("--interp", choices=["linlog", "spline", "eqexact"], default="linlog")
    ap.add_argument("--sigma-e", type=float, default=0.01)
    ap.add_argument("--c3-only", action="store_true", help="2<->3: the final side alone (3 C_3), the incorrect sum")
    ap.add_argument("--rel-width", action="store_true", help="relative width w (E_in + E_out)/2 with its controller")
    ap.add_argument("--precision", type=int, default=1, help="0 FP64, 1 FP32 integrand")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--record-every", type=int, default=10)
    ap.add_argument("--out", default="")
    a = ap.parse_args()
    res = run(a.process, n_grid=a.n_grid, n_samples=a.samples, n_iter=a.iters, steps=a.steps, eps=a.eps,
              sigma_E=a.sigma_e, side_mask=wl.SIDES_OUT if a.c3_only else wl.SIDES_AUTO,
              record_every=a.record_every, precision=a.precision, seed=a.seed, t_end=a.t_end, dt_max=a.dt_max,
              term_mode=wl.TERMS_NET if a.net else wl.TERMS_SPLIT,
              interp={"linlog": wl.INTERP_LINLOG, "spline": wl.INTERP_SPLINE, "eqexact": wl.INTERP_EQEXACT}[a.interp],
              width_mode=wl.WIDTH_REL if a.rel_width else wl.WIDTH_ABS, log=lambda s: print(s, flush=True))
    summary = {k: v for k, v in res.items() if k not in ("history", "f", "q")}
    print(json.dumps(summary), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(res, fh)


if __name__ == "__main__":
    main()
