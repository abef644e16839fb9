"""Python binding of libboltzmc (include/boltzmc.h): argument marshalling only.

Every evaluation runs in the HIP kernels of libboltzmc.so; this module loads that library (and fails
loudly if it is missing), passes plain pointers and sizes through ctypes, and uses PyTorch only to
allocate the device workspace and to name the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

from . import workloads as wl

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libboltzmc.so")

OK, EINVAL, ESTATE, ERANGE, ENOMEM, EHIP, EUNSUP = 0, -1, -2, -3, -4, -5, -6
MEM_HOST, MEM_DEVICE = 0, 1
FP64, FP32I = 0, 1
WIDTH_ABS, WIDTH_REL = 0, 1
INTERP_LINLOG, INTERP_SPLINE, INTERP_EQEXACT = 0, 1, 2
LAUNCH_BATCHED, LAUNCH_PLAIN = 0, 1
EULER, HEUN = 0, 1
MAXD, MAXITER = 12, 64


class ProcessParams(C.Structure):
    _fields_ = [("coupling", C.c_double), ("sigma_E", C.c_double), ("alpha", C.c_double), ("e_cut", C.c_double),
                ("n_bins", C.c_int), ("term_mode", C.c_int), ("side_mask", C.c_int), ("eval_stride", C.c_int),
                ("n_samples", C.c_int64), ("n_iter", C.c_int), ("width_mode", C.c_int), ("width_adapt", C.c_int),
                ("width_lo", C.c_double), ("width_hi", C.c_double), ("width_factor", C.c_double),
                ("width_min", C.c_double), ("width_max", C.c_double), ("vegas_plus", C.c_int), ("beta", C.c_double),
                ("m2_kind", C.c_int),
                ("m2_coef", C.c_double * 6)]


class RunOpts(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("n_iter", C.c_int), ("first_iter", C.c_int), ("seed", C.c_uint64),
                ("epoch", C.c_uint32), ("precision", C.c_int), ("launch", C.c_int), ("freeze_maps", C.c_int),
                ("eval_stride", C.c_int), ("eval_q", C.c_void_p), ("n_eval", C.c_int)]


class BmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("boltzmc error %d: %s" % (code, msg))
        self.code = code


_lib = None

_SIGS = {
    "bmc_create": [C.POINTER(C.c_void_p), C.c_int, C.c_void_p],
    "bmc_destroy": [C.c_void_p],
    "bmc_set_stream": [C.c_void_p, C.c_void_p],
    "bmc_workspace_query": [C.c_void_p, C.c_int64, C.c_int, C.POINTER(C.c_size_t)],
    "bmc_workspace_bind": [C.c_void_p, C.c_void_p, C.c_size_t],
    "bmc_add_species": [C.c_void_p, C.c_char_p, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                        C.POINTER(C.c_int)],
    "bmc_set_mass": [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double],
    "bmc_set_f": [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int],
    "bmc_get_f": [C.c_void_p, C.c_int, C.c_void_p, C.c_int, C.c_int],
    "bmc_add_process": [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_int), C.c_int,
                        C.POINTER(ProcessParams), C.POINTER(C.c_int)],
    "bmc_default_process_params": [C.POINTER(ProcessParams)],
    "bmc_set_coupling": [C.c_void_p, C.c_int, C.c_double],
    "bmc_set_interp": [C.c_void_p, C.c_int, C.c_int],
    "bmc_collision_noalloc": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_int],
    "bmc_collision_exact22": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_int],
    "bmc_get_width": [C.c_void_p, C.c_int, C.POINTER(C.c_double)],
    "bmc_set_width": [C.c_void_p, C.c_int, C.c_double],
    "bmc_set_expansion": [C.c_void_p, C.c_int, C.c_double, C.c_double],
    "bmc_set_time": [C.c_void_p, C.c_double],
    "bmc_get_time": [C.c_void_p, C.POINTER(C.c_double)],
    "bmc_plan_size": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.POINTER(C.c_int), C.POINTER(C.c_int)],
    "bmc_collision": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.c_void_p, C.c_void_p, C.c_size_t,
                      C.c_int],
    "bmc_item_results": [C.c_void_p, C.POINTER(C.c_uint32), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_int, C.c_int],
    "bmc_maps_get": [C.c_void_p, C.POINTER(C.c_uint32), C.c_int, C.c_void_p],
    "bmc_maps_set": [C.c_void_p, C.POINTER(C.c_uint32), C.c_int, C.c_void_p],
    "bmc_maps_reset": [C.c_void_p, C.c_int],
    "bmc_step": [C.c_void_p, C.c_int, C.c_double, C.c_double, C.c_double, C.POINTER(RunOpts),
                 C.POINTER(C.c_double)],
    "bmc_graph_capture_steps": [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                C.POINTER(RunOpts)],
    "bmc_graph_replay": [C.c_void_p],
    "bmc_graph_status": [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)],
    "bmc_vjp": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p,
                C.c_void_p, C.c_int],
    "bmc_set_timing": [C.c_void_p, C.c_int],
    "bmc_get_timing": [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)],
    "bmc_get_kernel_timing": [C.c_void_p, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double),
                              C.POINTER(C.c_int)],
    "bmc_get_sample_stats": [C.c_void_p, C.c_int, C.POINTER(C.c_int64)],
    "bmc_state_size": [C.c_void_p, C.POINTER(C.c_size_t)],
    "bmc_state_get": [C.c_void_p, C.c_void_p, C.c_size_t],
    "bmc_state_set": [C.c_void_p, C.c_void_p, C.c_size_t],
    "bmc_set_launch_tuning": [C.c_void_p, C.c_int, C.c_int],
    "bmc_autotune": [C.c_void_p, C.c_int, C.c_int, C.POINTER(RunOpts), C.POINTER(C.c_int), C.POINTER(C.c_int),
                     C.POINTER(C.c_double)],
    "bmc_last_error": [C.c_void_p],
    "bmc_version": [],
}


def lib():
    """The loaded libboltzmc.so.  Raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libboltzmc.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2603_28848_amd.build)")
        L = C.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.bmc_last_error.restype = C.c_char_p
        L.bmc_version.restype = C.c_char_p
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(C.c_void_p)
    return C.c_void_p(a.data_ptr())  # torch tensor


def default_opts(**kw) -> RunOpts:
    o = RunOpts(0, 0, 0, 0, 0, FP64, LAUNCH_BATCHED, 0, 0)
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Context:
    """Owns one bmc_ctx and its torch-allocated workspace."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        self._check(lib().bmc_create(C.byref(h), device, C.c_void_p(stream.cuda_stream)), None)
        self.h = h
        self.ws = None
        self.ws_bytes = 0

    def _check(self, rc, h="self"):
        if rc != OK:
            hh = self.h if h == "self" else h
            msg = lib().bmc_last_error(hh).decode() if hh is not None else ""
            raise BmcError(rc, msg)

    def close(self):
        if getattr(self, "h", None) is not None:
            lib().bmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- model -----------------------------------------------------------------------------------
    def add_species(self, name, stat, n_grid, q_min, q_max):
        sid = C.c_int()
        self._check(lib().bmc_add_species(self.h, name.encode(), stat, 0, n_grid, q_min, q_max, C.byref(sid)))
        self._n_f = getattr(self, "_n_f", 0) + n_grid
        self._n_species = getattr(self, "_n_species", 0) + 1
        self.grids = getattr(self, "grids", []) + [n_grid]
        self.masses = getattr(self, "masses", []) + [(0, 0.0, 0.0, 0.0)]
        return sid.value

    def set_mass(self, species, kind, m0, A=0.0, w=0.0):
        self._check(lib().bmc_set_mass(self.h, species, kind, m0, A, w))
        self.masses[species] = (kind, m0, A, w)

    def set_f_all(self, f):
        """f of every species, concatenated in species order (host array or device tensor)."""
        o = 0
        for s, n in enumerate(self.grids):
            self.set_f(s, f[o:o + n])
            o += n

    def get_f_all(self):
        return np.concatenate([self.get_f(s, n) for s, n in enumerate(self.grids)])

    def set_f(self, species, f):
        """f of one species from a host array or a torch tensor.  The library reads FP64 device memory: a tensor of
        another dtype, on the host or another device, or not contiguous is first copied to a contiguous FP64 tensor
        on the context's device (bmc_set_f is synchronous, so the copy lives long enough)."""
        if hasattr(f, "data_ptr"):
            t = self.torch
            if (f.dtype != t.float64 or f.device.type != "cuda" or f.device.index != self.device
                    or not f.is_contiguous()):
                f = f.detach().to(device="cuda:%d" % self.device, dtype=t.float64).contiguous()
            self._check(lib().bmc_set_f(self.h, species, _ptr(f), f.numel(), MEM_DEVICE))
        else:
            f = np.ascontiguousarray(f, dtype=np.float64)
            self._check(lib().bmc_set_f(self.h, species, _ptr(f), f.size, MEM_HOST))

    def get_f(self, species, n):
        out = np.zeros(n)
        self._check(lib().bmc_get_f(self.h, species, _ptr(out), n, MEM_HOST))
        return out

    def add_process(self, ins, outs, **params):
        p = ProcessParams()
        lib().bmc_default_process_params(C.byref(p))
        for k, v in params.items():
            setattr(p, k, v)
        a = (C.c_int * len(ins))(*ins)
        b = (C.c_int * len(outs))(*outs)
        pid = C.c_int()
        self._check(lib().bmc_add_process(self.h, a, len(ins), b, len(outs), C.byref(p), C.byref(pid)))
        self._n_proc = getattr(self, "_n_proc", 0) + 1
        return pid.value

    def set_coupling(self, process, coupling):
        self._check(lib().bmc_set_coupling(self.h, process, coupling))

    def set_interp(self, species, mode):
        self._check(lib().bmc_set_interp(self.h, species, mode))

    def get_width(self, process):
        w = C.c_double()
        self._check(lib().bmc_get_width(self.h, process, C.byref(w)))
        return w.value

    def set_width(self, process, width):
        self._check(lib().bmc_set_width(self.h, process, width))

    def set_expansion(self, kind, a0=1.0, t0=1.0):
        self._check(lib().bmc_set_expansion(self.h, kind, a0, t0))

    def set_time(self, t):
        self._check(lib().bmc_set_time(self.h, t))

    def get_time(self):
        t = C.c_double()
        self._check(lib().bmc_get_time(self.h, C.byref(t)))
        return t.value

    # ---- workspace -------------------------------------------------------------------------------
    def ensure_workspace(self, max_samples=0, max_iter=0):
        need = C.c_size_t()
        self._check(lib().bmc_workspace_query(self.h, max_samples, max_iter, C.byref(need)))
        if self.ws is None or need.value > self.ws_bytes:
            ws = self.torch.empty(int(need.value), dtype=self.torch.uint8, device="cuda:%d" % self.device)
            self._check(lib().bmc_workspace_bind(self.h, C.c_void_p(ws.data_ptr()), int(need.value)))
            self.ws = ws
            self.ws_bytes = int(need.value)

    # ---- evaluation ------------------------------------------------------------------------------
    def plan_size(self, process=-1, species=-1, opts: Optional[RunOpts] = None):
        opts = opts or default_opts()
        ni, no = C.c_int(), C.c_int()
        self._check(lib().bmc_plan_size(self.h, process, species, C.byref(opts), C.byref(ni), C.byref(no)))
        return ni.value, no.value

    def collision(self, process=-1, species=-1, opts: Optional[RunOpts] = None, out=None, sigma=None, eval_q=None):
        """C and sigma as host arrays (or into the given device tensors); with eval_q, at those comoving momenta
        of the one selected species instead of on its grid."""
        opts = opts or default_opts()
        if eval_q is not None:
            q = np.ascontiguousarray(eval_q, dtype=np.float64)
            opts = RunOpts.from_buffer_copy(opts)
            opts.eval_q = q.ctypes.data
            opts.n_eval = q.size
            self._eval_q_keep = q  # the library reads the points during the calls below
        ni, no = self.plan_size(process, species, opts)
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        self._last_items = ni
        if out is not None:
            for name, t in (("out", out), ("sigma", sigma)):
                if t is None:
                    continue
                if (not hasattr(t, "data_ptr") or t.dtype != self.torch.float64 or t.device.type != "cuda"
                        or t.device.index != self.device or not t.is_contiguous() or t.numel() < no):
                    raise ValueError("%s must be a contiguous float64 tensor of at least %d values on cuda:%d"
                                     % (name, no, self.device))
            self._check(lib().bmc_collision(self.h, process, species, C.byref(opts), _ptr(out), _ptr(sigma), no,
                                            MEM_DEVICE))
            return out, sigma
        Cv, S = np.zeros(no), np.zeros(no)
        self._check(lib().bmc_collision(self.h, process, species, C.byref(opts), _ptr(Cv), _ptr(S), no, MEM_HOST))
        return Cv, S

    def collision_noalloc(self, process=-1, species=-1, opts: Optional[RunOpts] = None):
        """C and sigma (host arrays) from the allocation-free entry point: per-call scratch in the library's static
        device array; the bound workspace holds only the persistent state."""
        opts = opts or default_opts()
        ni, no = self.plan_size(process, species, opts)
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        Cv, S = np.zeros(no), np.zeros(no)
        self._check(lib().bmc_collision_noalloc(self.h, process, species, C.byref(opts), _ptr(Cv), _ptr(S), no,
                                                MEM_HOST))
        return Cv, S

    def collision_exact22(self, process=-1, species=-1, opts: Optional[RunOpts] = None, eval_q=None):
        """C of 2->2 processes by the exact-delta reduction (host arrays; sigma is 0)."""
        opts = opts or default_opts()
        if eval_q is not None:
            q = np.ascontiguousarray(eval_q, dtype=np.float64)
            opts = RunOpts.from_buffer_copy(opts)
            opts.eval_q = q.ctypes.data
            opts.n_eval = q.size
            self._eval_q_keep = q
        ni, no = self.plan_size(process, species, opts)
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        self._last_items = ni
        Cv, S = np.zeros(no), np.zeros(no)
        self._check(lib().bmc_collision_exact22(self.h, process, species, C.byref(opts), _ptr(Cv), _ptr(S), no,
                                                MEM_HOST))
        return Cv, S

    def item_results(self, n_iter):
        n = self._n_items_last()
        uids = (C.c_uint32 * n)()
        Ib, sg = np.zeros(n), np.zeros(n)
        I_it, V_it = np.zeros((n, n_iter)), np.zeros((n, n_iter))
        self._check(lib().bmc_item_results(self.h, uids, _ptr(Ib), _ptr(sg), _ptr(I_it), _ptr(V_it), n, n_iter))
        return dict(uid=np.array(list(uids), dtype=np.uint32), Ibar=Ib, sigma=sg, I_it=I_it, V_it=V_it)

    def _n_items_last(self):
        if not hasattr(self, "_last_items"):
            raise BmcError(ESTATE, "no evaluation yet")
        return self._last_items

    def maps_get(self, uids: Sequence[int], nb: int):
        u = (C.c_uint32 * len(uids))(*[int(x) for x in uids])
        out = np.zeros((len(uids), MAXD * (nb + 1)))
        self._check(lib().bmc_maps_get(self.h, u, len(uids), _ptr(out)))
        return out

    def maps_set(self, uids: Sequence[int], maps: np.ndarray):
        u = (C.c_uint32 * len(uids))(*[int(x) for x in uids])
        maps = np.ascontiguousarray(maps, dtype=np.float64)
        self._check(lib().bmc_maps_set(self.h, u, len(uids), _ptr(maps)))

    def maps_reset(self, process=-1):
        self._check(lib().bmc_maps_reset(self.h, process))

    def step(self, method, dt, eps, dt_max, opts: Optional[RunOpts] = None):
        opts = opts or default_opts()
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        dtu = C.c_double()
        self._check(lib().bmc_step(self.h, method, dt, eps, dt_max, C.byref(opts), C.byref(dtu)))
        return dtu.value

    def graph_capture_steps(self, n_steps, method, dt, eps, dt_max, opts: Optional[RunOpts] = None):
        opts = opts or default_opts()
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        self._check(lib().bmc_graph_capture_steps(self.h, n_steps, method, dt, eps, dt_max, C.byref(opts)))

    def vjp(self, v, process=-1, species=-1, opts: Optional[RunOpts] = None, n_f=None):
        """dL/df (all grids concatenated), dL/dcoupling (per process), dL/dm0 (per species) of L = v . C with
        frozen maps and the counters of one iteration (opts.first_iter)."""
        opts = opts or default_opts()
        ni, no = self.plan_size(process, species, opts)
        self.ensure_workspace(opts.n_samples, 1)
        v = np.ascontiguousarray(v, dtype=np.float64)
        if v.size != no:
            raise ValueError("the cotangent has %d values, the plan's C has %d" % (v.size, no))
        n_f = n_f if n_f is not None else self._n_f
        gf, gl, gm = np.zeros(n_f), np.zeros(self._n_proc), np.zeros(self._n_species)
        self._check(lib().bmc_vjp(self.h, process, species, C.byref(opts), _ptr(v), no, _ptr(gf), _ptr(gl), _ptr(gm),
                                  MEM_HOST))
        return gf, gl, gm

    def set_timing(self, on=True, every=1):
        """Times the sample phases with HIP events: every `every`-th one while on (off: on=False)."""
        self._check(lib().bmc_set_timing(self.h, int(every) if on else 0))

    def get_timing(self, reset=True):
        ms, n = C.c_double(), C.c_int()
        self._check(lib().bmc_get_timing(self.h, int(reset), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def get_kernel_timing(self, reset=True):
        """(screening ms, second-pass ms, phases) summed over the timed sample phases."""
        a, b, n = C.c_double(), C.c_double(), C.c_int()
        self._check(lib().bmc_get_kernel_timing(self.h, int(reset), C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def state_get(self) -> bytes:
        """Checkpoint: f of every species, the time and epochs, every process's width and every Vegas map, as one
        byte string."""
        self.ensure_workspace()
        n = C.c_size_t()
        self._check(lib().bmc_state_size(self.h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._check(lib().bmc_state_get(self.h, buf, n.value))
        return buf.raw

    def state_set(self, blob: bytes):
        """Resume from a checkpoint of a context with the same species grids and processes."""
        self.ensure_workspace()
        buf = C.create_string_buffer(bytes(blob), len(blob))
        self._check(lib().bmc_state_set(self.h, buf, len(blob)))

    def get_sample_stats(self, reset=True):
        """Samples the second pass evaluated (in or near the energy shell) since the last reset."""
        n = C.c_int64()
        self._check(lib().bmc_get_sample_stats(self.h, int(reset), C.byref(n)))
        return n.value

    def set_launch_tuning(self, blocks_per_cu, chunk=4):
        self._check(lib().bmc_set_launch_tuning(self.h, blocks_per_cu, chunk))

    def autotune(self, process=-1, species=-1, opts: Optional[RunOpts] = None):
        """Picks the fastest persistent launch shape for this plan; returns (blocks_per_cu, chunk, ms)."""
        opts = opts or default_opts()
        self.plan_size(process, species, opts)
        self.ensure_workspace(opts.n_samples, opts.n_iter)
        b, ch, ms = C.c_int(), C.c_int(), C.c_double()
        self._check(lib().bmc_autotune(self.h, process, species, C.byref(opts), C.byref(b), C.byref(ch),
                                       C.byref(ms)))
        return b.value, ch.value, ms.value

    def graph_replay(self):
        self._check(lib().bmc_graph_replay(self.h))

    def graph_status(self):
        t, dt = C.c_double(), C.c_double()
        self._check(lib().bmc_graph_status(self.h, C.byref(t), C.byref(dt)))
        return t.value, dt.value


def from_workload(w: wl.Workload, device: int = 0, stream=None) -> Context:
    """A context with the species, masses, f tables, processes and expansion of a workload."""
    ctx = Context(device, stream)
    for s in w.species:
        sid = ctx.add_species(s.name, s.stat, s.n_grid, s.q_min, s.q_max)
        ctx.set_mass(sid, s.mass_kind, s.m0, s.mA, s.mw)
        if s.interp != INTERP_LINLOG:
            ctx.set_interp(sid, s.interp)
    for p in w.processes:
        ctx.add_process(p.ins, p.outs, coupling=p.coupling, sigma_E=p.sigma_E, alpha=p.alpha, e_cut=p.e_cut,
                        n_bins=p.n_bins, term_mode=p.term_mode, side_mask=p.side_mask, eval_stride=p.eval_stride,
                        n_samples=p.n_samples, n_iter=p.n_iter, width_mode=p.width_mode, width_adapt=p.width_adapt,
                        width_lo=p.width_lo, width_hi=p.width_hi, width_factor=p.width_factor,
                        width_min=p.width_min, width_max=p.width_max, vegas_plus=p.vegas_plus, beta=p.beta,
                        m2_kind=p.m2_kind,
                        m2_coef=(C.c_double * 6)(*p.m2_coef))
    if w.expansion:
        ctx.set_expansion(w.expansion, w.a0, w.t0)
    ctx.ensure_workspace()
    for i, s in enumerate(w.species):
        ctx.set_f(i, s.f)
    ctx.set_time(w.t)
    return ctx
