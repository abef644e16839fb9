/*
 * boltzmc.h -- C-ABI of the MI355X (gfx950) Monte-Carlo collision-integral library.
 *
 * The library evaluates the momentum-resolved collision integral
 *     C_a(q_i) = sum over processes of  n_alpha^a C_alpha(q_i) + n_beta^a C_beta(q_i)
 * (arXiv 2603.28848, Sec. II.C Eq. 7; Eq. 12 for self-reverse processes), each single-position term being
 * C^(k)(p) = (1/2E) Int dPi |M|^2 Lambda (Sec. II.B Eqs. 3-5), by Vegas adaptive Monte Carlo over the
 * 3(n_total - 2) dimensional space of Sec. II.D / Appendix A (observed momentum on z, one momentum fixed by
 * momentum conservation, Gaussian energy delta Eq. 15, phase-space weight Eq. 16), with separate gain and
 * loss integrators, and steps f in log space (Euler Eq. 18, Heun Eq. 19, adaptive step Eq. 20) in
 * comoving momenta with an optional radiation-dominated expansion (Sec. III.E).
 *
 * Conventions
 *   * Every function returns an int: BMC_OK (0) or a negative BMC_E* code.  bmc_last_error() describes the
 *     last failure of a context (the string is owned by the context and valid until its next call).
 *   * No exceptions cross this boundary.
 *   * Array arguments are borrowed.  `mem` says whether a pointer is host (BMC_MEM_HOST) or device
 *     (BMC_MEM_DEVICE) memory.  Device pointers are used asynchronously on the context's stream and must
 *     stay valid until the stream reaches that point; calls that return host results synchronise the stream.
 *   * The library allocates no device memory of its own: all device state (tables, Vegas maps, partial
 *     sums, results) lives in one workspace the caller allocates and binds (bmc_workspace_query / _bind).  The one
 *     exception is a static 64 MiB array per GPU that only bmc_collision_noalloc uses for its per-call scratch.
 *   * Results depend only on (inputs, seed, epoch, iteration indices, Vegas maps) and the launch mode; they do not
 *     depend on the launch tuning or on other items in the same call.  The batched and per-grid-point launch modes
 *     group the second pass's sums differently (4 and 64 groups per item), so for the same maps their results
 *     agree to rounding; each mode repeats itself bitwise.
 *   * Accuracy (BMC_FP64): an item's estimate I of one iteration differs from the same samples' estimate in
 *     correctly rounded arithmetic by at most 1e-12 |I| + 4 eps B1 (eps = 2^-52), B1 = (1/N) sum_n |W_n| s_n with
 *     s_n = (|dE_n| / sigma_E) (sum_i E_i / sigma_E): the energies carry a few ulps of the library's own sin, cos
 *     and square root, and the Gaussian energy delta (Eq. 15) amplifies an error in dE by dE / sigma_E^2.  Its
 *     variance V obeys the same with 1e-12 |V| + 4 eps B2, B2 = 2 / (N (N - 1)) sum_n W_n^2 s_n.
 *   * Work item: (process, observed species, pinned side, term, evaluation grid index).  Its identifier is
 *         uid = process << 24 | species << 20 | side << 19 | term << 18 | eval_index
 *     (side 0 = initial state, 1 = final state; term 0 = gain or net, 1 = loss).  Items of a call are
 *     ordered by uid.  The uniforms of iteration `it` of an item form one stream of 32-bit words: word k is
 *     output k mod 4 of Philox4x32-10 with key (lo32(seed), hi32(seed)) and counter (lo32(k/4), hi32(k/4),
 *     uid, 64 epoch + it); sample n takes words D n .. D n + D-1, and y = (word + 0.5) 2^-32.
 */
#ifndef BOLTZMC_H
#define BOLTZMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define BMC_OK 0
#define BMC_EINVAL (-1)   /* bad argument or id */
#define BMC_ESTATE (-2)   /* f not set, workspace not bound or too small, no processes */
#define BMC_ERANGE (-3)   /* f <= 0, Fermi-Dirac f >= 1, or an invalid extrapolation fit (Sec. III.B) */
#define BMC_ENOMEM (-4)   /* bound workspace smaller than the call needs (query again) */
#define BMC_EHIP (-5)     /* a HIP runtime call failed */
#define BMC_EUNSUP (-6)   /* valid request that the library does not implement */

/* ---- enumerations ---- */
#define BMC_MEM_HOST 0
#define BMC_MEM_DEVICE 1

#define BMC_BOSE 1        /* eta = +1 */
#define BMC_FERMI (-1)    /* eta = -1 */
#define BMC_MB 0          /* eta = 0 (no 1 +- f factors) */

#define BMC_GRID_LOG 0

#define BMC_MASS_CONST 0  /* m(t) = m0 */
#define BMC_MASS_SIN 1    /* m(t) = m0 + A sin(w t) */

#define BMC_EXP_NONE 0
#define BMC_EXP_RADIATION 1  /* a(t) = a0 (t / t0)^(1/2) */

#define BMC_TERMS_SPLIT 0 /* separate gain and loss integrators (Sec. II.D) */
#define BMC_TERMS_NET 1   /* one integrator of gain - loss */

#define BMC_SIDES_AUTO 0  /* both sides, or the initial side only for a self-reverse process (Eq. 12) */
#define BMC_SIDES_IN 1
#define BMC_SIDES_OUT 2
#define BMC_SIDES_BOTH 3

#define BMC_INTERP_LINLOG 0   /* f linear in ln q between grid nodes (default) */
#define BMC_INTERP_SPLINE 1   /* not-a-knot cubic spline of f in linear q (Sec. III.B) */
#define BMC_INTERP_EQEXACT 2  /* log(1/f + eta) linear in E between nodes: exact for equilibrium (the form of Eq. 17) */

#define BMC_M2_CONST 0    /* |M|^2 = coupling^2 */
#define BMC_M2_POLY 1     /* |M|^2 = coupling^2 P(s, t), P quadratic in the Mandelstam invariants (m2_coef) */

#define BMC_WIDTH_ABS 0   /* sigma_E is the width of the Gaussian energy delta (an energy) */
#define BMC_WIDTH_REL 1   /* sigma_E is a fraction w; the width at a point is w (E_in + E_out) / 2 (Appendix C) */

#define BMC_FP64 0        /* everything in IEEE double */
#define BMC_FP32I 1       /* FP32 integrand (f lookups, statistical factor, exponentials) with FP64
                             kinematics up to the delta argument and FP64 accumulation, for samples within
                             7 sigma_E (+ 1e-3 of the summed energies) of the energy shell.  Samples between that
                             and the FP64 underflow of the Gaussian factor (|dE| up to sqrt(2 746) sigma_E) are
                             finished wholly in FP32, conserved momentum and Gaussian argument included: their
                             factor is below e^-24.5 of the peak and the FP32 dE moves it by at most a few per
                             cent, so together they move an item's estimate by about 1e-12 of its size at most.
                             Samples beyond have W = 0 exactly, as in FP64. */

#define BMC_LAUNCH_BATCHED 0  /* all items of a call in one persistent launch per Vegas iteration */
#define BMC_LAUNCH_PLAIN 1    /* one launch per evaluation grid point per iteration */

#define BMC_EULER 0
#define BMC_HEUN 1

#define BMC_MAXN 6        /* particles per process (n_in + n_out <= 6, >= 3) */
#define BMC_MAXD 12       /* 3 (n - 2) */
#define BMC_MAXSPECIES 16
#define BMC_MAXBINS 64
#define BMC_MAXGRID 2048
#define BMC_MAXITER 64
#define BMC_MAXEVAL 256    /* evaluation points off the grid per call (bmc_run_opts.eval_q) */

typedef struct bmc_ctx bmc_ctx;

/* Per-process parameters (Sec. III.A "Processes are registered ..."; Appendix C). */
typedef struct {
  double coupling;     /* lambda; |M|^2 = lambda^2 includes the identical-particle symmetry factors */
  double sigma_E;      /* width of the Gaussian energy delta (Eq. 15), > 0: an energy (BMC_WIDTH_ABS) or the
                          fraction w of (E_in + E_out) / 2 at each point (BMC_WIDTH_REL, w <= 1); the initial value
                          when the width controller is on */
  double alpha;        /* Vegas damping exponent, in [0, 2] (paper: 0.5) */
  double e_cut;        /* points with any E_i < e_cut get weight 0 (Appendix A); default 0 */
  int n_bins;          /* Vegas bins per dimension, 2 .. BMC_MAXBINS (paper/workloads: 50) */
  int term_mode;       /* BMC_TERMS_SPLIT or BMC_TERMS_NET */
  int side_mask;       /* BMC_SIDES_* */
  int eval_stride;     /* evaluate every k-th grid point of the observed species (>= 1) */
  int64_t n_samples;   /* samples per item per iteration (>= 2, and D n_samples < 2^34) */
  int n_iter;          /* Vegas iterations per evaluation (1 .. BMC_MAXITER) */
  int width_mode;      /* BMC_WIDTH_ABS (default) or BMC_WIDTH_REL */
  /* Width controller (Appendix C), with width_adapt = 1: after every evaluation the width is divided by
   * width_factor when the relative Monte Carlo error r of the process's items is below width_lo, multiplied by it
   * when r exceeds width_hi, and clamped to [width_min, width_max].  r = sum sigma_i / sum |Ibar_i| over the
   * process's items of that evaluation.  Requires 0 < width_lo < width_hi, width_factor > 1,
   * 0 < width_min <= width_max (<= 1 for BMC_WIDTH_REL).  Defaults: 1e-3, 1e-2, 1.25, 1e-4, 0.2. */
  int width_adapt;
  double width_lo, width_hi, width_factor, width_min, width_max;
  /* VEGAS+ (Lepage 2021), with vegas_plus = 1: adaptive stratified sampling on top of the Vegas map.  y-space is
   * cut into M = k^D hypercubes, k the largest integer with k^D <= N / 2; an iteration draws n_h samples in
   * hypercube h (the first iteration of a call N / M each), estimates I = sum_h S1_h / (M n_h) with variance
   * sum_h (S2_h - S1_h^2 / n_h) / (n_h (n_h - 1) M^2), trains the map on (W N_it / (M n_h))^2, and (unless frozen)
   * reallocates n_h = 2 + floor((N - 2 M) sigma_h^beta / sum) with sigma_h the hypercube's standard deviation of
   * W / M.  Every sample is evaluated in full (no screening pass).  bmc_vjp does not take it.  beta in [0, 2]
   * (default 0.75). */
  int vegas_plus;
  double beta;
  /* Matrix element (Sec. III.A registers |M|^2 as a function of the momenta): BMC_M2_CONST (default), or
   * BMC_M2_POLY with |M|^2 = coupling^2 (c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2), c = m2_coef, where
   * s = (P_0 + P_1)^2 over the first two initial positions (m_0^2 with one initial particle) and
   * t = (P_0 - P_{n_in})^2 between the first initial and the first final position, from the physical
   * four-momenta of each sampled point.  Neither bmc_vjp nor bmc_collision_exact22 takes BMC_M2_POLY. */
  int m2_kind;
  double m2_coef[6];
} bmc_process_params;

/* Options of one evaluation. */
typedef struct {
  int64_t n_samples;   /* <= 0: each process's own n_samples */
  int n_iter;          /* <= 0: each process's own n_iter */
  int first_iter;      /* Philox iteration index of the first iteration (iterations first_iter .. +n_iter-1) */
  uint64_t seed;
  uint32_t epoch;      /* < 2^26 */
  int precision;       /* BMC_FP64 or BMC_FP32I */
  int launch;          /* BMC_LAUNCH_BATCHED or BMC_LAUNCH_PLAIN */
  int freeze_maps;     /* 1: the Vegas maps are used but not adapted */
  int eval_stride;     /* 0: each process's own stride, skipped nodes filled (linear in ln q; C/f held past
                          the last evaluated node); k >= 1: every k-th node of every process, no fill */
  const double* eval_q;  /* NULL: the grid (above).  Else n_eval comoving momenta (host, > 0, borrowed for the
                            call) at which C of the one selected species is evaluated: the observed leg sits at
                            q, its f interpolated linearly in ln q inside the grid and extrapolated by the fit
                            outside (the rule of every other particle).  Outputs are C(q_k) in order.  The maps
                            of these points are kept per index k and species (bmc_maps_reset when the points
                            change); the adjoint does not take them. */
  int n_eval;          /* number of eval_q points, 1 .. BMC_MAXEVAL */
} bmc_run_opts;

/* ---- context and workspace ---- */

/* Creates a context on HIP device `device` that launches on `hip_stream` (a hipStream_t; NULL = the null
 * stream).  The caller keeps the stream alive while the context exists. */
int bmc_create(bmc_ctx** out, int device, void* hip_stream);
int bmc_destroy(bmc_ctx* ctx);
int bmc_set_stream(bmc_ctx* ctx, void* hip_stream);

/* Bytes of device workspace needed by every call with at most `max_samples` samples per item per iteration
 * and at most `max_iter` iterations (<= 0: the registered processes' own values).  Species and processes
 * must be registered first; adding any afterwards requires a new query and bind. */
int bmc_workspace_query(bmc_ctx* ctx, int64_t max_samples, int max_iter, size_t* bytes);
/* Binds caller-owned device memory (256-byte aligned) of `bytes` bytes.  Rebinding a larger workspace
 * keeps the library's persistent state (f, maps, time): it is copied on the stream. */
int bmc_workspace_bind(bmc_ctx* ctx, void* dev_ptr, size_t bytes);

/* ---- model ---- */

/* Registers a species on a logarithmic comoving grid of n_grid nodes on [q_min, q_max] (Sec. III.A).
 * stat: BMC_BOSE / BMC_FERMI / BMC_MB.  Returns its id (0, 1, ...) in *species_id. */
int bmc_add_species(bmc_ctx* ctx, const char* name, int stat, int grid_kind, int n_grid, double q_min,
                    double q_max, int* species_id);
/* Mass of a species: BMC_MASS_CONST (m0) or BMC_MASS_SIN (m0 + A sin(w t)); m(t) >= 0 is required. */
int bmc_set_mass(bmc_ctx* ctx, int species, int kind, double m0, double A, double w);
/* Rule for f between grid nodes of a species (Sec. III.B): BMC_INTERP_LINLOG, _SPLINE or _EQEXACT.  Outside the
 * grid every rule uses the Eq. 17 fit; at the nodes every rule gives the table value.  The spline's second
 * derivatives are recomputed on the device before every evaluation.  bmc_vjp differentiates through every rule. */
int bmc_set_interp(bmc_ctx* ctx, int species, int mode);
/* Sets f on the species' grid (n values).  Validates f > 0 and, for Fermi-Dirac, f < 1 (BMC_ERANGE). */
int bmc_set_f(bmc_ctx* ctx, int species, const double* f, int n, int mem);
/* Copies the current f of a species (n values) to `f`. */
int bmc_get_f(bmc_ctx* ctx, int species, double* f, int n, int mem);

/* Registers the process in_sp[0..n_in-1] -> out_sp[0..n_out-1] (species ids), 3 <= n_in + n_out <= 6. */
int bmc_add_process(bmc_ctx* ctx, const int* in_sp, int n_in, const int* out_sp, int n_out,
                    const bmc_process_params* params, int* process_id);
int bmc_default_process_params(bmc_process_params* params);

/* Changes the coupling lambda of a process (|M|^2 = lambda^2). */
int bmc_set_coupling(bmc_ctx* ctx, int process, double coupling);

/* The current width parameter of a process (sigma_E, or w for BMC_WIDTH_REL): the registered value until the width
 * controller changes it on the device.  bmc_set_width replaces it (> 0; <= 1 for a relative width); either call
 * synchronises the context's stream when a workspace is bound. */
int bmc_get_width(bmc_ctx* ctx, int process, double* width);
int bmc_set_width(bmc_ctx* ctx, int process, double width);

/* Expansion (Sec. III.E): BMC_EXP_NONE (a = 1) or BMC_EXP_RADIATION with a0, t0 > 0. */
int bmc_set_expansion(bmc_ctx* ctx, int kind, double a0, double t0);
int bmc_set_time(bmc_ctx* ctx, double t);
int bmc_get_time(bmc_ctx* ctx, double* t);

/* ---- evaluation ---- */

/* Number of items and of output values bmc_collision produces for (process, species, opts):
 * process -1 = every process; species -1 = every species (outputs concatenated in species order); with
 * opts->eval_q set, n_out = opts->n_eval (one value per evaluation point). */
int bmc_plan_size(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, int* n_items, int* n_out);

/* Evaluates C and its Monte-Carlo sigma for the selected (process, species) pairs in one call.
 * Outputs (n_out values each, see bmc_plan_size): with opts->eval_stride >= 1, the values at grid nodes
 * 0, k, 2k, ... of each selected species in species order; with 0, the full grid of each species (the
 * per-process strided values filled).  sigma_out may be NULL.  Vegas maps are taken from and stored back to
 * the context (integrator reuse); maps start uniform.  BMC_EUNSUP when a block of the second pass would need more
 * than 64 KB of LDS: it holds the item's map (D N_b entries, twice), four per-wave W^2 histograms of D N_b doubles
 * and the f tables it reads; at D = 12 with 64 bins that leaves room for one FP64 table of up to 946 nodes with the
 * linear rule, or 315 when a species uses the spline or equilibrium-exact rule (or |M|^2 is a polynomial). */
int bmc_collision(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, double* C_out,
                  double* sigma_out, size_t n_out, int mem);

/* For callers that cannot allocate device memory at call time (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same evaluation, outputs and results as bmc_collision with the same
 * context state and options, but its per-call scratch (item records, task lists, screening lists, bin counts,
 * second-pass records, per-iteration estimates, slot sums, gather tables, output staging) lives in a static device
 * array of 64 MiB that the library holds on each GPU until the process ends, not in the bound workspace (which
 * still holds the persistent state: f, maps, time).  Calls no hipMalloc.  A call whose scratch exceeds 64 MiB
 * returns BMC_ENOMEM (the batched 2<->3 workload of 128 nodes x 2^18 samples fits; per-grid-point launches reserve
 * 8x more second-pass records).  Every call on one GPU shares the array, and the call synchronises the context's
 * stream before returning, so calls must not overlap on one GPU (concurrent calls from several threads or
 * contexts on the same GPU race).  bmc_item_results keeps reporting the last bmc_collision, not this call. */
int bmc_collision_noalloc(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, double* C_out,
                          double* sigma_out, size_t n_out, int mem);

/* Exact-delta 2->2 path (Sec. IV's two-dimensional reduction; Appendix B): the same outputs as bmc_collision for
 * the same selection and options, computed without Monte Carlo and without the Gaussian: per item, the integral
 * over two momentum magnitudes with energy conservation exact and the angular kinematic function in closed form,
 * by the trapezoidal rule in ln q on the grid nodes of the integrated species (the gain term over the opposite
 * side's momenta, the loss term over the partner's and one opposite momentum).  sigma_out is 0.  Every selected
 * process must be 2->2 with constant |M|^2 (BMC_EUNSUP otherwise).  Sampling options (n_samples, n_iter, seed,
 * epoch, precision, launch, freeze_maps) are ignored; Vegas maps and epochs are untouched.  bmc_item_results then
 * reports the per-item values with one iteration. */
int bmc_collision_exact22(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, double* C_out,
                          double* sigma_out, size_t n_out, int mem);

/* Per-item results of the last bmc_collision (items in uid order, n = its n_items): uid, multiplicity-free
 * estimate Ibar and sigma, and per-iteration I and V (n x n_iter each).  Any pointer may be NULL. */
int bmc_item_results(bmc_ctx* ctx, uint32_t* uids, double* Ibar, double* sigma, double* I_it, double* V_it,
                     int n, int n_iter);

/* Vegas map of items (uids[i]), each stored as BMC_MAXD x (n_bins + 1) edges (rows beyond D ignored).
 * An item that has no map yet reads as the uniform map.  Host memory. */
int bmc_maps_get(bmc_ctx* ctx, const uint32_t* uids, int n, double* maps);
int bmc_maps_set(bmc_ctx* ctx, const uint32_t* uids, int n, const double* maps);
/* Forgets the maps of a process (-1 = all): they restart uniform. */
int bmc_maps_reset(bmc_ctx* ctx, int process);

/* Checkpoint and resume: the state that an evolution carries from one call to the next -- every species' f, the
 * time and the device epoch counters, and every Vegas map the context holds -- as one host byte blob.
 * bmc_state_size gives the bytes bmc_state_get writes into the caller's buffer (synchronises the stream).
 * bmc_state_set restores a blob into a context with the same species grids and processes (checked: a blob of
 * another model, an invalid f or a map of an unknown work item is rejected with nothing changed); the masses,
 * couplings and expansion are the context's own.  Layout: a 48-byte header (magic "BMCS", version 2, species
 * count, map count, number of f values, t, epoch, next epoch, doubles per map, process count), the f values
 * (FP64, species concatenated), the current width parameter of every process (FP64), then per map its uid (as a
 * 64-bit word) and its edges (12 x 65 doubles, unused rows zero). */
int bmc_state_size(bmc_ctx* ctx, size_t* bytes);
int bmc_state_get(bmc_ctx* ctx, void* blob, size_t bytes);
int bmc_state_set(bmc_ctx* ctx, const void* blob, size_t bytes);

/* One Euler or Heun step of every species' f in log space over all processes (Sec. III.C):
 * dt > 0 fixed, dt <= 0: dt = min(dt_max, eps / max|k1/f|) (Eq. 20).  k1 uses opts->epoch at t, k2 uses
 * epoch + 1 at t + dt.  Strided processes are filled as in bmc_collision with eval_stride 0.  The time
 * advances by dt.  *dt_used (may be NULL) receives dt (host, synchronises). */
int bmc_step(bmc_ctx* ctx, int method, double dt, double eps, double dt_max, const bmc_run_opts* opts,
             double* dt_used);

/* Captures n_steps Heun/Euler steps (epochs opts->epoch + 2s, + 2s + 1 for step s) into a HIP graph held by
 * the context.  Time, step size, epoch and a(t), m(t) advance on the device, so each replay continues the
 * evolution.  bmc_graph_replay launches it on the context stream; bmc_graph_status reports a device-side
 * error flag set during replays (BMC_ERANGE for an invalid f) and the time reached. */
int bmc_graph_capture_steps(bmc_ctx* ctx, int n_steps, int method, double dt, double eps, double dt_max,
                            const bmc_run_opts* opts);
int bmc_graph_replay(bmc_ctx* ctx);
int bmc_graph_status(bmc_ctx* ctx, double* t, double* last_dt);

/* ---- differentiation ---- */

/* Vector-Jacobian product of the C of the last-planned items with frozen maps and common random numbers
 * (the same counters as bmc_collision with these opts and one iteration): given the cotangent v on C_out
 * (n_out values, layout as bmc_collision), returns dL/df (every species' grid, concatenated),
 * dL/dcoupling (one per process) and dL/dm0 (one per species).  BMC_EUNSUP for an FP32-integrand request,
 * evaluation points off the grid, a polynomial |M|^2, VEGAS+ sampling, a strided fill, or an adjoint block
 * that would need more than 64 KB of LDS. */
int bmc_vjp(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, const double* v_C,
            size_t n_out, double* grad_f, double* grad_coupling, double* grad_m0, int mem);

/* ---- measurement and tuning ---- */

/* Timing of the sample phase (screening and second pass of one iteration's launch) with HIP events on the context
 * stream (eager launches only; graph replays are not timed): on = 0 off, on = k >= 1 every k-th sample phase
 * (k = 1: all; each timed phase records an event before, between and after its two kernels).  BMC_EINVAL for
 * on < 0. */
int bmc_set_timing(bmc_ctx* ctx, int on);
/* Sum of the timed sample-phase durations (ms) and number of timed phases since the last reset;
 * synchronises the stream.  reset != 0 clears the counters after reading. */
int bmc_get_timing(bmc_ctx* ctx, int reset, double* sample_ms, int* n_launches);
/* The same timed sample phases split by kernel: the screening pass (from the event before it to the event between the
 * two kernels) and the second pass (from there to the event after it), summed in ms; synchronises the stream.  reset
 * != 0 clears every timing sum (bmc_get_timing's too) after reading. */
int bmc_get_kernel_timing(bmc_ctx* ctx, int reset, double* screen_ms, double* second_ms, int* n_launches);
/* Number of samples the second pass evaluated (those the screening pass found able to carry a nonzero W: in
 * the energy shell or near it) since the last reset, over all evaluations on the context, graph replays
 * included; synchronises the stream.  reset != 0 clears the counter after reading. */
int bmc_get_sample_stats(bmc_ctx* ctx, int reset, int64_t* n_listed);
/* Launch shape of the persistent batched sample kernel: resident blocks per compute unit (0 = from the LDS
 * need) and the number of consecutive tasks (units of samples) a block takes per visit.  Results do not
 * depend on either: every unit's partial sums are formed in the same fixed order by whichever block runs it. */
int bmc_set_launch_tuning(bmc_ctx* ctx, int blocks_per_cu, int chunk);
/* Times one frozen-map iteration of the (process, species, opts) plan for every launch shape (blocks per CU
 * 1 .. the LDS limit, chunk 1/2/4/8/16), keeps the fastest in the context and reports it.  No Vegas map,
 * f or time is changed. */
int bmc_autotune(bmc_ctx* ctx, int process, int species, const bmc_run_opts* opts, int* blocks_per_cu, int* chunk,
                 double* best_ms);

/* ---- misc ---- */
const char* bmc_last_error(bmc_ctx* ctx);
const char* bmc_version(void);

#ifdef __cplusplus
}
#endif
#endif
