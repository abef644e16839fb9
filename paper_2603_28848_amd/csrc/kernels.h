// kernels.h -- launch wrappers of the libboltzmc kernels (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace bmc {

struct SampleLaunch {
  const ItemRec* items;
  const Task* tasks;
  int n_tasks;
  int task_begin;        // first task of this launch
  const SpecDev* spec;
  const double* f64;
  const float* f32;
  const double* qnode;   // comoving grid nodes, same layout as f
  const DevState* st;
  const double* maps;
  uint32_t* counts;      // per item: the bin counts of the screening pass (D nb), added by the screening blocks;
                         // nullptr: not kept
  double* parts;         // adjoint: unit records
  const int64_t* unit_base;  // per item: index of its first unit
  int it;                // Philox iteration index
  uint32_t seed_lo, seed_hi;
  int nint_mask;         // bit (nint-1) set for every integrated-particle count present
  int precision;         // 0 FP64, 1 FP32I
  int any_interp;        // 1 if a species of the launch interpolates by the spline or the equilibrium-exact rule
  int grid;              // blocks
  int chunk;             // consecutive tasks per block visit
  size_t lds_bytes;       // sample blocks (VEGAS+)
  size_t shell_lds;       // second-pass blocks
  // FP32 integrand: in-shell lists of the screening pass and the in-shell pass
  uint16_t* shell_list;  // list_stride entries per task position of the launch (4 wave lists: in-shell samples
                         // from the front, near ones from the back)
  uint32_t* shell_cnt;   // per task position: 4 in-shell counts, then 4 near counts
  int64_t list_stride;   // largest unit size of the plan
  const ShellTask* sh_tasks;
  int sh_begin, n_sh;    // in-shell tasks (one per item) of this launch
  int sh_grid;
  int sh_tiles;          // tiles per second-pass group (blocks per group; kShellTiles batched, 1 per grid point)
  double* shell_rec;     // per second-pass group: S1, S2, then the D nb W^2 sums
  unsigned long long* n_listed;  // running count of the samples the second pass evaluates
  // VEGAS+ items: sample blocks of this iteration, per-hypercube allocation (n_h), offsets (sum of n before h),
  // sums of W and W^2, and per-block training records (S1, S2, 2 D nb doubles)
  const VpTask* vp_tasks;
  int n_vp;
  const int* vp_nh;
  const int64_t* vp_hoff;
  double* vp_S1;
  double* vp_S2;
  double* vp_rec;
};

// VEGAS+ sample blocks (every sample of the item evaluated in full, FP64 or FP32 integrand).
hipError_t launch_vplus(const SampleLaunch& L, hipStream_t s);
// VEGAS+: the uniform allocation n_h = N / M of the first iteration of a call, for the listed items.
hipError_t launch_vplus_init(const ItemRec* items, const int* which, int n, int* nh, int64_t* hoff, hipStream_t s);
// VEGAS+ per item: I and V of iteration `slot` from the hypercube sums; unless frozen, the map adapted from the
// blocks' training records and the next allocation n_h = 2 + floor((N - 2 M) sigma_h^beta / sum).
hipError_t launch_vplus_reduce(const ItemRec* items, const int* which, int n, int* nh, int64_t* hoff,
                               const double* S1, const double* S2, const double* rec, double* res_I, double* res_V,
                               int slot, double* maps, int freeze, hipStream_t s);

// Screening pass of a sample launch (FP32 kinematics; lists the samples whose W can be nonzero).
hipError_t launch_sample(const SampleLaunch& L, hipStream_t s);
// Second pass over the listed samples of the preceding screening launch (FP64, or the FP32 integrand).
hipError_t launch_shell(const SampleLaunch& L, hipStream_t s);

// Per item: S1, S2 and the W^2 histogram from its second-pass records in group order, the bin counts from the
// item's counts (the screening pass counts every sample; they are cleared here, frozen or not); stores I_it, V_it for
// iteration slot `slot` and (unless frozen) adapts the item's map.  `plain` names the grouping the records were
// written with (per-grid-point launch).
hipError_t launch_reduce_adapt(const ItemRec* items, int item_begin, int n_items, uint32_t* counts,
                               const double* shell_rec, double* res_I, double* res_V, int slot, double* maps,
                               int freeze, int plain, hipStream_t s);

// Initialises the maps of items (uniform edges over each dimension's range).
hipError_t launch_init_maps(const ItemRec* items, const int* which, int n, const SpecDev* spec, double* maps,
                            hipStream_t s);

// Per-slot combination: Ibar, sigma per item (inverse variance over n_iter iterations) and the slot sums
// C = sum mult sign Ibar, S2 = sum mult^2 sigma^2 over the slot's items (list slot_items[slot_begin[k]..]).
hipError_t launch_combine(const ItemRec* items, int n_items, const double* res_I, const double* res_V, int n_iter,
                          double* item_Ibar, double* item_sig, const int* slot_begin, const int* slot_items,
                          int n_slots, double* slot_C, double* slot_S2, hipStream_t s);

// Exact-delta 2->2: one block per item (2->2 items only), the estimate into iteration 0 of res_I with V = 0.
hipError_t launch_exact22(const ItemRec* items, int n_items, const SpecDev* spec, const double* f64,
                          const double* qnode, const DevState* st, double* res_I, double* res_V, hipStream_t s);

// Width controller after an evaluation (processes with adapt set): r = sum sigma / sum |Ibar| over the process's
// items in item order; the process's width in st->width is divided or multiplied by the factor and clamped.
hipError_t launch_width_control(const ItemRec* items, int n_items, const double* item_Ibar, const double* item_sig,
                                const WidthCtl* ctl, int n_proc, DevState* st, hipStream_t s);

// Output gather: out[o] for output node o of the plan, from the slot sums (stride-override or fill rule).
struct GatherEntry {
  int species;    // species of the output node
  int node;       // grid index
  int first;      // first process entry in gather_proc
  int count;
};
struct GatherProc {
  int slot_base;  // slot index of node 0 of this (process, species)
  int stride;     // evaluation stride
  int last;       // last evaluated node
  int fill;       // 1: apply the fill rule
};
hipError_t launch_gather(const GatherEntry* ge, int n_out, const GatherProc* gp, const double* slot_C,
                         const double* slot_S2, const SpecDev* spec, const double* f64, double* C_out,
                         double* sig_out, hipStream_t s);

// Recomputes a(t), m_s(t), the extrapolation fits and the FP32 copy of f; sets st->err on invalid tables.
hipError_t launch_prepare(DevState* st, const SpecDev* spec, int n_species, const double* f64, float* f32,
                          int64_t n_f, hipStream_t s);

int sample_lds_bytes(int D, int nb, int n_tab, int n_max, int precision);
// LDS bytes of a screening block (the FP32 map only).
int screen_lds_bytes();
// LDS bytes of a second-pass block (the sample layout without counts, plus the item's constants and the threads' word
// slots); alt = 0 for a launch whose tables all use the linear rule and whose |M|^2 is constant (tables of f alone).
int shell_lds_bytes(int D, int nb, int n_tab, int n_max, int precision, int alt);

// Adjoint (FP64, frozen maps): per-unit records of the sample derivatives, then per item (times coef/N),
// then per species node, fits, masses and couplings.
hipError_t launch_vjp(const SampleLaunch& L, hipStream_t s);
// spl: 1 if a table of the item is interpolated by the spline (its record then holds the d/dM slots too)
int vjp_lds_bytes(int D, int nb, int n_tab, int n_max, int spl);
int vjp_record_len(int n_tab, int n_max, int spl);
// work: 3 n_f doubles of scratch (the spline adjoint's right-hand sides and elimination rows)
hipError_t launch_vjp_finish(const ItemRec* items, int n_items, const double* coef, const double* parts,
                             const int* rec_len, const int* rec_nmax, double* item_rec, int rec_stride,
                             const SpecDev* spec, int n_species, const double* f64, const double* qnode,
                             const DevState* st, double* grad_f, int64_t n_f, double* work, double* grad_m,
                             double* grad_lam, const double* coupling, int n_proc, hipStream_t s);
hipError_t launch_next_epoch(DevState* st, hipStream_t s);

// Sets the next evaluation epoch (and optionally the time) on the device.
hipError_t launch_set_eval(DevState* st, double t, uint32_t epoch, int set_t, hipStream_t s);

// Step pieces (Sec. III.C).  stage_begin: dt from max|k1/f| (or fixed), f0 <- f, f <- f exp(dt k1 / f),
// t <- t0 + dt (Heun: epoch + 1).  finish: Heun combination.
hipError_t launch_step_begin(DevState* st, double* f64, double* f0, const double* k1, int64_t n_f, double dt_fixed,
                             double eps, double dt_max, int heun, hipStream_t s);
hipError_t launch_step_finish(DevState* st, double* f64, const double* f0, const double* fstar, const double* k1,
                              const double* k2, int64_t n_f, hipStream_t s);
hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s);

}  // namespace bmc
