// internal.h -- device-visible records shared by the host planner and the kernels of libboltzmc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmc {

constexpr int kMaxN = 6;          // particles per process
constexpr int kMaxInt = 4;        // integrated particles (n - 2)
constexpr int kMaxD = 12;         // 3 (n - 2)
constexpr int kMaxSpecies = 16;
constexpr int kMaxBins = 64;
constexpr int kMaxIter = 64;
constexpr int kBlock = 256;       // threads per sample block; part of the fixed summation order
constexpr int kWaves = kBlock / 64;
constexpr int kMaxTab = 4;        // distinct f tables one item reads (non-observed particles)
constexpr int kMaxProc = 256;     // processes per context (ids 0..254; the identifier keeps 8 bits)
// Second pass of a batched launch: the listed samples of each group of units are cut into this many equal tiles,
// one block and one record each.  One tile per group is the fastest measured: every block first stages the item's
// tables and constants in LDS (about 0.04 ms of a 0.2 ms pass at 2^26 samples), and 8 tiles doubled the pass.
constexpr int kShellTiles = 1;

// Species as the kernels see it: logarithmic grid q_j = exp(lq0 + h j), j = 0..n-1.
struct SpecDev {
  int stat;          // eta
  int n;             // nodes
  double q_min, q_max, lq0, inv_h;
  int mass_kind;     // 0 const, 1 m0 + A sin(w t)
  double m0, A, w;
  int64_t f_off;     // offset of the species' values in the f arrays
  int interp;        // 0 linear in ln q, 1 not-a-knot cubic spline in linear q, 2 log(1/f + eta) linear in E
  const double* qn;  // n comoving grid nodes
  double* aux;       // n doubles written by the prepare kernel: the spline's second derivatives, or the node
                     // energies of the equilibrium-exact rule
  double* tmp;       // n doubles: scratch of the spline solve, or log(1/f_j + eta) of the equilibrium-exact rule
};

// Time-dependent state read by every kernel (lives in device memory so graphs can advance it).
struct DevState {
  double t;          // time of the current evaluation
  double a;          // scale factor a(t)
  double inv_a;      // 1 / a(t)
  double a_m3n[5];   // a(t)^(-3 n), n = 0..4 (the a^-3 per integrated particle of the weight)
  double m[kMaxSpecies];          // masses at t
  double fit[kMaxSpecies][4];     // (a_lo, b_lo, a_hi, b_hi) of log(1/f + eta) = a + b E
  double dt;         // step size of the step in progress
  double t_step0;    // time at the start of the step in progress
  double rmax;       // max |k1/f| of the step in progress
  uint32_t epoch;    // epoch of the evaluation in progress
  uint32_t next_epoch;  // epoch the next evaluation consumes
  int err;           // sticky error flag (BMC_ERANGE ...)
  unsigned long long n_listed;  // samples evaluated by the second pass since the last read-out
  double expansion_a0, expansion_t0;
  int expansion;
  int n_species;
  double width[kMaxProc];  // current width parameter per process: sigma_E, or the fraction w of a relative width
};

// The width controller of one process (Appendix C): after an evaluation whose relative Monte Carlo error is r,
// the width is divided by `factor` if r < lo, multiplied by it if r > hi, and clamped to [wmin, wmax].
struct WidthCtl {
  int adapt;
  double lo, hi, factor, wmin, wmax;
};

// One work item.  Roles are stored by role, not by position: integrated k = 0..nint-1, then the
// conserved and the observed particle.
struct ItemRec {
  uint32_t uid;
  int proc;
  int nint;          // n - 2
  int D;             // 3 nint
  int nb;            // Vegas bins
  int term;          // 0 gain / net, 1 loss
  int net;           // 1: gain - loss
  int eval_idx;      // grid index of the observed momentum, or index k of an evaluation point off the grid
  int obs_at;        // 1: observed momentum q_obs off the grid, f there from the table's interpolation/fit
  int n_iter;        // Vegas iterations of this item in the call
  double q_obs;      // comoving observed momentum (the grid node)
  int obs_species;
  int mult;
  int n_units;       // partial-sum units of one iteration
  int unit_size;     // samples per unit
  int64_t N;         // samples per iteration
  int64_t map_off;   // doubles: Vegas map, kMaxD rows of (nb + 1) edges
  int64_t part_off;  // collision: the item's bin counts (D nb 32-bit counts); adjoint: doubles of the
                     // first unit record
  int64_t shell_off; // doubles: the item's second-pass records (S1, S2 and D nb W^2 sums each)
  int shell_units;   // units per second-pass record in a batched launch
  int shell_units_p; // units per second-pass record in a per-grid-point launch
  int64_t res_off;   // index of this item's per-iteration results
  int out_slot;      // output slot of the item's evaluation point (combine)
  int sign;          // +1 gain / net, -1 loss
  double coupling2;
  int rel;           // 1: the Gaussian's width at a point is w (E_in + E_out) / 2, w = DevState::width[proc]
  double e_cut;
  double twopi_pow;  // (2 pi)^(3(n-1)-4)
  double alpha;
  // role tables, index r: 0..nint-1 integrated, nint conserved, nint+1 observed
  int r_species[kMaxN];
  int r_tab[kMaxN];     // f-table slot (kMaxTab) of the role's species (integrated and conserved)
  int r_in[kMaxN];      // 1 if the role's particle is in the initial state
  int r_obsside[kMaxN]; // 1 if the role's particle is on the observed side
  int cons_in;          // conserved particle in the initial state
  // |M|^2 = coupling2 P(s, t) when m2poly: P = c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2, s = (sum_r cs_r P_r)^2,
  // t = (sum_r ct_r P_r)^2 over the roles' four-momenta (cs: the first two initial positions; ct: +1 the first
  // initial, -1 the first final position)
  // VEGAS+ (adaptive stratified sampling): vp_k strata per dimension, vp_M = vp_k^D hypercubes starting at index
  // vp_off of the plan's hypercube arrays, vp_blocks sample blocks whose records start at vp_rec (doubles)
  int vplus, vp_k, vp_M, vp_blocks;
  int64_t vp_off, vp_hb, vp_rec;  // hypercube base, offset-array base (M + 1 entries), record base
  double beta;
  int m2poly;
  double m2c[6];
  int r_cs[kMaxN], r_ct[kMaxN];
  int tab_species[kMaxTab];
  int n_tab;
};

// A VEGAS+ sample block: hypercubes [256 b, 256 (b + 1)) of item `item`.
struct VpTask {
  int item;
  int b;
};

// A unit of work: `unit` of item `item` in iteration order.
struct Task {
  int item;
  int unit;
};

// The in-shell pass over units [unit_begin, unit_end) of one item: `first_task` indexes unit `unit_begin` in the
// task list of the launch; the sums go to the record at `rec` (doubles into the in-shell records), tile t of the group
// (a batched launch's kShellTiles tiles) to the t-th record from there.
struct ShellTask {
  int item;
  int first_task;
  int unit_begin, unit_end;
  int64_t rec;
};

}  // namespace bmc
