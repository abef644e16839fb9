// api.hip -- C-ABI of libboltzmc: context, workspace, model registration, planner and launch sequencing.
//
// The planner turns (process, species, options) into work items (Sec. II.C Eq. 7 / Eq. 12 multiplicities and
// Appendix A particle roles), units of samples, output slots and the gather table; the launch sequence per
// evaluation is  next-epoch -> prepare (a(t), m(t), fits, FP32 f) -> [sample -> reduce/adapt] x n_iter ->
// combine -> gather.  All device memory is carved out of the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/boltzmc.h"
#include "internal.h"
#include "kernels.h"

using namespace bmc;

// The allocation-free evaluation (bmc_collision_noalloc) takes its per-call scratch from a static device array of
// kStaticScratchBytes, one per GPU, held until the process ends.  In host code the array's name is not a device
// address: the address of each GPU's copy comes from hipGetSymbolAddress (g_scratch_ptr below), resolved once per
// device when a context is created there.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {nullptr};

// Device address of `scratch` on `device` (the current device), resolved on the first call for that device.
hipError_t resolve_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr int kSlotDoubles = kMaxD * (kMaxBins + 1);
// FP32 integrand: bytes of in-shell lists one screening launch may fill (larger batches run in slices)
constexpr size_t kListCapBytes = size_t(1) << 30;
// Screening lists of one launch of the allocation-free evaluation: capped lower so that its launches are sliced to fit
// the static scratch.
constexpr size_t kStaticListCapBytes = size_t(16) << 20;
// Second pass: an item's units form groups, each one task of the pass with its own record.  A batched launch has
// many items and gives each few groups (every group pays for its barriers, histogram clear and record); a
// per-grid-point launch has a handful of items and needs many groups to fill the device.  Both depend on the item
// alone, so an item's results do not depend on the other items of its plan.
// Measured on the 2<->3 workload: 4 groups per item batched; 64 per grid point (32: 5 % slower, 16: 19 %).
constexpr int kShellGroupsBatched = 4;
constexpr int kShellGroupsPlain = 64;
constexpr int kMaxEvalPoints = BMC_MAXEVAL;  // map slots are reserved for this many points off the grid
constexpr int kVplusLdsExtra = 257 * 8 + 256 * 8;  // the VEGAS+ pass's hypercube offsets and chunk of W

// VEGAS+ strata per dimension: the largest k >= 1 with k^D <= N / 2.
int vplus_strata(int64_t N, int D) {
  int k = 1;
  for (;;) {
    int64_t p = 1;
    for (int d = 0; d < D && p <= N / 2; ++d) p *= (int64_t)(k + 1);
    if (p > N / 2) return k;
    ++k;
  }
}

// Units per group for at most `groups` groups, and the number of groups that makes.
int shell_units_for(int64_t n_units, int groups) { return std::max(1, (int)((n_units + groups - 1) / groups)); }
int64_t shell_groups(int64_t n_units, int su) { return (n_units + su - 1) / su; }
// Records an item reserves: enough for either launch's grouping (a batched group keeps kShellTiles records), or
// (launch >= 0) for that launch mode's only.
int64_t shell_records(int64_t n_units, int launch = -1) {
  const int64_t b = shell_groups(n_units, shell_units_for(n_units, kShellGroupsBatched)) * kShellTiles;
  const int64_t p = shell_groups(n_units, shell_units_for(n_units, kShellGroupsPlain));
  return launch == BMC_LAUNCH_BATCHED ? b : (launch == BMC_LAUNCH_PLAIN ? p : std::max(b, p));
}

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

struct Species {
  std::string name;
  int stat = 0;
  int n = 0;
  double q_min = 0, q_max = 0;
  int mass_kind = 0;
  double m0 = 0, A = 0, w = 0;
  std::vector<double> f;  // host mirror (authoritative until bound; refreshed from the device on demand)
  bool f_set = false;
  int64_t f_off = 0;
  int interp = BMC_INTERP_LINLOG;
};

struct Process {
  int n_in = 0, n_out = 0;
  int sp[kMaxN] = {0};
  bmc_process_params prm{};
  double width = 0.0;  // host mirror of the current width parameter (the device copy is authoritative while bound)
};

struct Plan {
  // key
  int process = -2, species = -2, stride = -1;
  int64_t n_samples = -1;
  int n_iter = -1;
  std::vector<double> eval_q;
  // content
  std::vector<ItemRec> items;
  std::vector<int> nodes_of_item;
  std::vector<Task> tasks_batched;            // item-major
  std::vector<Task> tasks_plain;              // node-major
  std::vector<int> plain_node_begin;          // ranges into tasks_plain per distinct node
  std::vector<int64_t> unit_base;
  std::vector<int> slot_begin, slot_items;
  std::vector<GatherEntry> gather;
  std::vector<GatherProc> gproc;
  std::vector<int> tasks_per_iter;            // batched tasks with item n_iter > k (prefix of item-major list)
  // FP32 integrand: in-shell tasks (one per item) in batched and plain order, slices of the batched launch
  std::vector<ShellTask> sh_batched, sh_plain;
  std::vector<int> plain_node_sh_begin;       // ranges into sh_plain per distinct node
  std::vector<int> sh_per_iter;               // batched in-shell tasks with item n_iter > k
  struct Slice {
    int tb, te, sb, se;  // task range and in-shell task range
  };
  std::vector<Slice> slices;
  int64_t list_stride = 0;  // largest unit size
  int64_t list_pos = 0;     // task positions the in-shell lists hold
  int64_t n_shell = 0;      // doubles of the in-shell records
  int n_iter_max = 0;
  int n_slots = 0;
  int n_out = 0;
  int nint_mask = 0;
  int64_t n_units = 0;
  int64_t n_parts = 0;   // 32-bit bin counts of all units
  int lds64 = 0, lds32 = 0;      // sample blocks (VEGAS+)
  int lds_sh64 = 0, lds_sh32 = 0;  // second-pass blocks (tables for every rule)
  int lds_sh64_lin = 0, lds_sh32_lin = 0;  // second-pass blocks of a launch with the linear rule only
  std::vector<int> new_maps;  // item indices whose maps need initialising
  // VEGAS+ items: sample blocks (items with more iterations first), blocks per iteration, the items themselves
  std::vector<VpTask> vp_tasks;
  std::vector<int> vp_per_iter, vp_items;
  int64_t vp_hc = 0, vp_hoffs = 0, vp_recd = 0;  // hypercubes, offset entries, record doubles
  VpTask* d_vpt = nullptr;
  int* d_vpi = nullptr;
  int* d_nh = nullptr;
  int64_t* d_hoff = nullptr;
  double *d_vS1 = nullptr, *d_vS2 = nullptr, *d_vrec = nullptr;
  // device pointers (inside the scratch region)
  ItemRec* d_items = nullptr;
  Task* d_tb = nullptr;
  Task* d_tp = nullptr;
  ShellTask* d_shb = nullptr;
  ShellTask* d_shp = nullptr;
  uint16_t* d_list = nullptr;
  uint32_t* d_cnt = nullptr;
  double* d_shell = nullptr;
  int64_t* d_unit_base = nullptr;
  uint32_t* d_counts = nullptr;
  int64_t n_counts = 0;  // 32-bit bin counts (D nb per item)
  double* d_res_I = nullptr;
  double* d_res_V = nullptr;
  double* d_item_Ibar = nullptr;
  double* d_item_sig = nullptr;
  int* d_slot_begin = nullptr;
  int* d_slot_items = nullptr;
  double* d_slot_C = nullptr;
  double* d_slot_S2 = nullptr;
  GatherEntry* d_gather = nullptr;
  GatherProc* d_gproc = nullptr;
  double* d_out_C = nullptr;
  double* d_out_S = nullptr;
  int* d_new = nullptr;
  size_t scratch_bytes = 0;
  bool uploaded = false;
  bool in_static = false;  // scratch in the library's static device array (bmc_collision_noalloc)
};

}  // namespace

struct bmc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::vector<Species> sp;
  std::vector<Process> pr;
  int expansion = BMC_EXP_NONE;
  double a0 = 1.0, t0 = 1.0;
  double t = 0.0;  // host mirror of the time (authoritative while unbound)
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false;
  size_t off_state = 0, off_spec = 0, off_f64 = 0, off_f32 = 0, off_f0 = 0, off_k1 = 0, off_k2 = 0, off_sig = 0,
         off_qnode = 0, off_maps = 0, off_wctl = 0, off_aux = 0, persist_bytes = 0;
  int64_t n_f = 0;
  int max_slots = 0;
  int n_sp_bound = -1, n_pr_bound = -1;
  std::unordered_map<uint32_t, int> slot_of_uid;
  Plan plan;       // last collision plan
  Plan step_plan;  // plan of bmc_step / graphs (all processes, all species, own strides)
  int last_n_iter = 0;
  std::string err;
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  // tuning
  int blocks_per_cu = 0;  // 0: from the LDS need
  int chunk = 4;          // consecutive tasks per block visit
  int n_cu = 0;
  // optional timing of the sample kernel (eager launches only)
  bool timing = false;
  int timing_every = 1;    // time every k-th sample phase
  int64_t phase_count = 0;  // sample phases launched while timing is on
  bool capturing = false;
  struct PhaseEvents {
    hipEvent_t a, m, b;  // before the screening pass, between the two kernels, after the second pass
  };
  std::vector<PhaseEvents> ev;
  double timed_ms = 0.0, timed_screen_ms = 0.0, timed_second_ms = 0.0;
  int timed_launches = 0;

  DevState* st() { return reinterpret_cast<DevState*>(ws + off_state); }
  SpecDev* spec() { return reinterpret_cast<SpecDev*>(ws + off_spec); }
  WidthCtl* wctl() { return reinterpret_cast<WidthCtl*>(ws + off_wctl); }
  double* f64() { return reinterpret_cast<double*>(ws + off_f64); }
  float* f32() { return reinterpret_cast<float*>(ws + off_f32); }
  double* f0() { return reinterpret_cast<double*>(ws + off_f0); }
  double* k1() { return reinterpret_cast<double*>(ws + off_k1); }
  double* k2() { return reinterpret_cast<double*>(ws + off_k2); }
  double* sig() { return reinterpret_cast<double*>(ws + off_sig); }
  double* qnode() { return reinterpret_cast<double*>(ws + off_qnode); }
  double* aux() { return reinterpret_cast<double*>(ws + off_aux); }  // 2 n_f: spline M, then solve scratch
  double* maps() { return reinterpret_cast<double*>(ws + off_maps); }
};

namespace {

int fail(bmc_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, x)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ != hipSuccess) return fail(ctx, BMC_EHIP, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

bool is_self_reverse(const Process& P) {
  if (P.n_in != P.n_out) return false;
  std::vector<int> a(P.sp, P.sp + P.n_in), b(P.sp + P.n_in, P.sp + P.n_in + P.n_out);
  std::sort(a.begin(), a.end());
  std::sort(b.begin(), b.end());
  return a == b;
}

int count_on_side(const Process& P, int a, int side) {
  int lo = side == 0 ? 0 : P.n_in, hi = side == 0 ? P.n_in : P.n_in + P.n_out, c = 0;
  for (int i = lo; i < hi; ++i) c += P.sp[i] == a;
  return c;
}

// Multiplicity of the side evaluation (0: not evaluated).
int multiplicity(const Process& P, int a, int side) {
  const int c = count_on_side(P, a, side);
  if (c == 0) return 0;
  const int mask = P.prm.side_mask;
  if (mask == BMC_SIDES_AUTO) return (is_self_reverse(P) && side == 1) ? 0 : c;
  return (mask & (1 << side)) ? c : 0;
}

// Observed: lowest index of species a on the side; conserved: lowest other index on the fewer-particle side
// (asymmetric) or on the observed side (symmetric), else the lowest other index on the opposite side.
bool assign_roles(const Process& P, int a, int side, int* obs, int* cons, int* integ) {
  const int n = P.n_in + P.n_out;
  auto range = [&](int s, int* lo, int* hi) {
    *lo = s == 0 ? 0 : P.n_in;
    *hi = s == 0 ? P.n_in : n;
  };
  int lo, hi;
  range(side, &lo, &hi);
  *obs = -1;
  for (int i = lo; i < hi && *obs < 0; ++i)
    if (P.sp[i] == a) *obs = i;
  if (*obs < 0) return false;
  const int cside = P.n_in != P.n_out ? (P.n_in < P.n_out ? 0 : 1) : side;
  *cons = -1;
  range(cside, &lo, &hi);
  for (int i = lo; i < hi && *cons < 0; ++i)
    if (i != *obs) *cons = i;
  if (*cons < 0) {
    range(1 - cside, &lo, &hi);
    for (int i = lo; i < hi && *cons < 0; ++i)
      if (i != *obs) *cons = i;
  }
  if (*cons < 0) return false;
  int k = 0;
  for (int i = 0; i < n; ++i)
    if (i != *obs && i != *cons) integ[k++] = i;
  return true;
}

int unit_size_for(int64_t N) {
  int64_t target = (N + 63) / 64;
  int64_t u = 4096;
  while (u < target && u < 65536) u <<= 1;
  return (int)u;
}

double grid_node(const Species& S, int j) {
  const double lq0 = std::log(S.q_min);
  const double h = (std::log(S.q_max) - lq0) / (double)(S.n - 1);
  return std::exp(lq0 + h * (double)j);
}

// Persistent layout from the registrations.
void layout_persistent(bmc_ctx* c) {
  size_t o = 0;
  c->off_state = o;
  o = align_up(o + sizeof(DevState));
  c->off_spec = o;
  o = align_up(o + sizeof(SpecDev) * kMaxSpecies);
  c->off_wctl = o;
  o = align_up(o + sizeof(WidthCtl) * std::max<size_t>(1, c->pr.size()));
  int64_t nf = 0;
  for (auto& s : c->sp) {
    s.f_off = nf;
    nf += s.n;
  }
  c->n_f = nf;
  c->off_f64 = o;
  o = align_up(o + 8 * nf);
  c->off_f32 = o;
  o = align_up(o + 4 * nf);
  c->off_f0 = o;
  o = align_up(o + 8 * nf);
  c->off_k1 = o;
  o = align_up(o + 8 * nf);
  c->off_k2 = o;
  o = align_up(o + 8 * nf);
  c->off_sig = o;
  o = align_up(o + 8 * nf);
  c->off_qnode = o;
  o = align_up(o + 8 * nf);
  c->off_aux = o;
  o = align_up(o + 16 * nf);
  // map slots: every item any call can plan (stride 1, both sides, both terms), at the grid nodes and at
  // kMaxEvalPoints evaluation points off the grid of every species
  int slots = 0;
  for (size_t p = 0; p < c->pr.size(); ++p)
    for (size_t a = 0; a < c->sp.size(); ++a)
      for (int side = 0; side < 2; ++side)
        if (multiplicity(c->pr[p], (int)a, side) > 0)
          slots += (c->sp[a].n + kMaxEvalPoints) * (c->pr[p].prm.term_mode == BMC_TERMS_NET ? 1 : 2);
  c->max_slots = slots;
  c->off_maps = o;
  o = align_up(o + sizeof(double) * (size_t)kSlotDoubles * (size_t)slots);
  c->persist_bytes = o;
}

SpecDev make_spec(bmc_ctx* c, const Species& S) {
  SpecDev d{};
  d.interp = S.interp;
  d.qn = c->qnode() + S.f_off;
  d.aux = c->aux() + S.f_off;
  d.tmp = c->aux() + c->n_f + S.f_off;
  d.stat = S.stat;
  d.n = S.n;
  d.q_min = S.q_min;
  d.q_max = S.q_max;
  d.lq0 = std::log(S.q_min);
  d.inv_h = (double)(S.n - 1) / (std::log(S.q_max) - d.lq0);
  d.mass_kind = S.mass_kind;
  d.m0 = S.m0;
  d.A = S.A;
  d.w = S.w;
  d.f_off = S.f_off;
  return d;
}

int upload_model(bmc_ctx* c) {
  std::vector<SpecDev> sd(kMaxSpecies);
  std::vector<double> qn;
  for (size_t i = 0; i < c->sp.size(); ++i) {
    sd[i] = make_spec(c, c->sp[i]);
    for (int j = 0; j < c->sp[i].n; ++j) qn.push_back(grid_node(c->sp[i], j));
  }
  HIPCHK(c, hipMemcpyAsync(c->spec(), sd.data(), sizeof(SpecDev) * kMaxSpecies, hipMemcpyHostToDevice, c->stream));
  std::vector<WidthCtl> wc(std::max<size_t>(1, c->pr.size()));
  for (size_t p = 0; p < c->pr.size(); ++p) {
    const bmc_process_params& q = c->pr[p].prm;
    wc[p] = WidthCtl{q.width_adapt, q.width_lo, q.width_hi, q.width_factor, q.width_min, q.width_max};
  }
  HIPCHK(c, hipMemcpyAsync(c->wctl(), wc.data(), sizeof(WidthCtl) * wc.size(), hipMemcpyHostToDevice, c->stream));
  if (!qn.empty())
    HIPCHK(c, hipMemcpyAsync(c->qnode(), qn.data(), 8 * qn.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BMC_OK;
}

int upload_state(bmc_ctx* c) {
  DevState s{};
  s.t = c->t;
  s.a = 1.0;
  s.inv_a = 1.0;
  for (int n = 0; n < 5; ++n) s.a_m3n[n] = 1.0;
  s.expansion = c->expansion;
  s.expansion_a0 = c->a0;
  s.expansion_t0 = c->t0;
  s.n_species = (int)c->sp.size();
  for (size_t i = 0; i < c->sp.size(); ++i) s.m[i] = c->sp[i].m0;
  for (size_t p = 0; p < c->pr.size(); ++p) s.width[p] = c->pr[p].width;
  HIPCHK(c, hipMemcpyAsync(c->st(), &s, sizeof(s), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BMC_OK;
}

int read_state(bmc_ctx* c, DevState* s) {
  HIPCHK(c, hipMemcpyAsync(s, c->st(), sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BMC_OK;
}

// Host mirrors of the device-side time and widths (before the device state is rebuilt).
void mirror_state(bmc_ctx* c, const DevState& s) {
  c->t = s.t;
  for (int p = 0; p < c->n_pr_bound && p < (int)c->pr.size(); ++p) c->pr[p].width = s.width[p];
}

int check_ready(bmc_ctx* c) {
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  if ((int)c->sp.size() != c->n_sp_bound || (int)c->pr.size() != c->n_pr_bound)
    return fail(c, BMC_ESTATE, "species or processes changed since the workspace was bound; query and bind again");
  if (c->pr.empty()) return fail(c, BMC_ESTATE, "no processes");
  for (auto& s : c->sp)
    if (!s.f_set) return fail(c, BMC_ESTATE, "f not set for species '" + s.name + "'");
  return BMC_OK;
}

// ---------------------------------------------------------------------------------------------- planner
struct PlanKey {
  int process, species, stride;
  int64_t n_samples;
  int n_iter;
  std::vector<double> eval_q;  // evaluation points off the grid (empty: the grid)
};

constexpr uint32_t kCustomBase = 1u << 17;  // identifier index of the first evaluation point off the grid

// scratch_base: where the plan's per-call scratch starts (nullptr: after the persistent part of the bound workspace);
// list_cap: bytes of screening lists one launch may fill; launch: the launch mode the second-pass records are
// reserved for (-1: either).
int build_plan(bmc_ctx* c, const PlanKey& k, Plan* P, char* scratch_base = nullptr,
               size_t list_cap = kListCapBytes, int launch = -1) {
  Plan Q;
  Q.process = k.process;
  Q.species = k.species;
  Q.stride = k.stride;
  Q.n_samples = k.n_samples;
  Q.n_iter = k.n_iter;
  Q.eval_q = k.eval_q;
  const int np = (int)c->pr.size(), ns = (int)c->sp.size();
  if (k.process < -1 || k.process >= np) return fail(c, BMC_EINVAL, "bad process id");
  if (k.species < -1 || k.species >= ns) return fail(c, BMC_EINVAL, "bad species id");
  const bool custom = !k.eval_q.empty();
  const int n_custom = (int)k.eval_q.size();
  if (custom && k.species < 0) return fail(c, BMC_EINVAL, "evaluation points need one species");
  for (double q : k.eval_q)
    if (!(q > 0.0) || !std::isfinite(q)) return fail(c, BMC_EINVAL, "evaluation points must be positive");
  // per (process, species): slot base for node 0 and its stride
  std::vector<std::vector<int>> slot_base(np, std::vector<int>(ns, -1));
  std::vector<std::vector<int>> pstride(np, std::vector<int>(ns, 0));
  int64_t part = 0, units = 0, shell = 0;
  int res = 0;
  std::vector<std::vector<int>> slot_lists;
  for (int p = 0; p < np; ++p) {
    if (k.process >= 0 && p != k.process) continue;
    const Process& Pr = c->pr[p];
    const int n = Pr.n_in + Pr.n_out;
    const int nint = n - 2;
    const int D = 3 * nint;
    const int nb = Pr.prm.n_bins;
    const int stride = k.stride > 0 ? k.stride : Pr.prm.eval_stride;
    const int64_t N = k.n_samples > 0 ? k.n_samples : Pr.prm.n_samples;
    const int nit = k.n_iter > 0 ? k.n_iter : Pr.prm.n_iter;
    if (N < 2) return fail(c, BMC_EINVAL, "n_samples < 2");
    // the word stream's block index D N / 4 stays below 2^32 (the device passes 0 as the counter's high word)
    if ((uint64_t)N * (uint64_t)D >= (1ull << 34)) return fail(c, BMC_EINVAL, "n_samples * D >= 2^34");
    if (nit < 1 || nit > kMaxIter) return fail(c, BMC_EINVAL, "n_iter out of range");
    for (int a = 0; a < ns; ++a) {
      if (k.species >= 0 && a != k.species) continue;
      const Species& S = c->sp[a];
      bool any = false;
      for (int side = 0; side < 2; ++side) any |= multiplicity(Pr, a, side) > 0;
      if (!any) continue;
      slot_base[p][a] = (int)slot_lists.size();
      pstride[p][a] = stride;
      const int n_nodes = custom ? n_custom : (S.n + stride - 1) / stride;
      const int first_slot = (int)slot_lists.size();
      slot_lists.resize(slot_lists.size() + n_nodes);
      for (int side = 0; side < 2; ++side) {
        const int mult = multiplicity(Pr, a, side);
        if (mult == 0) continue;
        int obs, cons, integ[kMaxInt];
        if (!assign_roles(Pr, a, side, &obs, &cons, integ)) return fail(c, BMC_EINVAL, "role assignment failed");
        const int n_terms = Pr.prm.term_mode == BMC_TERMS_NET ? 1 : 2;
        for (int term = 0; term < n_terms; ++term) {
          for (int pt = 0; pt < n_nodes; ++pt) {
            const int i = custom ? pt : pt * stride;
            ItemRec it{};
            it.uid = ((uint32_t)p << 24) | ((uint32_t)a << 20) | ((uint32_t)side << 19) | ((uint32_t)term << 18) |
                     (custom ? kCustomBase + (uint32_t)pt : (uint32_t)i);
            it.proc = p;
            it.nint = nint;
            it.D = D;
            it.nb = nb;
            it.term = term;
            it.net = Pr.prm.term_mode == BMC_TERMS_NET;
            it.eval_idx = i;
            it.obs_at = custom ? 1 : 0;
            it.n_iter = nit;
            it.q_obs = custom ? k.eval_q[pt] : grid_node(S, i);
            it.obs_species = a;
            it.mult = mult;
            it.N = N;
            it.unit_size = unit_size_for(N);
            it.n_units = Pr.prm.vegas_plus ? 0 : (int)((N + it.unit_size - 1) / it.unit_size);
            it.part_off = part;
            part += (int64_t)D * nb;  // the item's bin counts of the current iteration
            it.shell_off = shell;
            it.shell_units = shell_units_for(it.n_units, kShellGroupsBatched);
            it.shell_units_p = shell_units_for(it.n_units, kShellGroupsPlain);
            shell += shell_records(it.n_units, launch) * (2 + D * nb);
            it.res_off = res++;
            it.sign = (!it.net && term == 1) ? -1 : 1;
            it.coupling2 = Pr.prm.coupling * Pr.prm.coupling;
            it.rel = Pr.prm.width_mode == BMC_WIDTH_REL ? 1 : 0;
            it.vplus = Pr.prm.vegas_plus;
            it.beta = Pr.prm.beta;
            if (it.vplus) {
              it.vp_k = vplus_strata(N, D);
              int64_t M = 1;
              for (int d = 0; d < D; ++d) M *= it.vp_k;
              it.vp_M = (int)M;
              it.vp_blocks = (int)((M + kBlock - 1) / kBlock);
            }
            it.m2poly = Pr.prm.m2_kind == BMC_M2_POLY ? 1 : 0;
            for (int k2 = 0; k2 < 6; ++k2) it.m2c[k2] = Pr.prm.m2_coef[k2];
            it.e_cut = Pr.prm.e_cut;
            it.twopi_pow = std::pow(2.0 * M_PI, (double)(3 * (n - 1) - 4));
            it.alpha = Pr.prm.alpha;
            // roles
            int pos[kMaxN];
            for (int r = 0; r < nint; ++r) pos[r] = integ[r];
            pos[nint] = cons;
            pos[nint + 1] = obs;
            it.n_tab = 0;
            for (int r = 0; r < nint + 2; ++r) {
              const int q = pos[r];
              it.r_species[r] = Pr.sp[q];
              it.r_in[r] = q < Pr.n_in ? 1 : 0;
              it.r_obsside[r] = ((q < Pr.n_in) ? 0 : 1) == side ? 1 : 0;
              it.r_cs[r] = (q == 0 || (q == 1 && Pr.n_in >= 2)) ? 1 : 0;
              it.r_ct[r] = q == 0 ? 1 : (q == Pr.n_in ? -1 : 0);
              it.r_tab[r] = 0;
              if (r <= nint) {  // integrated and conserved particles read tables
                int slot = -1;
                for (int t = 0; t < it.n_tab; ++t)
                  if (it.tab_species[t] == Pr.sp[q]) slot = t;
                if (slot < 0) {
                  slot = it.n_tab++;
                  it.tab_species[slot] = Pr.sp[q];
                }
                it.r_tab[r] = slot;
              }
            }
            it.cons_in = cons < Pr.n_in ? 1 : 0;
            it.out_slot = first_slot + pt;
            // map slot
            auto f = c->slot_of_uid.find(it.uid);
            int ms;
            if (f == c->slot_of_uid.end()) {
              ms = (int)c->slot_of_uid.size();
              if (ms >= c->max_slots) return fail(c, BMC_ENOMEM, "map slots exhausted");
              c->slot_of_uid[it.uid] = ms;
              Q.new_maps.push_back((int)Q.items.size());
            } else {
              ms = f->second;
            }
            it.map_off = (int64_t)ms * kSlotDoubles;
            Q.nint_mask |= 1 << (nint - 1);
            Q.n_iter_max = std::max(Q.n_iter_max, nit);
            slot_lists[it.out_slot].push_back((int)Q.items.size());
            Q.items.push_back(it);
          }
        }
      }
    }
  }
  if (Q.items.empty()) return fail(c, BMC_EINVAL, "the selection has no work items");
  // units, tasks
  Q.unit_base.resize(Q.items.size());
  for (size_t i = 0; i < Q.items.size(); ++i) {
    Q.unit_base[i] = units;
    units += Q.items[i].n_units;
  }
  Q.n_units = units;
  Q.n_parts = part;
  // batched: item-major; items with more iterations first so that every iteration's tasks are a prefix
  std::vector<int> order(Q.items.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return Q.items[x].n_iter > Q.items[y].n_iter; });
  for (int i : order)
    for (int u = 0; u < Q.items[i].n_units; ++u) Q.tasks_batched.push_back(Task{i, u});
  Q.tasks_per_iter.assign(Q.n_iter_max, 0);
  for (int kk = 0; kk < Q.n_iter_max; ++kk) {
    int cnt = 0;
    for (int i : order)
      if (Q.items[i].n_iter > kk) cnt += Q.items[i].n_units;
    Q.tasks_per_iter[kk] = cnt;
  }
  // VEGAS+: hypercube arrays and sample blocks, items with more iterations first
  for (int i : order) {
    ItemRec& it = Q.items[i];
    if (!it.vplus) continue;
    it.vp_off = Q.vp_hc;
    it.vp_hb = Q.vp_hc + (int64_t)Q.vp_items.size();
    it.vp_rec = Q.vp_recd;
    Q.vp_hc += it.vp_M;
    Q.vp_recd += (int64_t)it.vp_blocks * (2 + 2 * (int64_t)it.D * it.nb);
    Q.vp_items.push_back(i);
    for (int b = 0; b < it.vp_blocks; ++b) Q.vp_tasks.push_back(VpTask{i, b});
  }
  // offsets: M + 1 entries per item, at vp_off + (the item's rank among the VEGAS+ items)
  Q.vp_hoffs = Q.vp_hc + (int64_t)Q.vp_items.size();
  Q.vp_per_iter.assign(Q.n_iter_max, 0);
  for (int kk = 0; kk < Q.n_iter_max; ++kk)
    for (int i : Q.vp_items)
      if (Q.items[i].n_iter > kk) Q.vp_per_iter[kk] += Q.items[i].vp_blocks;
  // plain: node-major
  {
    std::vector<int> byn(Q.items.size());
    for (size_t i = 0; i < byn.size(); ++i) byn[i] = (int)i;
    std::stable_sort(byn.begin(), byn.end(),
                     [&](int x, int y) { return Q.items[x].eval_idx < Q.items[y].eval_idx; });
    int last = -1;
    for (int i : byn) {
      if (Q.items[i].eval_idx != last) {
        Q.plain_node_begin.push_back((int)Q.tasks_plain.size());
        last = Q.items[i].eval_idx;
      }
      for (int u = 0; u < Q.items[i].n_units; ++u) Q.tasks_plain.push_back(Task{i, u});
    }
    Q.plain_node_begin.push_back((int)Q.tasks_plain.size());
  }
  // FP32 integrand: in-shell tasks, list sizing and slices of the batched launch
  {
    Q.n_shell = shell;
    std::vector<int> first_b(Q.items.size(), -1), first_p(Q.items.size(), -1);
    for (size_t t = 0; t < Q.tasks_batched.size(); ++t)
      if (Q.tasks_batched[t].unit == 0) first_b[Q.tasks_batched[t].item] = (int)t;
    for (size_t t = 0; t < Q.tasks_plain.size(); ++t)
      if (Q.tasks_plain[t].unit == 0) first_p[Q.tasks_plain[t].item] = (int)t;
    // groups of su consecutive units per second-pass task, in the order of the item's tasks
    auto groups = [&](int i, int first, int su, int tiles, std::vector<ShellTask>& out) {
      const ItemRec& it = Q.items[i];
      const int64_t stride = 2 + (int64_t)it.D * it.nb;
      for (int u = 0; u < it.n_units; u += su)
        out.push_back(
            ShellTask{i, first + u, u, std::min(it.n_units, u + su), it.shell_off + (u / su) * tiles * stride});
    };
    std::vector<int> sh_first(Q.items.size(), 0);
    for (int i : order) {
      sh_first[i] = (int)Q.sh_batched.size();
      groups(i, first_b[i], Q.items[i].shell_units, kShellTiles, Q.sh_batched);
    }
    Q.sh_per_iter.assign(Q.n_iter_max, 0);
    for (int kk = 0; kk < Q.n_iter_max; ++kk)
      for (int i : order)
        if (Q.items[i].n_iter > kk)
          Q.sh_per_iter[kk] += (int)shell_groups(Q.items[i].n_units, Q.items[i].shell_units);
    for (size_t g = 0; g + 1 < Q.plain_node_begin.size(); ++g) {
      Q.plain_node_sh_begin.push_back((int)Q.sh_plain.size());
      for (int t = Q.plain_node_begin[g]; t < Q.plain_node_begin[g + 1]; ++t)
        if (Q.tasks_plain[t].unit == 0)
          groups(Q.tasks_plain[t].item, t, Q.items[Q.tasks_plain[t].item].shell_units_p, 1, Q.sh_plain);
    }
    Q.plain_node_sh_begin.push_back((int)Q.sh_plain.size());
    int64_t umax = 0, pmin = 0;
    for (auto& it : Q.items) {
      umax = std::max<int64_t>(umax, it.unit_size);
      pmin = std::max<int64_t>(pmin, it.n_units);
    }
    for (size_t g = 0; g + 1 < Q.plain_node_begin.size(); ++g)
      pmin = std::max<int64_t>(pmin, Q.plain_node_begin[g + 1] - Q.plain_node_begin[g]);
    Q.list_stride = umax;
    Q.list_pos = std::min<int64_t>((int64_t)Q.tasks_batched.size(),
                                   std::max<int64_t>(pmin, (int64_t)(list_cap / (2 * (size_t)umax))));
    // slices: whole items in batched order, at most list_pos task positions each
    int tb = 0, sb = 0;
    for (size_t oi = 0; oi < order.size(); ++oi) {
      const int i = order[oi];
      const int te = first_b[i] + Q.items[i].n_units;
      if (te - tb > Q.list_pos) {
        Q.slices.push_back(Plan::Slice{tb, first_b[i], sb, sh_first[i]});
        tb = first_b[i];
        sb = sh_first[i];
      }
    }
    Q.slices.push_back(Plan::Slice{tb, (int)Q.tasks_batched.size(), sb, (int)Q.sh_batched.size()});
  }
  // slots
  Q.n_slots = (int)slot_lists.size();
  Q.slot_begin.push_back(0);
  for (auto& l : slot_lists) {
    for (int i : l) Q.slot_items.push_back(i);
    Q.slot_begin.push_back((int)Q.slot_items.size());
  }
  // gather
  for (int a = 0; a < ns; ++a) {
    if (k.species >= 0 && a != k.species) continue;
    const Species& S = c->sp[a];
    const int ostride = custom ? 1 : (k.stride > 0 ? k.stride : 1);
    const int n_pts = custom ? n_custom : S.n;
    for (int j = 0; j < n_pts; j += ostride) {
      GatherEntry g{};
      g.species = a;
      g.node = j;
      g.first = (int)Q.gproc.size();
      for (int p = 0; p < np; ++p) {
        if (slot_base[p][a] < 0) continue;
        GatherProc gp{};
        gp.slot_base = slot_base[p][a];
        gp.stride = custom ? 1 : pstride[p][a];
        gp.last = custom ? n_custom - 1 : ((S.n - 1) / gp.stride) * gp.stride;
        gp.fill = (custom || k.stride > 0) ? 0 : 1;
        Q.gproc.push_back(gp);
      }
      g.count = (int)Q.gproc.size() - g.first;
      Q.gather.push_back(g);
    }
  }
  Q.n_out = (int)Q.gather.size();
  // LDS bytes
  for (auto& it : Q.items) {
    int n_max = 0;
    for (int t = 0; t < it.n_tab; ++t) n_max = std::max(n_max, c->sp[it.tab_species[t]].n);
    Q.lds64 = std::max(Q.lds64, sample_lds_bytes(it.D, it.nb, it.n_tab, n_max, 0));
    Q.lds32 = std::max(Q.lds32, sample_lds_bytes(it.D, it.nb, it.n_tab, n_max, 1));
    Q.lds_sh64 = std::max(Q.lds_sh64, shell_lds_bytes(it.D, it.nb, it.n_tab, n_max, 0, 1));
    Q.lds_sh32 = std::max(Q.lds_sh32, shell_lds_bytes(it.D, it.nb, it.n_tab, n_max, 1, 1));
    Q.lds_sh64_lin = std::max(Q.lds_sh64_lin, shell_lds_bytes(it.D, it.nb, it.n_tab, n_max, 0, 0));
    Q.lds_sh32_lin = std::max(Q.lds_sh32_lin, shell_lds_bytes(it.D, it.nb, it.n_tab, n_max, 1, 0));
  }
  // the second pass's compact layout (every launch with the linear rule) is the least any plan needs; a launch with
  // the spline or equilibrium-exact rule is checked against its own layout when it is enqueued
  if (Q.lds_sh64_lin > 65536)
    return fail(c, BMC_EUNSUP, "per-block LDS need above 64 KB (grid or bins too large)");
  if (!Q.vp_items.empty() && ((Q.lds64 + 15) & ~15) + kVplusLdsExtra > 65536)
    return fail(c, BMC_EUNSUP, "per-block LDS of the VEGAS+ pass above 64 KB (grid or bins too large)");
  // scratch sizes
  size_t s = 0;
  auto take = [&](size_t bytes) {
    size_t o = s;
    s = align_up(s + bytes);
    return o;
  };
  const size_t nI = Q.items.size();
  size_t o_items = take(sizeof(ItemRec) * nI), o_tb = take(sizeof(Task) * Q.tasks_batched.size()),
         o_tp = take(sizeof(Task) * Q.tasks_plain.size()), o_shb = take(sizeof(ShellTask) * Q.sh_batched.size()),
         o_shp = take(sizeof(ShellTask) * Q.sh_plain.size()), o_list = take(2 * (size_t)(Q.list_pos * Q.list_stride)),
         o_cnt = take(8 * kWaves * (size_t)Q.list_pos), o_shell = take(8 * (size_t)Q.n_shell),
         o_ub = take(8 * nI), o_parts = take(4 * (size_t)part), o_rI = take(8 * kMaxIter * nI), o_rV = take(8 * kMaxIter * nI),
         o_ib = take(8 * nI), o_is = take(8 * nI), o_sb = take(4 * (Q.slot_begin.size())),
         o_si = take(4 * std::max<size_t>(1, Q.slot_items.size())), o_sC = take(8 * Q.n_slots),
         o_sS = take(8 * Q.n_slots), o_g = take(sizeof(GatherEntry) * Q.gather.size()),
         o_gp = take(sizeof(GatherProc) * std::max<size_t>(1, Q.gproc.size())), o_oC = take(8 * Q.n_out),
         o_oS = take(8 * Q.n_out), o_new = take(4 * std::max<size_t>(1, Q.new_maps.size()));
  const size_t o_vpt = take(sizeof(VpTask) * Q.vp_tasks.size()), o_vpi = take(4 * Q.vp_items.size()),
               o_nh = take(4 * (size_t)Q.vp_hc), o_hoff = take(8 * (size_t)Q.vp_hoffs),
               o_vS1 = take(8 * (size_t)Q.vp_hc), o_vS2 = take(8 * (size_t)Q.vp_hc), o_vrec = take(8 * (size_t)Q.vp_recd);
  Q.scratch_bytes = s;
  char* base = scratch_base ? scratch_base : (c->ws ? c->ws + c->persist_bytes : nullptr);
  Q.in_static = scratch_base != nullptr;
  if (base) {
    Q.d_items = reinterpret_cast<ItemRec*>(base + o_items);
    Q.d_tb = reinterpret_cast<Task*>(base + o_tb);
    Q.d_tp = reinterpret_cast<Task*>(base + o_tp);
    Q.d_shb = reinterpret_cast<ShellTask*>(base + o_shb);
    Q.d_shp = reinterpret_cast<ShellTask*>(base + o_shp);
    Q.d_list = reinterpret_cast<uint16_t*>(base + o_list);
    Q.d_cnt = reinterpret_cast<uint32_t*>(base + o_cnt);
    Q.d_shell = reinterpret_cast<double*>(base + o_shell);
    Q.d_unit_base = reinterpret_cast<int64_t*>(base + o_ub);
    Q.d_counts = reinterpret_cast<uint32_t*>(base + o_parts);
    Q.n_counts = part;
    Q.d_res_I = reinterpret_cast<double*>(base + o_rI);
    Q.d_res_V = reinterpret_cast<double*>(base + o_rV);
    Q.d_item_Ibar = reinterpret_cast<double*>(base + o_ib);
    Q.d_item_sig = reinterpret_cast<double*>(base + o_is);
    Q.d_slot_begin = reinterpret_cast<int*>(base + o_sb);
    Q.d_slot_items = reinterpret_cast<int*>(base + o_si);
    Q.d_slot_C = reinterpret_cast<double*>(base + o_sC);
    Q.d_slot_S2 = reinterpret_cast<double*>(base + o_sS);
    Q.d_gather = reinterpret_cast<GatherEntry*>(base + o_g);
    Q.d_gproc = reinterpret_cast<GatherProc*>(base + o_gp);
    Q.d_out_C = reinterpret_cast<double*>(base + o_oC);
    Q.d_out_S = reinterpret_cast<double*>(base + o_oS);
    Q.d_new = reinterpret_cast<int*>(base + o_new);
    Q.d_vpt = reinterpret_cast<VpTask*>(base + o_vpt);
    Q.d_vpi = reinterpret_cast<int*>(base + o_vpi);
    Q.d_nh = reinterpret_cast<int*>(base + o_nh);
    Q.d_hoff = reinterpret_cast<int64_t*>(base + o_hoff);
    Q.d_vS1 = reinterpret_cast<double*>(base + o_vS1);
    Q.d_vS2 = reinterpret_cast<double*>(base + o_vS2);
    Q.d_vrec = reinterpret_cast<double*>(base + o_vrec);
  }
  *P = std::move(Q);
  return BMC_OK;
}

// Worst-case scratch for the registered model.
size_t scratch_estimate(bmc_ctx* c, int64_t max_samples, int max_iter) {
  size_t s = 0;
  size_t items = 0, units = 0, part = 0, slots = 0, outs = 0, tasks = 0, shell = 0, umax = 0, per_node = 0,
         per_item = 0;
  for (auto& Pr : c->pr) {
    const int n = Pr.n_in + Pr.n_out;
    const int D = 3 * (n - 2);
    const int64_t N = std::max<int64_t>(max_samples > 0 ? max_samples : 0, Pr.prm.n_samples);
    const int U = unit_size_for(N);
    const int64_t nu = (N + U - 1) / U;
    umax = std::max<size_t>(umax, (size_t)U);
    per_item = std::max<size_t>(per_item, (size_t)nu);
    for (size_t a = 0; a < c->sp.size(); ++a) {
      int sides = 0;
      for (int side = 0; side < 2; ++side) sides += multiplicity(Pr, (int)a, side) > 0;
      if (!sides) continue;
      const int terms = Pr.prm.term_mode == BMC_TERMS_NET ? 1 : 2;
      const size_t ni = (size_t)c->sp[a].n * sides * terms;
      items += ni;
      units += ni * nu;
      tasks += ni * nu;
      part += ni * D * Pr.prm.n_bins;
      shell += ni * (size_t)shell_records(nu) * (2 + D * Pr.prm.n_bins);
      per_node += (size_t)sides * terms * nu;
      slots += c->sp[a].n;
    }
  }
  // VEGAS+ hypercube arrays (at most N / 2 hypercubes per item) and block records
  for (auto& Pr : c->pr) {
    if (!Pr.prm.vegas_plus) continue;
    const int D = 3 * (Pr.n_in + Pr.n_out - 2);
    const int64_t N = std::max<int64_t>(max_samples > 0 ? max_samples : 0, Pr.prm.n_samples);
    size_t ni = 0;
    for (size_t a = 0; a < c->sp.size(); ++a) {
      int sides = 0;
      for (int side = 0; side < 2; ++side) sides += multiplicity(Pr, (int)a, side) > 0;
      ni += (size_t)c->sp[a].n * sides * (Pr.prm.term_mode == BMC_TERMS_NET ? 1 : 2);
    }
    const size_t M = (size_t)(N / 2), blocks = (M + kBlock - 1) / kBlock;
    s += ni * (align_up(4 * M) + align_up(8 * (M + 1)) + 2 * align_up(8 * M) +
               align_up(8 * blocks * (2 + 2 * (size_t)D * Pr.prm.n_bins)) + sizeof(VpTask) * blocks + 4);
  }
  // in-shell lists of the FP32-integrand screening pass (one slice's task positions)
  const size_t list_pos =
      std::min(units, std::max(std::max(per_item, per_node), kListCapBytes / (2 * std::max<size_t>(1, umax))));
  s += align_up(2 * list_pos * umax) + align_up(8 * kWaves * list_pos) + align_up(8 * shell) +
       2 * align_up(sizeof(ShellTask) * units);
  for (auto& S : c->sp) outs += S.n;
  (void)max_iter;
  // adjoint records: per unit n_tab * n_max (twice that with a spline table) + 12 doubles (n_tab <= 4 tables of at
  // most the largest grid); the spline adjoint's 3 n_f doubles of scratch
  size_t gmax = 0, vjp_part = 0;
  for (auto& S : c->sp) gmax = std::max(gmax, (size_t)S.n);
  for (auto& Pr : c->pr) {
    const int64_t N = std::max<int64_t>(max_samples > 0 ? max_samples : 0, Pr.prm.n_samples);
    const int U = unit_size_for(N);
    const int64_t nu = (N + U - 1) / U;
    int ntab = 0, spl = 0;
    for (size_t a = 0; a < c->sp.size(); ++a) {
      bool used = false;
      for (int i = 0; i < Pr.n_in + Pr.n_out; ++i) used |= Pr.sp[i] == (int)a;
      ntab += used;
      spl |= used && c->sp[a].interp == BMC_INTERP_SPLINE ? 1 : 0;
    }
    for (size_t a = 0; a < c->sp.size(); ++a) {
      int sides = 0;
      for (int side = 0; side < 2; ++side) sides += multiplicity(Pr, (int)a, side) > 0;
      const size_t ni = (size_t)c->sp[a].n * sides * (Pr.prm.term_mode == BMC_TERMS_NET ? 1 : 2);
      vjp_part += ni * nu * (ntab * gmax * (1 + spl) + 12);
    }
  }
  s += align_up(8 * vjp_part) + align_up((sizeof(ItemRec) + 8 * (8 * gmax + 12) + 24) * items) +
       align_up(8 * (size_t)c->n_f) + align_up(24 * (size_t)c->n_f) + 4 * kAlign + 16 * c->pr.size();
  s += align_up(sizeof(ItemRec) * items) + 2 * align_up(sizeof(Task) * tasks) + align_up(8 * items) +
       align_up(4 * part) + 2 * align_up(8 * kMaxIter * items) + 2 * align_up(8 * items) +
       align_up(4 * (slots + 1)) + align_up(4 * items) + 2 * align_up(8 * slots) +
       align_up(sizeof(GatherEntry) * outs) + align_up(sizeof(GatherProc) * outs * std::max<size_t>(1, c->pr.size())) +
       2 * align_up(8 * outs) + align_up(4 * items) + 64 * kAlign;
  return s;
}

int upload_plan(bmc_ctx* c, Plan& P) {
  if (!P.in_static && c->persist_bytes + P.scratch_bytes > c->ws_bytes)
    return fail(c, BMC_ENOMEM, "workspace too small for this call: need " +
                                   std::to_string(c->persist_bytes + P.scratch_bytes) + " bytes");
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(P.d_items, P.items.data(), sizeof(ItemRec) * P.items.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(P.d_tb, P.tasks_batched.data(), sizeof(Task) * P.tasks_batched.size(),
                           hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(P.d_tp, P.tasks_plain.data(), sizeof(Task) * P.tasks_plain.size(), hipMemcpyHostToDevice,
                           s));
  HIPCHK(c, hipMemcpyAsync(P.d_unit_base, P.unit_base.data(), 8 * P.unit_base.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(P.d_shb, P.sh_batched.data(), sizeof(ShellTask) * P.sh_batched.size(),
                           hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(P.d_shp, P.sh_plain.data(), sizeof(ShellTask) * P.sh_plain.size(), hipMemcpyHostToDevice,
                           s));
  HIPCHK(c, hipMemcpyAsync(P.d_slot_begin, P.slot_begin.data(), 4 * P.slot_begin.size(), hipMemcpyHostToDevice, s));
  if (!P.vp_tasks.empty()) {
    HIPCHK(c, hipMemcpyAsync(P.d_vpt, P.vp_tasks.data(), sizeof(VpTask) * P.vp_tasks.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipMemcpyAsync(P.d_vpi, P.vp_items.data(), 4 * P.vp_items.size(), hipMemcpyHostToDevice, s));
  }
  if (!P.slot_items.empty())
    HIPCHK(c, hipMemcpyAsync(P.d_slot_items, P.slot_items.data(), 4 * P.slot_items.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(P.d_gather, P.gather.data(), sizeof(GatherEntry) * P.gather.size(), hipMemcpyHostToDevice,
                           s));
  if (!P.gproc.empty())
    HIPCHK(c, hipMemcpyAsync(P.d_gproc, P.gproc.data(), sizeof(GatherProc) * P.gproc.size(), hipMemcpyHostToDevice,
                             s));
  if (!P.new_maps.empty()) {
    HIPCHK(c, hipMemcpyAsync(P.d_new, P.new_maps.data(), 4 * P.new_maps.size(), hipMemcpyHostToDevice, s));
    HIPCHK(c, launch_init_maps(P.d_items, P.d_new, (int)P.new_maps.size(), c->spec(), c->maps(), s));
    P.new_maps.clear();
  }
  // the items' bin counts start at zero (each iteration's reduction reads and clears them)
  if (P.d_counts) HIPCHK(c, hipMemsetAsync(P.d_counts, 0, 4 * (size_t)P.n_counts, s));
  HIPCHK(c, hipStreamSynchronize(s));
  P.uploaded = true;
  return BMC_OK;
}

int grid_for(bmc_ctx* c, int precision, int lds, int mask) {
  if (c->n_cu <= 0) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return 256;
    c->n_cu = prop.multiProcessorCount;
  }
  int per_cu = c->blocks_per_cu;
  if (per_cu <= 0) {
    // LDS-limited residency (160 KB per CU), at most 8 blocks of 256 threads
    per_cu = std::max(1, std::min(8, (160 * 1024) / std::max(1, lds)));
    (void)precision;
    (void)mask;
  }
  return c->n_cu * per_cu;
}

// The sample phase of one launch: the screening pass and the second pass (FP64 or FP32 integrand).
// With timing on (eager launches only) the phase is bracketed by events on the launch stream.
hipError_t sample_phase(bmc_ctx* c, const SampleLaunch& L, hipStream_t s) {
  hipEvent_t a = nullptr, m = nullptr, b = nullptr;
  hipError_t e;
  const bool timed = c->timing && !c->capturing && (c->phase_count++ % c->timing_every) == 0;
  if (timed) {
    if ((e = hipEventCreate(&a)) != hipSuccess) return e;
    if ((e = hipEventCreate(&m)) != hipSuccess) return e;
    if ((e = hipEventCreate(&b)) != hipSuccess) return e;
    if ((e = hipEventRecord(a, s)) != hipSuccess) return e;
  }
  if ((e = launch_sample(L, s)) != hipSuccess) return e;
  if (timed && (e = hipEventRecord(m, s)) != hipSuccess) return e;
  if ((e = launch_shell(L, s)) != hipSuccess) return e;
  if (timed) {
    e = hipEventRecord(b, s);
    c->ev.push_back({a, m, b});
  }
  return e;
}

// Enqueues one evaluation of plan P (all iterations, combine, gather) on the context stream.  The screening pass
// counts the samples per bin where the maps adapt, or where count_bins forces it (the autotuner times frozen-map
// calls of a run that will adapt).
int enqueue_eval(bmc_ctx* c, Plan& P, const bmc_run_opts& o, double* out_C, double* out_S, bool count_bins = false) {
  hipStream_t s = c->stream;
  int any_interp = 0;
  for (auto& S : c->sp) any_interp |= S.interp != BMC_INTERP_LINLOG ? 1 : 0;
  for (auto& Pr : c->pr) any_interp |= Pr.prm.m2_kind != BMC_M2_CONST ? 1 : 0;
  const int shell_lds = any_interp ? (o.precision == BMC_FP64 ? P.lds_sh64 : P.lds_sh32)
                                   : (o.precision == BMC_FP64 ? P.lds_sh64_lin : P.lds_sh32_lin);
  if (shell_lds > 65536)  // checked before anything is enqueued
    return fail(c, BMC_EUNSUP,
                "per-block LDS of the second pass above 64 KB with the spline, equilibrium-exact rule or polynomial "
                "|M|^2 (grid or bins too large)");
  HIPCHK(c, launch_next_epoch(c->st(), s));
  HIPCHK(c, launch_prepare(c->st(), c->spec(), (int)c->sp.size(), c->f64(), c->f32(), c->n_f, s));
  SampleLaunch L{};
  L.items = P.d_items;
  L.spec = c->spec();
  L.f64 = c->f64();
  L.f32 = c->f32();
  L.qnode = c->qnode();
  L.st = c->st();
  L.maps = c->maps();
  // bin counts only where the maps adapt (frozen maps: the screening pass runs without its count atomics; the
  // reduction clears the counts either way)
  L.counts = (o.freeze_maps && !count_bins) ? nullptr : P.d_counts;
  L.unit_base = P.d_unit_base;
  L.seed_lo = (uint32_t)o.seed;
  L.seed_hi = (uint32_t)(o.seed >> 32);
  L.nint_mask = P.nint_mask;
  L.precision = o.precision;
  L.any_interp = any_interp;
  L.lds_bytes = o.precision == BMC_FP64 ? P.lds64 : P.lds32;
  // the second pass's layout follows its kernel instance: tables of f alone when every rule is the linear one
  L.shell_lds = shell_lds;
  L.shell_list = P.d_list;
  L.shell_cnt = P.d_cnt;
  L.list_stride = P.list_stride;
  L.shell_rec = P.d_shell;
  L.n_listed = &c->st()->n_listed;
  L.vp_tasks = P.d_vpt;
  L.vp_nh = P.d_nh;
  L.vp_hoff = P.d_hoff;
  L.vp_S1 = P.d_vS1;
  L.vp_S2 = P.d_vS2;
  L.vp_rec = P.d_vrec;
  const int n_vpi = (int)P.vp_items.size();
  if (n_vpi) HIPCHK(c, launch_vplus_init(P.d_items, P.d_vpi, n_vpi, P.d_nh, P.d_hoff, s));
  // persistent grid of the screening pass (its blocks hold the FP32 map only); the second pass's task grid is capped
  // by the same count
  const int max_grid = grid_for(c, o.precision, screen_lds_bytes(), P.nint_mask);
  for (int k = 0; k < P.n_iter_max; ++k) {
    L.it = o.first_iter + k;
    if (o.launch == BMC_LAUNCH_PLAIN) {
      L.tasks = P.d_tp;
      L.sh_tasks = P.d_shp;
      for (size_t g = 0; g + 1 < P.plain_node_begin.size(); ++g) {
        L.task_begin = P.plain_node_begin[g];
        L.n_tasks = P.plain_node_begin[g + 1] - P.plain_node_begin[g];
        L.grid = L.n_tasks;
        L.chunk = 1;
        L.sh_begin = P.plain_node_sh_begin[g];
        L.n_sh = P.plain_node_sh_begin[g + 1] - P.plain_node_sh_begin[g];
        L.sh_tiles = 1;
        L.sh_grid = L.n_sh;
        HIPCHK(c, sample_phase(c, L, s));
      }
    } else {
      L.tasks = P.d_tb;
      L.sh_tasks = P.d_shb;
      L.chunk = c->chunk;
      for (const Plan::Slice& sl : P.slices) {
        const int te = std::min(sl.te, P.tasks_per_iter[k]);
        if (sl.tb >= te) break;
        L.task_begin = sl.tb;
        L.n_tasks = te - sl.tb;
        L.grid = std::min((L.n_tasks + L.chunk - 1) / L.chunk, max_grid);
        L.sh_begin = sl.sb;
        L.n_sh = std::min(sl.se, P.sh_per_iter[k]) - sl.sb;
        L.sh_tiles = kShellTiles;  // each group in equal tiles, one block each
        L.sh_grid = L.n_sh * kShellTiles;
        HIPCHK(c, sample_phase(c, L, s));
      }
    }
    if (n_vpi && P.vp_per_iter[k] > 0) {  // VEGAS+ items: their own sample blocks and reduction
      L.n_vp = P.vp_per_iter[k];
      HIPCHK(c, launch_vplus(L, s));
      HIPCHK(c, launch_vplus_reduce(P.d_items, P.d_vpi, n_vpi, P.d_nh, P.d_hoff, P.d_vS1, P.d_vS2, P.d_vrec, P.d_res_I,
                                    P.d_res_V, k, c->maps(), o.freeze_maps, s));
    }
    HIPCHK(c, launch_reduce_adapt(P.d_items, 0, (int)P.items.size(), P.d_counts, P.d_shell, P.d_res_I, P.d_res_V, k,
                                  c->maps(), o.freeze_maps, o.launch == BMC_LAUNCH_PLAIN ? 1 : 0, s));
  }
  HIPCHK(c, launch_combine(P.d_items, (int)P.items.size(), P.d_res_I, P.d_res_V, P.n_iter_max, P.d_item_Ibar,
                           P.d_item_sig, P.d_slot_begin, P.d_slot_items, P.n_slots, P.d_slot_C, P.d_slot_S2, s));
  HIPCHK(c, launch_gather(P.d_gather, P.n_out, P.d_gproc, P.d_slot_C, P.d_slot_S2, c->spec(), c->f64(), out_C, out_S,
                          s));
  bool adapt = false;
  for (auto& pr : c->pr) adapt |= pr.prm.width_adapt != 0;
  if (adapt)
    HIPCHK(c, launch_width_control(P.d_items, (int)P.items.size(), P.d_item_Ibar, P.d_item_sig, c->wctl(),
                                   (int)c->pr.size(), c->st(), s));
  return BMC_OK;
}

int check_opts(bmc_ctx* c, const bmc_run_opts* o) {
  if (!o) return fail(c, BMC_EINVAL, "opts is NULL");
  if (o->precision != BMC_FP64 && o->precision != BMC_FP32I) return fail(c, BMC_EINVAL, "bad precision");
  if (o->launch != BMC_LAUNCH_BATCHED && o->launch != BMC_LAUNCH_PLAIN) return fail(c, BMC_EINVAL, "bad launch");
  if (o->epoch >= (1u << 26)) return fail(c, BMC_EINVAL, "epoch >= 2^26");
  if (o->first_iter < 0 || o->eval_stride < 0) return fail(c, BMC_EINVAL, "negative first_iter or eval_stride");
  if (o->eval_q && (o->n_eval < 1 || o->n_eval > kMaxEvalPoints))
    return fail(c, BMC_EINVAL, "n_eval must be in 1 .. " + std::to_string(kMaxEvalPoints) + " when eval_q is given");
  return BMC_OK;
}

PlanKey plan_key(int process, int species, const bmc_run_opts* o) {
  PlanKey k{process, species, o->eval_stride, o->n_samples, o->n_iter, {}};
  if (o->eval_q) k.eval_q.assign(o->eval_q, o->eval_q + o->n_eval);
  return k;
}

// The context's plan in `slot` is built for key k and uploaded (the calls that change the model reset it).
bool plan_matches(const Plan& slot, const PlanKey& k) {
  return slot.process == k.process && slot.species == k.species && slot.stride == k.stride &&
         slot.n_samples == k.n_samples && slot.n_iter == k.n_iter && slot.eval_q == k.eval_q && slot.uploaded;
}

int get_plan(bmc_ctx* c, Plan& slot, int process, int species, const bmc_run_opts* o) {
  const PlanKey k = plan_key(process, species, o);
  const bool same = plan_matches(slot, k);
  if (!same) {
    int rc = build_plan(c, k, &slot);
    if (rc) {
      slot = Plan();
      return rc;
    }
  }
  int nit_max = slot.n_iter_max;
  if (o->first_iter + nit_max > kMaxIter) return fail(c, BMC_EINVAL, "first_iter + n_iter > 64");
  if (!slot.uploaded || !slot.new_maps.empty()) return upload_plan(c, slot);
  return BMC_OK;
}

int finish_check(bmc_ctx* c) {
  DevState s;
  int rc = read_state(c, &s);
  if (rc) return rc;
  if (s.err) {
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(&c->st()->err, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return fail(c, BMC_ERANGE, "invalid distribution table (f <= 0, Fermi-Dirac f >= 1 or invalid extrapolation fit)");
  }
  return BMC_OK;
}

}  // namespace

// ================================================================================================ C-ABI
extern "C" {

int bmc_create(bmc_ctx** out, int device, void* hip_stream) {
  if (!out) return BMC_EINVAL;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return BMC_EINVAL;
  bmc_ctx* c = new (std::nothrow) bmc_ctx();
  if (!c) return BMC_ENOMEM;
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) {
    delete c;
    return BMC_EHIP;
  }
  if (device >= kMaxDevices || resolve_scratch(device) != hipSuccess) {
    delete c;
    return BMC_EHIP;
  }
  *out = c;
  return BMC_OK;
}

int bmc_destroy(bmc_ctx* c) {
  if (!c) return BMC_EINVAL;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  delete c;
  return BMC_OK;
}

int bmc_set_stream(bmc_ctx* c, void* hip_stream) {
  if (!c) return BMC_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return BMC_OK;
}

int bmc_default_process_params(bmc_process_params* p) {
  if (!p) return BMC_EINVAL;
  p->coupling = 1.0;
  p->sigma_E = 0.01;
  p->alpha = 0.5;
  p->e_cut = 0.0;
  p->n_bins = 50;
  p->term_mode = BMC_TERMS_SPLIT;
  p->side_mask = BMC_SIDES_AUTO;
  p->eval_stride = 1;
  p->n_samples = 1000000;
  p->n_iter = 2;
  p->width_mode = BMC_WIDTH_ABS;
  p->width_adapt = 0;
  p->width_lo = 1e-3;
  p->width_hi = 1e-2;
  p->width_factor = 1.25;
  p->width_min = 1e-4;
  p->width_max = 0.2;
  p->vegas_plus = 0;
  p->beta = 0.75;
  p->m2_kind = BMC_M2_CONST;
  p->m2_coef[0] = 1.0;
  for (int k = 1; k < 6; ++k) p->m2_coef[k] = 0.0;
  return BMC_OK;
}

int bmc_add_species(bmc_ctx* c, const char* name, int stat, int grid_kind, int n_grid, double q_min, double q_max,
                    int* species_id) {
  if (!c) return BMC_EINVAL;
  if (stat != BMC_BOSE && stat != BMC_FERMI && stat != BMC_MB) return fail(c, BMC_EINVAL, "bad statistics");
  if (grid_kind != BMC_GRID_LOG) return fail(c, BMC_EUNSUP, "only logarithmic grids are implemented");
  if (n_grid < 10 || n_grid > BMC_MAXGRID) return fail(c, BMC_EINVAL, "n_grid must be in [10, 2048]");
  if (!(q_min > 0.0) || !(q_max > q_min) || !std::isfinite(q_max)) return fail(c, BMC_EINVAL, "bad momentum range");
  if ((int)c->sp.size() >= kMaxSpecies) return fail(c, BMC_EINVAL, "too many species");
  Species s;
  s.name = name ? name : "";
  s.stat = stat;
  s.n = n_grid;
  s.q_min = q_min;
  s.q_max = q_max;
  s.m0 = 0.0;
  s.f.assign(n_grid, 0.0);
  c->sp.push_back(s);
  if (species_id) *species_id = (int)c->sp.size() - 1;
  return BMC_OK;
}

int bmc_set_mass(bmc_ctx* c, int species, int kind, double m0, double A, double w) {
  if (!c) return BMC_EINVAL;
  if (species < 0 || species >= (int)c->sp.size()) return fail(c, BMC_EINVAL, "bad species id");
  if (kind != BMC_MASS_CONST && kind != BMC_MASS_SIN) return fail(c, BMC_EINVAL, "bad mass kind");
  if (!(m0 >= 0.0) || !std::isfinite(A) || !std::isfinite(w) || (kind == BMC_MASS_SIN && m0 - std::fabs(A) < 0.0))
    return fail(c, BMC_EINVAL, "mass must stay non-negative");
  Species& s = c->sp[species];
  s.mass_kind = kind;
  s.m0 = m0;
  s.A = kind == BMC_MASS_SIN ? A : 0.0;
  s.w = kind == BMC_MASS_SIN ? w : 0.0;
  if (c->bound && species < c->n_sp_bound) {
    int rc = upload_model(c);
    if (rc) return rc;
  }
  return BMC_OK;
}

int bmc_set_interp(bmc_ctx* c, int species, int mode) {
  if (!c) return BMC_EINVAL;
  if (species < 0 || species >= (int)c->sp.size()) return fail(c, BMC_EINVAL, "bad species id");
  if (mode != BMC_INTERP_LINLOG && mode != BMC_INTERP_SPLINE && mode != BMC_INTERP_EQEXACT)
    return fail(c, BMC_EINVAL, "bad interpolation rule");
  c->sp[species].interp = mode;
  if (c->bound && species < c->n_sp_bound) {
    int rc = upload_model(c);
    if (rc) return rc;
  }
  return BMC_OK;
}

int bmc_set_f(bmc_ctx* c, int species, const double* f, int n, int mem) {
  if (!c || !f) return BMC_EINVAL;
  if (species < 0 || species >= (int)c->sp.size()) return fail(c, BMC_EINVAL, "bad species id");
  Species& s = c->sp[species];
  if (n != s.n) return fail(c, BMC_EINVAL, "n does not match the grid");
  std::vector<double> h(n);
  if (mem == BMC_MEM_DEVICE) {
    HIPCHK(c, hipMemcpyAsync(h.data(), f, 8 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::memcpy(h.data(), f, 8 * n);
  }
  for (int j = 0; j < n; ++j) {
    if (!(h[j] > 0.0) || !std::isfinite(h[j])) return fail(c, BMC_ERANGE, "f must be positive and finite");
    if (s.stat == BMC_FERMI && !(h[j] < 1.0)) return fail(c, BMC_ERANGE, "Fermi-Dirac f must be below 1");
  }
  s.f = h;
  s.f_set = true;
  if (c->bound && species < c->n_sp_bound) {
    HIPCHK(c, hipMemcpyAsync(c->f64() + s.f_off, s.f.data(), 8 * n, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return BMC_OK;
}

int bmc_get_f(bmc_ctx* c, int species, double* f, int n, int mem) {
  if (!c || !f) return BMC_EINVAL;
  if (species < 0 || species >= (int)c->sp.size()) return fail(c, BMC_EINVAL, "bad species id");
  Species& s = c->sp[species];
  if (n != s.n) return fail(c, BMC_EINVAL, "n does not match the grid");
  if (c->bound && species < c->n_sp_bound) {
    HIPCHK(c, hipMemcpyAsync(f, c->f64() + s.f_off, 8 * n,
                             mem == BMC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    HIPCHK(c, hipMemcpy(f, s.f.data(), 8 * n, mem == BMC_MEM_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost));
  }
  return BMC_OK;
}

int bmc_add_process(bmc_ctx* c, const int* in_sp, int n_in, const int* out_sp, int n_out,
                    const bmc_process_params* prm, int* process_id) {
  if (!c || !in_sp || !out_sp || !prm) return BMC_EINVAL;
  if (n_in < 1 || n_out < 1 || n_in + n_out < 3 || n_in + n_out > kMaxN)
    return fail(c, BMC_EINVAL, "need 1 <= n_in, n_out and 3 <= n_in + n_out <= 6");
  if ((int)c->pr.size() >= kMaxProc - 1) return fail(c, BMC_EINVAL, "too many processes");
  Process P;
  P.n_in = n_in;
  P.n_out = n_out;
  for (int i = 0; i < n_in; ++i) P.sp[i] = in_sp[i];
  for (int i = 0; i < n_out; ++i) P.sp[n_in + i] = out_sp[i];
  for (int i = 0; i < n_in + n_out; ++i)
    if (P.sp[i] < 0 || P.sp[i] >= (int)c->sp.size()) return fail(c, BMC_EINVAL, "process references an unknown species");
  const bmc_process_params& q = *prm;
  if (!(q.sigma_E > 0.0) || !(q.alpha >= 0.0 && q.alpha <= 2.0) || q.n_bins < 2 || q.n_bins > kMaxBins ||
      (q.term_mode != BMC_TERMS_SPLIT && q.term_mode != BMC_TERMS_NET) || q.side_mask < 0 || q.side_mask > 3 ||
      q.eval_stride < 1 || q.n_samples < 2 || q.n_iter < 1 || q.n_iter > kMaxIter || !std::isfinite(q.coupling))
    return fail(c, BMC_EINVAL, "bad process parameters");
  if ((uint64_t)q.n_samples * (uint64_t)(3 * (n_in + n_out - 2)) >= (1ull << 34))
    return fail(c, BMC_EINVAL, "n_samples * D >= 2^34");
  if (q.width_mode != BMC_WIDTH_ABS && q.width_mode != BMC_WIDTH_REL)
    return fail(c, BMC_EINVAL, "bad width_mode");
  // a relative width stays <= 1: the screening pass's energy margins assume it
  if (q.width_mode == BMC_WIDTH_REL && !(q.sigma_E <= 1.0)) return fail(c, BMC_EINVAL, "relative width above 1");
  if (q.width_adapt != 0 && q.width_adapt != 1) return fail(c, BMC_EINVAL, "width_adapt must be 0 or 1");
  if (q.m2_kind != BMC_M2_CONST && q.m2_kind != BMC_M2_POLY) return fail(c, BMC_EINVAL, "bad m2_kind");
  if ((q.vegas_plus != 0 && q.vegas_plus != 1) || !(q.beta >= 0.0 && q.beta <= 2.0))
    return fail(c, BMC_EINVAL, "vegas_plus must be 0 or 1 and beta in [0, 2]");
  for (int k = 0; k < 6; ++k)
    if (!std::isfinite(q.m2_coef[k])) return fail(c, BMC_EINVAL, "non-finite |M|^2 coefficient");
  if (q.width_adapt &&
      (!(q.width_lo > 0.0) || !(q.width_hi > q.width_lo) || !std::isfinite(q.width_hi) || !(q.width_factor > 1.0) ||
       !std::isfinite(q.width_factor) || !(q.width_min > 0.0) || !(q.width_max >= q.width_min) ||
       !std::isfinite(q.width_max) || (q.width_mode == BMC_WIDTH_REL && q.width_max > 1.0)))
    return fail(c, BMC_EINVAL, "bad width controller parameters");
  P.prm = q;
  P.width = q.sigma_E;
  c->pr.push_back(P);
  if (process_id) *process_id = (int)c->pr.size() - 1;
  return BMC_OK;
}

int bmc_set_coupling(bmc_ctx* c, int process, double coupling) {
  if (!c) return BMC_EINVAL;
  if (process < 0 || process >= (int)c->pr.size() || !std::isfinite(coupling))
    return fail(c, BMC_EINVAL, "bad process id or coupling");
  c->pr[process].prm.coupling = coupling;
  c->plan = Plan();
  c->step_plan = Plan();
  return BMC_OK;
}

int bmc_get_width(bmc_ctx* c, int process, double* width) {
  if (!c || !width) return BMC_EINVAL;
  if (process < 0 || process >= (int)c->pr.size()) return fail(c, BMC_EINVAL, "bad process id");
  if (c->bound && process < c->n_pr_bound) {
    DevState s;
    int rc = read_state(c, &s);
    if (rc) return rc;
    c->pr[process].width = s.width[process];
  }
  *width = c->pr[process].width;
  return BMC_OK;
}

int bmc_set_width(bmc_ctx* c, int process, double width) {
  if (!c) return BMC_EINVAL;
  if (process < 0 || process >= (int)c->pr.size()) return fail(c, BMC_EINVAL, "bad process id");
  if (!(width > 0.0) || !std::isfinite(width) || (c->pr[process].prm.width_mode == BMC_WIDTH_REL && width > 1.0))
    return fail(c, BMC_EINVAL, "width must be > 0 (and <= 1 for a relative width)");
  c->pr[process].width = width;
  if (c->bound && process < c->n_pr_bound) {
    HIPCHK(c, hipMemcpyAsync(&c->st()->width[process], &width, sizeof(double), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return BMC_OK;
}

int bmc_set_expansion(bmc_ctx* c, int kind, double a0, double t0) {
  if (!c) return BMC_EINVAL;
  if (kind != BMC_EXP_NONE && kind != BMC_EXP_RADIATION) return fail(c, BMC_EINVAL, "bad expansion kind");
  if (kind == BMC_EXP_RADIATION && (!(a0 > 0.0) || !(t0 > 0.0))) return fail(c, BMC_EINVAL, "a0, t0 must be > 0");
  c->expansion = kind;
  c->a0 = a0;
  c->t0 = t0;
  if (c->bound) {
    DevState s;
    int rc = read_state(c, &s);
    if (rc) return rc;
    mirror_state(c, s);
    return upload_state(c);
  }
  return BMC_OK;
}

int bmc_set_time(bmc_ctx* c, double t) {
  if (!c || !std::isfinite(t)) return BMC_EINVAL;
  c->t = t;
  if (c->bound) {
    HIPCHK(c, launch_set_eval(c->st(), t, 0, 1, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return BMC_OK;
}

int bmc_get_time(bmc_ctx* c, double* t) {
  if (!c || !t) return BMC_EINVAL;
  if (c->bound) {
    DevState s;
    int rc = read_state(c, &s);
    if (rc) return rc;
    c->t = s.t;
  }
  *t = c->t;
  return BMC_OK;
}

int bmc_workspace_query(bmc_ctx* c, int64_t max_samples, int max_iter, size_t* bytes) {
  if (!c || !bytes) return BMC_EINVAL;
  if (c->pr.empty()) return fail(c, BMC_ESTATE, "register processes first");
  std::vector<int64_t> offs;
  for (auto& s : c->sp) offs.push_back(s.f_off);
  // layout without touching the bound state
  bmc_ctx tmp;
  tmp.sp = c->sp;
  tmp.pr = c->pr;
  layout_persistent(&tmp);
  *bytes = tmp.persist_bytes + scratch_estimate(c, max_samples, max_iter);
  return BMC_OK;
}

int bmc_workspace_bind(bmc_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return BMC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(dev_ptr) & (kAlign - 1)) != 0) return fail(c, BMC_EINVAL, "workspace not 256-byte aligned");
  if (c->pr.empty()) return fail(c, BMC_ESTATE, "register processes first");
  HIPCHK(c, hipSetDevice(c->device));
  // save the persistent state of a previous binding
  std::vector<double> old_maps;
  size_t n_old_slots = 0;
  if (c->bound) {
    DevState s;
    int rc = read_state(c, &s);
    if (rc) return rc;
    mirror_state(c, s);
    for (int a = 0; a < c->n_sp_bound; ++a) {
      HIPCHK(c, hipMemcpy(c->sp[a].f.data(), c->f64() + c->sp[a].f_off, 8 * c->sp[a].n, hipMemcpyDeviceToHost));
    }
    n_old_slots = c->slot_of_uid.size();
    old_maps.resize(n_old_slots * kSlotDoubles);
    if (n_old_slots)
      HIPCHK(c, hipMemcpy(old_maps.data(), c->maps(), 8 * old_maps.size(), hipMemcpyDeviceToHost));
  }
  layout_persistent(c);
  if (bytes < c->persist_bytes) return fail(c, BMC_ENOMEM, "workspace smaller than the persistent state");
  c->ws = reinterpret_cast<char*>(dev_ptr);
  c->ws_bytes = bytes;
  c->bound = true;
  c->n_sp_bound = (int)c->sp.size();
  c->n_pr_bound = (int)c->pr.size();
  c->plan = Plan();
  c->step_plan = Plan();
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  int rc = upload_model(c);
  if (rc) return rc;
  rc = upload_state(c);
  if (rc) return rc;
  for (auto& s : c->sp)
    if (s.f_set) HIPCHK(c, hipMemcpyAsync(c->f64() + s.f_off, s.f.data(), 8 * s.n, hipMemcpyHostToDevice, c->stream));
  if (n_old_slots && n_old_slots <= (size_t)c->max_slots)
    HIPCHK(c, hipMemcpyAsync(c->maps(), old_maps.data(), 8 * old_maps.size(), hipMemcpyHostToDevice, c->stream));
  else
    c->slot_of_uid.clear();
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return BMC_OK;
}

int bmc_plan_size(bmc_ctx* c, int process, int species, const bmc_run_opts* o, int* n_items, int* n_out) {
  if (!c) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (plan_matches(c->plan, plan_key(process, species, o))) {  // the plan of the last call: its sizes
    if (n_items) *n_items = (int)c->plan.items.size();
    if (n_out) *n_out = c->plan.n_out;
    return BMC_OK;
  }
  Plan P;
  // a plan built without a workspace does not allocate map slots permanently
  auto saved = c->slot_of_uid;
  char* ws = c->ws;
  c->ws = nullptr;
  rc = build_plan(c, plan_key(process, species, o), &P);
  c->ws = ws;
  c->slot_of_uid = saved;
  if (rc) return rc;
  if (n_items) *n_items = (int)P.items.size();
  if (n_out) *n_out = P.n_out;
  return BMC_OK;
}

int bmc_collision(bmc_ctx* c, int process, int species, const bmc_run_opts* o, double* C_out, double* sigma_out,
                  size_t n_out, int mem) {
  if (!c || !C_out) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  rc = get_plan(c, c->plan, process, species, o);
  if (rc) return rc;
  Plan& P = c->plan;
  if ((size_t)P.n_out != n_out) return fail(c, BMC_EINVAL, "n_out does not match the plan (" + std::to_string(P.n_out) + ")");
  HIPCHK(c, launch_set_eval(c->st(), 0.0, o->epoch, 0, c->stream));
  rc = enqueue_eval(c, P, *o, P.d_out_C, P.d_out_S);
  if (rc) return rc;
  c->last_n_iter = P.n_iter_max;
  const hipMemcpyKind kind = mem == BMC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(c, hipMemcpyAsync(C_out, P.d_out_C, 8 * n_out, kind, c->stream));
  if (sigma_out) HIPCHK(c, hipMemcpyAsync(sigma_out, P.d_out_S, 8 * n_out, kind, c->stream));
  return finish_check(c);
}

int bmc_collision_noalloc(bmc_ctx* c, int process, int species, const bmc_run_opts* o, double* C_out,
                          double* sigma_out, size_t n_out, int mem) {
  if (!c || !C_out) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  char* base = static_cast<char*>(g_scratch_ptr[c->device]);
  if (!base) return fail(c, BMC_ESTATE, "static scratch not resolved for this device");
  // the array is shared by every call on this GPU: the plan is built and uploaded afresh each time
  Plan P;
  rc = build_plan(c, plan_key(process, species, o), &P, base, kStaticListCapBytes, o->launch);
  if (rc) return rc;
  if (P.scratch_bytes > kStaticScratchBytes)
    return fail(c, BMC_ENOMEM, "the call needs " + std::to_string(P.scratch_bytes) +
                                   " bytes of scratch; the allocation-free evaluation holds " +
                                   std::to_string(kStaticScratchBytes));
  if ((size_t)P.n_out != n_out) return fail(c, BMC_EINVAL, "n_out does not match the plan (" + std::to_string(P.n_out) + ")");
  if (o->first_iter + P.n_iter_max > kMaxIter) return fail(c, BMC_EINVAL, "first_iter + n_iter > 64");
  rc = upload_plan(c, P);  // also zeroes the bin counts
  if (rc) return rc;
  HIPCHK(c, launch_set_eval(c->st(), 0.0, o->epoch, 0, c->stream));
  rc = enqueue_eval(c, P, *o, P.d_out_C, P.d_out_S);
  if (rc) return rc;
  const hipMemcpyKind kind = mem == BMC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(c, hipMemcpyAsync(C_out, P.d_out_C, 8 * n_out, kind, c->stream));
  if (sigma_out) HIPCHK(c, hipMemcpyAsync(sigma_out, P.d_out_S, 8 * n_out, kind, c->stream));
  return finish_check(c);  // synchronises the stream: the scratch is free for the next call when this returns
}

int bmc_collision_exact22(bmc_ctx* c, int process, int species, const bmc_run_opts* o, double* C_out,
                          double* sigma_out, size_t n_out, int mem) {
  if (!c || !C_out) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  if (process < -1 || process >= (int)c->pr.size()) return fail(c, BMC_EINVAL, "bad process id");
  for (int p = 0; p < (int)c->pr.size(); ++p)
    if ((process < 0 || p == process) &&
        !(c->pr[p].n_in == 2 && c->pr[p].n_out == 2 && c->pr[p].prm.m2_kind == BMC_M2_CONST))
      return fail(c, BMC_EUNSUP, "the exact-delta path takes 2->2 processes with a constant |M|^2 only");
  HIPCHK(c, hipSetDevice(c->device));
  rc = get_plan(c, c->plan, process, species, o);
  if (rc) return rc;
  Plan& P = c->plan;
  if ((size_t)P.n_out != n_out) return fail(c, BMC_EINVAL, "n_out does not match the plan");
  hipStream_t s = c->stream;
  HIPCHK(c, launch_prepare(c->st(), c->spec(), (int)c->sp.size(), c->f64(), c->f32(), c->n_f, s));
  HIPCHK(c, launch_exact22(P.d_items, (int)P.items.size(), c->spec(), c->f64(), c->qnode(), c->st(), P.d_res_I,
                           P.d_res_V, s));
  HIPCHK(c, launch_combine(P.d_items, (int)P.items.size(), P.d_res_I, P.d_res_V, 1, P.d_item_Ibar, P.d_item_sig,
                           P.d_slot_begin, P.d_slot_items, P.n_slots, P.d_slot_C, P.d_slot_S2, s));
  HIPCHK(c, launch_gather(P.d_gather, P.n_out, P.d_gproc, P.d_slot_C, P.d_slot_S2, c->spec(), c->f64(), P.d_out_C,
                          P.d_out_S, s));
  c->last_n_iter = 1;
  const hipMemcpyKind kind = mem == BMC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIPCHK(c, hipMemcpyAsync(C_out, P.d_out_C, 8 * n_out, kind, s));
  if (sigma_out) HIPCHK(c, hipMemcpyAsync(sigma_out, P.d_out_S, 8 * n_out, kind, s));
  return finish_check(c);
}

int bmc_item_results(bmc_ctx* c, uint32_t* uids, double* Ibar, double* sigma, double* I_it, double* V_it, int n,
                     int n_iter) {
  if (!c) return BMC_EINVAL;
  Plan& P = c->plan;
  if (!P.uploaded) return fail(c, BMC_ESTATE, "no evaluation yet");
  if (n != (int)P.items.size()) return fail(c, BMC_EINVAL, "n does not match the last plan");
  if (n_iter < 0 || n_iter > kMaxIter) return fail(c, BMC_EINVAL, "bad n_iter");
  if (uids)
    for (int i = 0; i < n; ++i) uids[i] = P.items[i].uid;
  if (Ibar) HIPCHK(c, hipMemcpy(Ibar, P.d_item_Ibar, 8 * n, hipMemcpyDeviceToHost));
  if (sigma) HIPCHK(c, hipMemcpy(sigma, P.d_item_sig, 8 * n, hipMemcpyDeviceToHost));
  if (I_it || V_it) {
    std::vector<double> bI((size_t)n * kMaxIter), bV((size_t)n * kMaxIter);
    HIPCHK(c, hipMemcpy(bI.data(), P.d_res_I, 8 * bI.size(), hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(bV.data(), P.d_res_V, 8 * bV.size(), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < n_iter; ++t) {
        const int64_t r = P.items[i].res_off;
        if (I_it) I_it[(size_t)i * n_iter + t] = bI[r * kMaxIter + t];
        if (V_it) V_it[(size_t)i * n_iter + t] = bV[r * kMaxIter + t];
      }
  }
  return BMC_OK;
}

int bmc_maps_get(bmc_ctx* c, const uint32_t* uids, int n, double* maps) {
  if (!c || !uids || !maps || n < 0) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) {
    const uint32_t uid = uids[i];
    const int p = (int)(uid >> 24), a = (int)((uid >> 20) & 15), side = (int)((uid >> 19) & 1);
    const int node = (int)(uid & ((1u << 18) - 1));
    if (p >= (int)c->pr.size() || a >= (int)c->sp.size() || node >= c->sp[a].n || multiplicity(c->pr[p], a, side) == 0)
      return fail(c, BMC_EINVAL, "uid does not name a work item");
    const Process& Pr = c->pr[p];
    const int nb = Pr.prm.n_bins;
    double* dst = maps + (size_t)i * kMaxD * (nb + 1);
    auto f = c->slot_of_uid.find(uid);
    if (f != c->slot_of_uid.end()) {
      HIPCHK(c, hipMemcpy(dst, c->maps() + (size_t)f->second * kSlotDoubles, 8 * kMaxD * (nb + 1),
                          hipMemcpyDeviceToHost));
    } else {
      int obs, cons, integ[kMaxInt];
      assign_roles(Pr, a, side, &obs, &cons, integ);
      const int D = 3 * (Pr.n_in + Pr.n_out - 2);
      for (int d = 0; d < kMaxD; ++d)
        for (int j = 0; j <= nb; ++j) {
          double lo = 0, hi = 0;
          if (d < D) {
            if (d % 3 == 0) {
              lo = c->sp[Pr.sp[integ[d / 3]]].q_min;
              hi = c->sp[Pr.sp[integ[d / 3]]].q_max;
            } else {
              hi = d % 3 == 1 ? M_PI : 2.0 * M_PI;
            }
          }
          dst[d * (nb + 1) + j] = lo + (hi - lo) * (double)j / (double)nb;
        }
    }
  }
  return BMC_OK;
}

int bmc_maps_set(bmc_ctx* c, const uint32_t* uids, int n, const double* maps) {
  if (!c || !uids || !maps || n < 0) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < n; ++i) {
    const uint32_t uid = uids[i];
    const int p = (int)(uid >> 24), a = (int)((uid >> 20) & 15), side = (int)((uid >> 19) & 1);
    const int node = (int)(uid & ((1u << 18) - 1));
    if (p >= (int)c->pr.size() || a >= (int)c->sp.size() || node >= c->sp[a].n || multiplicity(c->pr[p], a, side) == 0)
      return fail(c, BMC_EINVAL, "uid does not name a work item");
    const int nb = c->pr[p].prm.n_bins;
    int slot;
    auto f = c->slot_of_uid.find(uid);
    if (f == c->slot_of_uid.end()) {
      slot = (int)c->slot_of_uid.size();
      if (slot >= c->max_slots) return fail(c, BMC_ENOMEM, "map slots exhausted");
      c->slot_of_uid[uid] = slot;
    } else {
      slot = f->second;
    }
    HIPCHK(c, hipMemcpy(c->maps() + (size_t)slot * kSlotDoubles, maps + (size_t)i * kMaxD * (nb + 1),
                        8 * kMaxD * (nb + 1), hipMemcpyHostToDevice));
  }
  // plans that were going to initialise these maps must not do so any more
  c->plan = Plan();
  c->step_plan = Plan();
  return BMC_OK;
}

namespace {
constexpr uint32_t kStateMagic = 0x53434d42u;  // "BMCS"
constexpr uint32_t kStateVersion = 2;
struct StateHeader {
  uint32_t magic, version, n_species, n_maps;
  int64_t n_f;
  double t;
  uint32_t epoch, next_epoch, slot_doubles, n_proc;
};
size_t state_bytes(const bmc_ctx* c) {
  return sizeof(StateHeader) + 8 * (size_t)c->n_f + 8 * c->pr.size() +
         c->slot_of_uid.size() * (8 + 8 * (size_t)kSlotDoubles);
}
}  // namespace

int bmc_state_size(bmc_ctx* c, size_t* bytes) {
  if (!c || !bytes) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  *bytes = state_bytes(c);
  return BMC_OK;
}

int bmc_state_get(bmc_ctx* c, void* blob, size_t bytes) {
  if (!c || !blob) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  if (bytes < state_bytes(c)) return fail(c, BMC_EINVAL, "state buffer too small");
  DevState s;
  int rc = read_state(c, &s);
  if (rc) return rc;
  char* p = static_cast<char*>(blob);
  StateHeader h{kStateMagic, kStateVersion, (uint32_t)c->sp.size(), (uint32_t)c->slot_of_uid.size(), c->n_f, s.t,
                s.epoch, s.next_epoch, (uint32_t)kSlotDoubles, (uint32_t)c->pr.size()};
  std::memcpy(p, &h, sizeof(h));
  p += sizeof(h);
  HIPCHK(c, hipMemcpy(p, c->f64(), 8 * (size_t)c->n_f, hipMemcpyDeviceToHost));
  p += 8 * (size_t)c->n_f;
  std::memcpy(p, s.width, 8 * c->pr.size());
  p += 8 * c->pr.size();
  std::vector<std::pair<uint32_t, int>> slots(c->slot_of_uid.begin(), c->slot_of_uid.end());
  std::sort(slots.begin(), slots.end());
  for (auto& us : slots) {
    const uint64_t uid = us.first;
    std::memcpy(p, &uid, 8);
    p += 8;
    HIPCHK(c, hipMemcpy(p, c->maps() + (size_t)us.second * kSlotDoubles, 8 * (size_t)kSlotDoubles,
                        hipMemcpyDeviceToHost));
    p += 8 * (size_t)kSlotDoubles;
  }
  return BMC_OK;
}

int bmc_state_set(bmc_ctx* c, const void* blob, size_t bytes) {
  if (!c || !blob) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  if (bytes < sizeof(StateHeader)) return fail(c, BMC_EINVAL, "state blob too short");
  StateHeader h;
  std::memcpy(&h, blob, sizeof(h));
  if (h.magic != kStateMagic || h.version != kStateVersion) return fail(c, BMC_EINVAL, "not a state blob");
  if (h.n_species != c->sp.size() || h.n_f != c->n_f || h.slot_doubles != (uint32_t)kSlotDoubles ||
      h.n_proc != c->pr.size())
    return fail(c, BMC_EINVAL, "the state blob belongs to a different model");
  if (bytes < sizeof(h) + 8 * (size_t)h.n_f + 8 * (size_t)h.n_proc + (size_t)h.n_maps * (8 + 8 * (size_t)kSlotDoubles))
    return fail(c, BMC_EINVAL, "state blob too short");
  if (!std::isfinite(h.t)) return fail(c, BMC_EINVAL, "non-finite time in the state blob");
  const char* p = static_cast<const char*>(blob) + sizeof(h);
  // validate everything before changing anything
  std::vector<double> f((size_t)h.n_f);
  std::memcpy(f.data(), p, 8 * f.size());
  p += 8 * f.size();
  for (auto& S : c->sp)
    for (int j = 0; j < S.n; ++j) {
      const double v = f[(size_t)S.f_off + j];
      if (!(v > 0.0) || !std::isfinite(v)) return fail(c, BMC_ERANGE, "f must be positive and finite");
      if (S.stat == BMC_FERMI && !(v < 1.0)) return fail(c, BMC_ERANGE, "Fermi-Dirac f must be below 1");
    }
  std::vector<double> widths(h.n_proc);
  std::memcpy(widths.data(), p, 8 * widths.size());
  p += 8 * widths.size();
  for (size_t q = 0; q < widths.size(); ++q)
    if (!(widths[q] > 0.0) || !std::isfinite(widths[q]) ||
        (c->pr[q].prm.width_mode == BMC_WIDTH_REL && widths[q] > 1.0))
      return fail(c, BMC_EINVAL, "invalid width in the state blob");
  std::vector<uint32_t> uids(h.n_maps);
  const char* pm = p;
  size_t new_slots = 0;
  for (uint32_t i = 0; i < h.n_maps; ++i) {
    uint64_t u;
    std::memcpy(&u, pm + (size_t)i * (8 + 8 * (size_t)kSlotDoubles), 8);
    const uint32_t uid = (uint32_t)u;
    const int pr = (int)(uid >> 24), a = (int)((uid >> 20) & 15), side = (int)((uid >> 19) & 1);
    const int node = (int)(uid & ((1u << 18) - 1));
    const bool node_ok = node < c->sp[a < (int)c->sp.size() ? a : 0].n ||
                         (node >= (int)kCustomBase && node < (int)kCustomBase + kMaxEvalPoints);
    if (u >> 32 || pr >= (int)c->pr.size() || a >= (int)c->sp.size() || !node_ok ||
        multiplicity(c->pr[pr], a, side) == 0)
      return fail(c, BMC_EINVAL, "a map in the state blob does not name a work item of this model");
    uids[i] = uid;
    new_slots += c->slot_of_uid.count(uid) ? 0 : 1;
  }
  if (c->slot_of_uid.size() + new_slots > (size_t)c->max_slots) return fail(c, BMC_ENOMEM, "map slots exhausted");
  for (auto& S : c->sp) {
    S.f.assign(f.begin() + S.f_off, f.begin() + S.f_off + S.n);
    S.f_set = true;
  }
  HIPCHK(c, hipMemcpy(c->f64(), f.data(), 8 * f.size(), hipMemcpyHostToDevice));
  for (uint32_t i = 0; i < h.n_maps; ++i) {
    auto it = c->slot_of_uid.find(uids[i]);
    int slot;
    if (it == c->slot_of_uid.end()) {
      slot = (int)c->slot_of_uid.size();
      c->slot_of_uid[uids[i]] = slot;
    } else {
      slot = it->second;
    }
    HIPCHK(c, hipMemcpy(c->maps() + (size_t)slot * kSlotDoubles, pm + (size_t)i * (8 + 8 * (size_t)kSlotDoubles) + 8,
                        8 * (size_t)kSlotDoubles, hipMemcpyHostToDevice));
  }
  c->t = h.t;
  DevState* st = c->st();
  for (size_t q = 0; q < widths.size(); ++q) c->pr[q].width = widths[q];
  if (!widths.empty()) HIPCHK(c, hipMemcpy(st->width, widths.data(), 8 * widths.size(), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(&st->t, &h.t, sizeof(double), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(&st->epoch, &h.epoch, sizeof(uint32_t), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(&st->next_epoch, &h.next_epoch, sizeof(uint32_t), hipMemcpyHostToDevice));
  c->plan = Plan();
  c->step_plan = Plan();
  return BMC_OK;
}

int bmc_maps_reset(bmc_ctx* c, int process) {
  if (!c) return BMC_EINVAL;
  if (process < -1 || process >= (int)c->pr.size()) return fail(c, BMC_EINVAL, "bad process id");
  // forgetting a slot makes the next plan re-initialise it (slots are never reused for other uids)
  std::vector<uint32_t> drop;
  for (auto& kv : c->slot_of_uid)
    if (process < 0 || (int)(kv.first >> 24) == process) drop.push_back(kv.first);
  if (process < 0) {
    c->slot_of_uid.clear();
  } else {
    // the dropped uids keep their slots (other processes keep theirs); their maps are rewritten as uniform now
    std::vector<double> buf;
    for (uint32_t u : drop) {
      const int nb = c->pr[u >> 24].prm.n_bins;
      buf.assign((size_t)kMaxD * (nb + 1), 0.0);
      int rc = 0;
      // bmc_maps_get of a uid without a slot returns the uniform map
      const int slot = c->slot_of_uid[u];
      c->slot_of_uid.erase(u);
      rc = bmc_maps_get(c, &u, 1, buf.data());
      c->slot_of_uid[u] = slot;
      if (rc) return rc;
      HIPCHK(c, hipMemcpy(c->maps() + (size_t)slot * kSlotDoubles, buf.data(), 8 * buf.size(), hipMemcpyHostToDevice));
    }
  }
  c->plan = Plan();
  c->step_plan = Plan();
  return BMC_OK;
}

int bmc_step(bmc_ctx* c, int method, double dt, double eps, double dt_max, const bmc_run_opts* o, double* dt_used) {
  if (!c) return BMC_EINVAL;
  if (method != BMC_EULER && method != BMC_HEUN) return fail(c, BMC_EINVAL, "bad method");
  if (!(dt > 0.0) && (!(eps > 0.0) || !(dt_max > 0.0))) return fail(c, BMC_EINVAL, "need dt > 0 or eps, dt_max > 0");
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  if (o->eval_q) return fail(c, BMC_EINVAL, "steps evaluate on the grids (eval_q must be NULL)");
  bmc_run_opts so = *o;
  so.eval_stride = 0;
  rc = get_plan(c, c->step_plan, -1, -1, &so);
  if (rc) return rc;
  Plan& P = c->step_plan;
  hipStream_t s = c->stream;
  DevState before;
  rc = read_state(c, &before);
  if (rc) return rc;
  // backup of f for error recovery (sig buffer is free outside evaluations)
  HIPCHK(c, launch_copy(c->sig(), c->f64(), c->n_f, s));
  HIPCHK(c, launch_set_eval(c->st(), 0.0, o->epoch, 0, s));
  rc = enqueue_eval(c, P, so, c->k1(), nullptr);
  if (rc) return rc;
  HIPCHK(c, launch_step_begin(c->st(), c->f64(), c->f0(), c->k1(), c->n_f, dt, eps, dt_max, method == BMC_HEUN, s));
  if (method == BMC_HEUN) {
    rc = enqueue_eval(c, P, so, c->k2(), nullptr);
    if (rc) return rc;
    HIPCHK(c, launch_step_finish(c->st(), c->f64(), c->f0(), c->f64(), c->k1(), c->k2(), c->n_f, s));
  }
  HIPCHK(c, launch_prepare(c->st(), c->spec(), (int)c->sp.size(), c->f64(), c->f32(), c->n_f, s));
  DevState after;
  rc = read_state(c, &after);
  if (rc) return rc;
  if (after.err) {
    HIPCHK(c, launch_copy(c->f64(), c->sig(), c->n_f, s));
    HIPCHK(c, launch_set_eval(c->st(), before.t, before.next_epoch, 1, s));
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(&c->st()->err, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(c, hipStreamSynchronize(s));
    return fail(c, BMC_ERANGE, "step produced an invalid distribution; f and t restored");
  }
  c->t = after.t;
  if (dt_used) *dt_used = after.dt;
  return BMC_OK;
}

int bmc_graph_capture_steps(bmc_ctx* c, int n_steps, int method, double dt, double eps, double dt_max,
                            const bmc_run_opts* o) {
  if (!c || n_steps < 1) return BMC_EINVAL;
  if (method != BMC_EULER && method != BMC_HEUN) return fail(c, BMC_EINVAL, "bad method");
  if (!(dt > 0.0) && (!(eps > 0.0) || !(dt_max > 0.0))) return fail(c, BMC_EINVAL, "need dt > 0 or eps, dt_max > 0");
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  if (c->stream == nullptr) return fail(c, BMC_EINVAL, "graph capture needs a non-null stream");
  if (o->eval_q) return fail(c, BMC_EINVAL, "steps evaluate on the grids (eval_q must be NULL)");
  bmc_run_opts so = *o;
  so.eval_stride = 0;
  rc = get_plan(c, c->step_plan, -1, -1, &so);
  if (rc) return rc;
  Plan& P = c->step_plan;
  hipStream_t s = c->stream;
  // epochs continue from the device counter: set it once, before the capture
  HIPCHK(c, launch_set_eval(c->st(), 0.0, o->epoch, 0, s));
  HIPCHK(c, hipStreamSynchronize(s));
  if (c->gexec) {
    (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
  }
  if (c->graph) {
    (void)hipGraphDestroy(c->graph);
    c->graph = nullptr;
  }
  HIPCHK(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  c->capturing = true;
  int crc = BMC_OK;
  for (int k = 0; k < n_steps && crc == BMC_OK; ++k) {
    crc = enqueue_eval(c, P, so, c->k1(), nullptr);
    if (crc) break;
    if (launch_step_begin(c->st(), c->f64(), c->f0(), c->k1(), c->n_f, dt, eps, dt_max, method == BMC_HEUN, s) !=
        hipSuccess) {
      crc = fail(c, BMC_EHIP, "launch in capture failed");
      break;
    }
    if (method == BMC_HEUN) {
      crc = enqueue_eval(c, P, so, c->k2(), nullptr);
      if (crc) break;
      if (launch_step_finish(c->st(), c->f64(), c->f0(), c->f64(), c->k1(), c->k2(), c->n_f, s) != hipSuccess) {
        crc = fail(c, BMC_EHIP, "launch in capture failed");
        break;
      }
    }
    if (launch_prepare(c->st(), c->spec(), (int)c->sp.size(), c->f64(), c->f32(), c->n_f, s) != hipSuccess) {
      crc = fail(c, BMC_EHIP, "launch in capture failed");
      break;
    }
  }
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(s, &g);
  c->capturing = false;
  if (crc) {
    if (g) (void)hipGraphDestroy(g);
    return crc;
  }
  if (e != hipSuccess) return fail(c, BMC_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  c->graph = g;
  HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
  return BMC_OK;
}

int bmc_graph_replay(bmc_ctx* c) {
  if (!c) return BMC_EINVAL;
  if (!c->gexec) return fail(c, BMC_ESTATE, "no captured graph");
  HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
  return BMC_OK;
}

int bmc_graph_status(bmc_ctx* c, double* t, double* last_dt) {
  if (!c) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  DevState s;
  int rc = read_state(c, &s);
  if (rc) return rc;
  c->t = s.t;
  if (t) *t = s.t;
  if (last_dt) *last_dt = s.dt;
  if (s.err) return fail(c, BMC_ERANGE, "a replayed step produced an invalid distribution");
  return BMC_OK;
}

int bmc_vjp(bmc_ctx* c, int process, int species, const bmc_run_opts* o, const double* v_C, size_t n_out,
            double* grad_f, double* grad_coupling, double* grad_m0, int mem) {
  if (!c || !v_C) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  if (o->precision != BMC_FP64) return fail(c, BMC_EUNSUP, "vector-Jacobian products are FP64 only");
  if (o->eval_q) return fail(c, BMC_EUNSUP, "vector-Jacobian products are on the grids only (eval_q must be NULL)");
  for (auto& Pr : c->pr)
    if (Pr.prm.m2_kind != BMC_M2_CONST || Pr.prm.vegas_plus)
      return fail(c, BMC_EUNSUP, "vector-Jacobian products need a constant |M|^2 and plain Vegas sampling");
  rc = check_ready(c);
  if (rc) return rc;
  HIPCHK(c, hipSetDevice(c->device));
  bmc_run_opts vo = *o;
  vo.n_iter = 1;
  vo.freeze_maps = 1;
  rc = get_plan(c, c->plan, process, species, &vo);
  if (rc) return rc;
  Plan& P = c->plan;
  if ((size_t)P.n_out != n_out) return fail(c, BMC_EINVAL, "n_out does not match the plan");
  for (auto& g : P.gproc)
    if (g.fill && g.stride > 1)
      return fail(c, BMC_EUNSUP, "strided evaluation with fill is not differentiated; use eval_stride >= 1");
  // cotangent on the host
  std::vector<double> v(n_out);
  if (mem == BMC_MEM_DEVICE) {
    HIPCHK(c, hipMemcpyAsync(v.data(), v_C, 8 * n_out, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  } else {
    std::memcpy(v.data(), v_C, 8 * n_out);
  }
  // output index of every item: the gather entry of its (species, node)
  std::unordered_map<int64_t, int> out_of;
  for (size_t k = 0; k < P.gather.size(); ++k) out_of[(int64_t)P.gather[k].species * 1000003 + P.gather[k].node] = (int)k;
  const size_t nI = P.items.size();
  std::vector<ItemRec> vitems = P.items;
  std::vector<double> coef(nI);
  std::vector<int> rec_len(nI), rec_nmax(2 * nI);  // n_max per item, then the offset of each record's tail
  int64_t part = 0;
  int rec_stride = 0, lds = 0;
  for (size_t i = 0; i < nI; ++i) {
    ItemRec& it = vitems[i];
    auto f = out_of.find((int64_t)it.obs_species * 1000003 + it.eval_idx);
    if (f == out_of.end()) return fail(c, BMC_EINVAL, "item without an output");
    coef[i] = v[f->second] * (double)it.mult * (double)it.sign;
    int n_max = 0, spl = 0;
    for (int t = 0; t < it.n_tab; ++t) {
      n_max = std::max(n_max, c->sp[it.tab_species[t]].n);
      spl |= c->sp[it.tab_species[t]].interp == BMC_INTERP_SPLINE ? 1 : 0;
    }
    rec_nmax[i] = n_max;
    rec_nmax[nI + i] = it.n_tab * n_max * (spl ? 2 : 1);
    rec_len[i] = vjp_record_len(it.n_tab, n_max, spl);
    rec_stride = std::max(rec_stride, rec_len[i]);
    it.part_off = part;  // one record per batched second-pass group of the item
    part += ((int64_t)it.n_units + it.shell_units - 1) / it.shell_units * rec_len[i];
    lds = std::max(lds, vjp_lds_bytes(it.D, it.nb, it.n_tab, n_max, spl));
  }
  if (lds > 65536) return fail(c, BMC_EUNSUP, "per-block LDS need of the adjoint above 64 KB");
  // scratch after the plan's own region
  size_t off = c->persist_bytes + P.scratch_bytes;
  auto take = [&](size_t bytes) {
    size_t o2 = off;
    off = align_up(off + bytes);
    return o2;
  };
  const size_t o_items = take(sizeof(ItemRec) * nI), o_parts = take(8 * (size_t)part),
               o_rec = take(8 * (size_t)rec_stride * nI), o_coef = take(8 * nI), o_len = take(4 * nI),
               o_nmax = take(8 * nI), o_gf = take(8 * (size_t)c->n_f), o_work = take(8 * 3 * (size_t)c->n_f),
               o_gm = take(8 * kMaxSpecies),
               o_gl = take(8 * c->pr.size()), o_cp = take(8 * c->pr.size());
  if (off > c->ws_bytes)
    return fail(c, BMC_ENOMEM, "workspace too small for the adjoint: need " + std::to_string(off) + " bytes");
  char* b = c->ws;
  ItemRec* d_items = reinterpret_cast<ItemRec*>(b + o_items);
  double* d_parts = reinterpret_cast<double*>(b + o_parts);
  double* d_rec = reinterpret_cast<double*>(b + o_rec);
  double* d_coef = reinterpret_cast<double*>(b + o_coef);
  int* d_len = reinterpret_cast<int*>(b + o_len);
  int* d_nmax = reinterpret_cast<int*>(b + o_nmax);
  double* d_gf = reinterpret_cast<double*>(b + o_gf);
  double* d_work = reinterpret_cast<double*>(b + o_work);
  double* d_gm = reinterpret_cast<double*>(b + o_gm);
  double* d_gl = reinterpret_cast<double*>(b + o_gl);
  double* d_cp = reinterpret_cast<double*>(b + o_cp);
  std::vector<double> cpl(c->pr.size());
  for (size_t p = 0; p < c->pr.size(); ++p) cpl[p] = c->pr[p].prm.coupling;
  hipStream_t s = c->stream;
  HIPCHK(c, hipMemcpyAsync(d_items, vitems.data(), sizeof(ItemRec) * nI, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(d_coef, coef.data(), 8 * nI, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(d_len, rec_len.data(), 4 * nI, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(d_nmax, rec_nmax.data(), 8 * nI, hipMemcpyHostToDevice, s));
  HIPCHK(c, hipMemcpyAsync(d_cp, cpl.data(), 8 * cpl.size(), hipMemcpyHostToDevice, s));
  HIPCHK(c, launch_set_eval(c->st(), 0.0, o->epoch, 0, s));
  HIPCHK(c, launch_next_epoch(c->st(), s));
  HIPCHK(c, launch_prepare(c->st(), c->spec(), (int)c->sp.size(), c->f64(), c->f32(), c->n_f, s));
  SampleLaunch L{};
  L.items = d_items;
  L.tasks = P.d_tb;
  L.task_begin = 0;
  L.n_tasks = (int)P.tasks_batched.size();
  L.spec = c->spec();
  L.f64 = c->f64();
  L.f32 = c->f32();
  L.qnode = c->qnode();
  L.st = c->st();
  L.maps = c->maps();
  L.parts = d_parts;
  L.unit_base = P.d_unit_base;
  L.it = o->first_iter;
  L.seed_lo = (uint32_t)o->seed;
  L.seed_hi = (uint32_t)(o->seed >> 32);
  L.nint_mask = P.nint_mask;
  L.precision = BMC_FP64;
  L.any_interp = 0;  // the adjoint kernel's general instance when a species uses the spline or equilibrium-exact rule
  for (auto& Sp : c->sp) L.any_interp |= Sp.interp != BMC_INTERP_LINLOG ? 1 : 0;
  L.lds_bytes = lds;
  L.chunk = 1;
  L.shell_list = P.d_list;
  L.shell_cnt = P.d_cnt;
  L.list_stride = P.list_stride;
  // screening launches of the collision plan list the samples whose W can be nonzero; the adjoint pass takes only
  // those (slice by slice, as the lists of one launch are bounded)
  SampleLaunch S = L;
  S.items = P.d_items;
  S.counts = nullptr;  // the collision's bin counts are not touched (no reduction follows)
  S.lds_bytes = P.lds32;
  S.chunk = c->chunk;
  S.n_listed = nullptr;
  L.sh_tasks = P.d_shb;  // the adjoint takes the batched second pass's groups of units, one block each
  for (const Plan::Slice& sl : P.slices) {
    S.task_begin = L.task_begin = sl.tb;
    S.n_tasks = L.n_tasks = sl.te - sl.tb;
    L.sh_begin = sl.sb;
    L.n_sh = sl.se - sl.sb;
    S.grid = std::min((S.n_tasks + S.chunk - 1) / S.chunk, grid_for(c, BMC_FP32I, screen_lds_bytes(), P.nint_mask));
    L.grid = std::min(L.n_sh, grid_for(c, BMC_FP64, lds, P.nint_mask));
    HIPCHK(c, launch_sample(S, s));
    HIPCHK(c, launch_vjp(L, s));
  }
  HIPCHK(c, launch_vjp_finish(d_items, (int)nI, d_coef, d_parts, d_len, d_nmax, d_rec, rec_stride, c->spec(),
                              (int)c->sp.size(), c->f64(), c->qnode(), c->st(), d_gf, c->n_f, d_work, d_gm, d_gl, d_cp,
                              (int)c->pr.size(), s));
  const hipMemcpyKind kind = mem == BMC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (grad_f) HIPCHK(c, hipMemcpyAsync(grad_f, d_gf, 8 * (size_t)c->n_f, kind, s));
  if (grad_m0) HIPCHK(c, hipMemcpyAsync(grad_m0, d_gm, 8 * c->sp.size(), kind, s));
  if (grad_coupling) HIPCHK(c, hipMemcpyAsync(grad_coupling, d_gl, 8 * c->pr.size(), kind, s));
  return finish_check(c);
}

int bmc_set_timing(bmc_ctx* c, int on) {
  if (!c || on < 0) return BMC_EINVAL;
  c->timing = on != 0;
  c->timing_every = on > 0 ? on : 1;
  c->phase_count = 0;
  return BMC_OK;
}

int bmc_get_sample_stats(bmc_ctx* c, int reset, int64_t* n_listed) {
  if (!c) return BMC_EINVAL;
  if (!c->bound) return fail(c, BMC_ESTATE, "workspace not bound");
  unsigned long long v = 0;
  HIPCHK(c, hipMemcpyAsync(&v, &c->st()->n_listed, sizeof(v), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (n_listed) *n_listed = (int64_t)v;
  if (reset) {
    const unsigned long long zero = 0;
    HIPCHK(c, hipMemcpyAsync(&c->st()->n_listed, &zero, sizeof(zero), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  return BMC_OK;
}

namespace {
// Folds the recorded phase events into the context's sums (synchronises the stream).
int collect_timing(bmc_ctx* c) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->ev) {
    float all = 0.0f, scr = 0.0f, sec = 0.0f;
    HIPCHK(c, hipEventElapsedTime(&all, p.a, p.b));
    HIPCHK(c, hipEventElapsedTime(&scr, p.a, p.m));
    HIPCHK(c, hipEventElapsedTime(&sec, p.m, p.b));
    c->timed_ms += all;
    c->timed_screen_ms += scr;
    c->timed_second_ms += sec;
    c->timed_launches += 1;
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.m);
    (void)hipEventDestroy(p.b);
  }
  c->ev.clear();
  return BMC_OK;
}

void reset_timing(bmc_ctx* c) {
  c->timed_ms = c->timed_screen_ms = c->timed_second_ms = 0.0;
  c->timed_launches = 0;
}
}  // namespace

int bmc_get_timing(bmc_ctx* c, int reset, double* sample_ms, int* n_launches) {
  if (!c) return BMC_EINVAL;
  int rc = collect_timing(c);
  if (rc) return rc;
  if (sample_ms) *sample_ms = c->timed_ms;
  if (n_launches) *n_launches = c->timed_launches;
  if (reset) reset_timing(c);
  return BMC_OK;
}

int bmc_get_kernel_timing(bmc_ctx* c, int reset, double* screen_ms, double* second_ms, int* n_launches) {
  if (!c) return BMC_EINVAL;
  int rc = collect_timing(c);
  if (rc) return rc;
  if (screen_ms) *screen_ms = c->timed_screen_ms;
  if (second_ms) *second_ms = c->timed_second_ms;
  if (n_launches) *n_launches = c->timed_launches;
  if (reset) reset_timing(c);
  return BMC_OK;
}

int bmc_set_launch_tuning(bmc_ctx* c, int blocks_per_cu, int chunk) {
  if (!c || blocks_per_cu < 0 || blocks_per_cu > 64 || chunk < 1 || chunk > 64) return BMC_EINVAL;
  c->blocks_per_cu = blocks_per_cu;
  c->chunk = chunk;
  return BMC_OK;
}

int bmc_autotune(bmc_ctx* c, int process, int species, const bmc_run_opts* o, int* blocks_per_cu, int* chunk,
                 double* best_ms) {
  if (!c) return BMC_EINVAL;
  int rc = check_opts(c, o);
  if (rc) return rc;
  rc = check_ready(c);
  if (rc) return rc;
  // calibration evaluations: one iteration, maps frozen (no state changes), a throw-away epoch
  bmc_run_opts q = *o;
  q.n_iter = 1;
  q.freeze_maps = 1;
  q.launch = BMC_LAUNCH_BATCHED;
  rc = get_plan(c, c->plan, process, species, &q);
  if (rc) return rc;
  Plan& P = c->plan;
  const int saved_b = c->blocks_per_cu, saved_c = c->chunk;
  const bool saved_timing = c->timing;
  const int max_b = std::max(1, std::min(8, (160 * 1024) / std::max(1, screen_lds_bytes())));
  double best = 1e300;
  int bb = saved_b, bc = saved_c;
  hipEvent_t e0, e1;
  HIPCHK(c, hipEventCreate(&e0));
  HIPCHK(c, hipEventCreate(&e1));
  c->timing = false;
  for (int b = 1; b <= max_b; ++b) {
    for (int ch : {1, 2, 4, 8, 16}) {
      c->blocks_per_cu = b;
      c->chunk = ch;
      HIPCHK(c, launch_set_eval(c->st(), 0.0, q.epoch, 0, c->stream));
      double ms_sum = 0.0;
      for (int rep = 0; rep < 2; ++rep) {
        HIPCHK(c, hipEventRecord(e0, c->stream));
        rc = enqueue_eval(c, P, q, P.d_out_C, P.d_out_S, o->freeze_maps == 0);
        if (rc) break;
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) ms_sum += ms;  // the first run warms the configuration up
      }
      if (rc) break;
      if (ms_sum < best) {
        best = ms_sum;
        bb = b;
        bc = ch;
      }
    }
    if (rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->timing = saved_timing;
  if (rc) {
    c->blocks_per_cu = saved_b;
    c->chunk = saved_c;
    return rc;
  }
  c->blocks_per_cu = bb;
  c->chunk = bc;
  if (blocks_per_cu) *blocks_per_cu = bb;
  if (chunk) *chunk = bc;
  if (best_ms) *best_ms = best;
  return finish_check(c);
}

const char* bmc_last_error(bmc_ctx* c) { return c ? c->err.c_str() : "null context"; }

const char* bmc_version(void) { return "boltzmc 0.1 (gfx950)"; }

}  // extern "C"
