// kernels.hip -- gfx950 kernels of the Vegas Monte-Carlo collision integral.
//
// Estimator (arXiv 2603.28848, Sec. II.D and Appendix A): for a work item (process, observed species, pinned
// side, term, grid node q_i) each sample y in [0,1)^D is mapped through the item's Vegas map to
// x = (r_k, theta_k, phi_k) of the integrated particles, the conserved particle's momentum follows from
// momentum conservation (Eq. 14), energy conservation is a Gaussian of width sigma_E (Eq. 15), and the
// weight is (Eq. 16)
//     W = J(y) prod_k r_k^2 sin(theta_k) a^-3 |M|^2 delta(E_in - E_out) / ((2 pi)^{3(n-1)-4} prod_i 2 E_i) * F
// with F the gain or loss product relative to the observed leg (Eq. 5 and the C_2 / C_3 lists of Sec. II.C).
//
// An iteration's sample phase is two kernels.  The screening pass (blocks of 256 threads over runs of units, a unit
// being a contiguous range of sample indices of one item) evaluates every sample's kinematics in FP32, adds every
// sample to its bins' counts (integers, so any order gives the same sums) and lists the samples whose W can be
// nonzero.  The second pass (one block per group of an item's units) evaluates the listed samples; its sums are
// formed in a fixed order that depends only on the item: per thread in list order, a butterfly over the wave, the
// four waves in order, then the groups in order (reduce kernel).  The Vegas training histograms of W^2 are
// accumulated per wave in LDS and summed over waves in order.
#include <math.h>

#include <type_traits>

#include "kernels.h"
#include "philox.h"

namespace bmc {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;
constexpr double kHistWMin = 0x1p-400;  // |W| below this enters the training histogram as 0

struct Lds {
  int off_e, off_w, off_m32, off_sc, off_tab, tab_stride, tab_f, off_h, off_c, off_red, off_q, off_k, off_wd, total;
};

// The three LDS layouts a block can use: the screening pass's, the general sample layout (VEGAS+ blocks and the
// per-wave counts they keep), and the second pass's (no counts; the item's constants and a slot of words per thread).
constexpr int kLayScreen = 0, kLaySample = 1, kLayShell = 2;

// FP32 map of the screening pass in LDS: three arrays of kMapSlots 32-bit entries (bin edge, bin width, the unit's
// bin count), so that one address serves all three (the other two by the instruction's constant offset) and a
// wave's random bins spread over all 32 banks.
constexpr int kMapSlots = kMaxD * kMaxBins;

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// LDS of a screening block: the FP32 map only (nothing else of the sample layout is read without the finish).
__host__ __device__ inline Lds screen_layout() {
  Lds L{};
  L.off_m32 = 0;
  L.total = align16(3 * kMapSlots * 4);
  return L;
}

// LDS of one sample block: map edges and widths (D x nb, FP64, and the screening pass's FP32 map), sin/cos of k pi/16
// (33 entries), per f table q_j, 1/q_j and f_j, per-wave training histograms (sum of W^2, counts), reduction
// scratch.
__host__ __device__ inline Lds lds_layout(int D, int nb, int n_tab, int n_max, int fbytes) {
  Lds L;
  const int DN = D * nb;
  int o = 0;
  L.off_e = o;
  o = align16(o + DN * 8);
  L.off_w = o;
  o = align16(o + DN * 8);
  L.off_m32 = o;
  o = align16(o + 3 * kMapSlots * 4);
  L.off_sc = o;
  o = align16(o + 33 * 16);
  L.off_tab = o;
  L.tab_stride = align16(n_max * (16 + fbytes));
  L.tab_f = 16 * n_max;
  o = align16(o + n_tab * L.tab_stride);
  L.off_h = o;
  o = align16(o + kWaves * DN * 8);
  L.off_c = o;
  o = align16(o + kWaves * DN * 4);
  L.off_red = o;
  o = align16(o + 2 * kWaves * 8);
  L.off_q = o;  // second pass: prefix sums over 256 lists and the four wave totals of the scan
  o = align16(o + (kBlock + 1 + kWaves) * 4);
  L.off_k = L.off_wd = o;
  L.total = o;
  return L;
}

// Bytes reserved for the per-item constants of a second-pass block (the largest instance).
constexpr int kItemConstsBytes = 1024;

// LDS of a second-pass block: the map (FP64 edges and widths, and the edges and widths of the FP32 map for the FP32
// finish; no counts), the sin/cos table, the f tables, the per-wave W^2 histograms, reduction and scan scratch, the
// item's constants (off_k) and, per thread, a slot of the D words of the sample it evaluates (off_wd, word d of thread t
// at index d kBlock + t).  alt = false (every table of the launch interpolates linearly in ln q): a table holds f_j
// alone, which keeps the 2<->3 workload's block within 40 KB, four blocks per CU.
__host__ __device__ inline Lds shell_layout(int D, int nb, int n_tab, int n_max, int fbytes, bool alt) {
  Lds L;
  const int DN = D * nb;
  int o = 0;
  L.off_e = o;
  o = align16(o + DN * 8);
  L.off_w = o;
  o = align16(o + DN * 8);
  L.off_m32 = o;
  o = align16(o + 2 * kMapSlots * 4);
  L.off_sc = o;
  o = align16(o + 33 * 16);
  L.off_tab = o;
  L.tab_stride = align16(n_max * (alt ? 16 + fbytes : fbytes));
  L.tab_f = alt ? 16 * n_max : 0;
  o = align16(o + n_tab * L.tab_stride);
  L.off_h = o;
  o = align16(o + kWaves * DN * 8);
  L.off_c = o;  // no counts
  L.off_red = o;
  o = align16(o + 2 * kWaves * 8);
  L.off_q = o;
  o = align16(o + (kBlock + 1 + kWaves) * 4);
  L.off_k = o;
  o = align16(o + kItemConstsBytes);
  L.off_wd = o;
  o = align16(o + kBlock * D * 4);
  L.total = o;
  return L;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// e^z for the FP32 integrand with the range reduction in FP64: z log2(e) = n + fr, fr in [0, 1), then
// 2^fr on the hardware exp2 and an exact scaling by 2^n.  Relative error ~1e-7 for any |z| (an FP32
// argument would lose |z| 2^-24).
__device__ __forceinline__ float exp_split(double z) {
  const double y = z * 1.4426950408889634074;
  double n = floor(y);
  const float fr = (float)(y - n);
  n = n > 200.0 ? 200.0 : (n < -200.0 ? -200.0 : n);
  return ldexpf(__builtin_amdgcn_exp2f(fr), (int)n);
}

// Pointers into a block's LDS (32-bit LDS addresses, read with LDS instructions wherever they are stored).
template <typename T>
using lds_ptr = T __attribute__((address_space(3)))*;
template <typename T>
__device__ __forceinline__ lds_ptr<T> to_lds(T* p) {
  return (lds_ptr<T>)p;
}

// sin(k pi/16), cos(k pi/16), k = 0..32 (correctly rounded; staged into LDS by every sample block).
__constant__ double kSinPi16[33] = {0.0, 0.19509032201612828, 0.3826834323650898, 0.5555702330196022, 0.7071067811865476, 0.8314696123025452, 0.9238795325112867, 0.9807852804032304, 1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452, 0.7071067811865476, 0.5555702330196022, 0.3826834323650898, 0.19509032201612828, 0.0, -0.19509032201612828, -0.3826834323650898, -0.5555702330196022, -0.7071067811865476, -0.8314696123025452, -0.9238795325112867, -0.9807852804032304, -1.0, -0.9807852804032304, -0.9238795325112867, -0.8314696123025452, -0.7071067811865476, -0.5555702330196022, -0.3826834323650898, -0.19509032201612828, 0.0};
__constant__ double kCosPi16[33] = {1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452, 0.7071067811865476, 0.5555702330196022, 0.3826834323650898, 0.19509032201612828, 0.0, -0.19509032201612828, -0.3826834323650898, -0.5555702330196022, -0.7071067811865476, -0.8314696123025452, -0.9238795325112867, -0.9807852804032304, -1.0, -0.9807852804032304, -0.9238795325112867, -0.8314696123025452, -0.7071067811865476, -0.5555702330196022, -0.3826834323650898, -0.19509032201612828, 0.0, 0.19509032201612828, 0.3826834323650898, 0.5555702330196022, 0.7071067811865476, 0.8314696123025452, 0.9238795325112867, 0.9807852804032304, 1.0};

// sin and cos of x in [0, 2 pi]: x = k pi/16 + tau with a two-part Cody-Waite reduction (k pi/16 exact in
// the first part), |tau| <= pi/32, Taylor series of sin(tau) to tau^11 and cos(tau) to tau^12 (truncation
// below 1e-22), then the angle-addition formulas with the tabulated sin/cos of k pi/16.
__device__ __forceinline__ void sincos_red(double x, lds_ptr<const double> tab, double* s, double* c) {
  const double kf = rint(x * 5.092958178940651);
  const double tau = fma(-kf, 9.304434350608279e-14, fma(-kf, 0.19634954084926903, x));
  int k = (int)kf;
  k = k < 0 ? 0 : (k > 32 ? 32 : k);
  const double t2 = tau * tau;
  double ps = -2.505210838544172e-08;
  ps = fma(ps, t2, 2.7557319223985893e-06);
  ps = fma(ps, t2, -0.0001984126984126984);
  ps = fma(ps, t2, 0.008333333333333333);
  ps = fma(ps, t2, -0.16666666666666666);
  const double st = fma(tau * t2, ps, tau);
  double pc = 2.08767569878681e-09;
  pc = fma(pc, t2, -2.755731922398589e-07);
  pc = fma(pc, t2, 2.48015873015873e-05);
  pc = fma(pc, t2, -0.001388888888888889);
  pc = fma(pc, t2, 0.041666666666666664);
  pc = fma(pc, t2, -0.5);
  const double ct = fma(pc, t2, 1.0);
  const double sk = tab[2 * k], ck = tab[2 * k + 1];  // the table holds (sin, cos) pairs
  *s = fma(sk, ct, ck * st);
  *c = fma(ck, ct, -(sk * st));
}

// Natural logarithm of q > 0: q = 2^e m with m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh((m-1)/(m+1)) by its
// Taylor series to z^19 (|z| <= 0.1716, truncation below 3e-17), e ln 2 in two parts.
__device__ __forceinline__ double log_pos(double q) {
  int e;
  double m = frexp(q, &e);
  if (m < 0.7071067811865476) {
    m *= 2.0;
    e -= 1;
  }
  const double z = (m - 1.0) / (m + 1.0);
  const double z2 = z * z;
  double p = 0.10526315789473684;  // 2/19
  p = fma(p, z2, 0.11764705882352941);
  p = fma(p, z2, 0.13333333333333333);
  p = fma(p, z2, 0.15384615384615385);
  p = fma(p, z2, 0.18181818181818182);
  p = fma(p, z2, 0.2222222222222222);
  p = fma(p, z2, 0.2857142857142857);
  p = fma(p, z2, 0.4);
  p = fma(p, z2, 0.6666666666666666);
  p = fma(p, z2, 2.0);
  const double de = (double)e;
  return fma(de, 0.6931471805592082, fma(de, 7.371002565167799e-13, z * p));
}

// A table of f on a logarithmic grid in LDS (q_j, 1/q_j, f_j).
// Per node, by rule: linear in ln q -- (unused, unused, f_j); spline -- (q_j, M_j, f_j) with M_j the second
// derivatives; equilibrium-exact -- (E_j, y_j = log(1/f_j + eta), unused).
template <typename T>
struct FTab {
  lds_ptr<const double> q;
  lds_ptr<const double> iq;
  lds_ptr<const T> f;
  int n;
  int mode;
  double lq0, inv_h, eta;
};

// Value between two nodes by the spline (mode 1: A = q, B = M) or the equilibrium-exact rule (mode 2: A = E,
// B = log(1/f + eta)); q is the comoving momentum, E the energy.
__device__ __forceinline__ double interp_alt64(int mode, double eta, double q, double E, double A0, double A1, double B0,
                                               double B1, double f0, double f1) {
  if (mode == 1) {
    const double hq = A1 - A0;
    const double b = (q - A0) / hq, a = 1.0 - b;
    return a * f0 + b * f1 + ((a * a * a - a) * B0 + (b * b * b - b) * B1) * (hq * hq / 6.0);
  }
  const double w = (E - A0) / (A1 - A0);
  return 1.0 / (exp(B0 + w * (B1 - B0)) - eta);
}

// FP64: position t = (ln q - ln q_0)/h on the grid, node j = floor(t), weight t - j.
// ALT = false: the linear rule only (every table of the launch uses it).
template <bool ALT>
__device__ __forceinline__ double interp64(const FTab<double>& t, double q, double E, int* jo, double* wo) {
  const double tp = (log_pos(q) - t.lq0) * t.inv_h;
  int j = (int)floor(tp);
  j = j < 0 ? 0 : (j > t.n - 2 ? t.n - 2 : j);
  const double w = tp - (double)j;
  *jo = j;
  *wo = w;
  if (ALT && t.mode != 0)
    return interp_alt64(t.mode, t.eta, q, E, t.q[j], t.q[j + 1], t.iq[j], t.iq[j + 1], t.f[j], t.f[j + 1]);
  const double f0 = t.f[j], f1 = t.f[j + 1];
  return f0 + w * (f1 - f0);
}

// f of species S (table f, global memory) at comoving momentum q with energy E by the rule of Sec. III.B: linear
// in ln q between the bracketing nodes inside [q_0, q_{N-1}], the fit f = 1 / (exp(a + b E) - eta) outside.
__device__ __forceinline__ double f_at_global(const SpecDev& S, const double* __restrict__ f, const double* qnode,
                                              const double* fit, double q, double E) {
  if (q < S.q_min) return 1.0 / (exp(fit[0] + fit[1] * E) - (double)S.stat);
  if (q > S.q_max) return 1.0 / (exp(fit[2] + fit[3] * E) - (double)S.stat);
  const double tp = (log_pos(q) - S.lq0) * S.inv_h;
  int j = (int)floor(tp);
  j = j < 0 ? 0 : (j > S.n - 2 ? S.n - 2 : j);
  if (S.interp == 1)
    return interp_alt64(1, (double)S.stat, q, E, qnode[j], qnode[j + 1], S.aux[j], S.aux[j + 1], f[j], f[j + 1]);
  if (S.interp == 2)
    return interp_alt64(2, (double)S.stat, q, E, S.aux[j], S.aux[j + 1], S.tmp[j], S.tmp[j + 1], f[j], f[j + 1]);
  const double w = tp - (double)j;
  return f[j] + w * (f[j + 1] - f[j]);
}

// FP32 integrand: the grid position in FP64 (an FP32 logarithm would move the weight by ~1e-6 / h, which the
// linear interpolation of a steep tail amplifies by f_j / f_{j+1}); interpolation of the FP32 table.
template <bool ALT>
__device__ __forceinline__ float interp32(const FTab<float>& t, double q, double E) {
  const double tp = (log_pos(q) - t.lq0) * t.inv_h;
  int j = (int)floor(tp);
  j = j < 0 ? 0 : (j > t.n - 2 ? t.n - 2 : j);
  if (ALT && t.mode == 1) {
    const double q0 = t.q[j], hq = t.q[j + 1] - q0;
    const float b = (float)((q - q0) / hq), a = 1.0f - b;
    const float h26 = (float)(hq * hq / 6.0);
    return fmaf(a, t.f[j], b * t.f[j + 1]) +
           ((a * a * a - a) * (float)t.iq[j] + (b * b * b - b) * (float)t.iq[j + 1]) * h26;
  }
  if (ALT && t.mode == 2) {
    const double w = (E - t.q[j]) / (t.q[j + 1] - t.q[j]);
    return __builtin_amdgcn_rcpf(exp_split(t.iq[j] + w * (t.iq[j + 1] - t.iq[j])) - (float)t.eta);
  }
  const float w = (float)(tp - (double)j);
  const float f0 = t.f[j], f1 = t.f[j + 1];
  return fmaf(w, f1 - f0, f0);
}

// Per-item constants of a sample block at the current time (uniform across the block).
template <int NI, typename FT>
struct ItemConsts {
  static constexpr int NR = NI + 2;  // roles: integrated 0..NI-1, conserved NI, observed NI+1
  lds_ptr<const double> e;    // LDS map edges (D x nb)
  lds_ptr<const double> w;    // LDS map widths
  lds_ptr<const double> sc;   // LDS (sin, cos) of k pi/16, k = 0..32
  lds_ptr<float> m32;         // LDS FP32 map (screening pass): edges [0, kMapSlots), widths x 2^-32 [kMapSlots,
                      // 2 kMapSlots) (radial values divided by a, angles in revolutions), the unit's bin counts
                      // (as bits) after them
  FTab<FT> tr[NI + 1];
  float lg1[NI + 1], lg0[NI + 1];  // grid position from log2: t = log2(q) ln2/h - ln(q_0)/h
  float ylog2;   // log2(e) / (2 sigma_E^2) (absolute width)
  float shell;   // 7 sigma_E (absolute width)
  float far;     // |dE| of the FP64 underflow of the Gaussian factor, sqrt(2 746) sigma_E (absolute width)
  float cin, cfar;  // per unit of the summed energies: the FP32 margin, plus 3.5 w and sqrt(2 746) w / 2 (relative)
  float wconst;  // a^-3n |M|^2 / ((2 pi)^(3(n-1)-4) sqrt(2 pi)), divided by sigma_E for an absolute width
  float whalf32;
  int rel;       // relative width: sigma_E = whalf (sum of the point's energies)
  double whalf;
  int m2poly;    // |M|^2 = coupling^2 P(s, t)
  double m2c[6], cs[NR], ct[NR];
  double a, inv_a, m2[NR], eta[NR], esg[NR];
  int obsside[NR];
  double p_obs, E_obs, f_obs, g_obs, l_obs, a3M2, e_cut;
  double fit[4], qc_min, qc_max;
  double inv2s2, dnorm, twopi_pow;
  double a3M2_tp;  // a3M2 / twopi_pow (the FP32 integrand's weight constant)
  int nb, net, term;
  uint32_t uid, c3, seed_lo, seed_hi;
};

// The uniforms of an item's iteration form one stream of 32-bit words: word w is output w & 3 of the
// Philox4x32-10 block with counter (lo32(w >> 2), hi32(w >> 2), uid, c3), and sample n takes words D n .. D n + D-1.
// A group of G = 4 / gcd(D, 4) consecutive samples, starting at a multiple of G, fills G D / 4 whole blocks.  The
// host keeps D N below 2^34, so the block index fits 32 bits and the counter's second word is 0 (which also makes
// the first round's second product, and the second round's first, the same for every lane).
template <int D>
struct WordStream {
  static constexpr int g = D % 4 == 0 ? 4 : (D % 2 == 0 ? 2 : 1);  // gcd(D, 4): a sample starts at w & 3 = k g
  static constexpr int G = 4 / g;                                 // samples per group
  static constexpr int GB = G * D / 4;                            // blocks per group
  static constexpr int NB = (4 - g + D - 1) / 4 + 1;              // blocks one sample can touch
};

// The D words of sample n (any n): its blocks, then the words from the sample's offset in the first.
template <int D>
__device__ __forceinline__ void sample_words(uint32_t* wd, uint64_t n, uint32_t uid, uint32_t c3, uint32_t k0,
                                             uint32_t k1) {
  using WS = WordStream<D>;
  const uint64_t w0 = n * (uint64_t)D;
  const uint64_t b0 = w0 >> 2;
  const int off = (int)(w0 & 3u);
  uint32_t all[4 * WS::NB];
#pragma unroll
  for (int b = 0; b < WS::NB; ++b) {
    const Philox4 r = philox4x32_10((uint32_t)(b0 + b), 0u, uid, c3, k0, k1);
#pragma unroll
    for (int s = 0; s < 4; ++s) all[4 * b + s] = r.v[s];
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    uint32_t v = all[i];
#pragma unroll
    for (int o = WS::g; o < 4; o += WS::g) v = off == o ? all[i + o] : v;
    wd[i] = v;
  }
}

// Of the G D words of the group of samples ng .. ng + G-1 (ng a multiple of G), the blocks whose first word belongs
// to sample s of the group (block b starts in sample 4 b / D): called for s = 0 .. G-1 in turn, just before sample
// s is used, it fills every word of the group once, with few of them live at a time.
template <int D>
__device__ __forceinline__ void group_blocks_for(uint32_t* wd, int s, uint64_t ng, uint32_t uid, uint32_t c3,
                                                 uint32_t k0, uint32_t k1) {
  using WS = WordStream<D>;
  const uint32_t b0 = (uint32_t)((ng * (uint64_t)D) >> 2);
#pragma unroll
  for (int b = 0; b < WS::GB; ++b) {
    if ((4 * b) / D != s) continue;
    const Philox4 r = philox4x32_10(b0 + (uint32_t)b, 0u, uid, c3, k0, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) wd[4 * b + q] = r.v[q];
  }
}

// One sample with FP64 kinematics (map, sin/cos, momenta, energies, dE and the Gaussian's argument); the f
// tables, interpolation and statistical factor in FT.  Returns W and, per dimension d, the histogram offset
// d nb + j of the sample's bin j.
// P(s, t) = c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2 from the four-momentum sums Ps and Pt (E, x, y, z).
template <typename T>
__device__ __forceinline__ T m2_poly(const double* c, const T* Ps, const T* Pt) {
  const T s = Ps[0] * Ps[0] - (Ps[1] * Ps[1] + Ps[2] * Ps[2] + Ps[3] * Ps[3]);
  const T t = Pt[0] * Pt[0] - (Pt[1] * Pt[1] + Pt[2] * Pt[2] + Pt[3] * Pt[3]);
  return (T)c[0] + (T)c[1] * s + (T)c[2] * t + (T)c[3] * s * s + (T)c[4] * s * t + (T)c[5] * t * t;
}

// Adds coefficient c times the four-momentum (E, x, y, z) to the sum P.
template <typename T>
__device__ __forceinline__ void add4(T* P, T c, T E, T x, T y, T z) {
  P[0] += c * E;
  P[1] += c * x;
  P[2] += c * y;
  P[3] += c * z;
}

// STRAT (VEGAS+): y_d = (dig_d + u_d) / kst, the sample inside hypercube dig of kst^D.
template <int NI, typename FT, bool ALT, bool STRAT = false>
__device__ __forceinline__ double eval_sample(const ItemConsts<NI, FT>& K, uint64_t n, int* hj,
                                              const int* dig = nullptr, int kst = 1) {
#pragma clang fp contract(off)
  constexpr int D = 3 * NI;
  uint32_t wd[D];
  sample_words<D>(wd, n, K.uid, K.c3, K.seed_lo, K.seed_hi);
  const int nb = K.nb;
  const double dnb = (double)nb;
  double J = 1.0, jac = 1.0;
  double sx = 0.0, sy = 0.0, sz = K.esg[NI + 1] * K.p_obs;  // sum_in - sum_out over all but the conserved
  double dE = K.esg[NI + 1] * K.E_obs;
  double prod2E = 2.0 * K.E_obs, sumE = K.E_obs;
  bool cut = K.E_obs < K.e_cut;
  FT gain = (FT)K.g_obs, loss = (FT)K.l_obs;
  double Ps[4] = {0.0, 0.0, 0.0, 0.0}, Pt[4] = {0.0, 0.0, 0.0, 0.0};  // Mandelstam sums (polynomial |M|^2)
  if constexpr (ALT) {
    if (K.m2poly) {
      add4(Ps, K.cs[NI + 1], K.E_obs, 0.0, 0.0, K.p_obs);
      add4(Pt, K.ct[NI + 1], K.E_obs, 0.0, 0.0, K.p_obs);
    }
  }
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    double x3[3], sc3[2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int d = 3 * k + c;
      double yn = (((double)wd[d] + 0.5) * 2.3283064365386962890625e-10) * dnb;
      if constexpr (STRAT) yn = (((double)dig[d] + ((double)wd[d] + 0.5) * 2.3283064365386962890625e-10) / (double)kst) * dnb;
      int j = (int)yn;
      j = j > nb - 1 ? nb - 1 : j;
      const double del = yn - (double)j;
      const double e0 = K.e[d * nb + j], w = K.w[d * nb + j];
      x3[c] = e0 + w * del;
      J *= dnb * w;
      hj[d] = d * nb + j;
      if (c != 0) sincos_red(x3[c], K.sc, &sc3[c - 1][0], &sc3[c - 1][1]);
    }
    const double r = x3[0];
    const double sth = sc3[0][0], cth = sc3[0][1], sph = sc3[1][0], cph = sc3[1][1];
    const double p = r * K.inv_a;
    const double ps = p * sth;
    sx += K.esg[k] * (ps * cph);
    sy += K.esg[k] * (ps * sph);
    sz += K.esg[k] * (p * cth);
    jac *= r * r * sth;
    const double E = sqrt(p * p + K.m2[k]);
    cut |= E < K.e_cut;
    dE += K.esg[k] * E;
    prod2E *= 2.0 * E;
    sumE += E;
    if constexpr (ALT) {
      if (K.m2poly) {
        add4(Ps, K.cs[k], E, ps * cph, ps * sph, p * cth);
        add4(Pt, K.ct[k], E, ps * cph, ps * sph, p * cth);
      }
    }
    FT f;
    if constexpr (std::is_same<FT, double>::value) {
      int jj;
      double ww;
      f = interp64<ALT>(K.tr[k], r, E, &jj, &ww);
    } else {
      f = interp32<ALT>(K.tr[k], r, E);
    }
    const FT bf = (FT)1.0 + (FT)K.eta[k] * f;
    gain *= K.obsside[k] ? bf : f;
    loss *= K.obsside[k] ? f : bf;
  }
  // ---- conserved particle ----
  const double P2 = sx * sx + sy * sy + sz * sz;
  const double Ec = sqrt(P2 + K.m2[NI]);
  cut |= Ec < K.e_cut;
  dE += K.esg[NI] * Ec;
  prod2E *= 2.0 * Ec;
  sumE += Ec;
  double m2f = 1.0;
  if constexpr (ALT) {
    if (K.m2poly) {
      // the conserved particle's momentum: sum_in - sum_out of the others, negated for an initial-state one
      const double sc = -K.esg[NI];
      add4(Ps, K.cs[NI], Ec, sc * sx, sc * sy, sc * sz);
      add4(Pt, K.ct[NI], Ec, sc * sx, sc * sy, sc * sz);
      m2f = m2_poly(K.m2c, Ps, Pt);
    }
  }
  const double qc = K.a * sqrt(P2);
  FT fc;
  if constexpr (std::is_same<FT, double>::value) {
    if (qc < K.qc_min) {
      fc = 1.0 / (exp(K.fit[0] + K.fit[1] * Ec) - K.eta[NI]);
    } else if (qc > K.qc_max) {
      fc = 1.0 / (exp(K.fit[2] + K.fit[3] * Ec) - K.eta[NI]);
    } else {
      int jj;
      double ww;
      fc = interp64<ALT>(K.tr[NI], qc, Ec, &jj, &ww);
    }
  } else {
    if (qc < K.qc_min) {
      fc = __builtin_amdgcn_rcpf(exp_split(K.fit[0] + K.fit[1] * Ec) - (float)K.eta[NI]);
    } else if (qc > K.qc_max) {
      fc = __builtin_amdgcn_rcpf(exp_split(K.fit[2] + K.fit[3] * Ec) - (float)K.eta[NI]);
    } else {
      fc = interp32<ALT>(K.tr[NI], qc, Ec);
    }
  }
  {
    const FT bf = (FT)1.0 + (FT)K.eta[NI] * fc;
    gain *= K.obsside[NI] ? bf : fc;
    loss *= K.obsside[NI] ? fc : bf;
  }
  const FT F = K.net ? gain - loss : (K.term == 0 ? gain : loss);
  double inv2s2 = K.inv2s2, dnorm = K.dnorm;
  if (K.rel) {
    const double sg = K.whalf * sumE;
    inv2s2 = 0.5 / (sg * sg);
    dnorm = 0.3989422804014327 / sg;
  }
  double W;
  if constexpr (std::is_same<FT, double>::value) {
    const double delta = exp(-dE * dE * inv2s2) * dnorm;
    W = J * (jac * K.a3M2 * delta / (K.twopi_pow * prod2E) * (double)F);
  } else {
    const float delta = exp_split(-dE * dE * inv2s2) * (float)dnorm;
    const float rcp = __builtin_amdgcn_rcpf((float)prod2E);
    W = J * jac * (K.a3M2 / K.twopi_pow) * ((double)delta * (double)rcp) * (double)F;
  }
  if constexpr (ALT) W *= m2f;
  return cut ? 0.0 : W;
}

// One listed sample of the second pass: the arithmetic of eval_sample, operation for operation (so results are the
// same bits), with the per-item constants read from the block's LDS copy K and the particle loop not unrolled, so
// that a thread keeps one particle's values live at a time.  The sample's D words are staged in the thread's LDS
// slot wl (word d at wl[d kBlock]); each is replaced by its bin's histogram index d nb + j once used.
template <int NI, typename FT, bool ALT>
__device__ __forceinline__ double eval_listed(const ItemConsts<NI, FT>* K, uint64_t n, uint32_t* wl) {
#pragma clang fp contract(off)
  constexpr int D = 3 * NI;
  {
    uint32_t wd[D];
    sample_words<D>(wd, n, K->uid, K->c3, K->seed_lo, K->seed_hi);
#pragma unroll
    for (int d = 0; d < D; ++d) wl[d * kBlock] = wd[d];
  }
  const int nb = K->nb;
  const double dnb = (double)nb;
  double J = 1.0, jac = 1.0;
  double sx = 0.0, sy = 0.0, sz = K->esg[NI + 1] * K->p_obs;  // sum_in - sum_out over all but the conserved
  double dE = K->esg[NI + 1] * K->E_obs;
  double prod2E = 2.0 * K->E_obs, sumE = K->E_obs;
  bool cut = K->E_obs < K->e_cut;
  FT gain = (FT)K->g_obs, loss = (FT)K->l_obs;
  double Ps[4] = {0.0, 0.0, 0.0, 0.0}, Pt[4] = {0.0, 0.0, 0.0, 0.0};  // Mandelstam sums (polynomial |M|^2)
  if constexpr (ALT) {
    if (K->m2poly) {
      add4(Ps, K->cs[NI + 1], K->E_obs, 0.0, 0.0, K->p_obs);
      add4(Pt, K->ct[NI + 1], K->E_obs, 0.0, 0.0, K->p_obs);
    }
  }
#pragma unroll 1
  for (int k = 0; k < NI; ++k) {
    double x3[3], sc3[2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int d = 3 * k + c;
      // y nb = (word + 1/2) nb 2^-32 in integers: bin j = high word of word nb + floor(nb/2), offset = (low word
      // + 1/2 for an odd nb) 2^-32 -- the same bits as the FP64 product (which is exact) and its floor
      const uint64_t t = (uint64_t)wl[d * kBlock] * (uint32_t)nb + (uint64_t)(nb >> 1);
      const int j = (int)(t >> 32);
      const double del = ((double)(uint32_t)t + 0.5 * (double)(nb & 1)) * 2.3283064365386962890625e-10;
      const double e0 = K->e[d * nb + j], w = K->w[d * nb + j];
      wl[d * kBlock] = (uint32_t)(d * nb + j);  // the word is spent: its slot keeps the bin for the accumulation
      x3[c] = e0 + w * del;
      J *= dnb * w;
      if (c != 0) sincos_red(x3[c], K->sc, &sc3[c - 1][0], &sc3[c - 1][1]);
    }
    const double r = x3[0];
    const double sth = sc3[0][0], cth = sc3[0][1], sph = sc3[1][0], cph = sc3[1][1];
    const double p = r * K->inv_a;
    const double ps = p * sth;
    const double sg = K->esg[k];
    sx += sg * (ps * cph);
    sy += sg * (ps * sph);
    sz += sg * (p * cth);
    jac *= r * r * sth;
    const double E = sqrt(p * p + K->m2[k]);
    cut |= E < K->e_cut;
    dE += sg * E;
    prod2E *= 2.0 * E;
    sumE += E;
    if constexpr (ALT) {
      if (K->m2poly) {
        add4(Ps, K->cs[k], E, ps * cph, ps * sph, p * cth);
        add4(Pt, K->ct[k], E, ps * cph, ps * sph, p * cth);
      }
    }
    FT f;
    if constexpr (std::is_same<FT, double>::value) {
      int jj;
      double ww;
      f = interp64<ALT>(K->tr[k], r, E, &jj, &ww);
    } else {
      f = interp32<ALT>(K->tr[k], r, E);
    }
    const FT bf = (FT)1.0 + (FT)K->eta[k] * f;
    const bool os = K->obsside[k];
    gain *= os ? bf : f;
    loss *= os ? f : bf;
  }
  // ---- conserved particle ----
  const double P2 = sx * sx + sy * sy + sz * sz;
  const double Ec = sqrt(P2 + K->m2[NI]);
  cut |= Ec < K->e_cut;
  dE += K->esg[NI] * Ec;
  prod2E *= 2.0 * Ec;
  sumE += Ec;
  double m2f = 1.0;
  if constexpr (ALT) {
    if (K->m2poly) {
      const double sc = -K->esg[NI];
      add4(Ps, K->cs[NI], Ec, sc * sx, sc * sy, sc * sz);
      add4(Pt, K->ct[NI], Ec, sc * sx, sc * sy, sc * sz);
      m2f = m2_poly(K->m2c, Ps, Pt);
    }
  }
  const double qc = K->a * sqrt(P2);
  FT fc;
  if constexpr (std::is_same<FT, double>::value) {
    if (qc < K->qc_min) {
      fc = 1.0 / (exp(K->fit[0] + K->fit[1] * Ec) - K->eta[NI]);
    } else if (qc > K->qc_max) {
      fc = 1.0 / (exp(K->fit[2] + K->fit[3] * Ec) - K->eta[NI]);
    } else {
      int jj;
      double ww;
      fc = interp64<ALT>(K->tr[NI], qc, Ec, &jj, &ww);
    }
  } else {
    if (qc < K->qc_min) {
      fc = __builtin_amdgcn_rcpf(exp_split(K->fit[0] + K->fit[1] * Ec) - (float)K->eta[NI]);
    } else if (qc > K->qc_max) {
      fc = __builtin_amdgcn_rcpf(exp_split(K->fit[2] + K->fit[3] * Ec) - (float)K->eta[NI]);
    } else {
      fc = interp32<ALT>(K->tr[NI], qc, Ec);
    }
  }
  {
    const FT bf = (FT)1.0 + (FT)K->eta[NI] * fc;
    gain *= K->obsside[NI] ? bf : fc;
    loss *= K->obsside[NI] ? fc : bf;
  }
  const FT F = K->net ? gain - loss : (K->term == 0 ? gain : loss);
  double inv2s2 = K->inv2s2, dnorm = K->dnorm;
  if (K->rel) {
    const double sg = K->whalf * sumE;
    inv2s2 = 0.5 / (sg * sg);
    dnorm = 0.3989422804014327 / sg;
  }
  double W;
  if constexpr (std::is_same<FT, double>::value) {
    const double delta = exp(-dE * dE * inv2s2) * dnorm;
    W = J * (jac * K->a3M2 * delta / (K->twopi_pow * prod2E) * (double)F);
  } else {
    const float delta = exp_split(-dE * dE * inv2s2) * (float)dnorm;
    const float rcp = __builtin_amdgcn_rcpf((float)prod2E);
    W = J * jac * K->a3M2_tp * ((double)delta * (double)rcp) * (double)F;
  }
  if constexpr (ALT) W *= m2f;
  return cut ? 0.0 : W;
}

// A listed near sample of the FP32-integrand second pass (7 sigma_E < |dE| < 38.6 sigma_E): the arithmetic of
// screen_sample's FP32 finish, operation for operation, with the constants read from the block's LDS copy K, the
// sample's words from the thread's LDS slot wl and the particle loop not unrolled.
template <int NI, bool ALT>
__device__ __forceinline__ double near_listed(const ItemConsts<NI, float>* K, uint32_t* wl) {
  const uint32_t nb = (uint32_t)K->nb;
  const uint64_t half_nb = nb >> 1;
  const float a32 = (float)K->a;
  const float fnb32 = (float)nb * 4294967296.0f, fnb32r = fnb32 * a32, fnb32rev = fnb32 * 6.2831853071795865f;
  float J = 1.0f, jac = 1.0f;
  float sx = 0.0f, sy = 0.0f, sz = (float)(K->esg[NI + 1] * K->p_obs);
  float dE = (float)(K->esg[NI + 1] * K->E_obs), sumE = (float)K->E_obs, prod2E = 2.0f * (float)K->E_obs;
  float gain = (float)K->g_obs, loss = (float)K->l_obs;
  bool cut = K->E_obs < K->e_cut;
  float Ps[4] = {0.0f, 0.0f, 0.0f, 0.0f}, Pt[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // Mandelstam sums
  if constexpr (ALT) {
    if (K->m2poly) {
      add4(Ps, (float)K->cs[NI + 1], (float)K->E_obs, 0.0f, 0.0f, (float)K->p_obs);
      add4(Pt, (float)K->ct[NI + 1], (float)K->E_obs, 0.0f, 0.0f, (float)K->p_obs);
    }
  }
  const lds_ptr<float> m32 = K->m32;
#pragma unroll 1
  for (int k = 0; k < NI; ++k) {
    float x3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int d = 3 * k + c;
      const uint64_t t = (uint64_t)wl[d * kBlock] * nb + (half_nb + ((uint64_t)(d * nb) << 32));
      const uint32_t jdu = (uint32_t)(t >> 32);
      wl[d * kBlock] = jdu;  // the word is spent: its slot keeps the bin (d nb + j) for the accumulation
      const float e0 = m32[jdu], ew = m32[kMapSlots + jdu];
      x3[c] = fmaf(ew, (float)(uint32_t)t, e0);
      J *= (c == 0 ? fnb32r : fnb32rev) * ew;
    }
    const float p = x3[0];
    const float r = p * a32;
    const float th = x3[1], ph = x3[2];
    const float sth = __builtin_amdgcn_sinf(th), cth = __builtin_amdgcn_cosf(th);
    const float sph = __builtin_amdgcn_sinf(ph), cph = __builtin_amdgcn_cosf(ph);
    const float ps = p * sth;
    const float sg = (float)K->esg[k];
    sx = fmaf(sg, ps * cph, sx);
    sy = fmaf(sg, ps * sph, sy);
    sz = fmaf(sg, p * cth, sz);
    jac *= r * r * sth;
    const float E = __builtin_amdgcn_sqrtf(fmaf(p, p, (float)K->m2[k]));
    cut |= E < (float)K->e_cut;
    dE = fmaf(sg, E, dE);
    sumE += E;
    prod2E *= 2.0f * E;
    if constexpr (ALT) {
      if (K->m2poly) {
        add4(Ps, (float)K->cs[k], E, ps * cph, ps * sph, p * cth);
        add4(Pt, (float)K->ct[k], E, ps * cph, ps * sph, p * cth);
      }
    }
    const FTab<float>& T = K->tr[k];
    float f;
    if (!ALT || T.mode == 0) {
      const float tp = fmaf(__builtin_amdgcn_logf(r), K->lg1[k], -K->lg0[k]);
      int jj = (int)tp;
      jj = jj < 0 ? 0 : (jj > T.n - 2 ? T.n - 2 : jj);
      const float wgt = tp - (float)jj;
      f = fmaf(wgt, T.f[jj + 1] - T.f[jj], T.f[jj]);
    } else {
      f = interp32<ALT>(T, (double)r, (double)E);
    }
    const float bf = fmaf((float)K->eta[k], f, 1.0f);
    const bool os = K->obsside[k];
    gain *= os ? bf : f;
    loss *= os ? f : bf;
  }
  const float P2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  const float Ec = __builtin_amdgcn_sqrtf(P2 + (float)K->m2[NI]);
  dE = fmaf((float)K->esg[NI], Ec, dE);
  sumE += Ec;
  prod2E *= 2.0f * Ec;
  float ylog2 = K->ylog2, wconst = K->wconst;
  if (K->rel) {
    const float isg = __builtin_amdgcn_rcpf(K->whalf32 * sumE);
    ylog2 = 0.72134752044448170f * isg * isg;
    wconst *= isg;
  }
  const float y = -(dE * dE) * ylog2;
  const float qc = (float)K->a * __builtin_amdgcn_sqrtf(P2);
  float fc;
  if (qc < (float)K->qc_min) {
    fc = __builtin_amdgcn_rcpf(exp_split((double)fmaf((float)K->fit[1], Ec, (float)K->fit[0])) - (float)K->eta[NI]);
  } else if (qc > (float)K->qc_max) {
    fc = __builtin_amdgcn_rcpf(exp_split((double)fmaf((float)K->fit[3], Ec, (float)K->fit[2])) - (float)K->eta[NI]);
  } else {
    const FTab<float>& T = K->tr[NI];
    if (!ALT || T.mode == 0) {
      const float tp = fmaf(__builtin_amdgcn_logf(qc), K->lg1[NI], -K->lg0[NI]);
      int jj = (int)tp;
      jj = jj < 0 ? 0 : (jj > T.n - 2 ? T.n - 2 : jj);
      fc = fmaf(tp - (float)jj, T.f[jj + 1] - T.f[jj], T.f[jj]);
    } else {
      fc = interp32<ALT>(T, (double)qc, (double)Ec);
    }
  }
  const float bf = fmaf((float)K->eta[NI], fc, 1.0f);
  gain *= K->obsside[NI] ? bf : fc;
  loss *= K->obsside[NI] ? fc : bf;
  float F = K->net ? gain - loss : (K->term == 0 ? gain : loss);
  if constexpr (ALT) {
    if (K->m2poly) {
      const float sc = -(float)K->esg[NI];
      add4(Ps, (float)K->cs[NI], Ec, sc * sx, sc * sy, sc * sz);
      add4(Pt, (float)K->ct[NI], Ec, sc * sx, sc * sy, sc * sz);
      F *= m2_poly(K->m2c, Ps, Pt);
    }
  }
  const float e = floorf(y);
  const float m = J * jac * wconst * __builtin_amdgcn_rcpf(prod2E) * __builtin_amdgcn_exp2f(__builtin_amdgcn_fractf(y));
  cut |= Ec < (float)K->e_cut;
  return cut ? 0.0 : ldexp((double)m, (int)e) * (double)F;
}

// The accumulation of one listed sample: S1 += W, S2 += W^2, and W^2 into the wave's histogram at the sample's bins,
// dimension by dimension as accumulate does.  eval_listed and near_listed leave each dimension's histogram index
// d nb + j in the thread's LDS slot in place of the word it came from.
template <int D>
__device__ __forceinline__ void accumulate_listed(double W, const uint32_t* wl, double& S1, double& S2,
                                                  double* my_h) {
  S1 += W;
  S2 += W * W;
  if (fabs(W) >= kHistWMin) {
    const double w2 = W * W;
#pragma unroll
    for (int d = 0; d < D; ++d) atomicAdd(&my_h[wl[d * kBlock]], w2);
  }
}

// FP32 screening pass of one sample: FP32 map, hardware sin/cos/log2/sqrt, momenta, energies and dE.  Returns the
// sample's class:
//   kInShell  |dE| < 7 sigma_E + m: W needs the FP64 kinematics;
//   kFar      |dE| > sqrt(2 746) sigma_E + m: the FP64 |dE| exceeds the point where the Gaussian factor
//             e^(-dE^2 / (2 sigma_E^2)) underflows to 0 in FP64, so W = 0 exactly;
//   kNear     the rest: with FINISH, W is finished in FP32.  Its Gaussian factor is below e^-24.5 = 2.3e-11 of the
//             peak, and the FP32 dE moves the factor by at most a few per cent there (|dE| eps_32 sum(E) / sigma_E^2
//             for sums of energies up to 100 and sigma_E = 0.005), so such a sample shifts the integral by ~1e-12 of
//             its size at most; W matters for the map's training histogram, where that accuracy is ample.
// m = 1e-3 of the summed energies bounds the difference of the FP32 and FP64 dE with a wide margin.  The bin of
// every dimension is exact (the same as with the FP64 map).  With COUNT the sample is added to the count of its bin
// in every dimension (the count word of the bin's map slot).
constexpr int kFar = 0, kNear = 1, kInShell = 2;

template <int NI, bool FINISH, bool ALT = false, bool COUNT = false>
__device__ __forceinline__ int screen_sample(const ItemConsts<NI, float>& K, const uint32_t* wd, int* hj,
                                             double* Wout) {
  const uint32_t nb = (uint32_t)__builtin_amdgcn_readfirstlane(K.nb);  // uniform (the item's), for the asm below
  const uint64_t half_nb = nb >> 1;
  // nb as a vector operand, so that the 64-bit multiply-add below can take its uniform addend from scalar registers
  uint32_t vnb;
  asm("v_mov_b32 %0, %1" : "=v"(vnb) : "s"(nb));
  const float a32 = (float)K.a;
  // per-dimension Jacobian factors (the radial widths carry 1/a, the angular ones 1/(2 pi))
  const float fnb32 = (float)nb * 4294967296.0f, fnb32r = fnb32 * a32, fnb32rev = fnb32 * 6.2831853071795865f;
  float J = 1.0f, jac = 1.0f;
  float sx = 0.0f, sy = 0.0f, sz = (float)(K.esg[NI + 1] * K.p_obs);
  float dE = (float)(K.esg[NI + 1] * K.E_obs), sumE = (float)K.E_obs, prod2E = 2.0f * (float)K.E_obs;
  float gain = (float)K.g_obs, loss = (float)K.l_obs;
  bool cut = K.E_obs < K.e_cut;
  float Ps[4] = {0.0f, 0.0f, 0.0f, 0.0f}, Pt[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // Mandelstam sums (FINISH)
  constexpr bool kPoly = FINISH && ALT;
  if constexpr (kPoly) {
    if (K.m2poly) {
      add4(Ps, (float)K.cs[NI + 1], (float)K.E_obs, 0.0f, 0.0f, (float)K.p_obs);
      add4(Pt, (float)K.ct[NI + 1], (float)K.E_obs, 0.0f, 0.0f, (float)K.p_obs);
    }
  }
#pragma unroll
  for (int k = 0; k < NI; ++k) {
    float x3[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int d = 3 * k + c;
      // y nb = (word + 1/2) nb / 2^32: the bin is the high word of word nb + floor(nb/2) (exact; an odd nb only
      // moves the in-bin offset by 2^-33), the offset comes from the low word; d nb added to the high word makes it
      // the histogram index d nb + j directly
      const uint64_t t = (uint64_t)wd[d] * vnb + (half_nb + ((uint64_t)(d * nb) << 32));
      uint32_t jdu = (uint32_t)(t >> 32);
      asm("" : "+v"(jdu));  // keeps the bin index as the product's high word (one shift-add to the address below)
      const int jd = (int)jdu;
      // one LDS address for the bin's edge, width and count (the last two at constant offsets)
      const lds_ptr<char> mp = (lds_ptr<char>)K.m32 + 4u * jdu;
      const float e0 = *(lds_ptr<const float>)mp;
      const float ew = *(lds_ptr<const float>)(mp + 4 * kMapSlots);
      if constexpr (COUNT) atomicAdd((uint32_t*)(mp + 8 * kMapSlots), 1u);  // the bin's count
      x3[c] = fmaf(ew, (float)(uint32_t)t, e0);
      J *= (c == 0 ? fnb32r : fnb32rev) * ew;
      hj[d] = jd;
    }
    const float p = x3[0];  // physical momentum: the radial map values carry 1/a
    const float r = p * a32;  // comoving momentum (the finish's Jacobian and f lookup)
    const float th = x3[1], ph = x3[2];  // revolutions
    const float sth = __builtin_amdgcn_sinf(th), cth = __builtin_amdgcn_cosf(th);
    const float sph = __builtin_amdgcn_sinf(ph), cph = __builtin_amdgcn_cosf(ph);
    const float ps = p * sth;
    const float sg = (float)K.esg[k];
    sx = fmaf(sg, ps * cph, sx);
    sy = fmaf(sg, ps * sph, sy);
    sz = fmaf(sg, p * cth, sz);
    jac *= r * r * sth;
    const float E = __builtin_amdgcn_sqrtf(fmaf(p, p, (float)K.m2[k]));
    cut |= E < (float)K.e_cut;
    dE = fmaf(sg, E, dE);
    sumE += E;
    prod2E *= 2.0f * E;
    if constexpr (kPoly) {
      if (K.m2poly) {
        add4(Ps, (float)K.cs[k], E, ps * cph, ps * sph, p * cth);
        add4(Pt, (float)K.ct[k], E, ps * cph, ps * sph, p * cth);
      }
    }
    if constexpr (FINISH) {  // the f tables are in LDS only for the finish (the screening layout has the map alone)
      const FTab<float>& T = K.tr[k];
      float f;
      if (!ALT || T.mode == 0) {
        const float tp = fmaf(__builtin_amdgcn_logf(r), K.lg1[k], -K.lg0[k]);
        int jj = (int)tp;
        jj = jj < 0 ? 0 : (jj > T.n - 2 ? T.n - 2 : jj);
        const float wgt = tp - (float)jj;
        f = fmaf(wgt, T.f[jj + 1] - T.f[jj], T.f[jj]);
      } else {
        f = interp32<ALT>(T, (double)r, (double)E);
      }
      const float bf = fmaf((float)K.eta[k], f, 1.0f);
      gain *= K.obsside[k] ? bf : f;
      loss *= K.obsside[k] ? f : bf;
    }
  }
  const float P2 = fmaf(sx, sx, fmaf(sy, sy, sz * sz));
  const float Ec = __builtin_amdgcn_sqrtf(P2 + (float)K.m2[NI]);
  dE = fmaf((float)K.esg[NI], Ec, dE);
  sumE += Ec;
  prod2E *= 2.0f * Ec;
  const float adE = fabsf(dE);
  if (adE < fmaf(K.cin, sumE, K.shell)) return kInShell;
  if (adE > fmaf(K.cfar, sumE, K.far)) return kFar;
  if constexpr (FINISH) {
    float ylog2 = K.ylog2, wconst = K.wconst;
    if (K.rel) {
      const float isg = __builtin_amdgcn_rcpf(K.whalf32 * sumE);
      ylog2 = 0.72134752044448170f * isg * isg;
      wconst *= isg;
    }
    const float y = -(dE * dE) * ylog2;
    const float qc = (float)K.a * __builtin_amdgcn_sqrtf(P2);
    float fc;
    if (qc < (float)K.qc_min) {
      fc = __builtin_amdgcn_rcpf(exp_split((double)fmaf((float)K.fit[1], Ec, (float)K.fit[0])) - (float)K.eta[NI]);
    } else if (qc > (float)K.qc_max) {
      fc = __builtin_amdgcn_rcpf(exp_split((double)fmaf((float)K.fit[3], Ec, (float)K.fit[2])) - (float)K.eta[NI]);
    } else {
      const FTab<float>& T = K.tr[NI];
      if (!ALT || T.mode == 0) {
        const float tp = fmaf(__builtin_amdgcn_logf(qc), K.lg1[NI], -K.lg0[NI]);
        int jj = (int)tp;
        jj = jj < 0 ? 0 : (jj > T.n - 2 ? T.n - 2 : jj);
        fc = fmaf(tp - (float)jj, T.f[jj + 1] - T.f[jj], T.f[jj]);
      } else {
        fc = interp32<ALT>(T, (double)qc, (double)Ec);
      }
    }
    const float bf = fmaf((float)K.eta[NI], fc, 1.0f);
    gain *= K.obsside[NI] ? bf : fc;
    loss *= K.obsside[NI] ? fc : bf;
    float F = K.net ? gain - loss : (K.term == 0 ? gain : loss);
    if constexpr (kPoly) {
      if (K.m2poly) {
        const float sc = -(float)K.esg[NI];
        add4(Ps, (float)K.cs[NI], Ec, sc * sx, sc * sy, sc * sz);
        add4(Pt, (float)K.ct[NI], Ec, sc * sx, sc * sy, sc * sz);
        F *= m2_poly(K.m2c, Ps, Pt);
      }
    }
    // W = m 2^e F: the Gaussian's exponent y = -dE^2 log2(e) / (2 sigma_E^2) = e + (y - e) with e integer, the
    // weight factors and 2^(y - e) in FP32 (their product stays well inside the FP32 range), the power of two and
    // F applied in FP64 (W itself can lie far below the FP32 range)
    // (y is rounded before it is split: a fused y - floor(y) could leave [0, 1) by up to half an ulp of y)
    const float e = floorf(y);
    const float m = J * jac * wconst * __builtin_amdgcn_rcpf(prod2E) * __builtin_amdgcn_exp2f(__builtin_amdgcn_fractf(y));
    cut |= Ec < (float)K.e_cut;
    *Wout = cut ? 0.0 : ldexp((double)m, (int)e) * (double)F;
  }
  return kNear;
}

// Clears the per-wave training histograms (W^2 sums and counts, contiguous up to the reduction scratch) with
// 16-byte stores.
__device__ __forceinline__ void clear_hist(const Lds& lay, unsigned char* smem) {
  uint4* p = reinterpret_cast<uint4*>(smem + lay.off_h);
  const int n16 = (lay.off_red - lay.off_h) / 16;
  for (int i = threadIdx.x; i < n16; i += kBlock) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Per-item set-up of a sample block: stages the map (FP64 edges and widths, FP32 map), the sin/cos table and the f
// tables into LDS unless the block's previous task staged the same item, clears the per-wave training histograms,
// and fills the per-item constants at the current time.  LAY: the block's layout -- kLayScreen (the screening pass:
// the FP32 map only), kLaySample, or kLayShell (the second pass: K is the block's LDS copy, filled by thread 0).
// Ends with a block barrier.
template <int NI, int PREC, int LAY = kLaySample, bool ALT = true>
__device__ __forceinline__ Lds setup_block(const SampleLaunch& L, const ItemRec* __restrict__ it,
                                           unsigned char* smem, bool stage,
                                           ItemConsts<NI, typename std::conditional<PREC == 0, double, float>::type>& K) {
  constexpr int D = 3 * NI;
  constexpr int NR = NI + 2;
  constexpr bool SCREEN = LAY == kLayScreen;
  using FT = typename std::conditional<PREC == 0, double, float>::type;
  static_assert(sizeof(ItemConsts<NI, FT>) <= kItemConstsBytes, "per-item constants exceed their LDS slot");
  const int tid = threadIdx.x;
  const int nb = it->nb;
  const int DN = D * nb;
  const int n_tab = it->n_tab;
  int n_max = 0;
  for (int k = 0; k < n_tab; ++k) n_max = max(n_max, L.spec[it->tab_species[k]].n);
  const Lds lay = SCREEN ? screen_layout()
                         : (LAY == kLayShell ? shell_layout(D, nb, n_tab, n_max, sizeof(FT), ALT)
                                             : lds_layout(D, nb, n_tab, n_max, sizeof(FT)));
  double* sm_e = reinterpret_cast<double*>(smem + lay.off_e);
  double* sm_w = reinterpret_cast<double*>(smem + lay.off_w);
  float* sm_m32 = reinterpret_cast<float*>(smem + lay.off_m32);
  double2* sm_sc = reinterpret_cast<double2*>(smem + lay.off_sc);

  const double* __restrict__ map = L.maps + it->map_off;
  for (int i = tid; stage && i < DN; i += kBlock) {
    const int d = i / nb, j = i - d * nb;
    const double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
    if constexpr (!SCREEN) {
      sm_e[i] = e0;
      sm_w[i] = e1 - e0;
    }
    // screening map: the width carries the 2^-32 of the uniform's low word, the radial values are physical momenta
    // (comoving / a) and the angles are in revolutions (the hardware sine takes them), so a momentum or an angle is
    // one fma of the low word; the bin's count starts at 0
    const double sc = (d % 3 == 0) ? L.st->inv_a : 0.15915494309189535;
    sm_m32[i] = (float)(e0 * sc);
    sm_m32[kMapSlots + i] = (float)((e1 - e0) * sc * 2.3283064365386962890625e-10);
    if constexpr (LAY != kLayShell) reinterpret_cast<uint32_t*>(sm_m32)[2 * kMapSlots + i] = 0u;
  }
  if (!SCREEN && stage && tid < 33) sm_sc[tid] = make_double2(kSinPi16[tid], kCosPi16[tid]);
  for (int k = 0; !SCREEN && stage && k < n_tab; ++k) {
    const SpecDev& S = L.spec[it->tab_species[k]];
    unsigned char* base = smem + lay.off_tab + k * lay.tab_stride;
    double* q = reinterpret_cast<double*>(base);
    double* iq = q + n_max;
    FT* f = reinterpret_cast<FT*>(base + lay.tab_f);
    const int md = S.interp;
    for (int j = tid; j < S.n; j += kBlock) {
      if (lay.tab_f != 0) {  // (the compact layout of a linear-rule second pass holds f alone)
        q[j] = md == 2 ? S.aux[j] : L.qnode[S.f_off + j];  // node energies (EQEXACT) or nodes
        iq[j] = md == 1 ? S.aux[j] : (md == 2 ? S.tmp[j] : 0.0);  // spline M_j, or log(1/f_j + eta)
      }
      if constexpr (PREC == 0) f[j] = L.f64[S.f_off + j];
      else f[j] = L.f32[S.f_off + j];
    }
  }
  if constexpr (!SCREEN) clear_hist(lay, smem);

  // the per-item constants: every thread fills its own copy, except in the second pass, whose K is the block's LDS
  // copy, written by thread 0 (every thread reaches the one barrier below)
  if (LAY != kLayShell || tid == 0) {
    K.e = to_lds<const double>(sm_e);
    K.w = to_lds<const double>(sm_w);
    K.sc = to_lds<const double>(reinterpret_cast<const double*>(sm_sc));
    K.m32 = to_lds<float>(sm_m32);
  #pragma unroll
    for (int r = 0; r <= NI; ++r) {
      const int k = it->r_tab[r];
      const SpecDev& S = L.spec[it->tab_species[k]];
      const unsigned char* base = smem + lay.off_tab + k * lay.tab_stride;
      K.tr[r].q = to_lds<const double>(reinterpret_cast<const double*>(base));
      K.tr[r].iq = K.tr[r].q + n_max;  // (not read by the linear rule)
      K.tr[r].f = to_lds<const FT>(reinterpret_cast<const FT*>(base + lay.tab_f));
      K.tr[r].n = S.n;
      K.tr[r].mode = S.interp;
      K.tr[r].eta = (double)S.stat;
      K.tr[r].lq0 = S.lq0;
      K.tr[r].inv_h = S.inv_h;
      K.lg1[r] = (float)(0.6931471805599453 * S.inv_h);
      K.lg0[r] = (float)(S.lq0 * S.inv_h);
    }
    const DevState* __restrict__ st = L.st;
    K.a = st->a;
    K.inv_a = st->inv_a;
  #pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double mr = st->m[it->r_species[r]];
      K.m2[r] = mr * mr;
      K.eta[r] = (double)L.spec[it->r_species[r]].stat;
      K.esg[r] = it->r_in[r] ? 1.0 : -1.0;
      K.obsside[r] = it->r_obsside[r];
      K.cs[r] = (double)it->r_cs[r];
      K.ct[r] = (double)it->r_ct[r];
    }
    K.m2poly = it->m2poly;
  #pragma unroll
    for (int k = 0; k < 6; ++k) K.m2c[k] = it->m2c[k];
    const SpecDev& So = L.spec[it->obs_species];
    K.p_obs = it->q_obs * K.inv_a;
    K.E_obs = sqrt(K.p_obs * K.p_obs + K.m2[NI + 1]);
    K.f_obs = it->obs_at ? f_at_global(So, L.f64 + So.f_off, L.qnode + So.f_off, st->fit[it->obs_species], it->q_obs,
                                       K.E_obs)
                          : L.f64[So.f_off + it->eval_idx];
    {
      const double obs_bf = 1.0 + K.eta[NI + 1] * K.f_obs;
      K.g_obs = K.obsside[NI + 1] ? obs_bf : K.f_obs;  // the observed leg is on the observed side
      K.l_obs = K.obsside[NI + 1] ? K.f_obs : obs_bf;
    }
    K.a3M2 = st->a_m3n[NI] * it->coupling2;
    K.e_cut = it->e_cut;
    const SpecDev& Sc = L.spec[it->r_species[NI]];
  #pragma unroll
    for (int k = 0; k < 4; ++k) K.fit[k] = st->fit[it->r_species[NI]][k];
    K.qc_min = Sc.q_min;
    K.qc_max = Sc.q_max;
    K.twopi_pow = it->twopi_pow;
    K.a3M2_tp = K.a3M2 / K.twopi_pow;
    {
      // the Gaussian energy delta: an absolute width, or w (E_in + E_out) / 2 at each point
      constexpr double kRs2pi = 0.3989422804014327, kFarK = 38.62641583165593;  // 1/sqrt(2 pi), sqrt(2 746)
      const double wd = st->width[it->proc];
      K.rel = it->rel;
      if (it->rel) {
        K.whalf = 0.5 * wd;
        K.inv2s2 = 0.0;
        K.dnorm = 0.0;
        K.shell = 0.0f;
        K.far = 0.0f;
        K.cin = (float)(1e-3 + 3.5 * wd);  // 7 sigma_E with sigma_E = w sum(E) / 2
        K.cfar = (float)(1e-3 + 0.5 * kFarK * wd);
        K.ylog2 = 0.0f;
        K.wconst = (float)(K.a3M2 / K.twopi_pow * kRs2pi);
      } else {
        K.whalf = 0.0;
        K.inv2s2 = 1.0 / (2.0 * wd * wd);
        K.dnorm = kRs2pi / wd;
        K.shell = (float)(7.0 * wd);
        K.far = (float)(kFarK * wd);
        K.cin = 1e-3f;
        K.cfar = 1e-3f;
        K.ylog2 = (float)(1.4426950408889634 * K.inv2s2);
        K.wconst = (float)(K.a3M2 / K.twopi_pow * K.dnorm);
      }
      K.whalf32 = (float)K.whalf;
    }
    K.nb = nb;
    K.net = it->net;
    K.term = it->term;
    K.uid = it->uid;
    K.c3 = st->epoch * 64u + (uint32_t)L.it;
    K.seed_lo = L.seed_lo;
    K.seed_hi = L.seed_hi;
  }
  __syncthreads();
  return lay;
}

// One sample's contribution: S1 += W, S2 += W^2 (registers), W^2 and (with COUNT) a count into the wave's
// histograms.  A zero W^2 (cut samples, and every |W| below the histogram floor: with sigma_E << E most off-shell
// samples) leaves the sums unchanged, so its atomics are skipped.
template <int D, bool COUNT = true>
__device__ __forceinline__ void accumulate(double W, const int* hj, double& S1, double& S2, double* my_h,
                                           uint32_t* my_c) {
  S1 += W;
  S2 += W * W;
  if (fabs(W) >= kHistWMin) {
    const double w2 = W * W;
#pragma unroll
    for (int d = 0; d < D; ++d) atomicAdd(&my_h[hj[d]], w2);
  }
  if constexpr (COUNT) {
#pragma unroll
    for (int d = 0; d < D; ++d) atomicAdd(&my_c[hj[d]], 1u);
  }
}

// End of a screening block's run of units of one item: the bin counts of the FP32 map added to the item's counts in
// global memory (integer atomics: any order gives the same sums; out = nullptr drops them) and cleared.
__device__ __forceinline__ void finish_counts(uint32_t* cnt, int DN, uint32_t* out) {
  __syncthreads();
  for (int i = threadIdx.x; i < DN; i += kBlock) {
    const uint32_t c = cnt[i];
    cnt[i] = 0u;
    if (out && c) atomicAdd(&out[i], c);
  }
  __syncthreads();
}

// Fixed-order end of a block's pass: butterfly wave sums of S1, S2, the four waves in order into s_out[0..1],
// and the wave histograms summed in wave order into rec[0 .. DN) (sums of W^2) and, with COUNTS, rec[DN .. 2 DN)
// (counts).
template <bool COUNTS>
__device__ __forceinline__ void finish_block(double S1, double S2, const Lds& lay, int DN, unsigned char* smem,
                                             double* s_out, double* rec) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double* sm_h = reinterpret_cast<const double*>(smem + lay.off_h);
  const uint32_t* sm_c = reinterpret_cast<const uint32_t*>(smem + lay.off_c);
  double* sm_red = reinterpret_cast<double*>(smem + lay.off_red);
  S1 = wave_sum(S1);
  S2 = wave_sum(S2);
  if (lane == 0) {
    sm_red[2 * wave] = S1;
    sm_red[2 * wave + 1] = S2;
  }
  __syncthreads();
  if (tid == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      s1 += sm_red[2 * w];
      s2 += sm_red[2 * w + 1];
    }
    s_out[0] = s1;
    s_out[1] = s2;
  }
  for (int i = tid; i < DN; i += kBlock) {
    double h = 0.0;
    uint32_t c = 0;
    for (int w = 0; w < kWaves; ++w) {
      h += sm_h[w * DN + i];
      if constexpr (COUNTS) c += sm_c[w * DN + i];
    }
    rec[i] = h;
    if constexpr (COUNTS) rec[DN + i] = (double)c;
  }
  __syncthreads();
}

// FP32 integrand, screening pass over the units of tasks t0 .. t1-1 (all of one item; launch positions t).
// A lane screens the G consecutive samples of one word group (G = 4 / gcd(D, 4): their uniforms fill whole Philox
// blocks); wave w takes rounds of 64 G samples (round k: samples n0 + 256 G k + 64 G w + G lane + s, s < G), so
// each wave screens a quarter of a unit.  With COUNT every sample adds to the counts of its bins (the unit's counts;
// a launch whose maps do not adapt passes no counts and runs without them); far samples (W = 0) do nothing else;
// the offsets n - n0 of in-shell samples are appended, in screening order (round, s, lane), to the front of the
// wave's list of the task position (list_stride / 4 entries per wave), those of near samples to its back, for the
// second pass; the wave's two counts are stored.
template <int NI, bool COUNT>
__device__ void screen_run(const SampleLaunch& L, int t0, int t1, unsigned char* smem, bool stage) {
  constexpr int D = 3 * NI;
  const int item = L.tasks[L.task_begin + t0].item;
  const ItemRec* __restrict__ it = &L.items[item];
  ItemConsts<NI, float> K;
  const Lds lay = setup_block<NI, 1, kLayScreen>(L, it, smem, stage, K);
  const int DN = D * it->nb, tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // bin counts of the current unit, in the FP32 map (all four waves add into them; zero when a unit starts: staged
  // as zero, and cleared by the previous unit's finish)
  uint32_t* slot_cnt = reinterpret_cast<uint32_t*>(smem + lay.off_m32) + 2 * kMapSlots;
  const uint64_t below = (1ull << lane) - 1ull;
  const int64_t wlen = L.list_stride / kWaves;
  for (int t = t0; t < t1; ++t) {
    const int unit = L.tasks[L.task_begin + t].unit;
    const int64_t n0 = (int64_t)unit * it->unit_size;
    const int64_t n1 = min(n0 + (int64_t)it->unit_size, it->N);
    uint16_t* lst = L.shell_list + (int64_t)t * L.list_stride + (int64_t)wave * wlen;
    uint32_t cin = 0, cnear = 0;  // wave-uniform
    constexpr int G = WordStream<D>::G;
    for (int64_t rbase = n0 + 64 * G * wave; rbase < n1; rbase += (int64_t)kBlock * G) {
      const int64_t ng = rbase + (int64_t)G * lane;  // the lane's group
      uint32_t wg[G * D];
#pragma unroll
      for (int s = 0; s < G; ++s) {
        group_blocks_for<D>(wg, s, (uint64_t)ng, K.uid, K.c3, K.seed_lo, K.seed_hi);
        const int64_t n = ng + s;
        int cls = kFar;
        if (n < n1) {
          int hj[D];
          double W;
          cls = screen_sample<NI, false, false, COUNT>(K, wg + s * D, hj, &W);
        }
        const uint64_t b_in = __ballot(cls == kInShell), b_near = __ballot(cls == kNear);
        if (cls == kInShell) lst[cin + (uint32_t)__popcll(b_in & below)] = (uint16_t)(n - n0);
        if (cls == kNear) lst[wlen - 1 - (cnear + (uint32_t)__popcll(b_near & below))] = (uint16_t)(n - n0);
        cin += (uint32_t)__popcll(b_in);
        cnear += (uint32_t)__popcll(b_near);
      }
    }
    if (lane == 0) {
      L.shell_cnt[(int64_t)t * 2 * kWaves + wave] = cin;
      L.shell_cnt[(int64_t)t * 2 * kWaves + kWaves + wave] = cnear;
    }
  }
  // the run's bin counts (all its units) into the item's counts
  if constexpr (COUNT) {
    finish_counts(slot_cnt, DN, L.counts + it->part_off);
  } else {
    __syncthreads();  // the next run restages the LDS
  }
}

// Second pass over the in-shell tasks k0 .. k1-1 (ranges of units of one item).  Per task: its in-shell lists, then
// its near lists (unit order, waves in order within a unit), read as one sequence in chunks of 256 lists; entry e of
// a chunk is evaluated by thread (e - first entry of the block's tile in the chunk) mod 256.  FP64 (PREC 0): every
// listed sample with FP64 kinematics and integrand.  FP32 integrand (PREC 1): in-shell samples with FP64
// kinematics, near samples with the FP32 finish.  The block's sums go to the task's record (tile t of the task: the
// t-th record from there).
template <int NI, int PREC, bool ALT>
__device__ void shell_run(const SampleLaunch& L, int k0, int k1, int tile, unsigned char* smem, bool stage) {
  constexpr int D = 3 * NI;
  constexpr int kLists = kBlock;  // lists per chunk: 64 units x 4 waves
  using FT = typename std::conditional<PREC == 0, double, float>::type;
  const ItemRec* __restrict__ it = &L.items[L.sh_tasks[L.sh_begin + k0].item];
  const int tid = threadIdx.x, wave = tid >> 6;
  int n_max = 0;
  for (int q = 0; q < it->n_tab; ++q) n_max = max(n_max, L.spec[it->tab_species[q]].n);
  // the item's constants live in LDS (read where needed, so that few stay in registers across a sample)
  ItemConsts<NI, FT>* K =
      reinterpret_cast<ItemConsts<NI, FT>*>(smem + shell_layout(D, it->nb, it->n_tab, n_max, sizeof(FT), ALT).off_k);
  const Lds lay = setup_block<NI, PREC, kLayShell, ALT>(L, it, smem, stage, *K);
  uint32_t* wl = reinterpret_cast<uint32_t*>(smem + lay.off_wd) + tid;  // this thread's word slot
  const int DN = D * it->nb;
  double* my_h = reinterpret_cast<double*>(smem + lay.off_h) + wave * DN;
  int* pre = reinterpret_cast<int*>(smem + lay.off_q);  // kLists + 1 prefix sums
  int* wtot = pre + kLists + 1;                          // per-wave totals of the scan
  const int lane = tid & 63;
  const int64_t wlen = L.list_stride / kWaves;
  const int tiles = L.sh_tiles;
  for (int k = k0; k < k1; ++k) {
    const ShellTask sht = L.sh_tasks[L.sh_begin + k];
    if (k > k0) {
      clear_hist(lay, smem);
      __syncthreads();
    }
    const int pos0 = sht.first_task - L.task_begin - sht.unit_begin;  // task position of unit 0
    // the group's listed samples form one sequence: the in-shell lists, then the near lists (unit order, waves in
    // order within a unit); this block evaluates entries [e_lo, e_hi), its tile of ceil(M / tiles) entries
    int e_lo = 0, e_hi = 0;
    {
      const int n_lists = 2 * (sht.unit_end - sht.unit_begin) * kWaves;
      int v = 0;
      for (int i = tid; i < n_lists; i += kBlock) {
        const int kind = i / (n_lists / 2), r = i % (n_lists / 2);
        const int u = sht.unit_begin + r / kWaves, w = r % kWaves;
        v += (int)L.shell_cnt[(int64_t)(pos0 + u) * 2 * kWaves + kind * kWaves + w];
      }
      #pragma unroll
      for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
      if (lane == 0) wtot[wave] = v;
      __syncthreads();
      int M = 0;
      for (int w = 0; w < kWaves; ++w) M += wtot[w];
      __syncthreads();  // wtot is rewritten by the scans below
      const int per = (M + tiles - 1) / tiles;
      e_lo = min(M, tile * per);
      e_hi = min(M, e_lo + per);
      if (tid == 0 && tile == 0 && L.n_listed) atomicAdd(L.n_listed, (unsigned long long)M);
    }
    int base = 0;  // position of the current chunk's first entry in the group's sequence
    double S1 = 0.0, S2 = 0.0;
    // the group's lists in sequence order: the in-shell lists of its units (unit order, waves in order within a
    // unit), then their near lists; taken kLists at a time, so that the two kinds share one entry loop (a wave
    // whose 64 entries straddle the boundary runs both evaluations)
    const int nu = sht.unit_end - sht.unit_begin, n_half = nu * kWaves;
    for (int c0 = 0; c0 < 2 * n_half && base < e_hi; c0 += kLists) {
      const int nl = min(kLists, 2 * n_half - c0);
      // block-wide inclusive scan of the list lengths: within each wave, then the wave totals in order
      int v = 0;
      if (tid < nl) {
        const int i = c0 + tid, kind = i >= n_half ? 1 : 0, r = i - kind * n_half;
        v = (int)L.shell_cnt[(int64_t)(pos0 + sht.unit_begin + r / kWaves) * 2 * kWaves + kind * kWaves +
                             r % kWaves];
      }
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
      }
      if (lane == 63) wtot[wave] = v;
      __syncthreads();
      for (int w = 0; w < wave; ++w) v += wtot[w];
      pre[tid + 1] = v;
      if (tid == 0) pre[0] = 0;
      __syncthreads();
      const int M = pre[nl];
      // this chunk's entries that fall in the tile: [lo, hi) of the chunk (entry e of the chunk is sequence entry
      // base + e), thread t taking lo + t, lo + t + 256, ...
      const int lo = max(0, e_lo - base), hi = min(M, e_hi - base);
      base += M;
      // sample index of chunk entry e, and whether it comes from a near list
      auto entry = [&](int e, bool& near) -> uint64_t {
        int a = 0, b = nl;  // pre[a] <= e < pre[b]
        while (b - a > 1) {
          const int mid = (a + b) >> 1;
          if (pre[mid] <= e) a = mid;
          else b = mid;
        }
        const int i = c0 + a, kind = i >= n_half ? 1 : 0, r = i - kind * n_half;
        const int u = sht.unit_begin + r / kWaves, w = r % kWaves, k = e - pre[a];
        const uint16_t* lst = L.shell_list + (int64_t)(pos0 + u) * L.list_stride + w * wlen;
        near = kind != 0;
        const uint32_t off = kind == 0 ? lst[k] : lst[wlen - 1 - k];
        return (uint64_t)((int64_t)u * it->unit_size + off);
      };
      for (int e = lo + tid; e < hi; e += kBlock) {
        bool near;
        const uint64_t n = entry(e, near);
        double W;
        if constexpr (PREC == 0) {
          W = eval_listed<NI, FT, ALT>(K, n, wl);
        } else if (!near) {
          W = eval_listed<NI, FT, ALT>(K, n, wl);
        } else {
          uint32_t wd[D];
          sample_words<D>(wd, n, K->uid, K->c3, K->seed_lo, K->seed_hi);
#pragma unroll
          for (int d = 0; d < D; ++d) wl[d * kBlock] = wd[d];
          W = near_listed<NI, ALT>(K, wl);
        }
        accumulate_listed<D>(W, wl, S1, S2, my_h);  // the screening pass counted every sample
      }
      __syncthreads();  // pre is rewritten by the next chunk
    }
    double* rec = L.shell_rec + sht.rec + (int64_t)tile * (2 + DN);
    finish_block<false>(S1, S2, lay, DN, smem, rec, rec + 2);
  }
}

// ------------------------------------------------------------------------------------------------------
// Adjoint of the frozen-map estimator (FP64).  For each sample, W and its partial derivatives with respect to
// the f values it reads (scattered to the grid through the interpolation rule of the species, or to the
// extrapolation line (a, b) of the conserved particle's species), the masses of the species of every particle
// (through E_i in the Gaussian, in 1/(2 E_i), in the extrapolated or equilibrium-exact f, and the node energies of
// the equilibrium-exact rule), and the coupling (2 W / lambda) are summed.  Table gradients by rule (Sec. III.B):
// linear in ln q -- d/df_j with weights 1 - w, w; spline -- d/df_j with weights A, B and d/dM_j with weights
// (A^3 - A) h^2/6, (B^3 - B) h^2/6 (M, the second derivatives, depend on every node; the finish kernel solves the
// transposed spline system); equilibrium-exact -- d/dy_j of y_j = log(1/f_j + eta) (the gather converts to f_j).
// Per group record (doubles): n_tab * n_max table gradients, as many d/dM slots when a table of the item is a
// spline, then g_obs, d/d(a_lo, b_lo, a_hi, b_hi), d/dm per role (kMaxN), sum W.
__host__ __device__ inline int vjp_tab_len(int n_tab, int n_max, int spl) { return n_tab * n_max * (spl ? 2 : 1); }
__host__ __device__ inline int vjp_rec_len(int n_tab, int n_max, int spl) {
  return vjp_tab_len(n_tab, n_max, spl) + 1 + 4 + kMaxN + 1;
}
// 1 if a table the item reads is interpolated by the spline
__device__ inline int item_spline(const ItemRec& it, const SpecDev* spec) {
  int spl = 0;
  for (int k = 0; k < it.n_tab; ++k) spl |= spec[it.tab_species[k]].interp == 1 ? 1 : 0;
  return spl;
}

// One block per group of consecutive units of one item (the batched second pass's groups): the map, tables and
// constants are staged once, the units' listed samples are taken unit by unit, and the group's sums go to record
// unit_begin / shell_units of the item.  ALT = false: every table of the launch uses the linear rule (the other
// rules' code is not compiled in).
template <int NI, bool ALT>
__device__ void vjp_group(const SampleLaunch& L, const ShellTask sht, unsigned char* smem) {
#pragma clang fp contract(off)
  constexpr int D = 3 * NI;
  constexpr int NR = NI + 2;
  const ItemRec* __restrict__ it = &L.items[sht.item];
  const int tid = threadIdx.x;
  const int nb = it->nb;
  const int DN = D * nb;
  const int n_tab = it->n_tab;
  int n_max = 0;
  for (int k = 0; k < n_tab; ++k) n_max = max(n_max, L.spec[it->tab_species[k]].n);
  const int spl = item_spline(*it, L.spec);
  // LDS: e, w, sin/cos table, f tables (q, iq, f by rule, as in the forward pass), per-wave table gradients,
  // reduction scratch
  int o = 0;
  double* sm_e = reinterpret_cast<double*>(smem + o);
  o = align16(o + DN * 8);
  double* sm_w = reinterpret_cast<double*>(smem + o);
  o = align16(o + DN * 8);
  double2* sm_sc = reinterpret_cast<double2*>(smem + o);
  o = align16(o + 33 * 16);
  const int tab_stride = align16(n_max * 24);
  const int off_tab = o;
  o = align16(o + n_tab * tab_stride);
  const int TG = n_tab * n_max, TG2 = vjp_tab_len(n_tab, n_max, spl);
  double* sm_g = reinterpret_cast<double*>(smem + o);
  o = align16(o + kWaves * TG2 * 8);
  double* sm_red = reinterpret_cast<double*>(smem + o);
  const double* __restrict__ map = L.maps + it->map_off;
  for (int i = tid; i < DN; i += kBlock) {
    const int d = i / nb, j = i - d * nb;
    const double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
    sm_e[i] = e0;
    sm_w[i] = e1 - e0;
  }
  if (tid < 33) sm_sc[tid] = make_double2(kSinPi16[tid], kCosPi16[tid]);
  for (int k = 0; k < n_tab; ++k) {
    const SpecDev& S = L.spec[it->tab_species[k]];
    double* q = reinterpret_cast<double*>(smem + off_tab + k * tab_stride);
    double* iq = q + n_max;
    double* f = iq + n_max;
    const int md = S.interp;
    for (int j = tid; j < S.n; j += kBlock) {
      q[j] = md == 2 ? S.aux[j] : L.qnode[S.f_off + j];  // node energies (equilibrium-exact) or nodes
      iq[j] = md == 1 ? S.aux[j] : (md == 2 ? S.tmp[j] : 0.0);  // spline M_j, or log(1/f_j + eta)
      f[j] = L.f64[S.f_off + j];
    }
  }
  for (int i = tid; i < kWaves * TG2; i += kBlock) sm_g[i] = 0.0;
  FTab<double> tr[NI + 1];
  int tslot[NI + 1];
#pragma unroll
  for (int r = 0; r <= NI; ++r) {
    const int k = it->r_tab[r];
    const SpecDev& S = L.spec[it->tab_species[k]];
    tr[r].q = to_lds<const double>(reinterpret_cast<const double*>(smem + off_tab + k * tab_stride));
    tr[r].iq = tr[r].q + n_max;
    tr[r].f = tr[r].iq + n_max;
    tr[r].n = S.n;
    tr[r].mode = S.interp;
    tr[r].eta = (double)S.stat;
    tr[r].lq0 = S.lq0;
    tr[r].inv_h = S.inv_h;
    tslot[r] = k;
  }
  const DevState* __restrict__ st = L.st;
  const double a = st->a, inv_a = 1.0 / a;
  double m[NR], eta[NR], esg[NR];
  int obsside[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    m[r] = st->m[it->r_species[r]];
    eta[r] = (double)L.spec[it->r_species[r]].stat;
    esg[r] = it->r_in[r] ? 1.0 : -1.0;
    obsside[r] = it->r_obsside[r];
  }
  const SpecDev& So = L.spec[it->obs_species];
  const double p_obs = it->q_obs * inv_a;
  const double E_obs = sqrt(p_obs * p_obs + m[NI + 1] * m[NI + 1]);
  const double f_obs = L.f64[So.f_off + it->eval_idx];
  const double a3M2 = pow(a, -3.0 * (double)NI) * it->coupling2;
  const SpecDev& Sc = L.spec[it->r_species[NI]];
  const double* fitc = st->fit[it->r_species[NI]];
  const uint32_t uid = it->uid;
  const uint32_t c3 = st->epoch * 64u + (uint32_t)L.it;
  const double dnb = (double)nb;
  const double wpar = st->width[it->proc];
  const int rel = it->rel;
  const int wave = tid >> 6;
  double* my_g = sm_g + wave * TG2;
  __syncthreads();

  double g_obs = 0.0, dfit[4] = {0.0, 0.0, 0.0, 0.0}, dm[NR], sumW = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) dm[r] = 0.0;
  // Only the samples the screening pass listed (in or near the energy shell): every other sample has W = 0 and
  // zero derivatives.  Per unit of the group, in unit order: the unit's eight lists (in-shell then near, waves in
  // order) form one sequence whose entry e is taken by thread e mod 256.
  const int pos0 = sht.first_task - L.task_begin - sht.unit_begin;  // launch position of unit 0
  const int64_t wlen = L.list_stride / kWaves;
  for (int un = sht.unit_begin; un < sht.unit_end; ++un) {
  const int pos = pos0 + un;
  const int64_t n0 = (int64_t)un * it->unit_size;
  const uint32_t* cnt = L.shell_cnt + (int64_t)pos * 2 * kWaves;
  const uint16_t* lst = L.shell_list + (int64_t)pos * L.list_stride;
  int M = 0;
  for (int l = 0; l < 2 * kWaves; ++l) M += (int)cnt[l];
  for (int e = tid; e < M; e += kBlock) {
    int l = 0, ke = e;  // list l of the unit (in-shell lists of waves 0..3, then near lists), entry ke in it
    while (ke >= (int)cnt[l]) {
      ke -= (int)cnt[l];
      ++l;
    }
    const int lw = l % kWaves;
    const uint32_t off = l < kWaves ? lst[lw * wlen + ke] : lst[lw * wlen + wlen - 1 - ke];
    const int64_t n = n0 + off;
    uint32_t wd[D];
    sample_words<D>(wd, (uint64_t)n, uid, c3, L.seed_lo, L.seed_hi);
    double J = 1.0, jac = 1.0, sx = 0.0, sy = 0.0, sz = esg[NI + 1] * p_obs;
    double E[NR], f[NR], wt[NR], qv[NR];
    int jn[NR], src[NR];  // src: 0 table node, 1 interpolated, 2 extrapolated low, 3 extrapolated high
    E[NI + 1] = E_obs;
    f[NI + 1] = f_obs;
    src[NI + 1] = 0;
    jn[NI + 1] = it->eval_idx;
    wt[NI + 1] = 0.0;
    bool cut = E_obs < it->e_cut;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      double x3[3], sc3[2][2];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int d = 3 * k + c;
        const double yn = (((double)wd[d] + 0.5) * 2.3283064365386962890625e-10) * dnb;
        int j = (int)yn;
        j = j > nb - 1 ? nb - 1 : j;
        const double del = yn - (double)j;
        const double e0 = sm_e[d * nb + j], w = sm_w[d * nb + j];
        x3[c] = e0 + w * del;
        J *= dnb * w;
        if (c != 0)
          sincos_red(x3[c], to_lds<const double>(reinterpret_cast<const double*>(sm_sc)), &sc3[c - 1][0],
                     &sc3[c - 1][1]);
      }
      const double r = x3[0];
      const double p = r * inv_a;
      const double ps = p * sc3[0][0];
      sx += esg[k] * (ps * sc3[1][1]);
      sy += esg[k] * (ps * sc3[1][0]);
      sz += esg[k] * (p * sc3[0][1]);
      jac *= r * r * sc3[0][0];
      E[k] = sqrt(p * p + m[k] * m[k]);
      cut |= E[k] < it->e_cut;
      f[k] = interp64<ALT>(tr[k], r, E[k], &jn[k], &wt[k]);
      qv[k] = r;
      src[k] = 1;
    }
    const double P2 = sx * sx + sy * sy + sz * sz;
    E[NI] = sqrt(P2 + m[NI] * m[NI]);
    cut |= E[NI] < it->e_cut;
    const double qc = a * sqrt(P2);
    if (qc < Sc.q_min) {
      f[NI] = 1.0 / (exp(fitc[0] + fitc[1] * E[NI]) - eta[NI]);
      src[NI] = 2;
    } else if (qc > Sc.q_max) {
      f[NI] = 1.0 / (exp(fitc[2] + fitc[3] * E[NI]) - eta[NI]);
      src[NI] = 3;
    } else {
      f[NI] = interp64<ALT>(tr[NI], qc, E[NI], &jn[NI], &wt[NI]);
      src[NI] = 1;
    }
    qv[NI] = qc;
    if (cut) continue;
    double dE = 0.0, prod2E = 1.0, sumE = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      dE += esg[r] * E[r];
      prod2E *= 2.0 * E[r];
      sumE += E[r];
    }
    // width of the Gaussian at this point; a relative one grows with every energy (d sigma / d E = w / 2)
    const double sg = rel ? 0.5 * wpar * sumE : wpar;
    const double sig2 = sg * sg;
    const double delta = exp(-dE * dE * (0.5 / sig2)) * (0.3989422804014327 / sg);
    const double dsig = rel ? (dE * dE / sig2 - 1.0) / sg * (0.5 * wpar) : 0.0;
    // factors and their derivatives
    double gv[2][NR], dg[2][NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double bf = 1.0 + eta[r] * f[r];
      gv[0][r] = obsside[r] ? bf : f[r];
      dg[0][r] = obsside[r] ? eta[r] : 1.0;
      gv[1][r] = obsside[r] ? f[r] : bf;
      dg[1][r] = obsside[r] ? 1.0 : eta[r];
    }
    double Fv[2], dF[2][NR];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      Fv[t] = 1.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) Fv[t] *= gv[t][r];
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double prod = dg[t][r];
#pragma unroll
        for (int r2 = 0; r2 < NR; ++r2)
          if (r2 != r) prod *= gv[t][r2];
        dF[t][r] = prod;
      }
    }
    const double F = it->net ? Fv[0] - Fv[1] : Fv[it->term];
    const double Wb = J * (jac * a3M2 * delta / (it->twopi_pow * prod2E));
    const double W = Wb * F;
    sumW += W;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double dWdf = Wb * (it->net ? dF[0][r] - dF[1][r] : dF[it->term][r]);
      double dWdE = W * (-dE / sig2 * esg[r] - 1.0 / E[r] + dsig);
      if (src[r] == 0) {
        g_obs += dWdf;
      } else if (src[r] == 1) {
        const int rr = r <= NI ? r : 0;  // (the observed role reads its node: src 0)
        const int base = tslot[rr] * n_max, j = jn[r], mode = ALT ? tr[rr].mode : 0;
        if (mode == 1) {
          const double q0 = tr[rr].q[j], hq = tr[rr].q[j + 1] - q0;
          const double b = (qv[r] - q0) / hq, a1 = 1.0 - b, h26 = hq * hq / 6.0;
          atomicAdd(&my_g[base + j], dWdf * a1);
          atomicAdd(&my_g[base + j + 1], dWdf * b);
          atomicAdd(&my_g[TG + base + j], dWdf * ((a1 * a1 * a1 - a1) * h26));
          atomicAdd(&my_g[TG + base + j + 1], dWdf * ((b * b * b - b) * h26));
        } else if (mode == 2) {
          // f = 1/(exp(y) - eta), y = (1 - u) y_j + u y_{j+1}, u = (E - E_j)/(E_{j+1} - E_j)
          const double E0 = tr[rr].q[j], E1 = tr[rr].q[j + 1], dEn = E1 - E0;
          const double u = (E[r] - E0) / dEn;
          const double dfdy = -f[r] * (1.0 + eta[r] * f[r]);
          atomicAdd(&my_g[base + j], dWdf * dfdy * (1.0 - u));
          atomicAdd(&my_g[base + j + 1], dWdf * dfdy * u);
          const double dfdu = dfdy * (tr[rr].iq[j + 1] - tr[rr].iq[j]);
          dWdE += dWdf * dfdu / dEn;
          // the node energies sqrt((q_j/a)^2 + m^2) move with m: du/dE_j = (u - 1)/dEn, du/dE_{j+1} = -u/dEn
          dm[r] += dWdf * dfdu * ((u - 1.0) / dEn * (m[r] / E0) - u / dEn * (m[r] / E1));
        } else {
          atomicAdd(&my_g[base + j], dWdf * (1.0 - wt[r]));
          atomicAdd(&my_g[base + j + 1], dWdf * wt[r]);
        }
      } else {
        const int sd = src[r] - 2;
        const double dfdz = -f[r] * (1.0 + eta[r] * f[r]);
        dfit[2 * sd] += dWdf * dfdz;
        dfit[2 * sd + 1] += dWdf * dfdz * E[r];
        dWdE += dWdf * (-fitc[2 * sd + 1] * f[r] * (1.0 + eta[r] * f[r]));
      }
      dm[r] += dWdE * m[r] / E[r];
    }
  }
  }  // units of the group
  // ---- fixed-order reductions into the group's record ----
  constexpr int NS = 1 + 4 + NR + 1;
  double vals[NS];
  vals[0] = g_obs;
#pragma unroll
  for (int k = 0; k < 4; ++k) vals[1 + k] = dfit[k];
#pragma unroll
  for (int r = 0; r < NR; ++r) vals[5 + r] = dm[r];
  vals[5 + NR] = sumW;
  double* rec = L.parts + it->part_off + (int64_t)(sht.unit_begin / it->shell_units) * vjp_rec_len(n_tab, n_max, spl);
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const double v = wave_sum(vals[k]);
    if ((tid & 63) == 0) sm_red[k * kWaves + wave] = v;
  }
  __syncthreads();
  if (tid < NS) {
    double acc = 0.0;
    for (int w = 0; w < kWaves; ++w) acc += sm_red[tid * kWaves + w];
    const int slot = tid < 5 + NR ? tid : 5 + kMaxN;  // g_obs, fit partials, d/dm by role; then sum W
    rec[TG2 + slot] = acc;
  }
  if (tid >= 5 + NR && tid < 5 + kMaxN) rec[TG2 + tid] = 0.0;  // roles this process does not have
  for (int i = tid; i < TG2; i += kBlock) {
    double g = 0.0;
    for (int w = 0; w < kWaves; ++w) g += sm_g[w * TG2 + i];
    rec[i] = g;
  }
  __syncthreads();
}

template <int MASK, bool ALT>
__global__ __launch_bounds__(kBlock, 2) void k_vjp(SampleLaunch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int g = blockIdx.x; g < L.n_sh; g += gridDim.x) {
    const ShellTask sht = L.sh_tasks[L.sh_begin + g];
    const int ni = L.items[sht.item].nint;
    if ((MASK & 1) && ni == 1) vjp_group<1, ALT>(L, sht, smem);
    if ((MASK & 2) && ni == 2) vjp_group<2, ALT>(L, sht, smem);
    if ((MASK & 4) && ni == 3) vjp_group<3, ALT>(L, sht, smem);
    if ((MASK & 8) && ni == 4) vjp_group<4, ALT>(L, sht, smem);
  }
}

// Per item: sum of its group records in group order, times coef_i / N.
__global__ void k_vjp_reduce(const ItemRec* items, int n_items, const double* coef, const double* parts,
                             const int* rec_len, double* item_rec, int rec_stride) {
  const int i = blockIdx.x;
  if (i >= n_items) return;
  const ItemRec& it = items[i];
  const int len = rec_len[i];
  const int n_groups = (it.n_units + it.shell_units - 1) / it.shell_units;
  const double c = coef[i] / (double)it.N;
  for (int k = threadIdx.x; k < len; k += blockDim.x) {
    double acc = 0.0;
    for (int g = 0; g < n_groups; ++g) acc += parts[it.part_off + (int64_t)g * len + k];
    item_rec[(int64_t)i * rec_stride + k] = c * acc;
  }
}

// Sum of one value per thread of a 256-thread block in a fixed order: a butterfly within each wave, then the four
// waves in order; every thread gets the sum.  red: 4 doubles of LDS.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = ((red[0] + red[1]) + red[2]) + red[3];
  __syncthreads();
  return t;
}

// Gradients: grad_f of every species node (one block per node: its 256 threads take the items i = t, t + 256, ...,
// then a fixed-order block sum), then (k_vjp_finish, one block per species and one per process) the chain through
// the extrapolation fits, the spline's second derivatives, the masses, and the couplings.  rec_nmax holds per item the
// table length n_max of its record, then (at n_items + i) the offset of the record's tail (g_obs, fit partials,
// masses, sum W) after the table gradients.
__global__ __launch_bounds__(256) void k_vjp_gather(const ItemRec* items, int n_items, const double* item_rec,
                                                    const int* rec_nmax, int rec_stride, const SpecDev* spec,
                                                    int n_species, const double* f64, double* grad_f, int64_t n_f) {
  __shared__ double red[4];
  for (int64_t g = blockIdx.x; g < n_f; g += gridDim.x) {
    int s = 0;
    while (s + 1 < n_species && g >= spec[s + 1].f_off) ++s;
    const int j = (int)(g - spec[s].f_off);
    double acc = 0.0, obs = 0.0;
    for (int i = threadIdx.x; i < n_items; i += blockDim.x) {
      const ItemRec& it = items[i];
      const double* rec = item_rec + (int64_t)i * rec_stride;
      const int nmax = rec_nmax[i];
      for (int k = 0; k < it.n_tab; ++k)
        if (it.tab_species[k] == s && j < spec[s].n) acc += rec[k * nmax + j];
      if (it.obs_species == s && it.eval_idx == j) obs += rec[rec_nmax[n_items + i]];
    }
    acc = block_sum256(acc, red);
    obs = block_sum256(obs, red);
    if (threadIdx.x == 0) {
      // equilibrium-exact tables hold d/dy_j, y_j = log(1/f_j + eta): dy_j/df_j = -1 / (f_j (1 + eta f_j))
      if (spec[s].interp == 2) {
        const double fj = f64[g];
        acc *= -1.0 / (fj * (1.0 + (double)spec[s].stat * fj));
      }
      grad_f[g] = acc + obs;
    }
  }
}

// Adjoint of the spline's second derivatives (spline_second_derivatives: the tridiagonal system T M_int = r(f) in
// M_1 .. M_{n-2}, then M_0 and M_{n-1} extrapolated from it).  Given g = dL/dM on the n nodes, folds g_0 and g_{n-1}
// back onto the interior, solves T^T z = g_int (forward elimination and back substitution; T^T is tridiagonal with
// the sub- and super-diagonals of T swapped), and adds r'^T z to grad_f: z_j reaches f_{j+1} with 1/h_j, f_j with
// -(1/h_j + 1/h_{j-1}) and f_{j-1} with 1/h_{j-1}.  One thread; g, cp and dp are n-double scratch arrays.
__device__ void spline_adjoint(int n, const double* qn, double* g, double* cp, double* dp, double* grad_f) {
  auto hs = [&](int j) { return qn[j + 1] - qn[j]; };
  // row j (1 <= j <= n-2) of T after the two folds, as the forward elimination builds it
  auto row = [&](int j, double& lo, double& di, double& up) {
    const double hl = hs(j - 1), hr = hs(j);
    lo = hl / 6.0;
    di = (hl + hr) / 3.0;
    up = hr / 6.0;
    if (j == 1) {
      const double r0 = hl / hr;
      di += lo * (1.0 + r0);
      up -= lo * r0;
      lo = 0.0;
    }
    if (j == n - 2) {
      const double r1 = hr / hl;
      di += up * (1.0 + r1);
      lo -= up * r1;
      up = 0.0;
    }
  };
  const double h0 = hs(0), h1 = hs(1), ha = hs(n - 3), hb = hs(n - 2);
  // M_0 = (1 + h0/h1) M_1 - (h0/h1) M_2 and M_{n-1} = (1 + hb/ha) M_{n-2} - (hb/ha) M_{n-3}
  g[1] += (1.0 + h0 / h1) * g[0];
  g[2] -= (h0 / h1) * g[0];
  g[n - 2] += (1.0 + hb / ha) * g[n - 1];
  g[n - 3] -= (hb / ha) * g[n - 1];
  double lo, di, up, lo_n, di_n, up_n, lo_p, di_p, up_p;
  for (int j = 1; j <= n - 2; ++j) {
    row(j, lo, di, up);
    double sub = 0.0, sup = 0.0;
    if (j > 1) {
      row(j - 1, lo_p, di_p, up_p);
      sub = up_p;
    }
    if (j < n - 2) {
      row(j + 1, lo_n, di_n, up_n);
      sup = lo_n;
    }
    const double den = di - (j > 1 ? sub * cp[j - 1] : 0.0);
    cp[j] = sup / den;
    dp[j] = (g[j] - (j > 1 ? sub * dp[j - 1] : 0.0)) / den;
  }
  for (int j = n - 3; j >= 1; --j) dp[j] -= cp[j] * dp[j + 1];
  for (int j = 1; j <= n - 2; ++j) {
    const double hl = hs(j - 1), hr = hs(j), z = dp[j];
    grad_f[j + 1] += z / hr;
    grad_f[j] -= z * (1.0 / hr + 1.0 / hl);
    grad_f[j - 1] += z / hl;
  }
}

__global__ __launch_bounds__(256) void k_vjp_finish(const ItemRec* items, int n_items, const double* item_rec,
                                                    const int* rec_nmax, int rec_stride, const SpecDev* spec,
                                                    int n_species, const double* f64, const double* qnode,
                                                    const DevState* st, double* grad_f, int64_t n_f, double* work,
                                                    double* grad_m, double* grad_lam, const double* coupling,
                                                    int n_proc) {
  __shared__ double red[4];
  const int b = blockIdx.x, tid = threadIdx.x;
  if (b >= n_species) {  // process b - n_species: dL/dlambda = 2 sum W / lambda over its items
    const int p = b - n_species;
    double acc = 0.0;
    for (int i = tid; i < n_items; i += blockDim.x)
      if (items[i].proc == p) acc += item_rec[(int64_t)i * rec_stride + rec_nmax[n_items + i] + 5 + kMaxN];
    acc = block_sum256(acc, red);
    if (tid == 0) grad_lam[p] = 2.0 * acc / coupling[p];
    return;
  }
  const int s = b;
  const SpecDev& S = spec[s];
  // the items' fit partials and mass derivatives of this species (threads over items, fixed-order block sums)
  double dfa[4] = {0.0, 0.0, 0.0, 0.0}, gm = 0.0;
  for (int i = tid; i < n_items; i += blockDim.x) {
    const ItemRec& it = items[i];
    const double* rec = item_rec + (int64_t)i * rec_stride + rec_nmax[n_items + i];
    if (it.r_species[it.nint] == s)
      for (int k = 0; k < 4; ++k) dfa[k] += rec[1 + k];
    for (int r = 0; r < it.nint + 2; ++r)
      if (it.r_species[r] == s) gm += rec[5 + r];
  }
  for (int k = 0; k < 4; ++k) dfa[k] = block_sum256(dfa[k], red);
  gm = block_sum256(gm, red);
  double* gM = work + S.f_off;  // the species' d/dM_j (spline), then the solve's two scratch rows
  if (S.interp == 1) {  // threads over nodes, each summing the items in order
    for (int j = tid; j < S.n; j += blockDim.x) {
      double g = 0.0;
      for (int i = 0; i < n_items; ++i) {
        const ItemRec& it = items[i];
        const int nmax = rec_nmax[i];
        if (rec_nmax[n_items + i] == it.n_tab * nmax) continue;  // no spline table in this item
        const double* rM = item_rec + (int64_t)i * rec_stride + it.n_tab * nmax;
        for (int k = 0; k < it.n_tab; ++k)
          if (it.tab_species[k] == s) g += rM[k * nmax + j];
      }
      gM[j] = g;
    }
    __syncthreads();
  }
  if (tid != 0) return;
  if (S.interp == 1) spline_adjoint(S.n, S.qn, gM, work + n_f + S.f_off, work + 2 * n_f + S.f_off, grad_f + S.f_off);
  // extrapolation fits: (a, b) least-squares line of y_k = log(1/f_k + eta) against E_k, 5 end nodes
  const double a = st->a, m = st->m[s], eta = (double)S.stat;
  const double* f = f64 + S.f_off;
  for (int side = 0; side < 2; ++side) {
    const double dWa = dfa[2 * side], dWb = dfa[2 * side + 1];
    if (dWa == 0.0 && dWb == 0.0) continue;
    const int j0 = side == 0 ? 0 : S.n - 5;
    double E[5], Y[5], mE = 0.0, mY = 0.0;
    for (int k = 0; k < 5; ++k) {
      const double p = qnode[S.f_off + j0 + k] / a;
      E[k] = sqrt(p * p + m * m);
      Y[k] = log(1.0 / f[j0 + k] + eta);
      mE += E[k] / 5.0;
      mY += Y[k] / 5.0;
    }
    double sxx = 0.0, sxy = 0.0;
    for (int k = 0; k < 5; ++k) {
      sxx += (E[k] - mE) * (E[k] - mE);
      sxy += (E[k] - mE) * (Y[k] - mY);
    }
    const double bb = sxy / sxx;
    for (int k = 0; k < 5; ++k) {
      const double db_dy = (E[k] - mE) / sxx;
      const double da_dy = 1.0 / 5.0 - mE * db_dy;
      const double db_dE = ((Y[k] - mY) - 2.0 * bb * (E[k] - mE)) / sxx;
      const double da_dE = -db_dE * mE - bb / 5.0;
      const double fk = f[j0 + k];
      const double dy_df = -1.0 / (fk * (1.0 + eta * fk));
      grad_f[S.f_off + j0 + k] += (dWa * da_dy + dWb * db_dy) * dy_df;
      gm += (dWa * da_dE + dWb * db_dE) * m / E[k];
    }
  }
  grad_m[s] = gm;
}

// Persistent screening kernel (both precisions): block b takes the chunks b, b + G, b + 2G, ... of `chunk`
// consecutive tasks (the units of one item are consecutive, so a chunk mostly re-uses the staged map and tables).
// Which block runs a task does not change its result.  Registers are capped per lane so that at least three
// (screening) or two (second pass) waves share a SIMD: above 256 the compiler moves values into accumulation
// registers and occupancy halves.
template <int MASK>
__global__ __launch_bounds__(kBlock, 4) void k_screen(SampleLaunch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int chunk = L.chunk > 0 ? L.chunk : 1;
  int prev_item = -1;
  for (int base = blockIdx.x * chunk; base < L.n_tasks; base += gridDim.x * chunk) {
    const int end = min(base + chunk, L.n_tasks);
    for (int t = base; t < end;) {
      const int item = L.tasks[L.task_begin + t].item;
      int t1 = t + 1;
      while (t1 < end && L.tasks[L.task_begin + t1].item == item) ++t1;
      const int ni = L.items[item].nint;
      const bool stage = item != prev_item;
      prev_item = item;
      if (L.counts) {
        if ((MASK & 1) && ni == 1) screen_run<1, true>(L, t, t1, smem, stage);
        if ((MASK & 2) && ni == 2) screen_run<2, true>(L, t, t1, smem, stage);
        if ((MASK & 4) && ni == 3) screen_run<3, true>(L, t, t1, smem, stage);
        if ((MASK & 8) && ni == 4) screen_run<4, true>(L, t, t1, smem, stage);
      } else {
        if ((MASK & 1) && ni == 1) screen_run<1, false>(L, t, t1, smem, stage);
        if ((MASK & 2) && ni == 2) screen_run<2, false>(L, t, t1, smem, stage);
        if ((MASK & 4) && ni == 3) screen_run<3, false>(L, t, t1, smem, stage);
        if ((MASK & 8) && ni == 4) screen_run<4, false>(L, t, t1, smem, stage);
      }
      t = t1;
    }
  }
}

// Second pass: block b takes tile b mod sh_tiles of second-pass group b / sh_tiles (one group of units of one item;
// every group of the launch has its own blocks).  Four blocks per CU with the linear rule (its compact LDS layout and
// at most 128 VGPRs) for up to three integrated particles, three
// otherwise (four integrated particles need more than 40 KB of LDS, so a tighter register cap would buy nothing).
// Which block runs a group does not change its result.
template <int MASK, int PREC, bool ALT>
__global__ __launch_bounds__(kBlock, (!ALT && MASK != 15 && MASK != 8) ? 4 : 3) void k_shell(SampleLaunch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = blockIdx.x / L.sh_tiles, tile = blockIdx.x % L.sh_tiles;  // grid = n_sh x sh_tiles
  if (k >= L.n_sh) return;
  const int ni = L.items[L.sh_tasks[L.sh_begin + k].item].nint;
  if ((MASK & 1) && ni == 1) shell_run<1, PREC, ALT>(L, k, k + 1, tile, smem, true);
  if ((MASK & 2) && ni == 2) shell_run<2, PREC, ALT>(L, k, k + 1, tile, smem, true);
  if ((MASK & 4) && ni == 3) shell_run<3, PREC, ALT>(L, k, k + 1, tile, smem, true);
  if ((MASK & 8) && ni == 4) shell_run<4, PREC, ALT>(L, k, k + 1, tile, smem, true);
}

// ------------------------------------------------------------------------------------------------------
// Vegas map adaptation of one dimension (Lepage): bin averages d = h/c, (7,1)/(1,6,1)/(1,7)/8 smoothing,
// normalisation, damping ((1-d)/ln(1/d))^alpha, new edges at equal cumulative damped weight placed linearly
// inside the old bins; the outer edges stay.
// Damped weight of a bin whose smoothed, normalised average is dh.
__device__ __forceinline__ double damped(double dh, double alpha) {
  if (dh <= 0.0) return 0.0;
  if (dh >= 1.0) return 1.0;
  const double base = (1.0 - dh) / log(1.0 / dh);
  return alpha == 0.5 ? sqrt(base) : pow(base, alpha);
}

// Lane l's value of v (l the same for every lane).
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

__device__ void adapt_item_map(const ItemRec& it, const double* sh, const double* sc, double* maps);

__global__ __launch_bounds__(512) void k_reduce_adapt(const ItemRec* items, int item_begin, uint32_t* counts,
                                                      const double* shell_rec, double* res_I, double* res_V,
                                                      int slot, double* maps, int freeze, int plain) {
  __shared__ double sh[kMaxD * kMaxBins], sc[kMaxD * kMaxBins];
  const int item = item_begin + blockIdx.x;
  const ItemRec& it = items[item];
  if (slot >= it.n_iter || it.vplus) return;  // finished, or a VEGAS+ item (its own reduction)
  const int D = it.D, nb = it.nb, DN = D * nb;
  const int64_t stride = 2 + (int64_t)DN;  // second-pass record: S1, S2, the W^2 sums
  // this launch's records of the item, contiguous: its groups in order (units of su each), and in a batched launch
  // each group's kShellTiles tiles in order
  const int su = plain ? it.shell_units_p : it.shell_units;
  const int n_rec = (int)((it.n_units + su - 1) / su) * (plain ? 1 : kShellTiles);
  if (threadIdx.x == 0) {
    double S1 = 0.0, S2 = 0.0;
    for (int q = 0; q < n_rec; ++q) {
      const int64_t r = it.shell_off + q * stride;
      S1 += shell_rec[r];
      S2 += shell_rec[r + 1];
    }
    const double Nd = (double)it.N;
    const double I = S1 / Nd;
    const double V = (S2 / Nd - I * I) / (Nd - 1.0);
    res_I[it.res_off * kMaxIter + slot] = I;
    res_V[it.res_off * kMaxIter + slot] = V;
  }
  // the item's bin counts of this iteration (every sample, from the screening pass), cleared for the next one
  uint32_t* cnt = counts + it.part_off;
  if (freeze) {
    for (int i = threadIdx.x; i < DN; i += blockDim.x) cnt[i] = 0u;
    return;
  }
  for (int i = threadIdx.x; i < DN; i += blockDim.x) {
    const uint32_t cu = cnt[i];
    cnt[i] = 0u;
    double h = 0.0;
    for (int q = 0; q < n_rec; ++q) h += shell_rec[it.shell_off + q * stride + 2 + i];
    const double c = (double)cu;
    sh[i] = h;
    sc[i] = c;
  }
  __syncthreads();
  adapt_item_map(it, sh, sc, maps);
}

// Vegas adaptation of an item's map from its training sums sh (W^2) and sc (counts), D x nb in LDS.  One wave per
// dimension, lane j holding bin j (nb <= 64): averages, smoothing from the neighbours' lanes, the sums over the
// bins in bin order (lane by lane, the order of a sequential loop), damping, the running sums in bin order, and
// new edge k (lane k) in the first bin whose running sum reaches k wsum / nb, found by a binary search over the
// lanes' running sums.  Every value is the one a sequential pass over the bins computes.  No block barrier: with
// nw waves in the block, wave w takes dimensions d = w, w + nw, ... (k_reduce_adapt's 512 threads: w, w + 8, so
// D = 9 and D = 12 give waves 0 and 0..3 a second dimension; a 256-thread block: w, w + 4, w + 8).
__device__ void adapt_item_map(const ItemRec& it, const double* sh, const double* sc, double* maps) {
  const int D = it.D, nb = it.nb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
  for (int d = wave; d < D; d += nw) {
    const int j = lane < nb ? lane : nb - 1;  // lanes past the last bin repeat it and write nothing
    const int i = d * nb + j;
    const double a = sc[i] > 0.0 ? sh[i] / sc[i] : 0.0;  // bin average h / c
    const double am = __shfl(a, j > 0 ? j - 1 : 0), ap = __shfl(a, j < nb - 1 ? j + 1 : nb - 1);
    // (7,1)/(1,6,1)/(1,7)/8 smoothing
    const double w0 = j == 0 ? (7.0 * a + ap) / 8.0 : (j == nb - 1 ? (am + 7.0 * a) / 8.0 : (am + 6.0 * a + ap) / 8.0);
    double sum = 0.0;
    for (int k = 0; k < nb; ++k) sum += lane_value(w0, k);
    if (!(sum > 0.0)) continue;  // a dimension without weight keeps its edges
    // normalisation and damping
    const double w = damped(w0 / sum, it.alpha);
    double wsum = 0.0;
    for (int k = 0; k < nb; ++k) wsum += lane_value(w, k);
    if (!(wsum > 0.0)) continue;
    // running sums: lane j gets w_0 + ... + w_{j-1} (pre_lo) and that plus w_j (pre_hi)
    double acc = 0.0, pre_lo = 0.0, pre_hi = 0.0;
    for (int k = 0; k < nb; ++k) {
      if (lane == k) pre_lo = acc;
      acc += lane_value(w, k);
      if (lane == k) pre_hi = acc;
    }
    double* edges = maps + it.map_off + d * (nb + 1);
    const double old_lo = edges[j], old_hi = edges[j + 1];  // read by every lane before any lane writes
    // edge k = lane: its bin is the number of bins j <= nb-2 whose running sum pre_hi stays below the target
    const double per = wsum / (double)nb;
    const double target = per * (double)lane;
    int pos = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
      const int cand = pos + step;
      const double v = __shfl(pre_hi, cand - 1 < 63 ? cand - 1 : 63);
      if (cand <= nb - 1 && v < target) pos = cand;
    }
    const double vj = __shfl(w, pos), acc_j = __shfl(pre_lo, pos);
    const double e0 = __shfl(old_lo, pos), e1 = __shfl(old_hi, pos);
    double frac = vj > 0.0 ? (target - acc_j) / vj : 0.0;
    frac = frac > 1.0 ? 1.0 : (frac < 0.0 ? 0.0 : frac);
    if (lane >= 1 && lane < nb) edges[lane] = e0 + frac * (e1 - e0);  // the outer edges stay
  }
}

// ------------------------------------------------------------------------------------------------------
// VEGAS+ (adaptive stratified sampling on top of the map).  y-space is cut into M = k^D hypercubes, hypercube
// h = sum_d h_d k^d (dimension 0 fastest); iteration samples s = off_h + i, i < n_h, lie in hypercube h with
// y_d = (h_d + u_d) / k.  A block takes 256 consecutive hypercubes and walks their samples in chunks of 256, one
// sample per thread (every sample in full: the allocation puts samples where W is not zero); after each chunk the
// thread that owns a hypercube adds the chunk's W of that hypercube in sample order, so S1_h and S2_h are summed
// exactly as a sequential loop over i would, whatever the allocation.  The training histograms take
// (W N_it / (M n_h))^2 per sample in the per-wave LDS histograms, summed per block into the block's record.
constexpr int kVpLds = (kBlock + 1) * 8 + kBlock * 8;  // LDS beyond the sample layout: offsets and a chunk of W

template <int NI, int PREC, bool ALT>
__device__ void vplus_run(const SampleLaunch& L, const VpTask task, unsigned char* smem) {
  constexpr int D = 3 * NI;
  using FT = typename std::conditional<PREC == 0, double, float>::type;
  const ItemRec* __restrict__ it = &L.items[task.item];
  ItemConsts<NI, FT> K;
  const Lds lay = setup_block<NI, PREC>(L, it, smem, true, K);
  const int DN = D * it->nb, tid = threadIdx.x, wave = tid >> 6;
  double* my_h = reinterpret_cast<double*>(smem + lay.off_h) + wave * DN;
  uint32_t* my_c = reinterpret_cast<uint32_t*>(smem + lay.off_c) + wave * DN;
  int64_t* s_off = reinterpret_cast<int64_t*>(smem + align16(lay.total));  // kBlock + 1 offsets
  double* s_W = reinterpret_cast<double*>(s_off + kBlock + 1);
  const int h0 = task.b * kBlock, nhc = min(kBlock, it->vp_M - h0);
  for (int i = tid; i <= nhc; i += kBlock) s_off[i] = L.vp_hoff[it->vp_hb + h0 + i];
  __syncthreads();
  const int64_t n_it = L.vp_hoff[it->vp_hb + it->vp_M];
  const double Mw = (double)it->vp_M;
  const int64_t s_begin = s_off[0], s_end = s_off[nhc];
  double t1 = 0.0, t2 = 0.0;  // weighted sums (the record's S1, S2 fields; not used by the estimate)
  double s1 = 0.0, s2 = 0.0;  // the owned hypercube's sums
  for (int64_t cs = s_begin; cs < s_end; cs += kBlock) {
    const int64_t smp = cs + tid;
    if (smp < s_end) {
      int lo = 0, hi = nhc;  // the local hypercube: s_off[lo] <= smp < s_off[lo + 1]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (s_off[mid] <= smp) lo = mid;
        else hi = mid;
      }
      int dig[D];
      int rem = h0 + lo;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        dig[d] = rem % it->vp_k;
        rem /= it->vp_k;
      }
      const double wt = (double)n_it / (Mw * (double)(s_off[lo + 1] - s_off[lo]));
      int hj[D];
      const double W = eval_sample<NI, FT, ALT, true>(K, (uint64_t)smp, hj, dig, it->vp_k);
      accumulate<D>(W * wt, hj, t1, t2, my_h, my_c);
      s_W[tid] = W;
    }
    __syncthreads();
    if (tid < nhc) {
      const int64_t a = max(s_off[tid], cs), e = min(s_off[tid + 1], cs + kBlock);
      for (int64_t i = a; i < e; ++i) {
        const double w = s_W[i - cs];
        s1 += w;
        s2 += w * w;
      }
    }
    __syncthreads();
  }
  if (tid < nhc) {
    L.vp_S1[it->vp_off + h0 + tid] = s1;
    L.vp_S2[it->vp_off + h0 + tid] = s2;
  }
  double* rec = L.vp_rec + it->vp_rec + (int64_t)task.b * (2 + 2 * (int64_t)DN);
  finish_block<true>(t1, t2, lay, DN, smem, rec, rec + 2);
}

template <int MASK, int PREC, bool ALT>
__global__ __launch_bounds__(kBlock, 2) void k_vplus(SampleLaunch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  const VpTask task = L.vp_tasks[blockIdx.x];
  const int ni = L.items[task.item].nint;
  if ((MASK & 1) && ni == 1) vplus_run<1, PREC, ALT>(L, task, smem);
  if ((MASK & 2) && ni == 2) vplus_run<2, PREC, ALT>(L, task, smem);
  if ((MASK & 4) && ni == 3) vplus_run<3, PREC, ALT>(L, task, smem);
  if ((MASK & 8) && ni == 4) vplus_run<4, PREC, ALT>(L, task, smem);
}

// First iteration of a call: n_h = N / M, offsets h N / M.
__global__ void k_vplus_init(const ItemRec* items, const int* which, int* nh, int64_t* hoff) {
  const ItemRec& it = items[which[blockIdx.x]];
  const int64_t n0 = it.N / it.vp_M;
  for (int h = threadIdx.x; h <= it.vp_M; h += blockDim.x) {
    if (h < it.vp_M) nh[it.vp_off + h] = (int)n0;
    hoff[it.vp_hb + h] = (int64_t)h * n0;
  }
}

// Per item: I = (1/M) sum_h S1_h / n_h and V = sum_h (S2_h - S1_h^2 / n_h) / (n_h (n_h - 1)) / M^2 (thread-strided
// partial sums, then the fixed wave tree); unless frozen, the map adapted from the blocks' records (block order)
// and the next allocation: d_h = (max(0, (S2_h - S1_h^2 / n_h) / (n_h - 1)) / M^2)^(beta / 2),
// n_h = 2 + floor((N - 2 M) d_h / sum d) (N / M if sum d = 0), offsets by a block scan over contiguous chunks.
__global__ __launch_bounds__(256) void k_vplus_reduce(const ItemRec* items, const int* which, int* nh,
                                                      int64_t* hoff, double* S1, const double* S2, const double* rec,
                                                      double* res_I, double* res_V, int slot, double* maps,
                                                      int freeze) {
  __shared__ double sh[kMaxD * kMaxBins], sc[kMaxD * kMaxBins];
  __shared__ double red[2 * kWaves];
  __shared__ int64_t scan[256];
  const ItemRec& it = items[which[blockIdx.x]];
  if (slot >= it.n_iter) return;
  const int tid = threadIdx.x, M = it.vp_M, wave = tid >> 6;
  const double Md = (double)M;
  double pI = 0.0, pV = 0.0;
  for (int h = tid; h < M; h += 256) {
    const double n = (double)nh[it.vp_off + h], s1 = S1[it.vp_off + h], s2 = S2[it.vp_off + h];
    pI += s1 / n;
    pV += (s2 - s1 * s1 / n) / (n * (n - 1.0));
  }
  pI = wave_sum(pI);
  pV = wave_sum(pV);
  if ((tid & 63) == 0) {
    red[wave] = pI;
    red[kWaves + wave] = pV;
  }
  __syncthreads();
  if (tid == 0) {
    double I = 0.0, V = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      I += red[w];
      V += red[kWaves + w];
    }
    res_I[it.res_off * kMaxIter + slot] = I / Md;
    res_V[it.res_off * kMaxIter + slot] = V / (Md * Md);
  }
  if (freeze) return;
  // training sums over the blocks' records, in block order
  const int DN = it.D * it.nb;
  const int64_t stride = 2 + 2 * (int64_t)DN;
  for (int i = tid; i < DN; i += 256) {
    double hs = 0.0, cs = 0.0;
    for (int b = 0; b < it.vp_blocks; ++b) {
      hs += rec[it.vp_rec + b * stride + 2 + i];
      cs += rec[it.vp_rec + b * stride + 2 + DN + i];
    }
    sh[i] = hs;
    sc[i] = cs;
  }
  __syncthreads();
  adapt_item_map(it, sh, sc, maps);
  // allocation: d_h into S1 (each h by the thread that read it above), then the sum of d
  double pd = 0.0;
  for (int h = tid; h < M; h += 256) {
    const double n = (double)nh[it.vp_off + h], s1 = S1[it.vp_off + h], s2 = S2[it.vp_off + h];
    double v = (s2 - s1 * s1 / n) / (n - 1.0) / (Md * Md);
    v = v > 0.0 ? v : 0.0;
    const double d = pow(v, 0.5 * it.beta);
    S1[it.vp_off + h] = d;
    pd += d;
  }
  pd = wave_sum(pd);
  __syncthreads();
  if ((tid & 63) == 0) red[wave] = pd;
  __syncthreads();
  double sumd = 0.0;
  for (int w = 0; w < kWaves; ++w) sumd += red[w];
  // new n_h over contiguous chunks, then the exclusive scan of the chunk totals
  const int chunk = (M + 255) / 256, h0 = tid * chunk, h1 = min(M, h0 + chunk);
  const int64_t spare = it.N - 2 * (int64_t)M, n0 = it.N / M;
  int64_t tot = 0;
  for (int h = h0; h < h1; ++h) {
    const int64_t n = sumd > 0.0 ? 2 + (int64_t)floor((double)spare * S1[it.vp_off + h] / sumd) : n0;
    nh[it.vp_off + h] = (int)n;
    tot += n;
  }
  scan[tid] = tot;
  __syncthreads();
  if (tid == 0) {
    int64_t acc = 0;
    for (int t = 0; t < 256; ++t) {
      const int64_t v = scan[t];
      scan[t] = acc;
      acc += v;
    }
    hoff[it.vp_hb + M] = acc;
  }
  __syncthreads();
  int64_t acc = scan[tid];
  for (int h = h0; h < h1; ++h) {
    hoff[it.vp_hb + h] = acc;
    acc += nh[it.vp_off + h];
  }
}

// Uniform maps: edge j of dimension d at lo + (hi - lo) j / nb with (lo, hi) = species range of r, [0, pi]
// for theta, [0, 2 pi] for phi.
__global__ void k_init_maps(const ItemRec* items, const int* which, int n, const SpecDev* spec, double* maps) {
  const int k = blockIdx.x;
  if (k >= n) return;
  const ItemRec& it = items[which[k]];
  const int nb = it.nb;
  for (int i = threadIdx.x; i < it.D * (nb + 1); i += blockDim.x) {
    const int d = i / (nb + 1), j = i - d * (nb + 1);
    double lo, hi;
    const int c = d % 3;
    if (c == 0) {
      const SpecDev& S = spec[it.r_species[d / 3]];
      lo = S.q_min;
      hi = S.q_max;
    } else if (c == 1) {
      lo = 0.0;
      hi = kPi;
    } else {
      lo = 0.0;
      hi = kTwoPi;
    }
    maps[it.map_off + i] = lo + (hi - lo) * (double)j / (double)nb;
  }
}

__global__ void k_combine(const ItemRec* items, const double* res_I, const double* res_V, int n_iter,
                          double* item_Ibar, double* item_sig, const int* slot_begin, const int* slot_items,
                          int n_slots, double* slot_C, double* slot_S2) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_slots) return;
  double C = 0.0, S2 = 0.0;
  for (int e = slot_begin[k]; e < slot_begin[k + 1]; ++e) {
    const int i = slot_items[e];
    const ItemRec& it = items[i];
    const double* I = res_I + it.res_off * kMaxIter;
    const double* V = res_V + it.res_off * kMaxIter;
    double sw = 0.0, swI = 0.0;
    int npos = 0;
    const int nit = it.n_iter < n_iter ? it.n_iter : n_iter;
    for (int t = 0; t < nit; ++t) {
      if (V[t] > 0.0) {
        sw += 1.0 / V[t];
        swI += I[t] / V[t];
        ++npos;
      }
    }
    double Ib, sg;
    if (npos > 0) {
      Ib = swI / sw;
      sg = 1.0 / sqrt(sw);
    } else {
      double mm = 0.0;
      for (int t = 0; t < nit; ++t) mm += I[t];
      Ib = mm / (double)nit;
      sg = 0.0;
    }
    item_Ibar[i] = Ib;
    item_sig[i] = sg;
    C += (double)it.mult * (double)it.sign * Ib;
    S2 += (double)it.mult * (double)it.mult * sg * sg;
  }
  slot_C[k] = C;
  slot_S2[k] = S2;
}

// ------------------------------------------------------------------------------------------------------
// Exact-delta 2->2 (the two-dimensional reduction of the 2->2 collision integral with energy conservation exact).
// Angular kinematic function in closed form: with kappa = p1^2 + p3^2 and G = Q + 2 gamma of the term, the allowed
// u = 2 p1 p3 cos(theta) lie between -(G + 2 px^2) -+ 2 px sqrt(G + px^2 + kappa), cut to [-2 p1 p3, 2 p1 p3], and
// F = |M|^2 pi (sqrt(kappa - u_lo) - sqrt(kappa - u_hi)) / (2 p1 p3 px).
__device__ __forceinline__ double kinematic_F(double p1, double p3, double px, double G, double M2) {
  const double kappa = p1 * p1 + p3 * p3;
  const double disc = G + px * px + kappa;
  if (!(disc >= 0.0)) return 0.0;
  const double mid = -(G + 2.0 * px * px), half = 2.0 * px * sqrt(disc);
  const double U = 2.0 * p1 * p3;
  const double lo = fmax(-U, mid - half), hi = fmin(U, mid + half);
  if (!(hi > lo)) return 0.0;
  return M2 * 3.141592653589793 * (sqrt(kappa - lo) - sqrt(kappa - hi)) / (U * px);
}

// One block per item.  Roles of a 2->2 item: integrated 0 and 1 (the opposite side, "3" and "4"), conserved 2 (the
// observed leg's partner, "2"), observed 3 ("1").  The gain term integrates over p3, p4 on the grid nodes of their
// species (E2 = E3 + E4 - E1 fixed), the loss term over p2, p3 (E4 = E1 + E2 - E3 fixed); the trapezoidal rule in
// ln q, h q_j / a per node (half at the ends).  The dependent particle's f comes by the species' interpolation rule
// or the fit.  Pairs are taken by thread index mod 256, then summed by the fixed wave tree; the estimate goes to
// iteration 0 of the item's results with V = 0.
__global__ __launch_bounds__(kBlock) void k_exact22(const ItemRec* items, const SpecDev* spec, const double* f64,
                                                    const double* qnode, const DevState* st, double* res_I,
                                                    double* res_V) {
  __shared__ double red[2 * kWaves];
  const ItemRec& it = items[blockIdx.x];
  const int tid = threadIdx.x;
  const double a = st->a, inv_a = st->inv_a, M2 = it.coupling2;
  int sp[4];
  double m[4], eta[4];
  for (int r = 0; r < 4; ++r) {
    sp[r] = it.r_species[r];
    m[r] = st->m[sp[r]];
    eta[r] = (double)spec[sp[r]].stat;
  }
  // positions 1..4 of the reduction -> roles 3, 2, 0, 1
  const SpecDev &S1 = spec[sp[3]], &S2 = spec[sp[2]], &S3 = spec[sp[0]], &S4 = spec[sp[1]];
  const double m1 = m[3], m2 = m[2], m3 = m[0], m4 = m[1];
  const double e1 = eta[3], e2 = eta[2], e3 = eta[0], e4 = eta[1];
  const double p1 = it.q_obs * inv_a, E1 = sqrt(p1 * p1 + m1 * m1);
  const double f1 = it.obs_at ? f_at_global(S1, f64 + S1.f_off, qnode + S1.f_off, st->fit[sp[3]], it.q_obs, E1)
                              : f64[S1.f_off + it.eval_idx];
  const bool want_gain = it.net || it.term == 0, want_loss = it.net || it.term == 1;
  double gain = 0.0, loss = 0.0;
  if (want_gain) {
    const int n3 = S3.n, n4 = S4.n;
    const double w3h = 1.0 / S3.inv_h * inv_a, w4h = 1.0 / S4.inv_h * inv_a;
    for (int idx = tid; idx < n3 * n4; idx += kBlock) {
      const int j3 = idx / n4, j4 = idx - j3 * n4;
      const double q3 = qnode[S3.f_off + j3], q4 = qnode[S4.f_off + j4];
      const double p3 = q3 * inv_a, p4 = q4 * inv_a;
      const double E3 = sqrt(p3 * p3 + m3 * m3), E4 = sqrt(p4 * p4 + m4 * m4);
      const double E2 = E3 + E4 - E1;
      if (!(E2 >= m2)) continue;
      const double p2 = sqrt(E2 * E2 - m2 * m2);
      const double f2 = f_at_global(S2, f64 + S2.f_off, qnode + S2.f_off, st->fit[sp[2]], a * p2, E2);
      const double G = m1 * m1 - m2 * m2 + m3 * m3 + m4 * m4 + 2.0 * (E3 * E4 - E1 * E3 - E1 * E4);
      const double F = kinematic_F(p1, p3, p4, G, M2);
      const double t3 = (j3 == 0 || j3 == n3 - 1) ? 0.5 : 1.0, t4 = (j4 == 0 || j4 == n4 - 1) ? 0.5 : 1.0;
      const double f3 = f64[S3.f_off + j3], f4 = f64[S4.f_off + j4];
      gain += (t3 * w3h * q3) * (t4 * w4h * q4) * (p3 * p3 / (2.0 * E3)) * (p4 * p4 / (2.0 * E4)) * F *
              (f3 * f4 * (1.0 + e1 * f1) * (1.0 + e2 * f2));
    }
  }
  if (want_loss) {
    const int n2 = S2.n, n3 = S3.n;
    const double w2h = 1.0 / S2.inv_h * inv_a, w3h = 1.0 / S3.inv_h * inv_a;
    for (int idx = tid; idx < n2 * n3; idx += kBlock) {
      const int j2 = idx / n3, j3 = idx - j2 * n3;
      const double q2 = qnode[S2.f_off + j2], q3 = qnode[S3.f_off + j3];
      const double p2 = q2 * inv_a, p3 = q3 * inv_a;
      const double E2 = sqrt(p2 * p2 + m2 * m2), E3 = sqrt(p3 * p3 + m3 * m3);
      const double E4 = E1 + E2 - E3;
      if (!(E4 >= m4)) continue;
      const double p4 = sqrt(E4 * E4 - m4 * m4);
      const double f4 = f_at_global(S4, f64 + S4.f_off, qnode + S4.f_off, st->fit[sp[1]], a * p4, E4);
      const double G = m1 * m1 + m2 * m2 + m3 * m3 - m4 * m4 + 2.0 * (E1 * E2 - E1 * E3 - E2 * E3);
      const double F = kinematic_F(p1, p3, p2, G, M2);
      const double t2 = (j2 == 0 || j2 == n2 - 1) ? 0.5 : 1.0, t3 = (j3 == 0 || j3 == n3 - 1) ? 0.5 : 1.0;
      const double f2 = f64[S2.f_off + j2], f3 = f64[S3.f_off + j3];
      loss += (t2 * w2h * q2) * (t3 * w3h * q3) * (p2 * p2 / (2.0 * E2)) * (p3 * p3 / (2.0 * E3)) * F *
              (f1 * f2 * (1.0 + e3 * f3) * (1.0 + e4 * f4));
    }
  }
  gain = wave_sum(gain);
  loss = wave_sum(loss);
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    red[wave] = gain;
    red[kWaves + wave] = loss;
  }
  __syncthreads();
  if (tid == 0) {
    double g = 0.0, l = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      g += red[w];
      l += red[kWaves + w];
    }
    const double pref = 2.0 / (1558.5454565440386 * 2.0 * E1);  // 2 / ((2 pi)^4 2 E1)
    const double I = pref * (it.net ? g - l : (it.term == 0 ? g : l));
    res_I[it.res_off * kMaxIter] = I;
    res_V[it.res_off * kMaxIter] = 0.0;
  }
}

// One thread per process; the sums run over the items in plan order (the same order as the evaluation's item
// results), so the decision depends on the results alone.
__global__ void k_width_control(const ItemRec* items, int n_items, const double* item_Ibar, const double* item_sig,
                                const WidthCtl* ctl, int n_proc, DevState* st) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_proc) return;
  const WidthCtl c = ctl[p];
  if (!c.adapt) return;
  double se = 0.0, si = 0.0;
  int n = 0;
  for (int i = 0; i < n_items; ++i) {
    if (items[i].proc != p) continue;
    se += item_sig[i];
    si += fabs(item_Ibar[i]);
    ++n;
  }
  if (n == 0 || !(si > 0.0)) return;
  const double r = se / si;
  double w = st->width[p];
  if (r < c.lo) w /= c.factor;
  else if (r > c.hi) w *= c.factor;
  w = w < c.wmin ? c.wmin : w;
  w = w > c.wmax ? c.wmax : w;
  st->width[p] = w;
}

__global__ void k_gather(const GatherEntry* ge, int n_out, const GatherProc* gp, const double* slot_C,
                         const double* slot_S2, const SpecDev* spec, const double* f64, double* C_out,
                         double* sig_out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  const GatherEntry g = ge[o];
  const SpecDev& S = spec[g.species];
  const double* f = f64 + S.f_off;
  const double h = (log(S.q_max) - S.lq0) / (double)(S.n - 1);
  double C = 0.0, V = 0.0;
  for (int e = g.first; e < g.first + g.count; ++e) {
    const GatherProc P = gp[e];
    double c, s;
    const int j = g.node;
    if (!P.fill || j % P.stride == 0) {
      const int k = P.slot_base + j / P.stride;
      c = slot_C[k];
      s = sqrt(slot_S2[k]);
    } else if (j > P.last) {
      const int k = P.slot_base + P.last / P.stride;
      c = slot_C[k] / f[P.last] * f[j];
      s = sqrt(slot_S2[k]) / f[P.last] * f[j];
    } else {
      const int i0 = (j / P.stride) * P.stride, i1 = i0 + P.stride;
      const int k0 = P.slot_base + i0 / P.stride;
      const double l0 = log(exp(S.lq0 + h * (double)i0)), l1 = log(exp(S.lq0 + h * (double)i1));
      const double lj = log(exp(S.lq0 + h * (double)j));
      const double u = (lj - l0) / (l1 - l0);
      const double c0 = slot_C[k0], c1 = slot_C[k0 + 1];
      const double s0 = sqrt(slot_S2[k0]), s1 = sqrt(slot_S2[k0 + 1]);
      c = c0 + u * (c1 - c0);
      s = s0 + u * (s1 - s0);
    }
    C += c;
    V += s * s;
  }
  C_out[o] = C;
  if (sig_out) sig_out[o] = sqrt(V);
}

// a(t), masses, extrapolation fits and the FP32 copy of f.  One block.
// Not-a-knot cubic spline through (q_j, f_j) on the logarithmic grid q_j = exp(lq0 + h j): second derivatives M_j.
// With h_j = q_{j+1} - q_j, continuity of S' at the interior nodes gives
//   h_{j-1}/6 M_{j-1} + (h_{j-1} + h_j)/3 M_j + h_j/6 M_{j+1} = (f_{j+1} - f_j)/h_j - (f_j - f_{j-1})/h_{j-1};
// a continuous third derivative at q_1 and q_{n-2} gives M_0 = (1 + h_0/h_1) M_1 - (h_0/h_1) M_2 and its mirror at
// the upper end, which fold into the first and last interior rows.  The tridiagonal system in M_1 .. M_{n-2} is
// diagonally dominant on a grid of growing spacing and is solved by forward elimination and back substitution
// (one thread; c holds the eliminated upper diagonal).
__device__ void spline_second_derivatives(int n, const double* qn, const double* f, double* M, double* c) {
  auto hs = [&](int j) { return qn[j + 1] - qn[j]; };
  double prev_c = 0.0, prev_d = 0.0;
  double hl = hs(0), hr = hs(1);
  for (int j = 1; j <= n - 2; ++j) {
    double lo = hl / 6.0, di = (hl + hr) / 3.0, up = hr / 6.0;
    const double rhs = (f[j + 1] - f[j]) / hr - (f[j] - f[j - 1]) / hl;
    if (j == 1) {  // M_0 folded in
      const double r0 = hl / hr;
      di += lo * (1.0 + r0);
      up -= lo * r0;
      lo = 0.0;
    }
    if (j == n - 2) {  // M_{n-1} folded in
      const double r1 = hr / hl;
      di += up * (1.0 + r1);
      lo -= up * r1;
      up = 0.0;
    }
    const double den = di - lo * prev_c;
    prev_c = up / den;
    prev_d = (rhs - lo * prev_d) / den;
    c[j] = prev_c;
    M[j] = prev_d;
    hl = hr;
    if (j + 2 <= n - 1) hr = hs(j + 1);
  }
  for (int j = n - 3; j >= 1; --j) M[j] -= c[j] * M[j + 1];
  const double h0 = hs(0), h1 = hs(1), ha = hs(n - 3), hb = hs(n - 2);
  M[0] = (1.0 + h0 / h1) * M[1] - (h0 / h1) * M[2];
  M[n - 1] = (1.0 + hb / ha) * M[n - 2] - (hb / ha) * M[n - 3];
}

__global__ void k_prepare(DevState* st, const SpecDev* spec, int n_species, const double* f64, float* f32,
                          int64_t n_f) {
  const double t = st->t;
  if (threadIdx.x == 0) {
    const double a = st->expansion == 1 ? st->expansion_a0 * sqrt(t / st->expansion_t0) : 1.0;
    st->a = a;
    st->inv_a = 1.0 / a;
    for (int n = 0; n < 5; ++n) st->a_m3n[n] = pow(a, -3.0 * (double)n);
  }
  __syncthreads();
  const double a = st->a;
  for (int64_t i = threadIdx.x; i < n_f; i += blockDim.x) f32[i] = (float)f64[i];
  if ((int)threadIdx.x < n_species) {
    const int s = threadIdx.x;
    const SpecDev& S = spec[s];
    const double m = S.mass_kind == 1 ? S.m0 + S.A * sin(S.w * t) : S.m0;
    st->m[s] = m;
    const double* f = f64 + S.f_off;
    const double eta = (double)S.stat;
    const double h = (log(S.q_max) - S.lq0) / (double)(S.n - 1);
    int bad = 0;
    for (int j = 0; j < S.n; ++j) {
      if (!(f[j] > 0.0) || !isfinite(f[j])) bad = 1;
      if (S.stat == -1 && !(f[j] < 1.0)) bad = 1;
    }
    double fit[4];
    for (int side = 0; side < 2 && !bad; ++side) {
      const int j0 = side == 0 ? 0 : S.n - 5;
      double E[5], Y[5], sE = 0.0, sY = 0.0;
      for (int k = 0; k < 5; ++k) {
        const double p = exp(S.lq0 + h * (double)(j0 + k)) / a;
        E[k] = sqrt(p * p + m * m);
        Y[k] = log(1.0 / f[j0 + k] + eta);
        sE += E[k];
        sY += Y[k];
      }
      const double mE = sE / 5.0, mY = sY / 5.0;
      double sxy = 0.0, sxx = 0.0;
      for (int k = 0; k < 5; ++k) {
        sxy += (E[k] - mE) * (Y[k] - mY);
        sxx += (E[k] - mE) * (E[k] - mE);
      }
      const double b = sxy / sxx, aa = mY - b * mE;
      if (!isfinite(b) || !isfinite(aa)) bad = 1;
      fit[2 * side] = aa;
      fit[2 * side + 1] = b;
    }
    if (!bad && !(fit[3] > 0.0)) bad = 1;
    if (!bad && S.stat == 1) {
      const double p0 = exp(S.lq0) / a, pN = exp(S.lq0 + h * (double)(S.n - 1)) / a;
      const double E0 = sqrt(p0 * p0 + m * m), EN = sqrt(pN * pN + m * m);
      if (!(fit[0] + fit[1] * m > 0.0) || !(fit[0] + fit[1] * E0 > 0.0) || !(fit[2] + fit[3] * EN > 0.0)) bad = 1;
    }
    if (bad) {
      atomicMax(&st->err, 3);
    } else {
      for (int k = 0; k < 4; ++k) st->fit[s][k] = fit[k];
    }
    if (S.interp == 1) spline_second_derivatives(S.n, S.qn, f, S.aux, S.tmp);
  }
  __syncthreads();
  // equilibrium-exact rule: node energies E_j = sqrt((q_j / a)^2 + m^2) and y_j = log(1/f_j + eta)
  for (int s = 0; s < n_species; ++s) {
    const SpecDev& S = spec[s];
    if (S.interp != 2) continue;
    const double m = st->m[s], eta = (double)S.stat;
    for (int j = threadIdx.x; j < S.n; j += blockDim.x) {
      const double p = S.qn[j] / a;
      S.aux[j] = sqrt(p * p + m * m);
      S.tmp[j] = log(1.0 / f64[S.f_off + j] + eta);
    }
  }
}

__global__ void k_set_eval(DevState* st, double t, uint32_t epoch, int set_t) {
  if (set_t) st->t = t;
  st->next_epoch = epoch;
}

// Start of an evaluation: consume the next epoch.
__global__ void k_next_epoch(DevState* st) {
  st->epoch = st->next_epoch;
  st->next_epoch = st->next_epoch + 1u;
}

__global__ void k_step_begin(DevState* st, double* f, double* f0, const double* k1, int64_t n, double dt_fixed,
                             double eps, double dt_max, int heun) {
  __shared__ double red[1024];
  double r = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) r = fmax(r, fabs(k1[i] / f[i]));
  red[threadIdx.x] = r;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  const double rmax = red[0];
  double h = dt_fixed;
  if (!(h > 0.0)) {
    h = rmax > 0.0 ? eps / rmax : dt_max;
    if (h > dt_max) h = dt_max;
  }
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double fv = f[i];
    f0[i] = fv;
    f[i] = exp(log(fv) + h * k1[i] / fv);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->rmax = rmax;
    st->dt = h;
    st->t_step0 = st->t;
    st->t = st->t + h;
    (void)heun;
  }
}

__global__ void k_step_finish(DevState* st, double* f, const double* f0, const double* fstar, const double* k1,
                              const double* k2, int64_t n) {
  const double h = st->dt;
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    f[i] = exp(log(f0[i]) + 0.5 * h * (k1[i] / f0[i] + k2[i] / fstar[i]));
  }
}

__global__ void k_copy(double* dst, const double* src, int64_t n) {
  for (int64_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

template <int MASK>
hipError_t launch_sample_t(const SampleLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_screen<MASK>), dim3(L.grid), dim3(kBlock), screen_layout().total, s, L);
  return hipGetLastError();
}

template <int MASK>
hipError_t launch_shell_t(const SampleLaunch& L, hipStream_t s) {
  const dim3 g(L.sh_grid), b(kBlock);
  if (L.any_interp) {
    if (L.precision == 0) hipLaunchKernelGGL((k_shell<MASK, 0, true>), g, b, L.shell_lds, s, L);
    else hipLaunchKernelGGL((k_shell<MASK, 1, true>), g, b, L.shell_lds, s, L);
  } else {
    if (L.precision == 0) hipLaunchKernelGGL((k_shell<MASK, 0, false>), g, b, L.shell_lds, s, L);
    else hipLaunchKernelGGL((k_shell<MASK, 1, false>), g, b, L.shell_lds, s, L);
  }
  return hipGetLastError();
}

template <int MASK>
hipError_t launch_vplus_t(const SampleLaunch& L, hipStream_t s) {
  const dim3 g(L.n_vp), b(kBlock);
  const size_t lds = align16((int)L.lds_bytes) + kVpLds;
  if (L.any_interp) {
    if (L.precision == 0) hipLaunchKernelGGL((k_vplus<MASK, 0, true>), g, b, lds, s, L);
    else hipLaunchKernelGGL((k_vplus<MASK, 1, true>), g, b, lds, s, L);
  } else {
    if (L.precision == 0) hipLaunchKernelGGL((k_vplus<MASK, 0, false>), g, b, lds, s, L);
    else hipLaunchKernelGGL((k_vplus<MASK, 1, false>), g, b, lds, s, L);
  }
  return hipGetLastError();
}

}  // namespace

int sample_lds_bytes(int D, int nb, int n_tab, int n_max, int precision) {
  return lds_layout(D, nb, n_tab, n_max, precision == 0 ? 8 : 4).total;
}

int screen_lds_bytes() { return screen_layout().total; }
int shell_lds_bytes(int D, int nb, int n_tab, int n_max, int precision, int alt) {
  return shell_layout(D, nb, n_tab, n_max, precision == 0 ? 8 : 4, alt != 0).total;
}

hipError_t launch_sample(const SampleLaunch& L, hipStream_t s) {
  if (L.n_tasks <= 0) return hipSuccess;
  switch (L.nint_mask) {
    case 1: return launch_sample_t<1>(L, s);
    case 2: return launch_sample_t<2>(L, s);
    case 4: return launch_sample_t<4>(L, s);
    case 8: return launch_sample_t<8>(L, s);
    default: return launch_sample_t<15>(L, s);
  }
}

hipError_t launch_vplus(const SampleLaunch& L, hipStream_t s) {
  if (L.n_vp <= 0) return hipSuccess;
  switch (L.nint_mask) {
    case 1: return launch_vplus_t<1>(L, s);
    case 2: return launch_vplus_t<2>(L, s);
    case 4: return launch_vplus_t<4>(L, s);
    case 8: return launch_vplus_t<8>(L, s);
    default: return launch_vplus_t<15>(L, s);
  }
}

hipError_t launch_shell(const SampleLaunch& L, hipStream_t s) {
  if (L.n_sh <= 0) return hipSuccess;
  switch (L.nint_mask) {
    case 1: return launch_shell_t<1>(L, s);
    case 2: return launch_shell_t<2>(L, s);
    case 4: return launch_shell_t<4>(L, s);
    case 8: return launch_shell_t<8>(L, s);
    default: return launch_shell_t<15>(L, s);
  }
}

template <int MASK>
void launch_vjp_mask(const SampleLaunch& L, hipStream_t s) {
  if (L.any_interp) hipLaunchKernelGGL((k_vjp<MASK, true>), dim3(L.grid), dim3(kBlock), L.lds_bytes, s, L);
  else hipLaunchKernelGGL((k_vjp<MASK, false>), dim3(L.grid), dim3(kBlock), L.lds_bytes, s, L);
}

hipError_t launch_vjp(const SampleLaunch& L, hipStream_t s) {
  if (L.n_sh <= 0) return hipSuccess;
  switch (L.nint_mask) {
    case 1: launch_vjp_mask<1>(L, s); break;
    case 2: launch_vjp_mask<2>(L, s); break;
    case 4: launch_vjp_mask<4>(L, s); break;
    case 8: launch_vjp_mask<8>(L, s); break;
    default:  // several particle counts: one launch per count (each skips the other counts' groups)
      if (L.nint_mask & 1) launch_vjp_mask<1>(L, s);
      if (L.nint_mask & 2) launch_vjp_mask<2>(L, s);
      if (L.nint_mask & 4) launch_vjp_mask<4>(L, s);
      if (L.nint_mask & 8) launch_vjp_mask<8>(L, s);
      break;
  }
  return hipGetLastError();
}

int vjp_lds_bytes(int D, int nb, int n_tab, int n_max, int spl) {
  int o = 0;
  o = align16(o + D * nb * 8);
  o = align16(o + D * nb * 8);
  o = align16(o + 33 * 16);
  o = align16(o + n_tab * align16(n_max * 24));
  o = align16(o + kWaves * vjp_tab_len(n_tab, n_max, spl) * 8);
  o = align16(o + (1 + 4 + kMaxN + 1) * kWaves * 8);
  return o;
}

int vjp_record_len(int n_tab, int n_max, int spl) { return vjp_rec_len(n_tab, n_max, spl); }

hipError_t launch_vjp_finish(const ItemRec* items, int n_items, const double* coef, const double* parts,
                             const int* rec_len, const int* rec_nmax, double* item_rec, int rec_stride,
                             const SpecDev* spec, int n_species, const double* f64, const double* qnode,
                             const DevState* st, double* grad_f, int64_t n_f, double* work, double* grad_m,
                             double* grad_lam, const double* coupling, int n_proc, hipStream_t s) {
  hipLaunchKernelGGL(k_vjp_reduce, dim3(n_items), dim3(256), 0, s, items, n_items, coef, parts, rec_len, item_rec,
                     rec_stride);
  hipLaunchKernelGGL(k_vjp_gather, dim3((unsigned)std::min<int64_t>(n_f, 65535)), dim3(256), 0, s, items, n_items,
                     item_rec, rec_nmax, rec_stride, spec, n_species, f64, grad_f, n_f);
  hipLaunchKernelGGL(k_vjp_finish, dim3(n_species + n_proc), dim3(256), 0, s, items, n_items, item_rec, rec_nmax,
                     rec_stride, spec, n_species, f64, qnode, st, grad_f, n_f, work, grad_m, grad_lam, coupling,
                     n_proc);
  return hipGetLastError();
}

hipError_t launch_reduce_adapt(const ItemRec* items, int item_begin, int n_items, uint32_t* counts,
                               const double* shell_rec, double* res_I, double* res_V, int slot, double* maps,
                               int freeze, int plain, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_adapt, dim3(n_items), dim3(512), 0, s, items, item_begin, counts, shell_rec, res_I,
                     res_V, slot, maps, freeze, plain);
  return hipGetLastError();
}

hipError_t launch_init_maps(const ItemRec* items, const int* which, int n, const SpecDev* spec, double* maps,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_maps, dim3(n), dim3(256), 0, s, items, which, n, spec, maps);
  return hipGetLastError();
}

hipError_t launch_combine(const ItemRec* items, int n_items, const double* res_I, const double* res_V, int n_iter,
                          double* item_Ibar, double* item_sig, const int* slot_begin, const int* slot_items,
                          int n_slots, double* slot_C, double* slot_S2, hipStream_t s) {
  (void)n_items;
  if (n_slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3((n_slots + 255) / 256), dim3(256), 0, s, items, res_I, res_V, n_iter, item_Ibar,
                     item_sig, slot_begin, slot_items, n_slots, slot_C, slot_S2);
  return hipGetLastError();
}

hipError_t launch_exact22(const ItemRec* items, int n_items, const SpecDev* spec, const double* f64,
                          const double* qnode, const DevState* st, double* res_I, double* res_V, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_exact22, dim3(n_items), dim3(kBlock), 0, s, items, spec, f64, qnode, st, res_I, res_V);
  return hipGetLastError();
}

hipError_t launch_vplus_init(const ItemRec* items, const int* which, int n, int* nh, int64_t* hoff, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vplus_init, dim3(n), dim3(256), 0, s, items, which, nh, hoff);
  return hipGetLastError();
}

hipError_t launch_vplus_reduce(const ItemRec* items, const int* which, int n, int* nh, int64_t* hoff,
                               const double* S1, const double* S2, const double* rec, double* res_I, double* res_V,
                               int slot, double* maps, int freeze, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vplus_reduce, dim3(n), dim3(256), 0, s, items, which, nh, hoff, const_cast<double*>(S1), S2,
                     rec, res_I, res_V, slot, maps, freeze);
  return hipGetLastError();
}

hipError_t launch_width_control(const ItemRec* items, int n_items, const double* item_Ibar, const double* item_sig,
                                const WidthCtl* ctl, int n_proc, DevState* st, hipStream_t s) {
  if (n_proc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_width_control, dim3((n_proc + 63) / 64), dim3(64), 0, s, items, n_items, item_Ibar, item_sig,
                     ctl, n_proc, st);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherEntry* ge, int n_out, const GatherProc* gp, const double* slot_C,
                         const double* slot_S2, const SpecDev* spec, const double* f64, double* C_out,
                         double* sig_out, hipStream_t s) {
  if (n_out <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather, dim3((n_out + 255) / 256), dim3(256), 0, s, ge, n_out, gp, slot_C, slot_S2, spec, f64,
                     C_out, sig_out);
  return hipGetLastError();
}

hipError_t launch_prepare(DevState* st, const SpecDev* spec, int n_species, const double* f64, float* f32,
                          int64_t n_f, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(1), dim3(256), 0, s, st, spec, n_species, f64, f32, n_f);
  return hipGetLastError();
}

hipError_t launch_set_eval(DevState* st, double t, uint32_t epoch, int set_t, hipStream_t s) {
  hipLaunchKernelGGL(k_set_eval, dim3(1), dim3(1), 0, s, st, t, epoch, set_t);
  return hipGetLastError();
}

hipError_t launch_next_epoch(DevState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_next_epoch, dim3(1), dim3(1), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_step_begin(DevState* st, double* f64, double* f0, const double* k1, int64_t n_f, double dt_fixed,
                             double eps, double dt_max, int heun, hipStream_t s) {
  hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1024), 0, s, st, f64, f0, k1, n_f, dt_fixed, eps, dt_max, heun);
  return hipGetLastError();
}

hipError_t launch_step_finish(DevState* st, double* f64, const double* f0, const double* fstar, const double* k1,
                              const double* k2, int64_t n_f, hipStream_t s) {
  hipLaunchKernelGGL(k_step_finish, dim3(8), dim3(256), 0, s, st, f64, f0, fstar, k1, k2, n_f);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, dim3(8), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

}  // namespace bmc
