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
// One block of 256 threads processes one unit (a contiguous range of sample indices) of one item.  Sums are
// formed in a fixed order that depends only on the unit size: per thread in sample order, a butterfly over
// the wave, the four waves in order, then the units in order (reduce kernel).  The Vegas training
// histograms are accumulated per wave in LDS and summed over waves in order.
#include <math.h>

#include "kernels.h"
#include "philox.h"

namespace bmc {

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;
constexpr double kHistWMin = 0x1p-400;  // |W| below this enters the training histogram as 0

struct Lds {
  int off_e, off_w, off_f, off_h, off_c, off_red, total;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline Lds lds_layout(int D, int nb, int n_tab, int n_max, int fbytes) {
  Lds L;
  int DN = D * nb;
  int o = 0;
  L.off_e = o;
  o = align16(o + DN * 8);
  L.off_w = o;
  o = align16(o + DN * 8);
  L.off_f = o;
  o = align16(o + n_tab * n_max * fbytes);
  L.off_h = o;
  o = align16(o + kWaves * DN * 8);
  L.off_c = o;
  o = align16(o + kWaves * DN * 4);
  L.off_red = o;
  o = align16(o + 2 * kWaves * 8);
  L.total = o;
  return L;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// f at a comoving momentum inside the grid: linear in ln q between the bracketing nodes (FP64).
__device__ __forceinline__ double interp64(const double* tab, int n, double lq0, double inv_h, double q) {
  double t = (log(q) - lq0) * inv_h;
  int j = (int)floor(t);
  j = j < 0 ? 0 : (j > n - 2 ? n - 2 : j);
  double w = t - (double)j;
  double f0 = tab[j], f1 = tab[j + 1];
  return f0 + w * (f1 - f0);
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

__device__ __forceinline__ float interp32(const float* tab, int n, float lq0, float inv_h, double q) {
  float t = (__logf((float)q) - lq0) * inv_h;
  int j = (int)floorf(t);
  j = j < 0 ? 0 : (j > n - 2 ? n - 2 : j);
  float w = t - (float)j;
  float f0 = tab[j], f1 = tab[j + 1];
  return fmaf(w, f1 - f0, f0);
}

template <int NI, int PREC>
__device__ void sample_task(const SampleLaunch& L, const Task task, unsigned char* smem) {
  // FP64 expressions are evaluated as written (no fused multiply-add contraction), like the reference
#pragma clang fp contract(off)
  constexpr int D = 3 * NI;
  constexpr int B = (D + 3) / 4;
  constexpr int NR = NI + 2;  // roles: integrated 0..NI-1, conserved NI, observed NI+1
  const ItemRec* __restrict__ it = &L.items[task.item];
  const int tid = threadIdx.x;
  const int nb = it->nb;
  const int DN = D * nb;
  const int n_tab = it->n_tab;
  int n_max = 0;
  for (int k = 0; k < n_tab; ++k) n_max = max(n_max, L.spec[it->tab_species[k]].n);
  const Lds lay = lds_layout(D, nb, n_tab, n_max, PREC == 0 ? 8 : 4);
  double* sm_e = reinterpret_cast<double*>(smem + lay.off_e);
  double* sm_w = reinterpret_cast<double*>(smem + lay.off_w);
  double* sm_h = reinterpret_cast<double*>(smem + lay.off_h);
  uint32_t* sm_c = reinterpret_cast<uint32_t*>(smem + lay.off_c);
  double* sm_red = reinterpret_cast<double*>(smem + lay.off_red);

  // ---- stage the map, the f tables and clear the histograms ----
  const double* __restrict__ map = L.maps + it->map_off;
  for (int i = tid; i < DN; i += kBlock) {
    int d = i / nb, j = i - d * nb;
    double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
    sm_e[i] = e0;
    sm_w[i] = e1 - e0;
  }
  for (int k = 0; k < n_tab; ++k) {
    const SpecDev& S = L.spec[it->tab_species[k]];
    if (PREC == 0) {
      double* dst = reinterpret_cast<double*>(smem + lay.off_f) + k * n_max;
      for (int j = tid; j < S.n; j += kBlock) dst[j] = L.f64[S.f_off + j];
    } else {
      float* dst = reinterpret_cast<float*>(smem + lay.off_f) + k * n_max;
      for (int j = tid; j < S.n; j += kBlock) dst[j] = L.f32[S.f_off + j];
    }
  }
  for (int i = tid; i < kWaves * DN; i += kBlock) {
    sm_h[i] = 0.0;
    sm_c[i] = 0u;
  }

  // ---- per-item constants at the current time ----
  const DevState* __restrict__ st = L.st;
  const double a = st->a;
  const double inv_a = 1.0 / a;
  double m[NR], eta[NR];
  int tabslot[NR], obsside[NR], isin[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    m[r] = st->m[it->r_species[r]];
    eta[r] = (double)L.spec[it->r_species[r]].stat;
    tabslot[r] = it->r_tab[r];
    obsside[r] = it->r_obsside[r];
    isin[r] = it->r_in[r];
  }
  const SpecDev& So = L.spec[it->obs_species];
  const double q_obs = it->q_obs;
  const double p_obs = q_obs * inv_a;
  const double E_obs = sqrt(p_obs * p_obs + m[NI + 1] * m[NI + 1]);
  const double f_obs = L.f64[So.f_off + it->eval_idx];
  const double a3 = pow(a, -3.0 * (double)NI);
  const double M2 = it->coupling2;
  const double e_cut = it->e_cut;
  // conserved particle: its species' table and fit
  const SpecDev& Sc = L.spec[it->r_species[NI]];
  const double fit_lo_a = st->fit[it->r_species[NI]][0], fit_lo_b = st->fit[it->r_species[NI]][1];
  const double fit_hi_a = st->fit[it->r_species[NI]][2], fit_hi_b = st->fit[it->r_species[NI]][3];
  const double cons_sign = it->cons_in ? -1.0 : 1.0;  // p_cons = s * (sum_in - sum_out) over the others
  const uint32_t uid = it->uid;
  const uint32_t c3 = st->epoch * 64u + (uint32_t)L.it;
  const int64_t N = it->N;
  const int64_t n0 = (int64_t)task.unit * it->unit_size;
  const int64_t n1 = min(n0 + (int64_t)it->unit_size, N);
  const double dnb = (double)nb;
  const int wave = tid >> 6;
  double* my_h = sm_h + wave * DN;
  uint32_t* my_c = sm_c + wave * DN;
  __syncthreads();

  double S1 = 0.0, S2 = 0.0;
  for (int64_t n = n0 + tid; n < n1; n += kBlock) {
    // ---- uniforms ----
    double y[4 * B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const uint64_t off = (uint64_t)n * (uint64_t)B + (uint64_t)b;
      Philox4 r = philox4x32_10((uint32_t)off, (uint32_t)(off >> 32), uid, c3, L.seed_lo, L.seed_hi);
#pragma unroll
      for (int s = 0; s < 4; ++s) y[4 * b + s] = ((double)r.v[s] + 0.5) * 2.3283064365386962890625e-10;
    }
    // ---- Vegas map ----
    double x[D];
    int jb[D];
    double J = 1.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      double yn = y[d] * dnb;
      int j = (int)yn;
      j = j > nb - 1 ? nb - 1 : j;
      double del = yn - (double)j;
      double e0 = sm_e[d * nb + j], w = sm_w[d * nb + j];
      x[d] = e0 + w * del;
      J *= dnb * w;
      jb[d] = j;
    }
    // ---- momenta ----
    double px[NR], py[NR], pz[NR], E[NR];
    double jac = 1.0;
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      double r = x[3 * k], th = x[3 * k + 1], ph = x[3 * k + 2];
      double p = r * inv_a;
      double sth, cth, sph, cph;
      sincos(th, &sth, &cth);
      sincos(ph, &sph, &cph);
      px[k] = p * sth * cph;
      py[k] = p * sth * sph;
      pz[k] = p * cth;
      jac *= r * r * sth;
      E[k] = sqrt(p * p + m[k] * m[k]);
    }
    px[NI + 1] = 0.0;
    py[NI + 1] = 0.0;
    pz[NI + 1] = p_obs;
    E[NI + 1] = E_obs;
    {
      double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (r == NI) continue;
        double sg = isin[r] ? 1.0 : -1.0;
        sx += sg * px[r];
        sy += sg * py[r];
        sz += sg * pz[r];
      }
      px[NI] = cons_sign * sx;
      py[NI] = cons_sign * sy;
      pz[NI] = cons_sign * sz;
    }
    const double P2 = px[NI] * px[NI] + py[NI] * py[NI] + pz[NI] * pz[NI];
    E[NI] = sqrt(P2 + m[NI] * m[NI]);
    bool cut = false;
    double dE = 0.0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      cut |= E[r] < e_cut;
      dE += isin[r] ? E[r] : -E[r];
    }
    const double q_cons = a * sqrt(P2);
    double W;
    if (PREC == 0) {
      const double delta = exp(-dE * dE * it->inv2s2) * it->dnorm;
      double f[NR];
#pragma unroll
      for (int r = 0; r < NI; ++r) {
        const SpecDev& S = L.spec[it->r_species[r]];
        const double* tab = reinterpret_cast<const double*>(smem + lay.off_f) + tabslot[r] * n_max;
        f[r] = interp64(tab, S.n, S.lq0, S.inv_h, x[3 * r]);
      }
      if (q_cons < Sc.q_min) {
        f[NI] = 1.0 / (exp(fit_lo_a + fit_lo_b * E[NI]) - eta[NI]);
      } else if (q_cons > Sc.q_max) {
        f[NI] = 1.0 / (exp(fit_hi_a + fit_hi_b * E[NI]) - eta[NI]);
      } else {
        const double* tab = reinterpret_cast<const double*>(smem + lay.off_f) + tabslot[NI] * n_max;
        f[NI] = interp64(tab, Sc.n, Sc.lq0, Sc.inv_h, q_cons);
      }
      f[NI + 1] = f_obs;
      double gain = 1.0, loss = 1.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        double bf = 1.0 + eta[r] * f[r];
        gain *= obsside[r] ? bf : f[r];
        loss *= obsside[r] ? f[r] : bf;
      }
      const double F = it->net ? gain - loss : (it->term == 0 ? gain : loss);
      double prod2E = 1.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) prod2E *= 2.0 * E[r];
      W = J * (jac * a3 * M2 * delta / (it->twopi_pow * prod2E) * F);
    } else {
      const float delta = exp_split(-dE * dE * it->inv2s2) * (float)it->dnorm;
      float f[NR];
#pragma unroll
      for (int r = 0; r < NI; ++r) {
        const SpecDev& S = L.spec[it->r_species[r]];
        const float* tab = reinterpret_cast<const float*>(smem + lay.off_f) + tabslot[r] * n_max;
        f[r] = interp32(tab, S.n, (float)S.lq0, (float)S.inv_h, x[3 * r]);
      }
      if (q_cons < Sc.q_min) {
        f[NI] = __builtin_amdgcn_rcpf(exp_split(fit_lo_a + fit_lo_b * E[NI]) - (float)eta[NI]);
      } else if (q_cons > Sc.q_max) {
        f[NI] = __builtin_amdgcn_rcpf(exp_split(fit_hi_a + fit_hi_b * E[NI]) - (float)eta[NI]);
      } else {
        const float* tab = reinterpret_cast<const float*>(smem + lay.off_f) + tabslot[NI] * n_max;
        f[NI] = interp32(tab, Sc.n, (float)Sc.lq0, (float)Sc.inv_h, q_cons);
      }
      f[NI + 1] = (float)f_obs;
      float gain = 1.0f, loss = 1.0f;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        float bf = fmaf((float)eta[r], f[r], 1.0f);
        gain *= obsside[r] ? bf : f[r];
        loss *= obsside[r] ? f[r] : bf;
      }
      const float F = it->net ? gain - loss : (it->term == 0 ? gain : loss);
      double prod2E = 1.0;
#pragma unroll
      for (int r = 0; r < NR; ++r) prod2E *= 2.0 * E[r];
      const float rcp = __builtin_amdgcn_rcpf((float)prod2E);
      W = J * jac * (a3 * M2 / it->twopi_pow) * ((double)delta * (double)rcp) * (double)F;
    }
    if (cut) W = 0.0;
    S1 += W;
    S2 += W * W;
    const double w2 = fabs(W) >= kHistWMin ? W * W : 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      atomicAdd(&my_h[d * nb + jb[d]], w2);
      atomicAdd(&my_c[d * nb + jb[d]], 1u);
    }
  }

  // ---- fixed-order reductions ----
  S1 = wave_sum(S1);
  S2 = wave_sum(S2);
  if ((tid & 63) == 0) {
    sm_red[2 * wave] = S1;
    sm_red[2 * wave + 1] = S2;
  }
  __syncthreads();
  const int64_t gu = L.unit_base[task.item] + task.unit;
  if (tid == 0) {
    double s1 = 0.0, s2 = 0.0;
    for (int w = 0; w < kWaves; ++w) {
      s1 += sm_red[2 * w];
      s2 += sm_red[2 * w + 1];
    }
    L.unit_s[2 * gu] = s1;
    L.unit_s[2 * gu + 1] = s2;
  }
  double* rec = L.parts + it->part_off + (int64_t)task.unit * 2 * DN;
  for (int i = tid; i < DN; i += kBlock) {
    double h = 0.0;
    uint32_t c = 0;
    for (int w = 0; w < kWaves; ++w) {
      h += sm_h[w * DN + i];
      c += sm_c[w * DN + i];
    }
    rec[i] = h;
    rec[DN + i] = (double)c;
  }
  __syncthreads();
}

template <int MASK, int PREC>
__global__ __launch_bounds__(kBlock) void k_sample(SampleLaunch L) {
  extern __shared__ __align__(16) unsigned char smem[];
  for (int t = blockIdx.x; t < L.n_tasks; t += gridDim.x) {
    const Task task = L.tasks[L.task_begin + t];
    const int ni = L.items[task.item].nint;
    if ((MASK & 1) && ni == 1) sample_task<1, PREC>(L, task, smem);
    if ((MASK & 2) && ni == 2) sample_task<2, PREC>(L, task, smem);
    if ((MASK & 4) && ni == 3) sample_task<3, PREC>(L, task, smem);
    if ((MASK & 8) && ni == 4) sample_task<4, PREC>(L, task, smem);
  }
}

// ------------------------------------------------------------------------------------------------------
// Vegas map adaptation of one dimension (Lepage): bin averages d = h/c, (7,1)/(1,6,1)/(1,7)/8 smoothing,
// normalisation, damping ((1-d)/ln(1/d))^alpha, new edges at equal cumulative damped weight placed linearly
// inside the old bins; the outer edges stay.
__device__ void adapt_dimension(double* edges, int nb, const double* h, const double* c, double alpha, double* d,
                                double* wgt, double* old) {
  for (int j = 0; j < nb; ++j) d[j] = c[j] > 0.0 ? h[j] / c[j] : 0.0;
  double sum = 0.0;
  // smoothed values go into wgt
  wgt[0] = (7.0 * d[0] + d[1]) / 8.0;
  wgt[nb - 1] = (d[nb - 2] + 7.0 * d[nb - 1]) / 8.0;
  for (int j = 1; j < nb - 1; ++j) wgt[j] = (d[j - 1] + 6.0 * d[j] + d[j + 1]) / 8.0;
  for (int j = 0; j < nb; ++j) sum += wgt[j];
  if (!(sum > 0.0)) return;
  double wsum = 0.0;
  for (int j = 0; j < nb; ++j) {
    double dh = wgt[j] / sum;
    double v;
    if (dh <= 0.0) {
      v = 0.0;
    } else if (dh >= 1.0) {
      v = 1.0;
    } else {
      double base = (1.0 - dh) / log(1.0 / dh);
      v = alpha == 0.5 ? sqrt(base) : pow(base, alpha);
    }
    wgt[j] = v;
    wsum += v;
  }
  if (!(wsum > 0.0)) return;
  for (int j = 0; j <= nb; ++j) old[j] = edges[j];
  const double per = wsum / (double)nb;
  int j = 0;
  double acc = 0.0;
  for (int k = 1; k < nb; ++k) {
    const double target = per * (double)k;
    while (j < nb - 1 && acc + wgt[j] < target) {
      acc += wgt[j];
      ++j;
    }
    double frac = wgt[j] > 0.0 ? (target - acc) / wgt[j] : 0.0;
    frac = frac > 1.0 ? 1.0 : (frac < 0.0 ? 0.0 : frac);
    edges[k] = old[j] + frac * (old[j + 1] - old[j]);
  }
}

__global__ __launch_bounds__(256) void k_reduce_adapt(const ItemRec* items, int item_begin, const double* unit_s,
                                                      const int64_t* unit_base, const double* parts, double* res_I,
                                                      double* res_V, int slot, double* maps, int freeze) {
  __shared__ double sh[kMaxD * kMaxBins], sc[kMaxD * kMaxBins];
  __shared__ double s_d[kMaxD][kMaxBins], s_w[kMaxD][kMaxBins], s_old[kMaxD][kMaxBins + 1];
  const int item = item_begin + blockIdx.x;
  const ItemRec& it = items[item];
  if (slot >= it.n_iter) return;  // the item has finished its iterations
  const int D = it.D, nb = it.nb, DN = D * nb;
  const int64_t u0 = unit_base[item];
  if (threadIdx.x == 0) {
    double S1 = 0.0, S2 = 0.0;
    for (int u = 0; u < it.n_units; ++u) {
      S1 += unit_s[2 * (u0 + u)];
      S2 += unit_s[2 * (u0 + u) + 1];
    }
    const double Nd = (double)it.N;
    const double I = S1 / Nd;
    const double V = (S2 / Nd - I * I) / (Nd - 1.0);
    res_I[it.res_off * kMaxIter + slot] = I;
    res_V[it.res_off * kMaxIter + slot] = V;
  }
  if (freeze) return;
  const double* rec = parts + it.part_off;
  for (int i = threadIdx.x; i < DN; i += blockDim.x) {
    double h = 0.0, c = 0.0;
    for (int u = 0; u < it.n_units; ++u) {
      h += rec[(int64_t)u * 2 * DN + i];
      c += rec[(int64_t)u * 2 * DN + DN + i];
    }
    sh[i] = h;
    sc[i] = c;
  }
  __syncthreads();
  if (threadIdx.x < D) {
    const int d = threadIdx.x;
    adapt_dimension(maps + it.map_off + d * (nb + 1), nb, sh + d * nb, sc + d * nb, it.alpha, s_d[d], s_w[d],
                    s_old[d]);
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
__global__ void k_prepare(DevState* st, const SpecDev* spec, int n_species, const double* f64, float* f32,
                          int64_t n_f) {
  const double t = st->t;
  if (threadIdx.x == 0) {
    st->a = st->expansion == 1 ? st->expansion_a0 * sqrt(t / st->expansion_t0) : 1.0;
  }
  __syncthreads();
  const double a = st->a;
  for (int64_t i = threadIdx.x; i < n_f; i += blockDim.x) f32[i] = (float)f64[i];
  if (threadIdx.x < n_species) {
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

template <int MASK, int PREC>
hipError_t launch_sample_t(const SampleLaunch& L, hipStream_t s) {
  hipLaunchKernelGGL((k_sample<MASK, PREC>), dim3(L.grid), dim3(kBlock), L.lds_bytes, s, L);
  return hipGetLastError();
}

}  // namespace

int sample_lds_bytes(int D, int nb, int n_tab, int n_max, int precision) {
  return lds_layout(D, nb, n_tab, n_max, precision == 0 ? 8 : 4).total;
}

hipError_t launch_sample(const SampleLaunch& L, hipStream_t s) {
  if (L.n_tasks <= 0) return hipSuccess;
  const int m = L.nint_mask;
  if (L.precision == 0) {
    switch (m) {
      case 1: return launch_sample_t<1, 0>(L, s);
      case 2: return launch_sample_t<2, 0>(L, s);
      case 4: return launch_sample_t<4, 0>(L, s);
      case 8: return launch_sample_t<8, 0>(L, s);
      default: return launch_sample_t<15, 0>(L, s);
    }
  }
  switch (m) {
    case 1: return launch_sample_t<1, 1>(L, s);
    case 2: return launch_sample_t<2, 1>(L, s);
    case 4: return launch_sample_t<4, 1>(L, s);
    case 8: return launch_sample_t<8, 1>(L, s);
    default: return launch_sample_t<15, 1>(L, s);
  }
}

hipError_t launch_reduce_adapt(const ItemRec* items, int item_begin, int n_items, const double* unit_s,
                               const int64_t* unit_base, const double* parts, double* res_I, double* res_V,
                               int slot, double* maps, int freeze, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_adapt, dim3(n_items), dim3(256), 0, s, items, item_begin, unit_s, unit_base, parts,
                     res_I, res_V, slot, maps, freeze);
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
