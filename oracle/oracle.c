/*
 * oracle.c -- plain, slow CPU FP64 reference of the Monte-Carlo collision-integral estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this file; only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark do.  It shares no code, header,
 * table or constant generator with the HIP implementation.
 *
 * What it computes (paper: "Boltzmann Equation Solver for Thermalization", arXiv 2603.28848):
 *   * the single-position collision integral C^(k)(p) = (1/2E) Int dPi |M|^2 Lambda     (Sec. II.B, Eqs. 3-5)
 *   * the identical-particle decomposition C_a = n_alpha^a C_{n_alpha} + n_beta^a C_{n_beta}, and the
 *     self-reverse rule C_a = n_alpha^a C_{n_alpha}                                     (Sec. II.C, Eqs. 7, 12)
 *   * the Monte-Carlo parametrisation: observed momentum on z, integrated particles in spherical
 *     coordinates, one momentum fixed by momentum conservation, a Gaussian energy delta, the
 *     phase-space weight                                         (Sec. II.D, Eqs. 14-16; Appendix A)
 *   * Vegas adaptive importance sampling (Lepage 1978, 2021), separate gain and loss integrators,
 *     alpha = 0.5                                                         (Sec. II.D; Appendix C)
 *   * interpolation of f and its extrapolation log(1/f + eta) = a + b E              (Sec. III.B, Eq. 17)
 *   * log-space Euler / Heun stepping with the adaptive time step                   (Sec. III.C, Eqs. 18-20)
 *   * comoving momenta and radiation-domination expansion                            (Sec. III.E)
 *
 * Every floating-point quantity is IEEE double; Monte-Carlo sums are accumulated in long double so that
 * the oracle's sums are (to ~1e-19 relative per term) the exact sums of its per-sample doubles.
 * Parallelism: OpenMP over work items only; each item's samples are processed serially in index order.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double TWO_PI = 6.283185307179586476925286766559;
static const double PI_D = 3.141592653589793238462643383279;

/* =====================================================================================================
 * Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
 * as 1, 2, 3", SC11, 2011).  One round: two 32x32->64 products of counter words 0 and 2 with the
 * multipliers 0xD2511F53 and 0xCD9E8D57; the high halves are xored with the other counter words and
 * the key, the low halves move into the odd slots.  The key is bumped by the Weyl constants
 * (0x9E3779B9, 0xBB67AE85) between rounds.  Ten rounds.
 * ===================================================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
    uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The D uniforms of sample n of iteration `it` of the item with identifier `uid`.  The iteration's words form
 * one stream: stream word k is output (k mod 4) of the Philox block with counter (lo32(k/4), hi32(k/4), uid,
 * epoch*64+it) and key (lo32(seed), hi32(seed)).  Sample n takes stream words D*n .. D*n + D-1, and word d of
 * the sample becomes y_d = (word + 0.5) 2^-32.  Each word is generated on its own, block by block. */
void orc_sample_uniforms(uint64_t seed, uint32_t uid, uint32_t epoch, int it, int64_t n, int D, double* y) {
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int d = 0; d < D; ++d) {
    uint64_t k = (uint64_t)n * (uint64_t)D + (uint64_t)d;
    uint64_t blk = k / 4;
    uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), uid, epoch * 64u + (uint32_t)it};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    y[d] = ((double)w[k % 4] + 0.5) * 2.3283064365386962890625e-10; /* 2^-32 */
  }
}

/* =====================================================================================================
 * Species: momentum grid, mass, statistics, distribution table.
 * ===================================================================================================== */

/* Comoving grid node j of a logarithmic grid on [q_min, q_max] with n nodes. */
double orc_grid_q(const orc_species* s, int j) {
  double lq0 = log(s->q_min);
  double h = (log(s->q_max) - lq0) / (double)(s->n_grid - 1);
  return exp(lq0 + h * (double)j);
}

/* Mass at time t: constant, or m0 + A sin(w t). */
double orc_mass(const orc_species* s, double t) {
  if (s->mass_kind == ORC_MASS_SIN) return s->m0 + s->mA * sin(s->mw * t);
  return s->m0;
}

/* Scale factor: 1 without expansion; radiation domination a(t) = a0 (t/t0)^(1/2)  (Sec. III.E). */
double orc_scale_factor(const orc_world* w, double t) {
  if (w->expansion == ORC_EXP_RADIATION) return w->a0 * sqrt(t / w->t0);
  return 1.0;
}

/* Extrapolation fit (Eq. 17): least-squares line y = a + b E through the points
 * (E_j, log(1/f_j + eta)), E_j = sqrt((q_j/a)^2 + m^2), over the ORC_NFIT lowest and the ORC_NFIT
 * highest grid nodes separately.  fit[0..3] = (a_lo, b_lo, a_hi, b_hi).
 * Returns ORC_ERANGE if a node value is not positive, a Fermi-Dirac value is >= 1, the fit is not
 * finite, the high-end slope is not positive, or (Bose-Einstein) the fitted exponent is not positive
 * at an end of the range where it is used. */
int orc_fit(const orc_species* s, double a, double t, double fit[4]) {
  const int n = s->n_grid;
  const double m = orc_mass(s, t);
  const double eta = (double)s->stat;
  if (n < 2 * ORC_NFIT) return ORC_EINVAL;
  for (int side = 0; side < 2; ++side) {
    int j0 = side == 0 ? 0 : n - ORC_NFIT;
    double sE = 0, sY = 0;
    double E[ORC_NFIT], Y[ORC_NFIT];
    for (int k = 0; k < ORC_NFIT; ++k) {
      int j = j0 + k;
      double f = s->f[j];
      if (!(f > 0.0)) return ORC_ERANGE;
      if (s->stat == ORC_FERMI && !(f < 1.0)) return ORC_ERANGE;
      double p = orc_grid_q(s, j) / a;
      E[k] = sqrt(p * p + m * m);
      Y[k] = log(1.0 / f + eta);
      sE += E[k];
      sY += Y[k];
    }
    double mE = sE / ORC_NFIT, mY = sY / ORC_NFIT;
    double sxy = 0, sxx = 0;
    for (int k = 0; k < ORC_NFIT; ++k) {
      sxy += (E[k] - mE) * (Y[k] - mY);
      sxx += (E[k] - mE) * (E[k] - mE);
    }
    double b = sxy / sxx;
    double aa = mY - b * mE;
    if (!isfinite(b) || !isfinite(aa)) return ORC_ERANGE;
    fit[2 * side] = aa;
    fit[2 * side + 1] = b;
  }
  if (!(fit[3] > 0.0)) return ORC_ERANGE;
  if (s->interp == ORC_INTERP_SPLINE || s->interp == ORC_INTERP_EQEXACT) {
    if (!s->aux) return ORC_EINVAL;
    if (s->interp == ORC_INTERP_EQEXACT) {
      for (int j = 0; j < n; ++j) {
        double p = orc_grid_q(s, j) / a;
        s->aux[j] = sqrt(p * p + m * m);
      }
    } else {
      double* q = (double*)malloc(sizeof(double) * (size_t)n);
      if (!q) return ORC_ENOMEM;
      for (int j = 0; j < n; ++j) q[j] = orc_grid_q(s, j);
      int rc = orc_spline_second_derivatives(n, q, s->f, s->aux);
      free(q);
      if (rc) return rc;
    }
  }
  if (s->stat == ORC_BOSE) {
    double p0 = orc_grid_q(s, 0) / a, pN = orc_grid_q(s, n - 1) / a;
    double E0 = sqrt(p0 * p0 + m * m), EN = sqrt(pN * pN + m * m);
    if (!(fit[0] + fit[1] * m > 0.0) || !(fit[0] + fit[1] * E0 > 0.0)) return ORC_ERANGE;
    if (!(fit[2] + fit[3] * EN > 0.0)) return ORC_ERANGE;
  }
  return ORC_OK;
}

/* Second derivatives of the not-a-knot cubic spline through (q_j, f_j), j = 0..n-1, n >= 4 (Sec. III.B: a cubic
 * spline in linear scale; not-a-knot ends are the usual default).  On [q_j, q_{j+1}], h_j = q_{j+1} - q_j, the
 * spline is A f_j + B f_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h_j^2 / 6 with B = (q - q_j) / h_j, A = 1 - B.
 * Conditions: S' continuous at q_1 .. q_{n-2} (rows 1 .. n-2); the third derivative continuous at q_1 (row 0) and
 * at q_{n-2} (row n-1).  The n x n system is solved by Gaussian elimination with partial pivoting. */
/* The matrix K of the spline conditions (row stride ld): K M = r(f), where r_j is the jump of the secant slopes at
 * interior node j and r_0 = r_{n-1} = 0 (the not-a-knot rows). */
static void spline_matrix(int n, const double* q, double* A, size_t ld) {
#define KE(r, c) A[(size_t)(r) * ld + (size_t)(c)]
  for (int j = 1; j < n - 1; ++j) {
    const double hl = q[j] - q[j - 1], hr = q[j + 1] - q[j];
    KE(j, j - 1) = hl / 6.0;
    KE(j, j) = (hl + hr) / 3.0;
    KE(j, j + 1) = hr / 6.0;
  }
  const double h0 = q[1] - q[0], h1 = q[2] - q[1];
  KE(0, 0) = -1.0 / h0;
  KE(0, 1) = 1.0 / h0 + 1.0 / h1;
  KE(0, 2) = -1.0 / h1;
  const double ha = q[n - 2] - q[n - 3], hb = q[n - 1] - q[n - 2];
  KE(n - 1, n - 3) = -1.0 / ha;
  KE(n - 1, n - 2) = 1.0 / ha + 1.0 / hb;
  KE(n - 1, n - 1) = -1.0 / hb;
#undef KE
}

/* Solves the n x n system whose augmented rows (n + 1 doubles each: the matrix row, then the right-hand side) are in
 * A, by Gaussian elimination with partial pivoting; A is overwritten. */
static int dense_solve(int n, double* A, double* x) {
#define AE(r, c) A[(size_t)(r) * (size_t)(n + 1) + (size_t)(c)]
  for (int col = 0; col < n; ++col) {
    int piv = col;
    for (int r = col + 1; r < n; ++r)
      if (fabs(AE(r, col)) > fabs(AE(piv, col))) piv = r;
    if (AE(piv, col) == 0.0) return ORC_ERANGE;
    if (piv != col)
      for (int c = 0; c <= n; ++c) {
        double tmp = AE(col, c);
        AE(col, c) = AE(piv, c);
        AE(piv, c) = tmp;
      }
    for (int r = col + 1; r < n; ++r) {
      const double fac = AE(r, col) / AE(col, col);
      if (fac == 0.0) continue;
      for (int c = col; c <= n; ++c) AE(r, c) -= fac * AE(col, c);
    }
  }
  for (int r = n - 1; r >= 0; --r) {
    double acc = AE(r, n);
    for (int c = r + 1; c < n; ++c) acc -= AE(r, c) * x[c];
    x[r] = acc / AE(r, r);
  }
#undef AE
  return ORC_OK;
}

int orc_spline_second_derivatives(int n, const double* q, const double* f, double* M) {
  if (n < 4) return ORC_EINVAL;
  double* A = (double*)calloc((size_t)n * (size_t)(n + 1), sizeof(double));  /* augmented rows of n + 1 */
  if (!A) return ORC_ENOMEM;
  spline_matrix(n, q, A, (size_t)(n + 1));
#define AE(r, c) A[(size_t)(r) * (size_t)(n + 1) + (size_t)(c)]
  for (int j = 1; j < n - 1; ++j) {
    const double hl = q[j] - q[j - 1], hr = q[j + 1] - q[j];
    AE(j, n) = (f[j + 1] - f[j]) / hr - (f[j] - f[j - 1]) / hl;
  }
#undef AE
  int rc = dense_solve(n, A, M);
  free(A);
  return rc;
}

/* Adjoint of the spline's second derivatives: given g_j = dL/dM_j, adds dL/df_j = sum_k g_k dM_k/df_j to gf.
 * M = K^-1 r(f) with r linear in f, so dL/df = r'^T z with K^T z = g; r_j = (f_{j+1} - f_j)/h_j - (f_j - f_{j-1})/h_{j-1}
 * sends z_j to f_{j+1} (1/h_j), f_j (-1/h_j - 1/h_{j-1}) and f_{j-1} (1/h_{j-1}). */
int orc_spline_adjoint(int n, const double* q, const double* g, double* gf) {
  if (n < 4) return ORC_EINVAL;
  double* K = (double*)calloc((size_t)n * (size_t)n, sizeof(double));
  double* A = (double*)calloc((size_t)n * (size_t)(n + 1), sizeof(double));
  double* z = (double*)malloc(sizeof(double) * (size_t)n);
  if (!K || !A || !z) {
    free(K); free(A); free(z);
    return ORC_ENOMEM;
  }
  spline_matrix(n, q, K, (size_t)n);
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) A[(size_t)r * (size_t)(n + 1) + (size_t)c] = K[(size_t)c * (size_t)n + (size_t)r];
    A[(size_t)r * (size_t)(n + 1) + (size_t)n] = g[r];
  }
  int rc = dense_solve(n, A, z);
  if (rc == ORC_OK)
    for (int j = 1; j < n - 1; ++j) {
      const double hl = q[j] - q[j - 1], hr = q[j + 1] - q[j];
      gf[j + 1] += z[j] / hr;
      gf[j] -= z[j] * (1.0 / hr + 1.0 / hl);
      gf[j - 1] += z[j] / hl;
    }
  free(K); free(A); free(z);
  return rc;
}

/* f at comoving momentum q with physical energy E (Sec. III.B):
 *   inside [q_0, q_{N-1}], on the segment [q_j, q_{j+1}] of the logarithmic grid that holds q:
 *     LINLOG   linear in ln q between f_j and f_{j+1};
 *     SPLINE   the not-a-knot cubic spline in linear q (second derivatives in s->aux);
 *     EQEXACT  y = log(1/f + eta) linear in E between (E_j, y_j) and (E_{j+1}, y_{j+1}) (E_j in s->aux),
 *              f = 1 / (exp(y) - eta);
 *   below / above: f = 1 / (exp(a + b E) - eta) with the low / high fit. */
double orc_f_at(const orc_species* s, const double fit[4], double q, double E) {
  const int n = s->n_grid;
  const double eta = (double)s->stat;
  if (q < s->q_min) return 1.0 / (exp(fit[0] + fit[1] * E) - eta);
  if (q > s->q_max) return 1.0 / (exp(fit[2] + fit[3] * E) - eta);
  double lq0 = log(s->q_min);
  double h = (log(s->q_max) - lq0) / (double)(n - 1);
  double tpos = (log(q) - lq0) / h;
  int j = (int)floor(tpos);
  if (j < 0) j = 0;
  if (j > n - 2) j = n - 2;
  if (s->interp == ORC_INTERP_SPLINE) {
    const double q0 = orc_grid_q(s, j), q1 = orc_grid_q(s, j + 1), hq = q1 - q0;
    const double B = (q - q0) / hq, A = 1.0 - B;
    return A * s->f[j] + B * s->f[j + 1] +
           ((A * A * A - A) * s->aux[j] + (B * B * B - B) * s->aux[j + 1]) * hq * hq / 6.0;
  }
  if (s->interp == ORC_INTERP_EQEXACT) {
    const double y0 = log(1.0 / s->f[j] + eta), y1 = log(1.0 / s->f[j + 1] + eta);
    const double w = (E - s->aux[j]) / (s->aux[j + 1] - s->aux[j]);
    return 1.0 / (exp(y0 + w * (y1 - y0)) - eta);
  }
  double w = tpos - (double)j;
  return s->f[j] + w * (s->f[j + 1] - s->f[j]);
}

/* f at n points (q[i], E[i]) -- the same rule as orc_f_at. */
void orc_f_batch(const orc_species* s, const double fit[4], int64_t n, const double* q, const double* E, double* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = orc_f_at(s, fit, q[i], E[i]);
}

/* =====================================================================================================
 * Roles (Sec. II.C; Appendix A "Particle roles").
 * ===================================================================================================== */

static int is_self_reverse(const orc_process* P) {
  if (P->n_in != P->n_out) return 0;
  int a[ORC_MAXN], b[ORC_MAXN];
  for (int i = 0; i < P->n_in; ++i) a[i] = P->sp[i];
  for (int i = 0; i < P->n_out; ++i) b[i] = P->sp[P->n_in + i];
  /* insertion sort both lists */
  for (int i = 1; i < P->n_in; ++i)
    for (int k = i; k > 0 && a[k] < a[k - 1]; --k) { int t = a[k]; a[k] = a[k - 1]; a[k - 1] = t; }
  for (int i = 1; i < P->n_out; ++i)
    for (int k = i; k > 0 && b[k] < b[k - 1]; --k) { int t = b[k]; b[k] = b[k - 1]; b[k - 1] = t; }
  for (int i = 0; i < P->n_in; ++i)
    if (a[i] != b[i]) return 0;
  return 1;
}

/* Number of times species a occupies side `side` (0 = initial state, 1 = final state). */
static int side_count(const orc_process* P, int a, int side) {
  int lo = side == 0 ? 0 : P->n_in, hi = side == 0 ? P->n_in : P->n_in + P->n_out, c = 0;
  for (int i = lo; i < hi; ++i) c += (P->sp[i] == a);
  return c;
}

/* Multiplicity with which the side-`side` evaluation of species a enters C_a (Eq. 7; Eq. 12 for
 * self-reverse processes under the automatic side selection).  0 means the side is not evaluated. */
int orc_side_multiplicity(const orc_process* P, int a, int side) {
  int n_s = side_count(P, a, side);
  if (n_s == 0) return 0;
  int mask = P->side_mask;
  if (mask == ORC_SIDES_AUTO) {
    if (is_self_reverse(P) && side == 1) return 0;
    return n_s;
  }
  if (!(mask & (1 << side))) return 0;
  return n_s;
}

/* Observed, conserved and integrated particle indices for species a pinned to side `side`. */
int orc_roles(const orc_process* P, int a, int side, int* i_obs, int* i_cons, int* integ) {
  const int n_in = P->n_in, n = P->n_in + P->n_out;
  int lo = side == 0 ? 0 : n_in, hi = side == 0 ? n_in : n;
  int obs = -1;
  for (int i = lo; i < hi; ++i)
    if (P->sp[i] == a) { obs = i; break; }
  if (obs < 0) return ORC_EINVAL;
  /* side that receives the conserved particle */
  int cside;
  if (P->n_in != P->n_out) cside = P->n_in < P->n_out ? 0 : 1; /* fewer-particle side */
  else cside = side;                                           /* same side as the observed one */
  int cons = -1;
  {
    int l = cside == 0 ? 0 : n_in, h = cside == 0 ? n_in : n;
    for (int i = l; i < h; ++i)
      if (i != obs) { cons = i; break; }
  }
  if (cons < 0) { /* fallback: lowest index on the opposite side */
    int os = 1 - cside;
    int l = os == 0 ? 0 : n_in, h = os == 0 ? n_in : n;
    for (int i = l; i < h; ++i)
      if (i != obs) { cons = i; break; }
  }
  if (cons < 0) return ORC_EINVAL;
  int k = 0;
  for (int i = 0; i < n; ++i)
    if (i != obs && i != cons) integ[k++] = i;
  *i_obs = obs;
  *i_cons = cons;
  return ORC_OK;
}

uint32_t orc_uid(int proc, int species, int side, int term, int eval_idx) {
  return ((uint32_t)proc << 24) | ((uint32_t)species << 20) | ((uint32_t)side << 19) | ((uint32_t)term << 18) |
         (uint32_t)eval_idx;
}

/* Work items for (process selection, species selection), ordered by identifier: process, species,
 * side, term, evaluation index.  Evaluation indices are {0, s, 2s, ...} below the observed species'
 * grid size, s = stride_override if > 0 else the process's own stride. */
int orc_list_items(const orc_world* w, int proc_sel, int species_sel, int stride_override, orc_item* out,
                   int cap) {
  int count = 0;
  for (int p = 0; p < w->n_proc; ++p) {
    if (proc_sel >= 0 && p != proc_sel) continue;
    const orc_process* P = &w->procs[p];
    for (int a = 0; a < w->n_species; ++a) {
      if (species_sel >= 0 && a != species_sel) continue;
      for (int side = 0; side < 2; ++side) {
        int mult = orc_side_multiplicity(P, a, side);
        if (mult == 0) continue;
        int n_terms = P->term_mode == ORC_TERMS_NET ? 1 : 2;
        int stride = stride_override > 0 ? stride_override : (P->eval_stride > 0 ? P->eval_stride : 1);
        for (int term = 0; term < n_terms; ++term) {
          for (int i = 0; i < w->species[a].n_grid; i += stride) {
            if (out && count < cap) {
              orc_item* it = &out[count];
              it->proc = p;
              it->species = a;
              it->side = side;
              it->term = term;
              it->eval_idx = i;
              it->mult = mult;
              it->uid = orc_uid(p, a, side, term, i);
              it->q_obs = 0.0;
            }
            ++count;
          }
        }
      }
    }
  }
  return count;
}

/* Evaluation points off the grid: the observed leg sits at the given comoving momentum q[k] and its f follows the
 * rule of every other particle (orc_f_at: interpolation inside the grid, the extrapolation fit outside). */
int orc_list_items_at(const orc_world* w, int proc_sel, int species, const double* q, int n_q, orc_item* out,
                      int cap) {
  int count = 0;
  if (species < 0 || species >= w->n_species || n_q < 0 || n_q > ORC_CUSTOM_BASE) return 0;
  for (int p = 0; p < w->n_proc; ++p) {
    if (proc_sel >= 0 && p != proc_sel) continue;
    const orc_process* P = &w->procs[p];
    for (int side = 0; side < 2; ++side) {
      int mult = orc_side_multiplicity(P, species, side);
      if (mult == 0) continue;
      int n_terms = P->term_mode == ORC_TERMS_NET ? 1 : 2;
      for (int term = 0; term < n_terms; ++term) {
        for (int k = 0; k < n_q; ++k) {
          if (out && count < cap) {
            orc_item* it = &out[count];
            it->proc = p;
            it->species = species;
            it->side = side;
            it->term = term;
            it->eval_idx = k;
            it->mult = mult;
            it->uid = orc_uid(p, species, side, term, ORC_CUSTOM_BASE + k);
            it->q_obs = q[k];
          }
          ++count;
        }
      }
    }
  }
  return count;
}

int orc_item_dims(const orc_world* w, const orc_item* it) {
  const orc_process* P = &w->procs[it->proc];
  return 3 * (P->n_in + P->n_out - 2);
}

/* Integration range of dimension d: r in [q_min, q_max] of the integrated particle's species,
 * theta in [0, pi], phi in [0, 2 pi)  (Appendix A). */
static void dim_range(const orc_world* w, const orc_process* P, const int* integ, int d, double* lo, double* hi) {
  int k = d / 3, c = d % 3;
  if (c == 0) {
    const orc_species* s = &w->species[P->sp[integ[k]]];
    *lo = s->q_min;
    *hi = s->q_max;
  } else if (c == 1) {
    *lo = 0.0;
    *hi = PI_D;
  } else {
    *lo = 0.0;
    *hi = TWO_PI;
  }
}

void orc_map_uniform(const orc_world* w, const orc_item* it, double* map) {
  const orc_process* P = &w->procs[it->proc];
  int i_obs, i_cons, integ[ORC_MAXN];
  orc_roles(P, it->species, it->side, &i_obs, &i_cons, integ);
  const int D = orc_item_dims(w, it), nb = P->n_bins;
  for (int d = 0; d < D; ++d) {
    double lo, hi;
    dim_range(w, P, integ, d, &lo, &hi);
    for (int j = 0; j <= nb; ++j) map[d * (nb + 1) + j] = lo + (hi - lo) * (double)j / (double)nb;
  }
}

/* =====================================================================================================
 * The integrand of one work item at a point x of the 3(n-2)-dimensional space.
 * ===================================================================================================== */

/* Statistical factor relative to the observed leg (Eq. 5 and the gain / loss lists of Sec. II.C):
 *   gain = prod_{opposite side} f_i * prod_{observed side} (1 + eta_i f_i)
 *   loss = prod_{observed side} f_i * prod_{opposite side} (1 + eta_i f_i)
 * f[i], eta[i] per position (initial state i < n_in).  SPLIT: term 0 = gain, 1 = loss; NET: gain - loss. */
double orc_stat_factor(int n_in, int n, int obs_side, int term_mode, int term, const double* f, const double* eta) {
  double gain = 1.0, loss = 1.0;
  for (int i = 0; i < n; ++i) {
    int on_obs_side = ((i < n_in) ? 0 : 1) == obs_side;
    if (on_obs_side) {
      gain *= 1.0 + eta[i] * f[i];
      loss *= f[i];
    } else {
      gain *= f[i];
      loss *= 1.0 + eta[i] * f[i];
    }
  }
  if (term_mode == ORC_TERMS_NET) return gain - loss;
  return term == 0 ? gain : loss;
}

typedef struct {
  const orc_world* w;
  const orc_process* P;
  int n, n_in, n_int;
  int i_obs, i_cons, integ[ORC_MAXN];
  int obs_side, term;
  double a;                   /* scale factor */
  double m[ORC_MAXN];         /* mass of each position */
  double eta[ORC_MAXN];       /* statistics of each position */
  const orc_species* sp[ORC_MAXN];
  const double* fit[ORC_MAXN];
  double q_obs, f_obs;        /* comoving observed momentum, table value of f there */
} item_ctx;

static int item_setup(item_ctx* c, const orc_world* w, const orc_item* it, double t, const double* fits) {
  c->w = w;
  c->P = &w->procs[it->proc];
  c->n_in = c->P->n_in;
  c->n = c->P->n_in + c->P->n_out;
  c->n_int = c->n - 2;
  c->obs_side = it->side;
  c->term = it->term;
  int rc = orc_roles(c->P, it->species, it->side, &c->i_obs, &c->i_cons, c->integ);
  if (rc) return rc;
  c->a = orc_scale_factor(w, t);
  for (int i = 0; i < c->n; ++i) {
    const orc_species* s = &w->species[c->P->sp[i]];
    c->sp[i] = s;
    c->m[i] = orc_mass(s, t);
    c->eta[i] = (double)s->stat;
    c->fit[i] = &fits[4 * c->P->sp[i]];
  }
  const orc_species* so = &w->species[it->species];
  if (it->q_obs > 0.0) {
    const double p = it->q_obs / c->a, m = c->m[c->i_obs];
    c->q_obs = it->q_obs;
    c->f_obs = orc_f_at(so, c->fit[c->i_obs], it->q_obs, sqrt(p * p + m * m));
  } else {
    c->q_obs = orc_grid_q(so, it->eval_idx);
    c->f_obs = so->f[it->eval_idx];
  }
  return ORC_OK;
}

/* Width of the Gaussian energy delta at one point (Eq. 15; Appendix C): the given sigma_E, or with a relative
 * width, sigma_E = w (E_in + E_out) / 2 where E_in and E_out are the summed initial and final energies. */
double orc_point_width(const orc_process* P, int n, const double* E) {
  if (P->width_mode != ORC_WIDTH_REL) return P->sigma_E;
  double sum = 0.0;
  for (int i = 0; i < n; ++i) sum += E[i];
  return P->sigma_E * 0.5 * sum;
}

/* Matrix-element factor (the paper registers |M|^2 as a function of the momenta; here a quadratic polynomial in
 * the Mandelstam invariants s and t of the process's positions): 1 for a constant |M|^2, else P(s, t). */
double orc_m2_factor(const orc_process* P, const double* E, const double* px, const double* py, const double* pz) {
  if (P->m2_kind != ORC_M2_POLY) return 1.0;
  double s;
  if (P->n_in >= 2) {
    const double e = E[0] + E[1], x = px[0] + px[1], y = py[0] + py[1], z = pz[0] + pz[1];
    s = e * e - (x * x + y * y + z * z);
  } else {
    s = E[0] * E[0] - (px[0] * px[0] + py[0] * py[0] + pz[0] * pz[0]);
  }
  const int j = P->n_in;
  const double e = E[0] - E[j], x = px[0] - px[j], y = py[0] - py[j], z = pz[0] - pz[j];
  const double t = e * e - (x * x + y * y + z * z);
  const double* c = P->m2_c;
  return c[0] + c[1] * s + c[2] * t + c[3] * s * s + c[4] * s * t + c[5] * t * t;
}

/* The width controller of Appendix C.  The relative Monte Carlo error of an evaluation is read as
 * sum_i sigma_i / sum_i |Ibar_i| over the process's items (the error relative to the gross rate, so that the
 * tiny items at the ends of the grid do not dominate).  Below width_lo the width narrows (w / width_factor),
 * above width_hi it widens (w width_factor), clamped to [width_min, width_max]. */
double orc_width_control(const orc_process* P, int n, const double* Ibar, const double* sigma, double w) {
  if (!P->width_adapt || n <= 0) return w;
  double se = 0.0, si = 0.0;
  for (int i = 0; i < n; ++i) {
    se += sigma[i];
    si += fabs(Ibar[i]);
  }
  if (!(si > 0.0)) return w;
  const double r = se / si;
  if (r < P->width_lo) w /= P->width_factor;
  else if (r > P->width_hi) w *= P->width_factor;
  if (w < P->width_min) w = P->width_min;
  if (w > P->width_max) w = P->width_max;
  return w;
}

/* Weight of the point x, excluding the Vegas Jacobian (Appendix A, Eq. A-weight):
 *   prod_k r_k^2 sin(theta_k) a^{-3} * |M|^2 * delta_sigma(E_in - E_out)
 *     / ((2 pi)^{3(n-1)-4} prod_{all i} 2 E_i) * F,
 * with F = gain or loss (SPLIT) or gain - loss (NET), gain/loss defined relative to the observed leg:
 *   gain = prod_{opposite side} f * prod_{observed side} (1 + eta f)
 *   loss = prod_{observed side} f * prod_{opposite side} (1 + eta f)       (Sec. II.C, the C_2 / C_3 lists)
 * Points with any E_i below the cut get weight 0 (Appendix A). */
static double item_point(const item_ctx* c, const double* x, double* sens);

static double item_integrand(const item_ctx* c, const double* x) { return item_point(c, x, NULL); }

/* The same weight; with sens != NULL also the point's sensitivity to rounding in the energies,
 * (|E_in - E_out| / sigma_E) (sum_i E_i / sigma_E): an absolute change e of E_in - E_out moves the Gaussian factor
 * by a relative (|E_in - E_out| / sigma_E^2) e, and two correct FP64 evaluations of the energies differ by e of a
 * few ulps of sum_i E_i. */
static double item_point(const item_ctx* c, const double* x, double* sens) {
  const int n = c->n, n_in = c->n_in;
  const double a = c->a;
  double px[ORC_MAXN], py[ORC_MAXN], pz[ORC_MAXN], E[ORC_MAXN] = {0}, f[ORC_MAXN] = {0};
  double jac = 1.0;
  if (sens) *sens = 0.0;
  /* observed particle on the z axis, physical momentum q/a */
  px[c->i_obs] = 0.0;
  py[c->i_obs] = 0.0;
  pz[c->i_obs] = c->q_obs / a;
  /* integrated particles: spherical coordinates, comoving r, physical p = r / a */
  for (int k = 0; k < c->n_int; ++k) {
    int i = c->integ[k];
    double r = x[3 * k], th = x[3 * k + 1], ph = x[3 * k + 2];
    double p = r / a;
    px[i] = p * sin(th) * cos(ph);
    py[i] = p * sin(th) * sin(ph);
    pz[i] = p * cos(th);
    jac *= r * r * sin(th);
  }
  /* conserved particle (Eq. 14 / Appendix A momentum conservation) */
  {
    double sx = 0, sy = 0, sz = 0;
    for (int i = 0; i < n; ++i) {
      if (i == c->i_cons) continue;
      double sgn = (i < n_in) ? 1.0 : -1.0; /* sum_in - sum_out */
      sx += sgn * px[i];
      sy += sgn * py[i];
      sz += sgn * pz[i];
    }
    if (c->i_cons < n_in) { sx = -sx; sy = -sy; sz = -sz; } /* sum_out - sum_in for an initial-state one */
    px[c->i_cons] = sx;
    py[c->i_cons] = sy;
    pz[c->i_cons] = sz;
  }
  /* energies: E = sqrt(|p|^2 + m^2); an integrated particle's |p| is r/a by construction */
  for (int i = 0; i < n; ++i) {
    double p2 = px[i] * px[i] + py[i] * py[i] + pz[i] * pz[i];
    for (int k = 0; k < c->n_int; ++k)
      if (c->integ[k] == i) {
        double p = x[3 * k] / a;
        p2 = p * p;
      }
    E[i] = sqrt(p2 + c->m[i] * c->m[i]);
    if (E[i] < c->P->e_cut) return 0.0;
  }
  double dE = 0.0;
  for (int i = 0; i < n; ++i) dE += (i < n_in) ? E[i] : -E[i];
  const double sig = orc_point_width(c->P, n, E);
  double delta = exp(-dE * dE / (2.0 * sig * sig)) / (sig * sqrt(TWO_PI));
  if (sens) {
    double sumE = 0.0;
    for (int i = 0; i < n; ++i) sumE += E[i];
    *sens = (fabs(dE) / sig) * (sumE / sig);
  }
  /* distribution values */
  for (int i = 0; i < n; ++i) {
    if (i == c->i_obs) {
      f[i] = c->f_obs;
    } else if (i == c->i_cons) {
      double pabs = sqrt(px[i] * px[i] + py[i] * py[i] + pz[i] * pz[i]);
      f[i] = orc_f_at(c->sp[i], c->fit[i], a * pabs, E[i]);
    } else {
      int k = -1;
      for (int kk = 0; kk < c->n_int; ++kk)
        if (c->integ[kk] == i) k = kk;
      f[i] = orc_f_at(c->sp[i], c->fit[i], x[3 * k], E[i]);
    }
  }
  double F = orc_stat_factor(n_in, n, c->obs_side, c->P->term_mode, c->term, f, c->eta);
  double prod2E = 1.0;
  for (int i = 0; i < n; ++i) prod2E *= 2.0 * E[i];
  double twopi_pow = pow(TWO_PI, (double)(3 * (n - 1) - 4));
  double a3 = pow(a, -3.0 * (double)c->n_int);
  double M2 = c->P->coupling * c->P->coupling * orc_m2_factor(c->P, E, px, py, pz);
  return jac * a3 * M2 * delta / (twopi_pow * prod2E) * F;
}

/* Fit parameters of every species at time t (4 doubles each). */
int orc_fits_all(const orc_world* w, double t, double* fits) {
  double a = orc_scale_factor(w, t);
  for (int s = 0; s < w->n_species; ++s) {
    int rc = orc_fit(&w->species[s], a, t, &fits[4 * s]);
    if (rc) return rc;
  }
  return ORC_OK;
}

int orc_integrand_at(const orc_world* w, const orc_item* it, const double* x, double* value) {
  double fits[4 * ORC_MAXSPECIES];
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  item_ctx c;
  rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  *value = item_integrand(&c, x);
  return ORC_OK;
}

/* The integrand (without Vegas Jacobian) at n points x[n][D] of one item, OpenMP over points. */
int orc_integrand_batch(const orc_world* w, const orc_item* it, int64_t n, const double* x, double* value) {
  double fits[4 * ORC_MAXSPECIES];
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  item_ctx c;
  rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  const int D = 3 * c.n_int;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) value[i] = item_integrand(&c, &x[i * D]);
  return ORC_OK;
}

/* =====================================================================================================
 * Vegas (Lepage, J. Comput. Phys. 27 (1978) 192; 439 (2021) 110386) for one work item.
 * ===================================================================================================== */

/* Map adaptation of one dimension from the per-bin sums h_j (of squared weights) and counts c_j:
 * average d_j = h_j / c_j, (7,1)/(1,6,1)/(1,7) / 8 smoothing, normalisation to unit sum, damping
 * w_j = ((1 - d_j) / ln(1/d_j))^alpha, then new interior edges at equal cumulative w, placed linearly
 * inside the old bins.  Dimensions whose smoothed sum is zero keep their edges. */
static void adapt_dim(double* edges, int nb, const long double* h, const long double* cnt, double alpha) {
  double d[ORC_MAXBINS], ds[ORC_MAXBINS], wgt[ORC_MAXBINS], old[ORC_MAXBINS + 1];
  for (int j = 0; j < nb; ++j) d[j] = cnt[j] > 0 ? (double)(h[j] / cnt[j]) : 0.0;
  if (nb == 1) return;
  ds[0] = (7.0 * d[0] + d[1]) / 8.0;
  ds[nb - 1] = (d[nb - 2] + 7.0 * d[nb - 1]) / 8.0;
  for (int j = 1; j < nb - 1; ++j) ds[j] = (d[j - 1] + 6.0 * d[j] + d[j + 1]) / 8.0;
  double sum = 0.0;
  for (int j = 0; j < nb; ++j) sum += ds[j];
  if (!(sum > 0.0)) return;
  double wsum = 0.0;
  for (int j = 0; j < nb; ++j) {
    double dh = ds[j] / sum;
    double v;
    if (dh <= 0.0) v = 0.0;
    else if (dh >= 1.0) v = 1.0;
    else {
      double base = (1.0 - dh) / log(1.0 / dh);
      v = alpha == 0.5 ? sqrt(base) : pow(base, alpha);
    }
    wgt[j] = v;
    wsum += v;
  }
  if (!(wsum > 0.0)) return;
  for (int j = 0; j <= nb; ++j) old[j] = edges[j];
  const double per_bin = wsum / (double)nb;
  int j = 0;           /* current old bin */
  double acc = 0.0;    /* cumulative weight up to the start of old bin j */
  for (int k = 1; k < nb; ++k) {
    double target = per_bin * (double)k;
    while (j < nb - 1 && acc + wgt[j] < target) {
      acc += wgt[j];
      ++j;
    }
    double frac = wgt[j] > 0.0 ? (target - acc) / wgt[j] : 0.0;
    if (frac > 1.0) frac = 1.0;
    if (frac < 0.0) frac = 0.0;
    edges[k] = old[j] + frac * (old[j + 1] - old[j]);
  }
  edges[0] = old[0];
  edges[nb] = old[nb];
}

/* The adaptation of one dimension from per-bin sums h[0..nb-1] and counts cnt[0..nb-1] given as doubles (edges:
 * nb + 1 values, in/out). */
void orc_adapt_dim(double* edges, int nb, const double* h, const double* cnt, double alpha) {
  long double hl[ORC_MAXBINS], cl[ORC_MAXBINS];
  if (nb < 1 || nb > ORC_MAXBINS) return;
  for (int j = 0; j < nb; ++j) {
    hl[j] = (long double)h[j];
    cl[j] = (long double)cnt[j];
  }
  adapt_dim(edges, nb, hl, cl, alpha);
}

/* VEGAS+ (Lepage, J. Comput. Phys. 439 (2021) 110386): adaptive stratified sampling on top of the Vegas map.
 * y-space is cut into M = k^D hypercubes, k = orc_vplus_strata(N, D) per dimension, each of volume 1/M; hypercube
 * h = sum_d h_d k^d (dimension 0 fastest).  An iteration draws n_h samples in hypercube h, sample s = off_h + i
 * (off_h = sum of n over the hypercubes before h) with y_d = (h_d + u_d) / k from the sample's uniforms u.
 *   estimate   I = sum_h (1/M) S1_h / n_h,  variance V = sum_h (S2_h - S1_h^2 / n_h) / (n_h (n_h - 1)) / M^2;
 *   map training data: per sample (W N_it / (M n_h))^2, the squared weight of the sample in the plain-Vegas
 *   normalisation (N_it = sum_h n_h), and a count;
 *   allocation: the first iteration of a call takes n_h = N / M (integer division); after an adapted iteration,
 *   sigma_h^2 = max(0, (S2_h - S1_h^2 / n_h) / (n_h - 1)) / M^2, d_h = (sigma_h^2)^(beta/2), and
 *   n_h = 2 + floor((N - 2 M) d_h / sum d) (every hypercube keeps two samples; the uniform allocation again if
 *   sum d = 0).  Frozen runs (adapt = 0) keep the uniform allocation. */
int orc_vplus_strata(int64_t N, int D) {
  int k = 1;
  for (;;) {
    int64_t p = 1;
    for (int d = 0; d < D && p <= N / 2; ++d) p *= (int64_t)(k + 1);
    if (p > N / 2) return k;
    ++k;
  }
}

static int item_vegas_plus(const item_ctx* c, const orc_item* it, int64_t N, int first_iter, int nitn, uint64_t seed,
                           uint32_t epoch, int adapt, double* map, double* I_it, double* V_it) {
  const int D = 3 * c->n_int, nb = c->P->n_bins;
  const int k = orc_vplus_strata(N, D);
  int64_t M = 1;
  for (int d = 0; d < D; ++d) M *= k;
  int64_t* nh = (int64_t*)malloc(sizeof(int64_t) * (size_t)M);
  double* S1 = (double*)malloc(sizeof(double) * (size_t)M);
  double* S2 = (double*)malloc(sizeof(double) * (size_t)M);
  long double* h = (long double*)calloc((size_t)D * nb, sizeof(long double));
  long double* cn = (long double*)calloc((size_t)D * nb, sizeof(long double));
  if (!nh || !S1 || !S2 || !h || !cn) {
    free(nh); free(S1); free(S2); free(h); free(cn);
    return ORC_ENOMEM;
  }
  for (int64_t q = 0; q < M; ++q) nh[q] = N / M;
  double y[ORC_MAXD], x[ORC_MAXD];
  int jb[ORC_MAXD];
  for (int itn = 0; itn < nitn; ++itn) {
    int64_t Nit = 0;
    for (int64_t q = 0; q < M; ++q) Nit += nh[q];
    memset(h, 0, sizeof(long double) * (size_t)D * nb);
    memset(cn, 0, sizeof(long double) * (size_t)D * nb);
    int64_t off = 0;
    for (int64_t q = 0; q < M; ++q) {
      int dig[ORC_MAXD];
      int64_t rem = q;
      for (int d = 0; d < D; ++d) {
        dig[d] = (int)(rem % k);
        rem /= k;
      }
      const double wt = (double)Nit / ((double)M * (double)nh[q]);
      double s1 = 0.0, s2 = 0.0;
      for (int64_t i = 0; i < nh[q]; ++i) {
        orc_sample_uniforms(seed, it->uid, epoch, first_iter + itn, off + i, D, y);
        double J = 1.0;
        for (int d = 0; d < D; ++d) {
          double yn = ((double)dig[d] + y[d]) / (double)k * (double)nb;
          int j = (int)floor(yn);
          if (j > nb - 1) j = nb - 1;
          double del = yn - (double)j;
          double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
          x[d] = e0 + (e1 - e0) * del;
          J *= (double)nb * (e1 - e0);
          jb[d] = j;
        }
        double W = J * item_integrand(c, x);
        s1 += W;
        s2 += W * W;
        double Wt = W * wt;
        double w2 = fabs(Wt) >= ORC_HIST_WMIN ? Wt * Wt : 0.0;
        for (int d = 0; d < D; ++d) {
          h[d * nb + jb[d]] += (long double)w2;
          cn[d * nb + jb[d]] += 1.0L;
        }
      }
      S1[q] = s1;
      S2[q] = s2;
      off += nh[q];
    }
    long double I = 0.0L, V = 0.0L;
    for (int64_t q = 0; q < M; ++q) {
      const double n = (double)nh[q];
      I += (long double)(S1[q] / n);
      V += (long double)((S2[q] - S1[q] * S1[q] / n) / (n * (n - 1.0)));
    }
    I_it[itn] = (double)(I / (long double)M);
    V_it[itn] = (double)(V / ((long double)M * (long double)M));
    if (adapt) {
      for (int d = 0; d < D; ++d) adapt_dim(&map[d * (nb + 1)], nb, &h[d * nb], &cn[d * nb], c->P->alpha);
      double sumd = 0.0;
      for (int64_t q = 0; q < M; ++q) {
        const double n = (double)nh[q];
        double s2 = (S2[q] - S1[q] * S1[q] / n) / (n - 1.0) / ((double)M * (double)M);
        s2 = s2 > 0.0 ? s2 : 0.0;
        S1[q] = pow(s2, 0.5 * c->P->beta);  /* d_h, reusing the array */
        sumd += S1[q];
      }
      for (int64_t q = 0; q < M; ++q)
        nh[q] = sumd > 0.0 ? 2 + (int64_t)floor((double)(N - 2 * M) * S1[q] / sumd) : N / M;
    }
  }
  free(nh); free(S1); free(S2); free(h); free(cn);
  return ORC_OK;
}

/* Runs Vegas iterations first_iter .. first_iter + nitn - 1 of N samples for one item.  map: D x (nb+1)
 * edges (in: current map; out: map adapted after every iteration, or unchanged when adapt == 0).  I_it, V_it: per-iteration estimate and its variance
 * V = (S2/N - I^2)/(N-1).  Ibar, sigma: inverse-variance weighted combination over the iterations with
 * V > 0 (plain mean and sigma 0 if there is none). */
int orc_item_vegas(const orc_world* w, const orc_item* it, const double* fits, int64_t N, int first_iter, int nitn,
                   uint64_t seed, uint32_t epoch, int adapt, double* map, double* I_it, double* V_it, double* Ibar,
                   double* sigma) {
  item_ctx c;
  int rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  const int D = 3 * c.n_int, nb = c.P->n_bins;
  if (c.P->vegas_plus) {
    rc = item_vegas_plus(&c, it, N, first_iter, nitn, seed, epoch, adapt, map, I_it, V_it);
    if (rc) return rc;
    nitn = -nitn;  /* iterations done: skip the plain loop below */
  }
  long double* h = (long double*)calloc((size_t)D * nb, sizeof(long double));
  long double* cn = (long double*)calloc((size_t)D * nb, sizeof(long double));
  if (!h || !cn) { free(h); free(cn); return ORC_ENOMEM; }
  double y[ORC_MAXD], x[ORC_MAXD];
  int jb[ORC_MAXD];
  for (int itn = 0; itn < nitn; ++itn) {
    long double S1 = 0.0L, S2 = 0.0L;
    memset(h, 0, sizeof(long double) * (size_t)D * nb);
    memset(cn, 0, sizeof(long double) * (size_t)D * nb);
    for (int64_t s = 0; s < N; ++s) {
      orc_sample_uniforms(seed, it->uid, epoch, first_iter + itn, s, D, y);
      double J = 1.0;
      for (int d = 0; d < D; ++d) {
        double yn = y[d] * (double)nb;
        int j = (int)floor(yn);
        if (j > nb - 1) j = nb - 1;
        double del = yn - (double)j;
        double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
        x[d] = e0 + (e1 - e0) * del;
        J *= (double)nb * (e1 - e0);
        jb[d] = j;
      }
      double W = J * item_integrand(&c, x);
      S1 += (long double)W;
      S2 += (long double)W * (long double)W;
      /* training data of the map: W^2, with weights below 2^-400 in magnitude counted as 0 so that every
       * contribution is a normal double (sub-normal squares carry rounding-order-dependent relative
       * errors of order one, which the logarithm of the damping step would turn into edge shifts) */
      double w2 = fabs(W) >= ORC_HIST_WMIN ? W * W : 0.0;
      for (int d = 0; d < D; ++d) {
        h[d * nb + jb[d]] += (long double)w2;
        cn[d * nb + jb[d]] += 1.0L;
      }
    }
    double Id = (double)(S1 / (long double)N);
    double Vd = (double)(((S2 / (long double)N) - (long double)Id * (long double)Id) / (long double)(N - 1));
    I_it[itn] = Id;
    V_it[itn] = Vd;
    if (adapt)
      for (int d = 0; d < D; ++d) adapt_dim(&map[d * (nb + 1)], nb, &h[d * nb], &cn[d * nb], c.P->alpha);
  }
  free(h);
  free(cn);
  if (nitn < 0) nitn = -nitn;
  double sw = 0.0, swI = 0.0;
  int npos = 0;
  for (int itn = 0; itn < nitn; ++itn) {
    if (V_it[itn] > 0.0) {
      sw += 1.0 / V_it[itn];
      swI += I_it[itn] / V_it[itn];
      ++npos;
    }
  }
  if (npos > 0) {
    *Ibar = swI / sw;
    *sigma = 1.0 / sqrt(sw);
  } else {
    double m = 0.0;
    for (int itn = 0; itn < nitn; ++itn) m += I_it[itn];
    *Ibar = nitn > 0 ? m / nitn : 0.0;
    *sigma = 0.0;
  }
  return ORC_OK;
}

/* Rounding sensitivity of the plain-Vegas estimate of one item over iterations first_iter .. + nitn - 1 on a fixed
 * map (no adaptation), from the same samples as orc_item_vegas: per iteration
 *   B1 = (1/N) sum_n |W_n| s_n,   B2 = (2 / (N (N - 1))) sum_n W_n^2 s_n,
 * with s_n the point's sensitivity (item_point).  If another correct FP64 evaluation moves each sample's
 * E_in - E_out by at most c eps sum_i E_i, its I differs by at most c eps B1 (first order) and its V by about
 * c eps B2.  Test infrastructure for the tolerance of GPU parity; not part of the estimator. */
int orc_item_sensitivity(const orc_world* w, const orc_item* it, int64_t N, int first_iter, int nitn, uint64_t seed,
                         uint32_t epoch, const double* map, double* B1, double* B2) {
  double fits[4 * ORC_MAXSPECIES];
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  item_ctx c;
  rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  if (c.P->vegas_plus) return ORC_EINVAL;
  const int D = 3 * c.n_int, nb = c.P->n_bins;
  double y[ORC_MAXD], x[ORC_MAXD];
  for (int itn = 0; itn < nitn; ++itn) {
    long double b1 = 0.0L, b2 = 0.0L;
    for (int64_t s = 0; s < N; ++s) {
      orc_sample_uniforms(seed, it->uid, epoch, first_iter + itn, s, D, y);
      double J = 1.0;
      for (int d = 0; d < D; ++d) {
        double yn = y[d] * (double)nb;
        int j = (int)floor(yn);
        if (j > nb - 1) j = nb - 1;
        double del = yn - (double)j;
        double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
        x[d] = e0 + (e1 - e0) * del;
        J *= (double)nb * (e1 - e0);
      }
      double sn = 0.0;
      const double W = J * item_point(&c, x, &sn);
      b1 += (long double)(fabs(W) * sn);
      b2 += (long double)(W * W * sn);
    }
    B1[itn] = (double)(b1 / (long double)N);
    B2[itn] = (double)(2.0L * b2 / ((long double)N * (long double)(N - 1)));
  }
  return ORC_OK;
}

/* orc_item_sensitivity for n_items items (OpenMP over items); maps: n_items x ORC_MAP_STRIDE(nb), B1, B2:
 * n_items x nitn. */
int orc_items_sensitivity(const orc_world* w, int n_items, const orc_item* items, int64_t N, int first_iter, int nitn,
                          uint64_t seed, uint32_t epoch, const double* maps, double* B1, double* B2, int n_threads) {
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_items; ++i) {
    const orc_process* P = &w->procs[items[i].proc];
    int r = orc_item_sensitivity(w, &items[i], N, first_iter, nitn, seed, epoch,
                                 &maps[(size_t)i * ORC_MAP_STRIDE(P->n_bins)], &B1[(size_t)i * nitn],
                                 &B2[(size_t)i * nitn]);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  return err;
}

/* Runs every item of `items` (OpenMP over items).  maps: n_items x ORC_MAP_STRIDE(nb) doubles (in/out;
 * a row whose first edge is NaN is initialised to the uniform map first).  I_it, V_it: n_items x nitn. */
int orc_run_items(const orc_world* w, int n_items, const orc_item* items, int64_t N, int first_iter, int nitn,
                  uint64_t seed, uint32_t epoch, int adapt, double* maps, double* I_it, double* V_it, double* Ibar,
                  double* sigma, int n_threads) {
  double fits[4 * ORC_MAXSPECIES];
  if (w->n_species > ORC_MAXSPECIES) return ORC_EINVAL;
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  if (N < 2 || nitn < 1 || first_iter < 0 || first_iter + nitn > 64) return ORC_EINVAL;
  int err = 0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_items; ++i) {
    const orc_process* P = &w->procs[items[i].proc];
    double* map = &maps[(size_t)i * ORC_MAP_STRIDE(P->n_bins)];
    if (isnan(map[0])) orc_map_uniform(w, &items[i], map);
    int r = orc_item_vegas(w, &items[i], fits, N, first_iter, nitn, seed, epoch, adapt, map,
                           &I_it[(size_t)i * nitn], &V_it[(size_t)i * nitn], &Ibar[i], &sigma[i]);
    if (r) {
#pragma omp atomic write
      err = r;
    }
  }
  return err;
}

/* Combination of item results into C_a on the evaluation points (Eq. 7, Eq. 12):
 *   C(q_i) = sum over items at point i of mult * (+Ibar for gain / net, -Ibar for loss),
 *   sigma(q_i)^2 = sum of mult^2 sigma_item^2.
 * C and sigma are indexed by grid index (n_grid entries); points that are not evaluated are left 0. */
void orc_combine(const orc_world* w, int n_items, const orc_item* items, const double* Ibar, const double* sig,
                 int species, double* C, double* sigma) {
  int n = w->species[species].n_grid;
  for (int j = 0; j < n; ++j) { C[j] = 0.0; sigma[j] = 0.0; }
  for (int i = 0; i < n_items; ++i) {
    const orc_item* it = &items[i];
    if (it->species != species) continue;
    const orc_process* P = &w->procs[it->proc];
    double sgn = (P->term_mode == ORC_TERMS_SPLIT && it->term == 1) ? -1.0 : 1.0;
    C[it->eval_idx] += (double)it->mult * sgn * Ibar[i];
    sigma[it->eval_idx] += (double)it->mult * (double)it->mult * sig[i] * sig[i];
  }
  for (int j = 0; j < n; ++j) sigma[j] = sqrt(sigma[j]);
}

/* Fill rule for a strided evaluation of one process on the grid of species a: between evaluated
 * neighbours C is linear in ln q; beyond the last evaluated index, C/f of that index is held. */
static void fill_strided(const orc_species* s, int stride, double* C, double* sg) {
  const int n = s->n_grid;
  if (stride <= 1) return;
  int last = ((n - 1) / stride) * stride;
  for (int j = 0; j < n; ++j) {
    if (j % stride == 0) continue;
    if (j > last) {
      C[j] = C[last] / s->f[last] * s->f[j];
      sg[j] = sg[last] / s->f[last] * s->f[j];
      continue;
    }
    int i0 = (j / stride) * stride, i1 = i0 + stride;
    double l0 = log(orc_grid_q(s, i0)), l1 = log(orc_grid_q(s, i1)), lj = log(orc_grid_q(s, j));
    double u = (lj - l0) / (l1 - l0);
    C[j] = C[i0] + u * (C[i1] - C[i0]);
    sg[j] = sg[i0] + u * (sg[i1] - sg[i0]);
  }
}

/* Full-grid collision term of every species from all processes at the world's current time:
 * per process, its items are run and combined, the strided fill rule is applied, and the processes'
 * contributions are summed (sigma in quadrature).  C_all / sig_all: concatenation over species of
 * n_grid entries each.  maps: per item of orc_list_items(w, -1, -1, 0) order (in/out). */
int orc_collision_all(const orc_world* w, int64_t N, int nitn, uint64_t seed, uint32_t epoch, int adapt,
                      double* maps, double* C_all, double* sig_all, int n_threads) {
  int n_items = orc_list_items(w, -1, -1, 0, NULL, 0);
  orc_item* items = (orc_item*)malloc(sizeof(orc_item) * (size_t)(n_items > 0 ? n_items : 1));
  double* I_it = (double*)malloc(sizeof(double) * (size_t)(n_items > 0 ? n_items : 1) * (size_t)nitn);
  double* V_it = (double*)malloc(sizeof(double) * (size_t)(n_items > 0 ? n_items : 1) * (size_t)nitn);
  double* Ib = (double*)malloc(sizeof(double) * (size_t)(n_items > 0 ? n_items : 1));
  double* sg = (double*)malloc(sizeof(double) * (size_t)(n_items > 0 ? n_items : 1));
  if (!items || !I_it || !V_it || !Ib || !sg) {
    free(items); free(I_it); free(V_it); free(Ib); free(sg);
    return ORC_ENOMEM;
  }
  orc_list_items(w, -1, -1, 0, items, n_items);
  int rc = orc_run_items(w, n_items, items, N, 0, nitn, seed, epoch, adapt, maps, I_it, V_it, Ib, sg, n_threads);
  if (rc == ORC_OK) {
    size_t off = 0;
    for (int a = 0; a < w->n_species; ++a) {
      int n = w->species[a].n_grid;
      for (int j = 0; j < n; ++j) { C_all[off + j] = 0.0; sig_all[off + j] = 0.0; }
      double* Cp = (double*)malloc(sizeof(double) * (size_t)n);
      double* Sp = (double*)malloc(sizeof(double) * (size_t)n);
      for (int p = 0; p < w->n_proc; ++p) {
        /* items of process p and species a */
        int first = -1, cnt = 0;
        for (int i = 0; i < n_items; ++i)
          if (items[i].proc == p && items[i].species == a) { if (first < 0) first = i; ++cnt; }
        if (cnt == 0) continue;
        orc_combine(w, cnt, &items[first], &Ib[first], &sg[first], a, Cp, Sp);
        int stride = w->procs[p].eval_stride > 0 ? w->procs[p].eval_stride : 1;
        fill_strided(&w->species[a], stride, Cp, Sp);
        for (int j = 0; j < n; ++j) {
          C_all[off + j] += Cp[j];
          sig_all[off + j] = sqrt(sig_all[off + j] * sig_all[off + j] + Sp[j] * Sp[j]);
        }
      }
      free(Cp);
      free(Sp);
      off += (size_t)n;
    }
  }
  free(items); free(I_it); free(V_it); free(Ib); free(sg);
  return rc;
}

/* =====================================================================================================
 * Vector-Jacobian product of the frozen-map estimator (common random numbers).
 *
 * With the map frozen, item i's estimate of one iteration is I_i = (1/N) sum_n W_n, and C at an evaluation
 * point is sum over its items of mult * sign * I_i.  Given coef_i = v_point * mult * sign, this accumulates
 *   grad_f[s][j] += coef_i/N sum_n dW_n/df_{s,j},   grad_m[s] += coef_i/N sum_n dW_n/dm_s,
 *   grad_lambda[p] += coef_i/N sum_n 2 W_n / lambda_p.
 * f enters W through the statistical factor: the observed leg's table value, the interpolation rule of the
 * particle's species between the bracketing nodes (Sec. III.B: linear in ln q; the not-a-knot cubic spline in q,
 * whose second derivatives depend on every node through the spline conditions; the equilibrium-exact rule, linear
 * in E for log(1/f + eta)), or the extrapolation f = 1/(exp(a + b E) - eta) whose (a, b) are the least-squares line
 * through (E_k, log(1/f_k + eta)) of the end nodes.  m enters through every energy E_i = sqrt(p_i^2 + m^2) of a
 * particle of that species (Gaussian delta, 1/(2 E_i), the extrapolated or equilibrium-exact f) and through the
 * energies E_k of the fit nodes and of the equilibrium-exact rule's bracketing nodes.
 * ===================================================================================================== */

/* Derivatives of the end-node fit (a, b) of one side: da/dy_k, db/dy_k, da/dE_k, db/dE_k, the node
 * energies E_k and values y_k.  side 0 = low end, 1 = high end. */
static void fit_derivatives(const orc_species* s, double a_scale, double m, int side, double* da_dy, double* db_dy,
                            double* da_dE, double* db_dE, double* Ek, int* j0_out) {
  const int n = s->n_grid;
  const int j0 = side == 0 ? 0 : n - ORC_NFIT;
  const double eta = (double)s->stat;
  double E[ORC_NFIT], Y[ORC_NFIT], mE = 0, mY = 0;
  for (int k = 0; k < ORC_NFIT; ++k) {
    double p = orc_grid_q(s, j0 + k) / a_scale;
    E[k] = sqrt(p * p + m * m);
    Y[k] = log(1.0 / s->f[j0 + k] + eta);
    mE += E[k] / ORC_NFIT;
    mY += Y[k] / ORC_NFIT;
  }
  double sxx = 0, sxy = 0;
  for (int k = 0; k < ORC_NFIT; ++k) {
    sxx += (E[k] - mE) * (E[k] - mE);
    sxy += (E[k] - mE) * (Y[k] - mY);
  }
  const double b = sxy / sxx;
  for (int k = 0; k < ORC_NFIT; ++k) {
    db_dy[k] = (E[k] - mE) / sxx;
    da_dy[k] = 1.0 / ORC_NFIT - mE * db_dy[k];
    db_dE[k] = ((Y[k] - mY) - 2.0 * b * (E[k] - mE)) / sxx;
    da_dE[k] = -db_dE[k] * mE - b / ORC_NFIT;
    Ek[k] = E[k];
  }
  *j0_out = j0;
}

/* One item: accumulates into grad_f (concatenated species grids, offsets f_off), grad_m, grad_lam. */
int orc_item_vjp(const orc_world* w, const orc_item* it, const double* fits, int64_t N, int iter, uint64_t seed,
                 uint32_t epoch, const double* map, double coef, const int64_t* f_off, double* grad_f, double* grad_M,
                 double* grad_m, double* grad_lam) {
  item_ctx c;
  int rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  const int n = c.n, n_in = c.n_in, D = 3 * c.n_int, nb = c.P->n_bins;
  const double a = c.a;
  const double cN = coef / (double)N;
  /* per-species accumulators of dW/da, dW/db for the low and high fits */
  double dfit[ORC_MAXSPECIES][4];
  memset(dfit, 0, sizeof dfit);
  double y[ORC_MAXD], x[ORC_MAXD];
  for (int64_t sidx = 0; sidx < N; ++sidx) {
    orc_sample_uniforms(seed, it->uid, epoch, iter, sidx, D, y);
    double J = 1.0;
    for (int d = 0; d < D; ++d) {
      double yn = y[d] * (double)nb;
      int j = (int)floor(yn);
      if (j > nb - 1) j = nb - 1;
      double del = yn - (double)j;
      double e0 = map[d * (nb + 1) + j], e1 = map[d * (nb + 1) + j + 1];
      x[d] = e0 + (e1 - e0) * del;
      J *= (double)nb * (e1 - e0);
    }
    /* kinematics (as item_integrand) */
    double px[ORC_MAXN], py[ORC_MAXN], pz[ORC_MAXN], E[ORC_MAXN], f[ORC_MAXN] = {0};
    double jac = 1.0;
    px[c.i_obs] = 0.0;
    py[c.i_obs] = 0.0;
    pz[c.i_obs] = c.q_obs / a;
    int kof[ORC_MAXN];
    for (int i = 0; i < n; ++i) kof[i] = -1;
    for (int k = 0; k < c.n_int; ++k) {
      int i = c.integ[k];
      kof[i] = k;
      double r = x[3 * k], th = x[3 * k + 1], ph = x[3 * k + 2];
      double p = r / a;
      px[i] = p * sin(th) * cos(ph);
      py[i] = p * sin(th) * sin(ph);
      pz[i] = p * cos(th);
      jac *= r * r * sin(th);
    }
    {
      double sx = 0, sy = 0, sz = 0;
      for (int i = 0; i < n; ++i) {
        if (i == c.i_cons) continue;
        double sg = (i < n_in) ? 1.0 : -1.0;
        sx += sg * px[i];
        sy += sg * py[i];
        sz += sg * pz[i];
      }
      if (c.i_cons < n_in) { sx = -sx; sy = -sy; sz = -sz; }
      px[c.i_cons] = sx;
      py[c.i_cons] = sy;
      pz[c.i_cons] = sz;
    }
    int cut = 0;
    for (int i = 0; i < n; ++i) {
      double p2 = px[i] * px[i] + py[i] * py[i] + pz[i] * pz[i];
      if (kof[i] >= 0) {
        double p = x[3 * kof[i]] / a;
        p2 = p * p;
      }
      E[i] = sqrt(p2 + c.m[i] * c.m[i]);
      if (E[i] < c.P->e_cut) cut = 1;
    }
    if (cut) continue;
    double dE = 0.0;
    for (int i = 0; i < n; ++i) dE += (i < n_in) ? E[i] : -E[i];
    const double sig = orc_point_width(c.P, n, E);
    double delta = exp(-dE * dE / (2.0 * sig * sig)) / (sig * sqrt(TWO_PI));
    /* f values and where they come from */
    int src[ORC_MAXN], node[ORC_MAXN], eside[ORC_MAXN];
    double wgt[ORC_MAXN], qat[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
      const orc_species* S = c.sp[i];
      double q;
      if (i == c.i_obs) {
        f[i] = c.f_obs;
        src[i] = 0;
        node[i] = it->eval_idx;
        continue;
      }
      if (i == c.i_cons) q = a * sqrt(px[i] * px[i] + py[i] * py[i] + pz[i] * pz[i]);
      else q = x[3 * kof[i]];
      qat[i] = q;
      f[i] = orc_f_at(S, c.fit[i], q, E[i]);
      if (q < S->q_min || q > S->q_max) {
        src[i] = 2;
        eside[i] = q < S->q_min ? 0 : 1;
      } else {
        src[i] = 1;
        double lq0 = log(S->q_min), h = (log(S->q_max) - lq0) / (double)(S->n_grid - 1);
        double tpos = (log(q) - lq0) / h;
        int j = (int)floor(tpos);
        if (j < 0) j = 0;
        if (j > S->n_grid - 2) j = S->n_grid - 2;
        node[i] = j;
        wgt[i] = tpos - (double)j;
      }
    }
    /* statistical factor and its partials */
    double g[2][ORC_MAXN], dg[2][ORC_MAXN]; /* [gain/loss][position]: factor value, d factor / d f */
    for (int i = 0; i < n; ++i) {
      int on_obs = ((i < n_in) ? 0 : 1) == c.obs_side;
      double bf = 1.0 + c.eta[i] * f[i];
      g[0][i] = on_obs ? bf : f[i];
      dg[0][i] = on_obs ? c.eta[i] : 1.0;
      g[1][i] = on_obs ? f[i] : bf;
      dg[1][i] = on_obs ? 1.0 : c.eta[i];
    }
    double Fv[2], dF[2][ORC_MAXN];
    for (int t = 0; t < 2; ++t) {
      Fv[t] = 1.0;
      for (int i = 0; i < n; ++i) Fv[t] *= g[t][i];
      for (int i = 0; i < n; ++i) {
        double prod = dg[t][i];
        for (int k = 0; k < n; ++k)
          if (k != i) prod *= g[t][k];
        dF[t][i] = prod;
      }
    }
    double F, dFdf[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
      if (c.P->term_mode == ORC_TERMS_NET) dFdf[i] = dF[0][i] - dF[1][i];
      else dFdf[i] = dF[c.term][i];
    }
    F = c.P->term_mode == ORC_TERMS_NET ? Fv[0] - Fv[1] : Fv[c.term];
    double prod2E = 1.0;
    for (int i = 0; i < n; ++i) prod2E *= 2.0 * E[i];
    const double twopi_pow = pow(TWO_PI, (double)(3 * (n - 1) - 4));
    const double a3 = pow(a, -3.0 * (double)c.n_int);
    const double M2 = c.P->coupling * c.P->coupling;
    const double Wb = J * (jac * a3 * M2 * delta / (twopi_pow * prod2E));
    const double W = Wb * F;
    /* coupling */
    grad_lam[it->proc] += cN * 2.0 * W / c.P->coupling;
    /* f */
    double dWdf[ORC_MAXN];
    for (int i = 0; i < n; ++i) {
      dWdf[i] = Wb * dFdf[i];
      int spc = c.P->sp[i];
      double gsum = cN * dWdf[i];
      const orc_species* S = c.sp[i];
      const int j = node[i];
      if (src[i] == 0) {
        grad_f[f_off[spc] + j] += gsum;
      } else if (src[i] == 1 && S->interp == ORC_INTERP_SPLINE) {
        /* A f_j + B f_{j+1} + ((A^3 - A) M_j + (B^3 - B) M_{j+1}) h^2/6: the f_j directly, the M_j through grad_M */
        const double q0 = orc_grid_q(S, j), hq = orc_grid_q(S, j + 1) - q0;
        const double B = (qat[i] - q0) / hq, A = 1.0 - B;
        grad_f[f_off[spc] + j] += gsum * A;
        grad_f[f_off[spc] + j + 1] += gsum * B;
        grad_M[f_off[spc] + j] += gsum * (A * A * A - A) * hq * hq / 6.0;
        grad_M[f_off[spc] + j + 1] += gsum * (B * B * B - B) * hq * hq / 6.0;
      } else if (src[i] == 1 && S->interp == ORC_INTERP_EQEXACT) {
        /* f = 1/(exp(y) - eta), y = (1 - u) y_j + u y_{j+1}, u = (E - E_j)/(E_{j+1} - E_j), y_k = log(1/f_k + eta):
         * df/dy = -f (1 + eta f), dy_k/df_k = -1 / (f_k (1 + eta f_k)) */
        const double u = (E[i] - S->aux[j]) / (S->aux[j + 1] - S->aux[j]);
        const double dfdy = -f[i] * (1.0 + c.eta[i] * f[i]);
        const double f0 = S->f[j], f1 = S->f[j + 1];
        grad_f[f_off[spc] + j] += gsum * dfdy * (1.0 - u) * (-1.0 / (f0 * (1.0 + c.eta[i] * f0)));
        grad_f[f_off[spc] + j + 1] += gsum * dfdy * u * (-1.0 / (f1 * (1.0 + c.eta[i] * f1)));
      } else if (src[i] == 1) {
        grad_f[f_off[spc] + j] += gsum * (1.0 - wgt[i]);
        grad_f[f_off[spc] + j + 1] += gsum * wgt[i];
      } else {
        double dfdz = -f[i] * (1.0 + c.eta[i] * f[i]);
        dfit[spc][2 * eside[i]] += gsum * dfdz;
        dfit[spc][2 * eside[i] + 1] += gsum * dfdz * E[i];
      }
    }
    /* mass: energies of every particle, and the extrapolated f's energy dependence */
    for (int i = 0; i < n; ++i) {
      double dWdE = W * (-dE / (sig * sig) * ((i < n_in) ? 1.0 : -1.0) - 1.0 / E[i]);
      /* a relative width grows with every energy: d sigma / d E_i = w / 2 */
      if (c.P->width_mode == ORC_WIDTH_REL) dWdE += W * (dE * dE / (sig * sig) - 1.0) / sig * (0.5 * c.P->sigma_E);
      if (src[i] == 2) {
        double b = c.fit[i][2 * eside[i] + 1];
        dWdE += dWdf[i] * (-b * f[i] * (1.0 + c.eta[i] * f[i]));
      }
      if (src[i] == 1 && c.sp[i]->interp == ORC_INTERP_EQEXACT) {
        /* y is linear in E between the node energies E_j = sqrt((q_j/a)^2 + m^2), which move with m too:
         * du/dE = 1/dE_n, du/dE_j = (u - 1)/dE_n, du/dE_{j+1} = -u/dE_n with dE_n = E_{j+1} - E_j */
        const orc_species* S = c.sp[i];
        const int j = node[i];
        const double Ej = S->aux[j], Ej1 = S->aux[j + 1], dEn = Ej1 - Ej;
        const double u = (E[i] - Ej) / dEn;
        const double y0 = log(1.0 / S->f[j] + c.eta[i]), y1 = log(1.0 / S->f[j + 1] + c.eta[i]);
        const double dfdu = -f[i] * (1.0 + c.eta[i] * f[i]) * (y1 - y0);
        dWdE += dWdf[i] * dfdu / dEn;
        grad_m[c.P->sp[i]] += cN * dWdf[i] * dfdu * ((u - 1.0) / dEn * c.m[i] / Ej - u / dEn * c.m[i] / Ej1);
      }
      grad_m[c.P->sp[i]] += cN * dWdE * c.m[i] / E[i];
    }
  }
  /* chain of the extrapolation fits */
  for (int spc = 0; spc < w->n_species; ++spc) {
    for (int side = 0; side < 2; ++side) {
      double dWa = dfit[spc][2 * side], dWb = dfit[spc][2 * side + 1];
      if (dWa == 0.0 && dWb == 0.0) continue;
      const orc_species* S = &w->species[spc];
      double m = orc_mass(S, w->t);
      double da_dy[ORC_NFIT], db_dy[ORC_NFIT], da_dE[ORC_NFIT], db_dE[ORC_NFIT], Ek[ORC_NFIT];
      int j0;
      fit_derivatives(S, a, m, side, da_dy, db_dy, da_dE, db_dE, Ek, &j0);
      const double eta = (double)S->stat;
      for (int k = 0; k < ORC_NFIT; ++k) {
        double fk = S->f[j0 + k];
        double dy_df = -1.0 / (fk * (1.0 + eta * fk));
        grad_f[f_off[spc] + j0 + k] += (dWa * da_dy[k] + dWb * db_dy[k]) * dy_df;
        grad_m[spc] += (dWa * da_dE[k] + dWb * db_dE[k]) * m / Ek[k];
      }
    }
  }
  return ORC_OK;
}

/* VJP over a list of items with per-item coefficients (v * mult * sign), frozen maps (one map row per item,
 * ORC_MAP_STRIDE(nb) doubles; NaN first edge = uniform), iteration index `iter`.  grad_f: all species grids
 * concatenated; grad_m: per species; grad_lam: per process.  Outputs are overwritten. */
int orc_vjp(const orc_world* w, int n_items, const orc_item* items, const double* coef, int64_t N, int iter,
            uint64_t seed, uint32_t epoch, const double* maps, double* grad_f, double* grad_m, double* grad_lam,
            int n_threads) {
  /* the gradient's chain is written for a constant |M|^2 */
  for (int p = 0; p < w->n_proc; ++p)
    if (w->procs[p].m2_kind != ORC_M2_CONST) return ORC_EINVAL;
  double fits[4 * ORC_MAXSPECIES];
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  int64_t f_off[ORC_MAXSPECIES];
  int64_t tot = 0;
  for (int s = 0; s < w->n_species; ++s) {
    f_off[s] = tot;
    tot += w->species[s].n_grid;
  }
  for (int64_t j = 0; j < tot; ++j) grad_f[j] = 0.0;
  double* grad_M = (double*)calloc((size_t)(tot > 0 ? tot : 1), sizeof(double));  /* dL/dM_j of spline species */
  if (!grad_M) return ORC_ENOMEM;
  for (int s = 0; s < w->n_species; ++s) grad_m[s] = 0.0;
  for (int p = 0; p < w->n_proc; ++p) grad_lam[p] = 0.0;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
  int err = 0;
#pragma omp parallel
  {
    double* gf = (double*)calloc((size_t)tot, sizeof(double));
    double* gM = (double*)calloc((size_t)tot, sizeof(double));
    double gm[ORC_MAXSPECIES] = {0}, gl[256] = {0};
#pragma omp for schedule(dynamic, 1)
    for (int i = 0; i < n_items; ++i) {
      const orc_process* P = &w->procs[items[i].proc];
      const size_t stride = ORC_MAP_STRIDE(P->n_bins);
      double* mp = (double*)malloc(sizeof(double) * stride);
      memcpy(mp, &maps[(size_t)i * stride], sizeof(double) * stride);
      if (isnan(mp[0])) orc_map_uniform(w, &items[i], mp);
      int r = orc_item_vjp(w, &items[i], fits, N, iter, seed, epoch, mp, coef[i], f_off, gf, gM, gm, gl);
      free(mp);
      if (r) {
#pragma omp atomic write
        err = r;
      }
    }
#pragma omp critical
    {
      for (int64_t j = 0; j < tot; ++j) grad_f[j] += gf[j];
      for (int64_t j = 0; j < tot; ++j) grad_M[j] += gM[j];
      for (int s = 0; s < w->n_species; ++s) grad_m[s] += gm[s];
      for (int p = 0; p < w->n_proc && p < 256; ++p) grad_lam[p] += gl[p];
    }
    free(gf);
    free(gM);
  }
  /* the spline's second derivatives depend on every node of their species */
  for (int s = 0; s < w->n_species && !err; ++s) {
    const orc_species* S = &w->species[s];
    if (S->interp != ORC_INTERP_SPLINE) continue;
    double* q = (double*)malloc(sizeof(double) * (size_t)S->n_grid);
    for (int j = 0; j < S->n_grid; ++j) q[j] = orc_grid_q(S, j);
    err = orc_spline_adjoint(S->n_grid, q, &grad_M[f_off[s]], &grad_f[f_off[s]]);
    free(q);
  }
  free(grad_M);
  return err;
}

/* =====================================================================================================
 * Exact-delta 2->2 (Sec. IV "semi-analytical" reduction, Eq. 22; Appendix B).
 * ===================================================================================================== */

/* The angular kinematic function F = int_{-1}^{1} dcos(theta) |M|^2 pi / sqrt(-a) Theta(b^2 - 4ac) of Appendix B, in
 * closed form.  With eps = p1 p3 cos(theta), kappa = p1^2 + p3^2 and u = 2 eps:
 *   -a = 4 px^2 (kappa - u), so pi / sqrt(-a) = pi / (2 px sqrt(kappa - u));
 *   b^2 - 4ac = 16 px^2 p3^2 sin^2(theta) (4 px^2 (kappa - u) - (G + u)^2), G = Q + 2 gamma,
 * so the allowed u form the interval between the roots of (G + u)^2 = 4 px^2 (kappa - u),
 *   u = -(G + 2 px^2) -+ 2 px sqrt(G + px^2 + kappa),
 * cut to [-2 p1 p3, 2 p1 p3], and
 *   F = |M|^2 pi (sqrt(kappa - u_lo) - sqrt(kappa - u_hi)) / (2 p1 p3 px). */
double orc_kinematic_F(double p1, double p3, double px, double G, double M2) {
  const double kappa = p1 * p1 + p3 * p3;
  const double disc = G + px * px + kappa;
  if (!(disc >= 0.0)) return 0.0;
  const double mid = -(G + 2.0 * px * px), half = 2.0 * px * sqrt(disc);
  const double U = 2.0 * p1 * p3;
  const double lo = fmax(-U, mid - half), hi = fmin(U, mid + half);
  if (!(hi > lo)) return 0.0;
  return M2 * (0.5 * TWO_PI) * (sqrt(kappa - lo) - sqrt(kappa - hi)) / (2.0 * p1 * p3 * px);
}

/* Trapezoid weight of node j of a species grid for int dp (physical p = q / a): the rule in ln q,
 * int g dq = int g q dln q, gives h q_j (1/2 at the two ends), and dp = dq / a. */
static double trap_weight(const orc_species* s, int j, double a) {
  const double h = (log(s->q_max) - log(s->q_min)) / (double)(s->n_grid - 1);
  const double t = (j == 0 || j == s->n_grid - 1) ? 0.5 : 1.0;
  return t * h * orc_grid_q(s, j) / a;
}

/* One item.  Positions: 1 the observed particle, 2 its partner on the same side (the conserved particle of the
 * Monte Carlo roles), 3 and 4 the opposite side in index order.
 *   backward (gain) term: C_BW = 2/(2 pi)^4 1/(2 E1) int dp3 p3^2/(2E3) int dp4 p4^2/(2E4) F f3 f4 (1 + eta1 f1)(1 + eta2 f2)
 *     with E2 = E3 + E4 - E1 >= m2, Q = m1^2 - m2^2 + m3^2 + m4^2, gamma = E3 E4 - E1 E3 - E1 E4;
 *   forward (loss) term: C_FW = 2/(2 pi)^4 1/(2 E1) int dp2 p2^2/(2E2) int dp3 p3^2/(2E3) F' f1 f2 (1 + eta3 f3)(1 + eta4 f4)
 *     with E4 = E1 + E2 - E3 >= m4, Q' = m1^2 + m2^2 + m3^2 - m4^2, gamma' = E1 E2 - E1 E3 - E2 E3 and p2 in the
 *     place of p4.
 * The dependent particle's f comes from orc_f_at (interpolation or fit); the integrated momenta run over the grid
 * nodes of their species. */
static int exact22_item(const orc_world* w, const orc_item* it, const double* fits, double* out) {
  const orc_process* P = &w->procs[it->proc];
  if (P->n_in != 2 || P->n_out != 2 || P->m2_kind != ORC_M2_CONST) return ORC_EINVAL;
  item_ctx c;
  int rc = item_setup(&c, w, it, w->t, fits);
  if (rc) return rc;
  const int i1 = c.i_obs, i2 = c.i_cons, i3 = c.integ[0], i4 = c.integ[1];
  const double a = c.a, M2 = P->coupling * P->coupling;
  const double m1 = c.m[i1], m2 = c.m[i2], m3 = c.m[i3], m4 = c.m[i4];
  const double e1 = c.eta[i1], e2 = c.eta[i2], e3 = c.eta[i3], e4 = c.eta[i4];
  const double p1 = c.q_obs / a, E1 = sqrt(p1 * p1 + m1 * m1), f1 = c.f_obs;
  const orc_species *s2 = c.sp[i2], *s3 = c.sp[i3], *s4 = c.sp[i4];
  const int want_gain = P->term_mode == ORC_TERMS_NET || it->term == 0;
  const int want_loss = P->term_mode == ORC_TERMS_NET || it->term == 1;
  long double gain = 0.0L, loss = 0.0L;
  if (want_gain)
    for (int j3 = 0; j3 < s3->n_grid; ++j3) {
      const double p3 = orc_grid_q(s3, j3) / a, E3 = sqrt(p3 * p3 + m3 * m3), f3 = s3->f[j3];
      for (int j4 = 0; j4 < s4->n_grid; ++j4) {
        const double p4 = orc_grid_q(s4, j4) / a, E4 = sqrt(p4 * p4 + m4 * m4), f4 = s4->f[j4];
        const double E2 = E3 + E4 - E1;
        if (!(E2 >= m2)) continue;
        const double p2 = sqrt(E2 * E2 - m2 * m2);
        const double f2 = orc_f_at(s2, c.fit[i2], a * p2, E2);
        const double G = m1 * m1 - m2 * m2 + m3 * m3 + m4 * m4 + 2.0 * (E3 * E4 - E1 * E3 - E1 * E4);
        const double F = orc_kinematic_F(p1, p3, p4, G, M2);
        gain += (long double)(trap_weight(s3, j3, a) * trap_weight(s4, j4, a) * (p3 * p3 / (2.0 * E3)) *
                              (p4 * p4 / (2.0 * E4)) * F * (f3 * f4 * (1.0 + e1 * f1) * (1.0 + e2 * f2)));
      }
    }
  if (want_loss)
    for (int j2 = 0; j2 < s2->n_grid; ++j2) {
      const double p2 = orc_grid_q(s2, j2) / a, E2 = sqrt(p2 * p2 + m2 * m2), f2 = s2->f[j2];
      for (int j3 = 0; j3 < s3->n_grid; ++j3) {
        const double p3 = orc_grid_q(s3, j3) / a, E3 = sqrt(p3 * p3 + m3 * m3), f3 = s3->f[j3];
        const double E4 = E1 + E2 - E3;
        if (!(E4 >= m4)) continue;
        const double p4 = sqrt(E4 * E4 - m4 * m4);
        const double f4 = orc_f_at(s4, c.fit[i4], a * p4, E4);
        const double G = m1 * m1 + m2 * m2 + m3 * m3 - m4 * m4 + 2.0 * (E1 * E2 - E1 * E3 - E2 * E3);
        const double F = orc_kinematic_F(p1, p3, p2, G, M2);
        loss += (long double)(trap_weight(s2, j2, a) * trap_weight(s3, j3, a) * (p2 * p2 / (2.0 * E2)) *
                              (p3 * p3 / (2.0 * E3)) * F * (f1 * f2 * (1.0 + e3 * f3) * (1.0 + e4 * f4)));
      }
    }
  const double pref = 2.0 / pow(TWO_PI, 4.0) / (2.0 * E1);
  if (P->term_mode == ORC_TERMS_NET) *out = pref * (double)(gain - loss);
  else *out = pref * (double)(it->term == 0 ? gain : loss);
  return ORC_OK;
}

int orc_exact22(const orc_world* w, int n_items, const orc_item* items, double* I) {
  double fits[4 * ORC_MAXSPECIES];
  int rc = orc_fits_all(w, w->t, fits);
  if (rc) return rc;
  for (int i = 0; i < n_items; ++i) {
    rc = exact22_item(w, &items[i], fits, &I[i]);
    if (rc) return rc;
  }
  return ORC_OK;
}

/* Full-grid exact-delta collision term of every species from all processes (each 2->2 with a constant |M|^2): the
 * items of orc_list_items, their exact-delta estimates combined per process as in orc_collision_all (strided fill
 * included); sig_all is 0. */
int orc_collision_exact22_all(const orc_world* w, double* C_all, double* sig_all) {
  int n_items = orc_list_items(w, -1, -1, 0, NULL, 0);
  orc_item* items = (orc_item*)malloc(sizeof(orc_item) * (size_t)(n_items > 0 ? n_items : 1));
  double* I = (double*)malloc(sizeof(double) * (size_t)(n_items > 0 ? n_items : 1));
  double* z = (double*)calloc((size_t)(n_items > 0 ? n_items : 1), sizeof(double));
  if (!items || !I || !z) {
    free(items); free(I); free(z);
    return ORC_ENOMEM;
  }
  orc_list_items(w, -1, -1, 0, items, n_items);
  int rc = orc_exact22(w, n_items, items, I);
  if (rc == ORC_OK) {
    size_t off = 0;
    for (int a = 0; a < w->n_species; ++a) {
      int n = w->species[a].n_grid;
      for (int j = 0; j < n; ++j) { C_all[off + j] = 0.0; sig_all[off + j] = 0.0; }
      double* Cp = (double*)malloc(sizeof(double) * (size_t)n);
      double* Sp = (double*)malloc(sizeof(double) * (size_t)n);
      for (int p = 0; p < w->n_proc; ++p) {
        int first = -1, cnt = 0;
        for (int i = 0; i < n_items; ++i)
          if (items[i].proc == p && items[i].species == a) { if (first < 0) first = i; ++cnt; }
        if (cnt == 0) continue;
        orc_combine(w, cnt, &items[first], &I[first], &z[first], a, Cp, Sp);
        int stride = w->procs[p].eval_stride > 0 ? w->procs[p].eval_stride : 1;
        fill_strided(&w->species[a], stride, Cp, Sp);
        for (int j = 0; j < n; ++j) C_all[off + j] += Cp[j];
      }
      free(Cp);
      free(Sp);
      off += (size_t)n;
    }
  }
  free(items); free(I); free(z);
  return rc;
}

/* =====================================================================================================
 * Log-space time stepping (Sec. III.C).
 * ===================================================================================================== */

/* One evaluation of the collision operator on every species' full grid (C_all, sigma in sig_all).  The Monte Carlo
 * operator of orc_collision_all, or the exact-delta 2->2 reduction of orc_collision_exact22_all. */
typedef struct {
  int exact;
  int64_t N;
  int nitn, adapt, n_threads;
  uint64_t seed;
  double* maps;
} step_op;

static int apply_op(const step_op* op, const orc_world* w, uint32_t epoch, double* C_all, double* sig_all) {
  if (op->exact) return orc_collision_exact22_all(w, C_all, sig_all);
  return orc_collision_all(w, op->N, op->nitn, op->seed, epoch, op->adapt, op->maps, C_all, sig_all, op->n_threads);
}

/* One Euler or Heun step of every species' f (in place, via the species' f pointers, which must be writable),
 * advancing w->t (Sec. III.C).  k1 = C[f] at t; dt > 0: a fixed step; dt <= 0: dt = min(dt_max, eps / max |k1/f|)
 * (Eq. 20).
 *   Euler (Eq. 18):  log f <- log f + dt k1/f;
 *   Heun (Eq. 19):   the predictor f* = f exp(dt k1/f), k2 = C[f*] at t + dt (epoch + 1 for the Monte Carlo
 *                    operator), then log f <- log f + dt/2 (k1/f + k2/f*). */
static int step_core(orc_world* w, int method, double dt, double eps, double dt_max, uint32_t epoch,
                     const step_op* op, double* dt_used) {
  size_t tot = 0;
  for (int a = 0; a < w->n_species; ++a) tot += (size_t)w->species[a].n_grid;
  double* k1 = (double*)malloc(sizeof(double) * tot);
  double* k2 = (double*)malloc(sizeof(double) * tot);
  double* sg = (double*)malloc(sizeof(double) * tot);
  double* f0 = (double*)malloc(sizeof(double) * tot);
  double* fs = (double*)malloc(sizeof(double) * tot);
  if (!k1 || !k2 || !sg || !f0 || !fs) {
    free(k1); free(k2); free(sg); free(f0); free(fs);
    return ORC_ENOMEM;
  }
  int rc = apply_op(op, w, epoch, k1, sg);
  if (rc) goto done;
  {
    size_t off = 0;
    double rmax = 0.0;
    for (int a = 0; a < w->n_species; ++a) {
      const orc_species* s = &w->species[a];
      for (int j = 0; j < s->n_grid; ++j) {
        f0[off + j] = s->f[j];
        double r = fabs(k1[off + j] / s->f[j]);
        if (r > rmax) rmax = r;
      }
      off += (size_t)s->n_grid;
    }
    double h = dt;
    if (!(h > 0.0)) {
      h = rmax > 0.0 ? eps / rmax : dt_max;
      if (h > dt_max) h = dt_max;
    }
    *dt_used = h;
    if (method == ORC_EULER) {
      off = 0;
      for (int a = 0; a < w->n_species; ++a) {
        double* f = (double*)w->species[a].f;
        for (int j = 0; j < w->species[a].n_grid; ++j) f[j] = exp(log(f0[off + j]) + h * k1[off + j] / f0[off + j]);
        off += (size_t)w->species[a].n_grid;
      }
      w->t += h;
    } else {
      off = 0;
      for (int a = 0; a < w->n_species; ++a) {
        double* f = (double*)w->species[a].f;
        for (int j = 0; j < w->species[a].n_grid; ++j) {
          fs[off + j] = exp(log(f0[off + j]) + h * k1[off + j] / f0[off + j]);
          f[j] = fs[off + j];
        }
        off += (size_t)w->species[a].n_grid;
      }
      double t0 = w->t;
      w->t = t0 + h;
      rc = apply_op(op, w, epoch + 1u, k2, sg);
      if (rc) {
        w->t = t0;
        off = 0;
        for (int a = 0; a < w->n_species; ++a) {
          double* f = (double*)w->species[a].f;
          for (int j = 0; j < w->species[a].n_grid; ++j) f[j] = f0[off + j];
          off += (size_t)w->species[a].n_grid;
        }
        goto done;
      }
      off = 0;
      for (int a = 0; a < w->n_species; ++a) {
        double* f = (double*)w->species[a].f;
        for (int j = 0; j < w->species[a].n_grid; ++j)
          f[j] = exp(log(f0[off + j]) + 0.5 * h * (k1[off + j] / f0[off + j] + k2[off + j] / fs[off + j]));
        off += (size_t)w->species[a].n_grid;
      }
    }
  }
done:
  free(k1); free(k2); free(sg); free(f0); free(fs);
  return rc;
}

/* The Monte Carlo step: k1 with `epoch`, k2 with epoch + 1; maps are reused and updated in place. */
int orc_step(orc_world* w, int method, double dt, double eps, double dt_max, int64_t N, int nitn, uint64_t seed,
             uint32_t epoch, int adapt, double* maps, double* dt_used, int n_threads) {
  step_op op = {0, N, nitn, adapt, n_threads, seed, maps};
  return step_core(w, method, dt, eps, dt_max, epoch, &op, dt_used);
}

/* The same step with the deterministic exact-delta 2->2 operator (every process 2->2 with a constant |M|^2). */
int orc_step_exact22(orc_world* w, int method, double dt, double eps, double dt_max, double* dt_used) {
  step_op op = {1, 0, 0, 0, 0, 0, NULL};
  return step_core(w, method, dt, eps, dt_max, 0u, &op, dt_used);
}
