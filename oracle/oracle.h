/*
 * oracle.h -- declarations of the CPU FP64 reference (test infrastructure only; see oracle.c).
 * This header is private to oracle/ and the test suite; the product library never includes it.
 */
#ifndef BOLTZ_ORACLE_H
#define BOLTZ_ORACLE_H

#include <stdint.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ESTATE (-2)
#define ORC_ERANGE (-3)
#define ORC_ENOMEM (-4)

#define ORC_MAXN 6          /* particles per process */
#define ORC_MAXD 12         /* 3 (n - 2) */
#define ORC_MAXBINS 256
#define ORC_MAXSPECIES 16
#define ORC_NFIT 5          /* nodes per end in the extrapolation fit */
#define ORC_HIST_WMIN 0x1p-400 /* smallest |W| whose square enters the Vegas histogram */
#define ORC_MAP_STRIDE(nb) (ORC_MAXD * ((nb) + 1))

#define ORC_BOSE 1
#define ORC_FERMI (-1)
#define ORC_MB 0

#define ORC_INTERP_LINLOG 0  /* f linear in ln q between nodes */
#define ORC_INTERP_SPLINE 1  /* not-a-knot cubic spline of f in linear q (Sec. III.B) */
#define ORC_INTERP_EQEXACT 2 /* log(1/f + eta) linear in E between nodes (exact for equilibrium, like Eq. 17) */

#define ORC_MASS_CONST 0
#define ORC_MASS_SIN 1

#define ORC_EXP_NONE 0
#define ORC_EXP_RADIATION 1

#define ORC_TERMS_SPLIT 0
#define ORC_TERMS_NET 1

#define ORC_SIDES_AUTO 0    /* self-reverse -> initial side only; else both sides */

#define ORC_WIDTH_ABS 0     /* sigma_E is the Gaussian's width (an energy) */
#define ORC_WIDTH_REL 1     /* sigma_E is the fraction w: width w (E_in + E_out) / 2 per point (Appendix C) */

#define ORC_M2_CONST 0      /* |M|^2 = coupling^2 */
#define ORC_M2_POLY 1       /* |M|^2 = coupling^2 P(s, t), P a quadratic polynomial in the Mandelstam invariants */

#define ORC_EULER 0
#define ORC_HEUN 1

typedef struct {
  int stat;                 /* eta: +1 Bose-Einstein, -1 Fermi-Dirac, 0 Maxwell-Boltzmann */
  int n_grid;               /* logarithmic grid nodes */
  double q_min, q_max;      /* comoving momentum range */
  int mass_kind;            /* ORC_MASS_CONST or ORC_MASS_SIN (m0 + mA sin(mw t)) */
  double m0, mA, mw;
  const double* f;          /* n_grid values of f on the grid */
  int interp;               /* ORC_INTERP_* */
  double* aux;              /* n_grid doubles owned by the caller, written by orc_fit: the spline's second
                               derivatives (SPLINE) or the node energies E_j at the fit's time (EQEXACT) */
} orc_species;

typedef struct {
  int n_in, n_out;
  int sp[ORC_MAXN];         /* species of positions 0..n-1 (initial state first) */
  double coupling;          /* |M|^2 = coupling^2 */
  double sigma_E;           /* Gaussian width (ORC_WIDTH_ABS) or its fraction w of (E_in + E_out) / 2 (REL) */
  double alpha;             /* Vegas damping exponent */
  double e_cut;             /* energy cut */
  int n_bins;               /* Vegas bins per dimension */
  int term_mode;            /* ORC_TERMS_SPLIT (gain and loss items) or ORC_TERMS_NET */
  int side_mask;            /* ORC_SIDES_AUTO, or bit 0 = initial side, bit 1 = final side */
  int eval_stride;          /* evaluate every k-th grid point of the observed species */
  int width_mode;           /* ORC_WIDTH_ABS or ORC_WIDTH_REL */
  /* width controller (Appendix C): after an evaluation, narrow the width by width_factor when the relative Monte
   * Carlo error is below width_lo, widen it when above width_hi, within [width_min, width_max] */
  int width_adapt;
  double width_lo, width_hi, width_factor, width_min, width_max;
  int vegas_plus;           /* 1: adaptive stratified sampling (VEGAS+) on top of the map */
  double beta;              /* VEGAS+ allocation exponent: n_h ~ sigma_h^beta */
  int m2_kind;              /* ORC_M2_CONST or ORC_M2_POLY */
  /* P(s, t) = c0 + c1 s + c2 t + c3 s^2 + c4 s t + c5 t^2 with s = (P_0 + P_1)^2 (the first two initial
   * positions; m_0^2 for one initial particle) and t = (P_0 - P_{n_in})^2 (the first initial and the first final
   * position), four-momenta physical */
  double m2_c[6];
} orc_process;

typedef struct {
  int n_species;
  const orc_species* species;
  int n_proc;
  const orc_process* procs;
  double t;
  int expansion;            /* ORC_EXP_NONE or ORC_EXP_RADIATION */
  double a0, t0;
} orc_world;

typedef struct {
  int proc, species, side, term, eval_idx, mult;
  uint32_t uid;
  double q_obs;  /* > 0: an evaluation point off the grid (comoving momentum); 0: grid node eval_idx */
} orc_item;

/* Identifier index of the k-th evaluation point off the grid: above every grid index. */
#define ORC_CUSTOM_BASE (1 << 17)

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_sample_uniforms(uint64_t seed, uint32_t uid, uint32_t epoch, int it, int64_t n, int D, double* y);
double orc_grid_q(const orc_species* s, int j);
double orc_mass(const orc_species* s, double t);
double orc_scale_factor(const orc_world* w, double t);
int orc_fit(const orc_species* s, double a, double t, double fit[4]);
double orc_f_at(const orc_species* s, const double fit[4], double q, double E);
/* Second derivatives M[0..n-1] of the not-a-knot cubic spline through (q_j, f_j). */
int orc_spline_second_derivatives(int n, const double* q, const double* f, double* M);
void orc_f_batch(const orc_species* s, const double fit[4], int64_t n, const double* q, const double* E, double* out);
int orc_side_multiplicity(const orc_process* P, int a, int side);
int orc_roles(const orc_process* P, int a, int side, int* i_obs, int* i_cons, int* integ);
uint32_t orc_uid(int proc, int species, int side, int term, int eval_idx);
int orc_list_items(const orc_world* w, int proc_sel, int species_sel, int stride_override, orc_item* out, int cap);
/* Work items at n_q evaluation momenta q[k] of one species (eval_idx = k, identifier index ORC_CUSTOM_BASE + k),
 * in the order of orc_list_items. */
int orc_list_items_at(const orc_world* w, int proc_sel, int species, const double* q, int n_q, orc_item* out,
                      int cap);
int orc_item_dims(const orc_world* w, const orc_item* it);
void orc_map_uniform(const orc_world* w, const orc_item* it, double* map);
int orc_fits_all(const orc_world* w, double t, double* fits);
double orc_stat_factor(int n_in, int n, int obs_side, int term_mode, int term, const double* f, const double* eta);
int orc_integrand_batch(const orc_world* w, const orc_item* it, int64_t n, const double* x, double* value);
int orc_integrand_at(const orc_world* w, const orc_item* it, const double* x, double* value);
/* Strata per dimension of VEGAS+ for N samples in D dimensions: the largest k >= 1 with k^D <= N / 2. */
int orc_vplus_strata(int64_t N, int D);
int orc_item_vegas(const orc_world* w, const orc_item* it, const double* fits, int64_t N, int first_iter, int nitn,
                   uint64_t seed, uint32_t epoch, int adapt, double* map, double* I_it, double* V_it, double* Ibar,
                   double* sigma);
/* Per iteration on a fixed map: B1 = (1/N) sum |W_n| s_n and B2 = (2/(N(N-1))) sum W_n^2 s_n, s_n = (|dE|/sigma_E)
 * (sum E / sigma_E) the sample's sensitivity to rounding in the energies (bounds of another FP64 evaluation's
 * difference in I and V per unit of relative energy rounding). */
int orc_item_sensitivity(const orc_world* w, const orc_item* it, int64_t N, int first_iter, int nitn, uint64_t seed,
                         uint32_t epoch, const double* map, double* B1, double* B2);
int orc_items_sensitivity(const orc_world* w, int n_items, const orc_item* items, int64_t N, int first_iter, int nitn,
                          uint64_t seed, uint32_t epoch, const double* maps, double* B1, double* B2, int n_threads);
int orc_run_items(const orc_world* w, int n_items, const orc_item* items, int64_t N, int first_iter, int nitn,
                  uint64_t seed, uint32_t epoch, int adapt, double* maps, double* I_it, double* V_it, double* Ibar,
                  double* sigma, int n_threads);
/* Exact-delta 2->2 (Sec. IV; Appendix B): the angular kinematic function for observed momentum p1, integrated
 * momentum p3 and the other integrated momentum px (p4 of the backward term, p2 of the forward term), with
 * G = Q + 2 gamma of that term, and |M|^2 = M2. */
double orc_kinematic_F(double p1, double p3, double px, double G, double M2);
/* Per item of a 2->2 process, the exact-delta estimate of the same single-position contribution the Monte Carlo
 * items estimate: the two-dimensional reduction with the trapezoidal rule in ln q on the grid nodes of the two
 * integrated species.  I[i] for items[i]; ORC_EINVAL for an item of another process kind. */
int orc_exact22(const orc_world* w, int n_items, const orc_item* items, double* I);
void orc_combine(const orc_world* w, int n_items, const orc_item* items, const double* Ibar, const double* sig,
                 int species, double* C, double* sigma);
int orc_collision_all(const orc_world* w, int64_t N, int nitn, uint64_t seed, uint32_t epoch, int adapt,
                      double* maps, double* C_all, double* sig_all, int n_threads);
/* Gaussian width of one point with energies E[0..n-1]: sigma_E, or w (E_in + E_out) / 2 for ORC_WIDTH_REL. */
double orc_point_width(const orc_process* P, int n, const double* E);
/* |M|^2 / coupling^2 at one point with position four-momenta (E, px, py, pz): 1, or P(s, t). */
double orc_m2_factor(const orc_process* P, const double* E, const double* px, const double* py, const double* pz);
/* The width controller: the width after an evaluation whose items of process P had estimates Ibar[i] and Monte
 * Carlo errors sigma[i] (i < n), starting from width w. */
double orc_width_control(const orc_process* P, int n, const double* Ibar, const double* sigma, double w);
/* One item's share of the vector-Jacobian product (grad_M: the gradient with respect to the second derivatives
 * M_j of spline species, on their nodes, taken to f by orc_spline_adjoint). */
int orc_item_vjp(const orc_world* w, const orc_item* it, const double* fits, int64_t N, int iter, uint64_t seed,
                 uint32_t epoch, const double* map, double coef, const int64_t* f_off, double* grad_f, double* grad_M,
                 double* grad_m, double* grad_lam);
/* Adds to gf (n nodes) the gradient with respect to f of a loss whose gradient with respect to the not-a-knot
 * spline's second derivatives M_j on the nodes q is g. */
int orc_spline_adjoint(int n, const double* q, const double* g, double* gf);
int orc_vjp(const orc_world* w, int n_items, const orc_item* items, const double* coef, int64_t N, int iter,
            uint64_t seed, uint32_t epoch, const double* maps, double* grad_f, double* grad_m, double* grad_lam,
            int n_threads);
/* Vegas map adaptation of one dimension (smoothing, normalisation, damping, rebinning; Appendix C alpha) from
 * per-bin training sums h and counts cnt; edges[0..nb] in/out. */
void orc_adapt_dim(double* edges, int nb, const double* h, const double* cnt, double alpha);
/* Full-grid collision term of every species by the exact-delta 2->2 reduction (sigma 0). */
int orc_collision_exact22_all(const orc_world* w, double* C_all, double* sig_all);
/* One Euler or Heun step (Sec. III.C) with the exact-delta 2->2 operator in place of the Monte Carlo one. */
int orc_step_exact22(orc_world* w, int method, double dt, double eps, double dt_max, double* dt_used);
int orc_step(orc_world* w, int method, double dt, double eps, double dt_max, int64_t N, int nitn, uint64_t seed,
             uint32_t epoch, int adapt, double* maps, double* dt_used, int n_threads);

#endif
