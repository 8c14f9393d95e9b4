/*
 * kr_oracle.h -- plain FP64 CPU oracle for per-cell implicit thermochemistry.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this code; it exists so tests (and the CPU baseline timing) can
 * check the HIP path against a slow, obviously correct implementation.
 *
 * What it computes (paper Sec. 2.2, eq. method-ode-thermochem, Sec. 2.2.1
 * rates and analytic Jacobian, Sec. 2.2.2 pre-processing, Sec. 2.2.3
 * post-processing and retry, Algorithm algo:lu-decomp for the LU):
 * backward-Euler substeps solved by Newton iteration on the unknowns
 * y = (n_1..n_S, T), with mass-action Arrhenius rates, detailed-balance
 * reverse rates, optional tabulated rate factors, and an energy equation
 * written in eps = sum_s n_s e_s(T) (T sum_s c_s n_s for constant c_s).
 *
 * Conventions: cgs; energies divided by k_B (so in K); row-major matrices.
 */
#ifndef KR_ORACLE_H
#define KR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kro_net kro_net;

/* Builds the oracle's own copy of a network description.  Returns NULL and
 * sets *err (1 bad sizes/indices, 2 non-conserving reaction, 3 reservoir not
 * single-row) on invalid input. */
kro_net *kro_net_create(int S, int n_rows, int n_elem, const int32_t *comp,
                        const int32_t *reservoir, const double *cv,
                        const double *h_form, const double *s_form, int R,
                        const int32_t *reac, const int32_t *prod,
                        const double *arr_f, const double *arr_r,
                        double p_ref, double T_min, double T_max, int *err);
void kro_net_destroy(kro_net *net);

/* Optional temperature-dependent heat capacities (paper Sec. 4.2: c_V as
 * NASA-style piecewise polynomials in T): cv_poly[S][2][5] holds, per
 * species, c_V/k_B = sum_k a_k T^k for T < T_mid and for T >= T_mid.  The
 * thermal energy per particle is e_s(T) = its integral from 0 (upper piece
 * shifted to be continuous at T_mid) and the energy equation is written in
 * eps = sum_s n_s e_s(T).  Returns 0, or 1 for invalid input. */
int kro_net_set_heat_capacity(kro_net *net, double T_mid, const double *cv_poly);
/* Optional tabulated rate factors (paper Sec. 2.2.1, third rate type): the
 * coefficient of reaction r with tab_of[r] = t >= 0 is its Arrhenius form
 * times tau_t(T), log2 tau_t linear in log2 T between the nodes
 * log2 T = log2T0 + i dlog2T (values tab[t][i], end segments extended); with
 * detailed-balance reverse rates the reverse coefficient carries the same
 * factor.  Returns 0, or 1 for invalid input. */
int kro_net_set_tables(kro_net *net, int n_tab, int n_nodes, double log2T0, double dlog2T,
                       const int32_t *tab_of, const double *tab);
/* Optional photoreactions and radiative heat terms (paper Sec. 2.2.1, the
 * second rate type, and the heating/cooling of eq. method-ode-thermochem):
 *   sigma[S]           photo-absorption cross-section of each species (cm^2)
 *   photo[R]           1: the forward coefficient is A F_eff (A the
 *                      reaction's cross-section, b = E = 0), no reverse;
 *                      F_eff = F (1 - exp(-tau)) / tau, tau = L sum_s
 *                      sigma_s n_s, the path average over the cell of eq.
 *                      method-rad-equiv-flux (F, L per cell: kro_extras)
 *   heat_extra[R][3]   gas heating per net forward event besides the
 *                      formation energies, q0 + q1 T + q2 T ln T (K): the
 *                      absorbed photon energy, radiated recombination
 *                      energy and the like.
 * Any of the three may be NULL (photo needs sigma).  Returns 0 or 1. */
int kro_net_set_photo(kro_net *net, const double *sigma, const int32_t *photo,
                      const double *heat_extra);
/* kro_rhs / kro_jacobian in a radiation field (F, L). */
void kro_rhs_photo(const kro_net *net, const double *y, double F, double L, double *f, double *Q);
void kro_jacobian_photo(const kro_net *net, const double *y, double F, double L, double *J);
/* e_s(T) and c_V,s(T) of every species (k_B units). */
void kro_species_thermo(const kro_net *net, double T, double *e, double *c);

/* Arrhenius parameters actually used: out[r][dir][3] = (A, b, E), dir 0 fwd,
 * 1 reverse (derived by detailed balance unless given explicitly). */
void kro_arrhenius(const kro_net *net, double *out);
void kro_rate_coeffs(const kro_net *net, double T, double *kf, double *kr);
/* f[S] = dn/dt, *Q = d eps/dt at y = (n, T). */
void kro_rhs(const kro_net *net, const double *y, double *f, double *Q);
/* J[(S+1)^2] = d(f_0..f_{S-1}, Q)/d(n_0..n_{S-1}, T). */
void kro_jacobian(const kro_net *net, const double *y, double *J);
/* Backward-Euler residual and its derivative (the Newton matrix). */
void kro_residual(const kro_net *net, const double *y, const double *yn,
                  double h, double *R);
void kro_newton_matrix(const kro_net *net, const double *y, double h,
                       double *M);

/* Crout LU with implicit (scaled) partial pivoting, in place.  Returns 0, or
 * -1 for a zero / non-finite pivot or a zero row.  p[j] = row swapped with
 * row j at step j. */
int kro_lu_decompose(int N, double *a, int32_t *p);
void kro_lu_solve(int N, const double *a, const int32_t *p, double *b);
/* Brute-force Gaussian elimination with full (row and column) pivoting. */
int kro_gauss_full_pivot(int N, const double *a, const double *b, double *x);

/* Substep control: adaptive (error controller), fixed (n_fixed equal
 * substeps), or replay (a given sequence of substep lengths per cell, no
 * error control; a Newton failure reverts the cell). */
enum { KRO_ADAPTIVE = 0, KRO_FIXED = 1, KRO_REPLAY = 2 };

typedef struct {
  double rtol;        /* relative tolerance (error control and Newton) */
  double floor;       /* absolute tolerance, as a fraction of n_nuc */
  double newton_tol;  /* weighted-norm threshold on the Newton update */
  double rho_floor;   /* density floor for pre-processing (0: none) */
  int32_t max_newton;
  int32_t max_substeps;
  int32_t mode;       /* KRO_ADAPTIVE, KRO_FIXED or KRO_REPLAY */
  int32_t n_fixed;    /* substeps in fixed mode */
} kro_opts;

void kro_default_opts(kro_opts *o);

/* Integrates every cell over its step.  states: [S][ld] SoA, in/out;
 * T in/out; dt per cell (or NULL => dt_scalar).  status[c]: 0 ok, 1 ok after
 * retry, 2 reverted to the input.  cell_stats[c][4] (may be NULL): accepted
 * substeps, Newton iterations, rejected substeps, Newton failures.
 * nthreads <= 0 uses the OpenMP default.  Returns 0 or -1 (bad args). */
int kro_integrate(const kro_net *net, int64_t n_cells, double *states,
                  int64_t ld, double *T, const double *rho, const double *dt,
                  double dt_scalar, const kro_opts *o, int32_t *status,
                  int32_t *cell_stats, int nthreads);

/* Per-cell extras of kro_integrate_ex (every pointer may be NULL):
 *   h_hint   [n_cells] in/out: first substep length of the first attempt
 *            when positive and finite (else dt); on return the controller's
 *            proposed length after the last accepted substep (adaptive mode,
 *            cells not reverted; others keep their value)
 *   h_log    [h_log_cap][h_log_ld]: the accepted substep lengths, in order,
 *            of the attempt that produced the result (out), or the lengths
 *            to replay (in, mode KRO_REPLAY)
 *   h_log_n  [n_cells]: their number (out: may exceed h_log_cap, 0 for
 *            reverted cells; in for KRO_REPLAY, <= h_log_cap)
 *   post     [n_cells] out: post-processing flags (KRO_POST_*) */
typedef struct {
  double *h_hint;
  double *h_log;
  int64_t h_log_ld;
  int32_t h_log_cap;
  int32_t *h_log_n;
  int32_t *post;
  const double *photo_flux;    /* [n_cells] optically thin photon flux (cm^-2 s^-1) */
  const double *photo_length;  /* [n_cells] path length through the cell (cm) */
} kro_extras;

enum { KRO_POST_CLIPPED = 1,      /* stage 1 set a negative abundance to 0 */
       KRO_POST_BROKEN_UP = 2 };  /* stage 3 broke up a species */

int kro_integrate_ex(const kro_net *net, int64_t n_cells, double *states,
                     int64_t ld, double *T, const double *rho, const double *dt,
                     double dt_scalar, const kro_opts *o, int32_t *status,
                     int32_t *cell_stats, const kro_extras *ex, int nthreads);

/* One backward-Euler substep of length h from yn (plain initial guess);
 * returns 0 on convergence (y holds the root) or -1.  *iters counts
 * Newton iterations.  atol[N] per unknown. */
int kro_be_substep(const kro_net *net, const kro_opts *o, const double *yn,
                   const double *atol, double h, double *y, int32_t *iters);

/* Per-cell element/charge residual: max over conserved rows of
 * |sum_s N_vs (after-before)_s| / D_v (D_v = sum_s |N_vs| before_s for an
 * element row, n_nuc for a charge row). */
void kro_element_residual(const kro_net *net, int64_t n_cells,
                          const double *before, const double *after,
                          int64_t ld, double *resid);

/* Post-processing stages 1-3 on one cell's abundances, given the conserved
 * totals E0[n_rows] of the initial state. */
void kro_postprocess(const kro_net *net, const double *E0, double *n);
/* The same, returning which stages changed anything (KRO_POST_*). */
int kro_postprocess_flags(const kro_net *net, const double *E0, double *n);

/* Fastest self-coupling timescale at y: 1 / max(max_s |d f_s/d n_s|,
 * |dQ/dT| / c_V), capped at 1e7 s (also returned when it is undefined). */
double kro_fastest_timescale(const kro_net *net, const double *y);

#ifdef __cplusplus
}
#endif
#endif
