/*
 * kr_oracle.c -- plain FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).
 *
 * Only tests, the package smoke check and the benchmark's CPU-baseline leg
 * use this file.  It shares no code with the HIP library: it parses the
 * network description itself, derives reverse rates itself and implements
 * every step of the per-cell integration sequentially, in FP64, in the order
 * the method takes them.  It is deliberately unoptimised: no blocking, no
 * fusion, no reordering.
 *
 * Method (paper Sec. 2.2):
 *   dn^i/dt = sum_r nu_ri w_r(n, T)                    (eq. method-ode-thermochem,
 *   d eps/dt = Q(n, T) = sum_r qhat_r w_r                mass-action form)
 *   eps = T * sum_s c_s n_s                              (T = eps / c_V)
 * with w_r = k_f(T) prod_{reac} n - k_r(T) prod_{prod} n and modified
 * Arrhenius coefficients k = A T^b exp(-E/T) (Sec. 2.2.1, item 1).  The
 * reverse coefficient follows from detailed balance with per-species
 * formation energy h_s and entropy s_s at the standard-state pressure p_ref
 * (reference density n_ref = p_ref / (k_B T)); with dnu = #products -
 * #reactants, K_eq = n_ref^dnu exp(dS - dH/T) and
 *   k_r = k_f / K_eq  =>  A_r = A (k_B/p_ref)^dnu e^{-dS}, b_r = b + dnu,
 *                          E_r = E - dH.
 * qhat_r = -dH_r is the heat released per forward event, which makes
 * U = sum_s n_s (c_s T + h_s) an exact invariant of each BE substep.
 *
 * Each substep is backward Euler, R(y) = 0 with
 *   R_s = n_s - n_s^(n) - h f_s(y),   R_E = eps(y) - eps(y^(n)) - h Q(y),
 * solved by Newton iteration with the analytic Jacobian (Sec. 2.2.1,
 * eq. method-jacobian; T is the energy unknown so the thermal column is
 * d/dT, the paper's dk/deps = (1/c_V) dk/dT being the same column rescaled)
 * and an LU decomposition with implicit row scaling and partial pivoting
 * (Algorithm algo:lu-decomp, taken sequentially).  The substep size is set by
 * an error controller; pre-processing follows Sec. 2.2.2 (floors, T limits)
 * and post-processing and the retry/revert ladder follow Sec. 2.2.3.
 */
#include "kr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KRO_MAXN 64
#define KRO_KB 1.380649e-16   /* Boltzmann constant, erg/K */

struct kro_net {
  int S, n_rows, n_elem, R;
  int32_t *comp;     /* [n_rows][S] */
  int32_t *res;      /* [n_rows] */
  double *cv, *h, *s;
  int32_t *reac, *prod; /* [R][3] */
  int32_t *nu;       /* [R][S] net stoichiometry */
  double *par;       /* [R][2][3] (A, b, E) forward / reverse */
  double *qhat;      /* [R] heat released per forward event (K) */
  double T_min, T_max;
  int explicit_rev;  /* reverse parameters given, not by detailed balance */
  /* temperature-dependent heat capacities (cvp NULL: constant cv) */
  double *cvp;       /* [S][2][5] c_V/k_B = sum_k a_k T^k, T < T_mid / >= */
  double *econ;      /* [S] constant of the upper piece of e_s(T) */
  double T_mid;
  /* tabulated rate factors (tab_of NULL: none) */
  int n_tab, n_nodes;
  int32_t *tab_of;   /* [R] table of reaction r, or -1 */
  double *tab;       /* [n_tab][n_nodes] log2 of the factor at the nodes */
  double tab_x0, tab_dx;   /* node i at log2 T = tab_x0 + i tab_dx */
  /* photoreactions and radiative heat terms (NULL: none) */
  double *sigma;     /* [S] photo-absorption cross-section (cm^2) */
  int32_t *photo;    /* [R] 1: forward coefficient A F_eff, no reverse */
  double *qx;        /* [R][3] extra gas heating per event q0 + q1 T + q2 T ln T (K) */
};

/* The radiation field of one cell: the optically thin photon flux F
 * (cm^-2 s^-1) and the path length L (cm) of the cell along the rays. */
typedef struct {
  double F, L;
} kro_rad;

/* ------------------------------------------------------------------------ */
/* network                                                                   */
/* ------------------------------------------------------------------------ */

kro_net *kro_net_create(int S, int n_rows, int n_elem, const int32_t *comp,
                        const int32_t *reservoir, const double *cv,
                        const double *h_form, const double *s_form, int R,
                        const int32_t *reac, const int32_t *prod,
                        const double *arr_f, const double *arr_r,
                        double p_ref, double T_min, double T_max, int *err) {
  *err = 0;
  if (S < 1 || S + 1 > KRO_MAXN || n_rows < 0 || n_elem < 0 ||
      n_elem > n_rows || R < 0 || !(p_ref > 0.0)) {
    *err = 1;
    return NULL;
  }
  for (int r = 0; r < R; ++r)
    for (int k = 0; k < 3; ++k) {
      if (reac[3 * r + k] >= S || prod[3 * r + k] >= S) { *err = 1; return NULL; }
    }
  kro_net *n = (kro_net *)calloc(1, sizeof(kro_net));
  n->S = S; n->n_rows = n_rows; n->n_elem = n_elem; n->R = R;
  n->T_min = T_min; n->T_max = T_max;
  n->comp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows * S + 1));
  n->res = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_rows + 1));
  n->cv = (double *)malloc(sizeof(double) * S);
  n->h = (double *)malloc(sizeof(double) * S);
  n->s = (double *)malloc(sizeof(double) * S);
  n->reac = (int32_t *)malloc(sizeof(int32_t) * (size_t)(3 * R + 1));
  n->prod = (int32_t *)malloc(sizeof(int32_t) * (size_t)(3 * R + 1));
  n->nu = (int32_t *)calloc((size_t)(R * S + 1), sizeof(int32_t));
  n->par = (double *)malloc(sizeof(double) * (size_t)(6 * R + 1));
  n->qhat = (double *)malloc(sizeof(double) * (size_t)(R + 1));
  memcpy(n->comp, comp, sizeof(int32_t) * (size_t)(n_rows * S));
  memcpy(n->res, reservoir, sizeof(int32_t) * (size_t)n_rows);
  memcpy(n->cv, cv, sizeof(double) * S);
  memcpy(n->h, h_form, sizeof(double) * S);
  memcpy(n->s, s_form, sizeof(double) * S);
  memcpy(n->reac, reac, sizeof(int32_t) * (size_t)(3 * R));
  memcpy(n->prod, prod, sizeof(int32_t) * (size_t)(3 * R));

  for (int r = 0; r < R; ++r) {
    for (int k = 0; k < 3; ++k) {
      if (reac[3 * r + k] >= 0) n->nu[r * S + reac[3 * r + k]] -= 1;
      if (prod[3 * r + k] >= 0) n->nu[r * S + prod[3 * r + k]] += 1;
    }
    /* every reaction must conserve every row (elements and charge) */
    for (int v = 0; v < n_rows; ++v) {
      long sum = 0;
      for (int sp = 0; sp < S; ++sp) sum += (long)comp[v * S + sp] * n->nu[r * S + sp];
      if (sum != 0) { *err = 2; kro_net_destroy(n); return NULL; }
    }
    double dH = 0.0, dS = 0.0;
    int dnu = 0;
    for (int sp = 0; sp < S; ++sp) {
      dH += n->nu[r * S + sp] * h_form[sp];
      dS += n->nu[r * S + sp] * s_form[sp];
      dnu += n->nu[r * S + sp];
    }
    n->qhat[r] = -dH;
    double *pf = n->par + 6 * r, *pr = pf + 3;
    pf[0] = arr_f[3 * r]; pf[1] = arr_f[3 * r + 1]; pf[2] = arr_f[3 * r + 2];
    n->explicit_rev = arr_r != NULL;
    if (arr_r) {
      pr[0] = arr_r[3 * r]; pr[1] = arr_r[3 * r + 1]; pr[2] = arr_r[3 * r + 2];
    } else {
      /* detailed balance: k_r = k_f / K_eq,
       * K_eq = (p_ref / (k_B T))^dnu exp(dS - dH/T) */
      pr[0] = pf[0] * pow(KRO_KB / p_ref, dnu) * exp(-dS);
      pr[1] = pf[1] + dnu;
      pr[2] = pf[2] - dH;
    }
  }
  /* a reservoir must carry only its own row */
  for (int v = 0; v < n_rows; ++v) {
    int rs = reservoir[v];
    if (rs < 0 || rs >= S || comp[v * S + rs] == 0) { *err = 3; kro_net_destroy(n); return NULL; }
    for (int u = 0; u < n_rows; ++u)
      if (u != v && comp[u * S + rs] != 0) { *err = 3; kro_net_destroy(n); return NULL; }
  }
  return n;
}

void kro_net_destroy(kro_net *n) {
  if (!n) return;
  free(n->comp); free(n->res); free(n->cv); free(n->h); free(n->s);
  free(n->cvp); free(n->econ); free(n->tab_of); free(n->tab);
  free(n->sigma); free(n->photo); free(n->qx);
  free(n->reac); free(n->prod); free(n->nu); free(n->par); free(n->qhat);
  free(n);
}

void kro_arrhenius(const kro_net *n, double *out) {
  memcpy(out, n->par, sizeof(double) * (size_t)(6 * n->R));
}

/* e_s(T) = integral from 0 to T of c_V,s: on the lower piece the integral of
 * its polynomial, on the upper piece the integral of that one plus the
 * constant that makes e_s continuous at T_mid. */
static double poly_energy(const double *a, double T) {
  double e = 0.0, Tk = T;
  for (int k = 0; k < 5; ++k) {
    e += a[k] * Tk / (k + 1);
    Tk *= T;
  }
  return e;
}

int kro_net_set_heat_capacity(kro_net *n, double T_mid, const double *cv_poly) {
  if (!(T_mid > 0.0) || !isfinite(T_mid) || !cv_poly) return 1;
  const int S = n->S;
  for (int i = 0; i < 10 * S; ++i)
    if (!isfinite(cv_poly[i])) return 1;
  free(n->cvp); free(n->econ);
  n->cvp = (double *)malloc(sizeof(double) * 10 * (size_t)S);
  n->econ = (double *)malloc(sizeof(double) * (size_t)S);
  memcpy(n->cvp, cv_poly, sizeof(double) * 10 * (size_t)S);
  n->T_mid = T_mid;
  for (int s = 0; s < S; ++s)
    n->econ[s] = poly_energy(n->cvp + 10 * s, T_mid) - poly_energy(n->cvp + 10 * s + 5, T_mid);
  return 0;
}

int kro_net_set_tables(kro_net *n, int n_tab, int n_nodes, double log2T0, double dlog2T,
                       const int32_t *tab_of, const double *tab) {
  if (n_tab < 1 || n_nodes < 2 || !(dlog2T > 0.0) || !isfinite(log2T0) || !tab_of || !tab) return 1;
  for (int r = 0; r < n->R; ++r)
    if (tab_of[r] < -1 || tab_of[r] >= n_tab) return 1;
  for (long i = 0; i < (long)n_tab * n_nodes; ++i)
    if (!isfinite(tab[i])) return 1;
  free(n->tab_of); free(n->tab);
  n->tab_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n->R + 1));
  n->tab = (double *)malloc(sizeof(double) * (size_t)n_tab * n_nodes);
  memcpy(n->tab_of, tab_of, sizeof(int32_t) * (size_t)n->R);
  memcpy(n->tab, tab, sizeof(double) * (size_t)n_tab * n_nodes);
  n->n_tab = n_tab; n->n_nodes = n_nodes;
  n->tab_x0 = log2T0; n->tab_dx = dlog2T;
  return 0;
}

/* c_V,s(T) and e_s(T) of one species (constant cv: c_s and c_s T). */
static void species_thermo(const kro_net *n, int s, double T, double *e, double *c) {
  if (!n->cvp) {
    *c = n->cv[s];
    *e = n->cv[s] * T;
    return;
  }
  const int upper = T >= n->T_mid;
  const double *a = n->cvp + 10 * s + 5 * upper;
  double cc = 0.0, Tk = 1.0;
  for (int k = 0; k < 5; ++k) {
    cc += a[k] * Tk;
    Tk *= T;
  }
  *c = cc;
  *e = poly_energy(a, T) + (upper ? n->econ[s] : 0.0);
}

void kro_species_thermo(const kro_net *n, double T, double *e, double *c) {
  for (int s = 0; s < n->S; ++s) species_thermo(n, s, T, &e[s], &c[s]);
}

int kro_net_set_photo(kro_net *n, const double *sigma, const int32_t *photo, const double *heat_extra) {
  const int S = n->S, R = n->R;
  if (!sigma && !photo && !heat_extra) return 1;
  if (photo) {
    if (!sigma) return 1;
    for (int r = 0; r < R; ++r) {
      if (photo[r] != 0 && photo[r] != 1) return 1;
      /* a photoreaction's forward coefficient is A F_eff: no T dependence */
      if (photo[r] && (n->par[6 * r + 1] != 0.0 || n->par[6 * r + 2] != 0.0)) return 1;
    }
  }
  if (sigma)
    for (int s = 0; s < S; ++s)
      if (!(sigma[s] >= 0.0) || !isfinite(sigma[s])) return 1;
  if (heat_extra)
    for (int i = 0; i < 3 * R; ++i)
      if (!isfinite(heat_extra[i])) return 1;
  free(n->sigma); free(n->photo); free(n->qx);
  n->sigma = NULL; n->photo = NULL; n->qx = NULL;
  if (sigma) {
    n->sigma = (double *)malloc(sizeof(double) * (size_t)S);
    memcpy(n->sigma, sigma, sizeof(double) * (size_t)S);
  }
  if (photo) {
    n->photo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(R + 1));
    memcpy(n->photo, photo, sizeof(int32_t) * (size_t)R);
  }
  if (heat_extra) {
    n->qx = (double *)malloc(sizeof(double) * (size_t)(3 * R + 1));
    memcpy(n->qx, heat_extra, sizeof(double) * (size_t)(3 * R));
  }
  return 0;
}

/* Effective photon flux of a cell whose own absorbers have inverse
 * absorption length linv (eq. method-rad-equiv-flux, the path average over
 * the cell): F_eff = F (1 - exp(-tau)) / tau with tau = L linv; *dF =
 * d F_eff / d linv.  Below tau = 1e-4 the two-term series of both. */
static double photo_flux(const kro_rad *rad, double linv, double *dF) {
  *dF = 0.0;
  if (!rad || rad->F == 0.0) return 0.0;
  const double tau = rad->L * linv;
  double g, dg;
  if (tau < 1e-4) {
    g = 1.0 - tau / 2.0 + tau * tau / 6.0;
    dg = -0.5 + tau / 3.0 - tau * tau / 8.0;
  } else {
    const double em = expm1(-tau);
    g = -em / tau;
    dg = (tau * exp(-tau) + em) / (tau * tau);
  }
  *dF = rad->F * rad->L * dg;
  return rad->F * g;
}

/* inverse absorption length sum_s sigma_s n_s */
static double absorption(const kro_net *n, const double *y) {
  double l = 0.0;
  if (n->sigma)
    for (int s = 0; s < n->S; ++s) l += n->sigma[s] * y[s];
  return l;
}

/* extra heat per event of reaction r at T and its T derivative */
static double extra_heat(const kro_net *n, int r, double T, double *dq) {
  if (!n->qx) { *dq = 0.0; return 0.0; }
  const double *q = n->qx + 3 * r;
  const double lnT = log(T);
  *dq = q[1] + q[2] * (lnT + 1.0);
  return q[0] + q[1] * T + q[2] * T * lnT;
}

/* Tabulated factor tau(T) of table t: log2 tau linear in log2 T between
 * nodes (the end segments extended); *slope = d ln tau / d ln T. */
static double table_factor(const kro_net *n, int t, double T, double *slope) {
  const double *L = n->tab + (size_t)t * n->n_nodes;
  const double u = (log2(T) - n->tab_x0) / n->tab_dx;
  int i = (int)floor(u);
  if (i < 0) i = 0;
  if (i > n->n_nodes - 2) i = n->n_nodes - 2;
  const double f = u - i;
  *slope = (L[i + 1] - L[i]) / n->tab_dx;
  return exp2(L[i] + f * (L[i + 1] - L[i]));
}

/* ------------------------------------------------------------------------ */
/* rates, right-hand side, Jacobian                                          */
/* ------------------------------------------------------------------------ */

/* modified Arrhenius coefficient A T^b exp(-E/T) */
static double arrhenius(const double *p, double T) {
  return p[0] * exp(p[1] * log(T) - p[2] / T);
}

/* Rate coefficient of direction dir (0 forward, 1 reverse) of reaction r
 * and, if dk is given, its derivative in T: the Arrhenius form, times the
 * reaction's tabulated factor (both directions with detailed-balance reverse
 * rates, so that the equilibrium constant is untouched; the forward one only
 * when the reverse parameters were given). */
static double rate_coeff(const kro_net *n, int r, int dir, double T, double *dk) {
  const double *p = n->par + 6 * r + 3 * dir;
  double k = arrhenius(p, T);
  double tl = p[1] + p[2] / T;          /* T dk/dT / k */
  if (n->tab_of && n->tab_of[r] >= 0 && (dir == 0 || !n->explicit_rev)) {
    double slope;
    k *= table_factor(n, n->tab_of[r], T, &slope);
    tl += slope;
  }
  if (dk) *dk = k * tl / T;
  return k;
}

void kro_rate_coeffs(const kro_net *n, double T, double *kf, double *kr) {
  for (int r = 0; r < n->R; ++r) {
    kf[r] = rate_coeff(n, r, 0, T, NULL);
    kr[r] = rate_coeff(n, r, 1, T, NULL);
  }
}

/* rate of one direction: q = k * product over the side's species slots */
static double side_rate(double k, const int32_t *side, const double *nn) {
  double q = k;
  for (int i = 0; i < 3; ++i)
    if (side[i] >= 0) q *= nn[side[i]];
  return q;
}

/* d q / d n_m by the product rule over the side's slots */
static double side_rate_dn(double k, const int32_t *side, const double *nn, int m) {
  double d = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (side[i] != m) continue;
    double t = k;
    for (int j = 0; j < 3; ++j)
      if (j != i && side[j] >= 0) t *= nn[side[j]];
    d += t;
  }
  return d;
}

/* Coefficients of reaction r's two directions at y: photoreactions take
 * A F_eff (no reverse), the others rate_coeff; dk receive d/dT. */
static void coeffs(const kro_net *n, int r, const double *y, double Feff, double *kf, double *kr,
                   double *dkf, double *dkr) {
  const double T = y[n->S];
  if (n->photo && n->photo[r]) {
    *kf = n->par[6 * r] * Feff;
    *kr = 0.0;
    if (dkf) *dkf = 0.0;
    if (dkr) *dkr = 0.0;
    return;
  }
  *kf = rate_coeff(n, r, 0, T, dkf);
  *kr = rate_coeff(n, r, 1, T, dkr);
}

static void rhs_rad(const kro_net *n, const double *y, const kro_rad *rad, double *f, double *Q) {
  const int S = n->S;
  const double T = y[S];
  double dF;
  const double Feff = photo_flux(rad, absorption(n, y), &dF);
  for (int s = 0; s < S; ++s) f[s] = 0.0;
  double q = 0.0;
  for (int r = 0; r < n->R; ++r) {
    double kf, kr, dq;
    coeffs(n, r, y, Feff, &kf, &kr, NULL, NULL);
    double w = side_rate(kf, n->reac + 3 * r, y) - side_rate(kr, n->prod + 3 * r, y);
    for (int s = 0; s < S; ++s) f[s] += n->nu[r * S + s] * w;
    q += (n->qhat[r] + extra_heat(n, r, T, &dq)) * w;
  }
  *Q = q;
}

/* The analytic Jacobian.  A photoreaction's coefficient depends on the
 * abundances through F_eff(lambda^-1): its derivative in n_i is taken as
 * A (dF_eff / dlambda^-1) sigma_i min{1, n_i sigma_i / lambda^-1} (the
 * paper's dominant-absorber cutoff, Sec. 2.2.1; 1 where lambda^-1 = 0). */
static void jacobian_rad(const kro_net *n, const double *y, const kro_rad *rad, double *J) {
  const int S = n->S, N = S + 1;
  const double T = y[S];
  memset(J, 0, sizeof(double) * (size_t)(N * N));
  double dF;
  const double linv = absorption(n, y);
  const double Feff = photo_flux(rad, linv, &dF);
  for (int r = 0; r < n->R; ++r) {
    double dkf, dkr, kf, kr;
    coeffs(n, r, y, Feff, &kf, &kr, &dkf, &dkr);
    const int32_t *rc = n->reac + 3 * r, *pd = n->prod + 3 * r;
    /* d q/dT = (d k/dT) times the same product of abundances */
    double dwdT = side_rate(dkf, rc, y) - side_rate(dkr, pd, y);
    double dwdn[KRO_MAXN];
    for (int m = 0; m < S; ++m)
      dwdn[m] = side_rate_dn(kf, rc, y, m) - side_rate_dn(kr, pd, y, m);
    if (n->photo && n->photo[r] && dF != 0.0) {
      const double prod = side_rate(n->par[6 * r] * dF, rc, y);   /* A dF prod n */
      for (int m = 0; m < S; ++m) {
        if (n->sigma[m] == 0.0) continue;
        const double cut = linv > 0.0 ? fmin(1.0, y[m] * n->sigma[m] / linv) : 1.0;
        dwdn[m] += prod * n->sigma[m] * cut;
      }
    }
    double dq;
    const double qr = n->qhat[r] + extra_heat(n, r, T, &dq);
    const double w = side_rate(kf, rc, y) - side_rate(kr, pd, y);
    for (int s = 0; s < S; ++s) {
      int v = n->nu[r * S + s];
      if (!v) continue;
      for (int m = 0; m < S; ++m) J[s * N + m] += v * dwdn[m];
      J[s * N + S] += v * dwdT;
    }
    for (int m = 0; m < S; ++m) J[S * N + m] += qr * dwdn[m];
    J[S * N + S] += qr * dwdT + dq * w;
  }
}

void kro_rhs(const kro_net *n, const double *y, double *f, double *Q) { rhs_rad(n, y, NULL, f, Q); }
void kro_jacobian(const kro_net *n, const double *y, double *J) { jacobian_rad(n, y, NULL, J); }
void kro_rhs_photo(const kro_net *n, const double *y, double F, double L, double *f, double *Q) {
  const kro_rad rad = {F, L};
  rhs_rad(n, y, &rad, f, Q);
}
void kro_jacobian_photo(const kro_net *n, const double *y, double F, double L, double *J) {
  const kro_rad rad = {F, L};
  jacobian_rad(n, y, &rad, J);
}

/* c_V = sum_s n_s c_V,s(T) */
static double heat_capacity(const kro_net *n, const double *y) {
  double c = 0.0;
  for (int s = 0; s < n->S; ++s) {
    double es, cs;
    species_thermo(n, s, y[n->S], &es, &cs);
    c += cs * y[s];
  }
  return c;
}

/* thermal energy eps = sum_s n_s e_s(T) (= T c_V for constant cv) */
static double thermal_energy(const kro_net *n, const double *y) {
  if (!n->cvp) return y[n->S] * heat_capacity(n, y);
  double e = 0.0;
  for (int s = 0; s < n->S; ++s) {
    double es, cs;
    species_thermo(n, s, y[n->S], &es, &cs);
    e += es * y[s];
  }
  return e;
}

static void residual_rad(const kro_net *n, const double *y, const double *yn, double h,
                         const kro_rad *rad, double *R) {
  const int S = n->S;
  double f[KRO_MAXN], Q;
  rhs_rad(n, y, rad, f, &Q);
  for (int s = 0; s < S; ++s) R[s] = y[s] - yn[s] - h * f[s];
  R[S] = thermal_energy(n, y) - thermal_energy(n, yn) - h * Q;
}

void kro_residual(const kro_net *n, const double *y, const double *yn, double h, double *R) {
  residual_rad(n, y, yn, h, NULL, R);
}

static void newton_matrix_rad(const kro_net *n, const double *y, double h, const kro_rad *rad,
                              double *M) {
  const int S = n->S, N = S + 1;
  double J[KRO_MAXN * KRO_MAXN];
  jacobian_rad(n, y, rad, J);
  for (int s = 0; s < S; ++s) {
    for (int m = 0; m < N; ++m) M[s * N + m] = (s == m ? 1.0 : 0.0) - h * J[s * N + m];
  }
  /* d eps / d n_m = e_m(T) ; d eps / d T = c_V */
  for (int m = 0; m < S; ++m) {
    double em, cm;
    species_thermo(n, m, y[S], &em, &cm);
    M[S * N + m] = em - h * J[S * N + m];
  }
  M[S * N + S] = heat_capacity(n, y) - h * J[S * N + S];
}

void kro_newton_matrix(const kro_net *n, const double *y, double h, double *M) {
  newton_matrix_rad(n, y, h, NULL, M);
}

/* ------------------------------------------------------------------------ */
/* dense linear algebra                                                      */
/* ------------------------------------------------------------------------ */

/* Crout's method with implicit row scaling: for each column j compute the
 * U entries (rows <= j) and the not-yet-divided L entries (rows > j) from
 * already finished columns; pick as pivot the row i >= j with the largest
 * |a_ij| / v_i (v_i = largest magnitude in the original row i; the lowest
 * row wins ties); exchange rows (and their scales); divide the L entries by
 * the pivot. */
int kro_lu_decompose(int N, double *a, int32_t *p) {
  double v[KRO_MAXN];
  for (int i = 0; i < N; ++i) {
    double m = 0.0;
    for (int j = 0; j < N; ++j) m = fmax(m, fabs(a[i * N + j]));
    if (!(m > 0.0) || !isfinite(m)) return -1;
    v[i] = m;
  }
  for (int j = 0; j < N; ++j) {
    for (int i = 0; i < N; ++i) {
      int kmax = (i < j ? i : j);
      double sum = a[i * N + j];
      for (int k = 0; k < kmax; ++k) sum -= a[i * N + k] * a[k * N + j];
      a[i * N + j] = sum;
    }
    int imax = j;
    double best = fabs(a[j * N + j]) / v[j];
    for (int i = j + 1; i < N; ++i) {
      double t = fabs(a[i * N + j]) / v[i];
      if (t > best) { best = t; imax = i; }
    }
    if (imax != j) {
      for (int k = 0; k < N; ++k) {
        double tmp = a[imax * N + k]; a[imax * N + k] = a[j * N + k]; a[j * N + k] = tmp;
      }
      double tv = v[imax]; v[imax] = v[j]; v[j] = tv;
    }
    p[j] = imax;
    double piv = a[j * N + j];
    if (piv == 0.0 || !isfinite(piv)) return -1;
    for (int i = j + 1; i < N; ++i) a[i * N + j] /= piv;
  }
  return 0;
}

void kro_lu_solve(int N, const double *a, const int32_t *p, double *b) {
  for (int j = 0; j < N; ++j) {
    int q = p[j];
    if (q != j) { double t = b[q]; b[q] = b[j]; b[j] = t; }
  }
  for (int i = 0; i < N; ++i) {             /* L y = P b, unit diagonal */
    double sum = b[i];
    for (int k = 0; k < i; ++k) sum -= a[i * N + k] * b[k];
    b[i] = sum;
  }
  for (int i = N - 1; i >= 0; --i) {        /* U x = y */
    double sum = b[i];
    for (int k = i + 1; k < N; ++k) sum -= a[i * N + k] * b[k];
    b[i] = sum / a[i * N + i];
  }
}

int kro_gauss_full_pivot(int N, const double *a_in, const double *b_in, double *x) {
  double a[KRO_MAXN * KRO_MAXN], b[KRO_MAXN];
  int col[KRO_MAXN];
  memcpy(a, a_in, sizeof(double) * (size_t)(N * N));
  memcpy(b, b_in, sizeof(double) * (size_t)N);
  for (int j = 0; j < N; ++j) col[j] = j;
  for (int k = 0; k < N; ++k) {
    int pr = k, pc = k;
    double best = -1.0;
    for (int i = k; i < N; ++i)
      for (int j = k; j < N; ++j)
        if (fabs(a[i * N + j]) > best) { best = fabs(a[i * N + j]); pr = i; pc = j; }
    if (!(best > 0.0)) return -1;
    if (pr != k) {
      for (int j = 0; j < N; ++j) { double t = a[pr * N + j]; a[pr * N + j] = a[k * N + j]; a[k * N + j] = t; }
      double t = b[pr]; b[pr] = b[k]; b[k] = t;
    }
    if (pc != k) {
      for (int i = 0; i < N; ++i) { double t = a[i * N + pc]; a[i * N + pc] = a[i * N + k]; a[i * N + k] = t; }
      int t = col[pc]; col[pc] = col[k]; col[k] = t;
    }
    for (int i = k + 1; i < N; ++i) {
      double l = a[i * N + k] / a[k * N + k];
      for (int j = k; j < N; ++j) a[i * N + j] -= l * a[k * N + j];
      b[i] -= l * b[k];
    }
  }
  double z[KRO_MAXN];
  for (int i = N - 1; i >= 0; --i) {
    double sum = b[i];
    for (int j = i + 1; j < N; ++j) sum -= a[i * N + j] * z[j];
    z[i] = sum / a[i * N + i];
  }
  for (int j = 0; j < N; ++j) x[col[j]] = z[j];
  return 0;
}

/* ------------------------------------------------------------------------ */
/* backward-Euler substep by Newton iteration                                */
/* ------------------------------------------------------------------------ */

void kro_default_opts(kro_opts *o) {
  o->rtol = 1e-6;
  o->floor = 1e-20;
  o->newton_tol = 1e-3;
  o->rho_floor = 0.0;
  o->max_newton = 10;
  o->max_substeps = 100000;
  o->mode = KRO_ADAPTIVE;
  o->n_fixed = 1;
}

/* Newton from the plain guess y = yn.  Each iteration solves M d = -R and
 * applies d.  Converged when max_i |d_i| / w_i <= newton_tol with
 * w_i = atol_i + rtol * max(|yn_i|, |y_i|).  Fails on a singular matrix, a
 * non-finite value, T <= 0, two consecutive growths of the update norm, or
 * no convergence within max_newton iterations. */
static int be_substep_rad(const kro_net *n, const kro_opts *o, const double *yn,
                          const double *atol, double h, const kro_rad *rad, double *y,
                          int32_t *iters) {
  const int N = n->S + 1;
  double R[KRO_MAXN], M[KRO_MAXN * KRO_MAXN], d[KRO_MAXN];
  int32_t p[KRO_MAXN];
  for (int i = 0; i < N; ++i) y[i] = yn[i];
  double prev = INFINITY;
  int grow = 0;
  for (int k = 0; k < o->max_newton; ++k) {
    residual_rad(n, y, yn, h, rad, R);
    newton_matrix_rad(n, y, h, rad, M);
    *iters += 1;
    if (kro_lu_decompose(N, M, p) != 0) return -1;
    for (int i = 0; i < N; ++i) d[i] = -R[i];
    kro_lu_solve(N, M, p, d);
    double norm = 0.0;
    int finite = 1;
    for (int i = 0; i < N; ++i) {
      y[i] += d[i];
      if (!isfinite(d[i]) || !isfinite(y[i])) finite = 0;
    }
    if (!finite || !(y[N - 1] > 0.0)) return -1;
    for (int i = 0; i < N; ++i) {
      double w = atol[i] + o->rtol * fmax(fabs(yn[i]), fabs(y[i]));
      double e = fabs(d[i]) / w;
      if (e > norm) norm = e;
    }
    if (norm <= o->newton_tol) return 0;
    if (norm > prev) {
      if (++grow >= 2) return -1;
    } else {
      grow = 0;
    }
    prev = norm;
  }
  return -1;
}

int kro_be_substep(const kro_net *n, const kro_opts *o, const double *yn,
                   const double *atol, double h, double *y, int32_t *iters) {
  return be_substep_rad(n, o, yn, atol, h, NULL, y, iters);
}

/* g = (f_0..f_{S-1}, Q / c_V): the rate of change of each unknown */
static void unknown_rates(const kro_net *n, const double *y, const kro_rad *rad, double *g) {
  double Q;
  rhs_rad(n, y, rad, g, &Q);
  g[n->S] = Q / heat_capacity(n, y);
}

typedef struct {
  double h0, safety, growth;
} attempt_params;

/* Record of one attempt: the accepted substep lengths in order (the first
 * cap of them are stored), their number, and the controller's proposed
 * length of the substep after the last accepted one. */
typedef struct {
  double *h;             /* [cap] with stride ld, or NULL */
  int64_t ld;
  int32_t cap, n;
  double h_next;
} substep_log;

static void log_substep(substep_log *lg, double h) {
  if (lg->h && lg->n < lg->cap) lg->h[lg->n * lg->ld] = h;
  lg->n++;
}

/* One attempt over [0, dt].  Adaptive: after each converged substep the
 * local error estimate err = max_i |(h/2)(g_i(y_new) - g_i(y_old))| / w_i
 * (w_i from both end points) decides; accepted when err <= 1, after which
 * h *= min(growth, max(0.2, safety/sqrt(max(err,1e-10)))); a rejected step
 * uses h *= max(0.2, safety/sqrt(err)); a Newton failure quarters h.  The
 * step is clipped to land on dt exactly.  Fails when h < 1e-12 dt or the
 * number of substep attempts reaches max_substeps.  The proposed next
 * length after the last substep is the same update of the accepted length;
 * when that substep was clipped to land on dt, the unclipped length is kept
 * if it is larger.  Fixed mode: n_fixed substeps of dt / n_fixed.  Replay
 * mode: the n_replay given lengths in order, no error control. */
static int integrate_attempt(const kro_net *n, const kro_opts *o, const double *y0,
                             const double *atol, double dt, const kro_rad *rad, attempt_params ap,
                             const double *replay, int64_t replay_ld, int32_t n_replay,
                             double *y_out, int32_t *st, substep_log *lg) {
  const int N = n->S + 1;
  double yn[KRO_MAXN], y[KRO_MAXN], gn[KRO_MAXN], g[KRO_MAXN];
  memcpy(yn, y0, sizeof(double) * (size_t)N);
  lg->n = 0;
  lg->h_next = 0.0;
  if (o->mode == KRO_FIXED || o->mode == KRO_REPLAY) {
    const int m = o->mode == KRO_FIXED ? o->n_fixed : n_replay;
    for (int k = 0; k < m; ++k) {
      double h = o->mode == KRO_FIXED ? dt / (double)o->n_fixed : replay[k * replay_ld];
      if (be_substep_rad(n, o, yn, atol, h, rad, y, &st[1]) != 0) { st[3]++; return -1; }
      memcpy(yn, y, sizeof(double) * (size_t)N);
      st[0]++;
      log_substep(lg, h);
    }
    memcpy(y_out, yn, sizeof(double) * (size_t)N);
    return 0;
  }
  unknown_rates(n, yn, rad, gn);
  double t = 0.0, h = ap.h0;
  int attempts = 0;
  for (;;) {
    if (attempts >= o->max_substeps) return -1;
    int final = 0;
    double h_free = h;             /* the controller's length before the clip */
    if (h >= dt - t) { h = dt - t; final = 1; }
    else if (h < 1e-12 * dt) return -1;
    attempts++;
    if (be_substep_rad(n, o, yn, atol, h, rad, y, &st[1]) != 0) {
      st[3]++;
      h *= 0.25;
      continue;
    }
    unknown_rates(n, y, rad, g);
    double err = 0.0;
    for (int i = 0; i < N; ++i) {
      double w = atol[i] + o->rtol * fmax(fabs(yn[i]), fabs(y[i]));
      double e = fabs(0.5 * h * (g[i] - gn[i])) / w;
      if (e > err) err = e;
    }
    if (!isfinite(err)) { st[2]++; h *= 0.2; continue; }
    if (err <= 1.0) {
      memcpy(yn, y, sizeof(double) * (size_t)N);
      memcpy(gn, g, sizeof(double) * (size_t)N);
      st[0]++;
      log_substep(lg, h);
      double h_new = h * fmin(ap.growth, fmax(0.2, ap.safety / sqrt(fmax(err, 1e-10))));
      if (final) {
        lg->h_next = h_free > h_new ? h_free : h_new;
        break;
      }
      t += h;
      h = h_new;
    } else {
      st[2]++;
      h *= fmax(0.2, ap.safety / sqrt(err));
    }
  }
  memcpy(y_out, yn, sizeof(double) * (size_t)N);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* conservation, post-processing                                             */
/* ------------------------------------------------------------------------ */

static double nuclei(const kro_net *n, const double *nn) {
  double t = 0.0;
  for (int s = 0; s < n->S; ++s) {
    int atoms = 0;
    for (int v = 0; v < n->n_elem; ++v) atoms += n->comp[v * n->S + s];
    t += atoms * nn[s];
  }
  return t;
}

static void row_totals(const kro_net *n, const double *nn, double *E) {
  for (int v = 0; v < n->n_rows; ++v) {
    double t = 0.0;
    for (int s = 0; s < n->S; ++s) t += n->comp[v * n->S + s] * nn[s];
    E[v] = t;
  }
}

static double cell_element_residual(const kro_net *n, const double *before,
                                     const double *after) {
  double nn = nuclei(n, before), worst = 0.0;
  for (int v = 0; v < n->n_rows; ++v) {
    double diff = 0.0, D = 0.0;
    for (int s = 0; s < n->S; ++s) {
      diff += n->comp[v * n->S + s] * (after[s] - before[s]);
      D += abs(n->comp[v * n->S + s]) * before[s];
    }
    if (v >= n->n_elem) D = nn;
    double e = fabs(diff) / fmax(D, 1e-300);
    if (!(e <= worst)) worst = e;   /* NaN propagates */
  }
  return worst;
}

void kro_element_residual(const kro_net *n, int64_t n_cells, const double *before,
                          const double *after, int64_t ld, double *resid) {
  double b[KRO_MAXN], a[KRO_MAXN];
  for (int64_t c = 0; c < n_cells; ++c) {
    for (int s = 0; s < n->S; ++s) { b[s] = before[s * ld + c]; a[s] = after[s * ld + c]; }
    resid[c] = cell_element_residual(n, b, a);
  }
}

/* Stage 1: negative abundances become zero.  Stage 2: for each conserved row
 * in order, the row's reservoir species absorbs the difference between the
 * initial and current totals.  Stage 3: if a reservoir is then negative, the
 * most abundant species that carries the row with the reservoir's sign is
 * broken up into the reservoirs of all its rows, just enough to bring the
 * reservoir to zero (moving to the next most abundant if one is used up). */
int kro_postprocess_flags(const kro_net *n, const double *E0, double *nn) {
  const int S = n->S;
  int flags = 0;
  for (int s = 0; s < S; ++s)
    if (nn[s] < 0.0) { nn[s] = 0.0; flags |= KRO_POST_CLIPPED; }
  for (int v = 0; v < n->n_rows; ++v) {
    double E = 0.0;
    for (int s = 0; s < S; ++s) E += n->comp[v * S + s] * nn[s];
    int rs = n->res[v];
    nn[rs] += (E0[v] - E) / n->comp[v * S + rs];
  }
  for (int v = 0; v < n->n_rows; ++v) {
    int rs = n->res[v];
    int sign_r = n->comp[v * S + rs] > 0 ? 1 : -1;
    int used[KRO_MAXN] = {0};
    while (nn[rs] < 0.0) {
      int best = -1;
      for (int s = 0; s < S; ++s) {
        if (s == rs || used[s]) continue;
        int a = n->comp[v * S + s];
        if (a == 0 || (a > 0 ? 1 : -1) != sign_r) continue;
        if (nn[s] <= 0.0) continue;
        if (best < 0 || nn[s] > nn[best]) best = s;
      }
      if (best < 0) break;
      used[best] = 1;
      flags |= KRO_POST_BROKEN_UP;
      /* converting x of species `best` changes the reservoir of row v by
       * x * N_v,best / N_v,rs; the x that brings it to zero */
      double need = -nn[rs] * n->comp[v * S + rs] / n->comp[v * S + best];
      double x = need < nn[best] ? need : nn[best];
      nn[best] -= x;
      for (int u = 0; u < n->n_rows; ++u) {
        int a = n->comp[u * S + best];
        if (a) nn[n->res[u]] += x * a / n->comp[u * S + n->res[u]];
      }
      if (x == need) nn[rs] = 0.0;   /* drop the rounding residue */
    }
  }
  return flags;
}

void kro_postprocess(const kro_net *n, const double *E0, double *nn) {
  (void)kro_postprocess_flags(n, E0, nn);
}

double kro_fastest_timescale(const kro_net *n, const double *y) {
  const int S = n->S, N = S + 1;
  double J[KRO_MAXN * KRO_MAXN];
  jacobian_rad(n, y, NULL, J);
  /* the largest self-coupling rate: species diagonal, and the thermal mode
   * d(Q/c_V)/dT ~ (dQ/dT)/c_V */
  double m = 0.0;
  for (int s = 0; s < S; ++s) m = fmax(m, fabs(J[s * N + s]));
  double cv = heat_capacity(n, y);
  if (cv > 0.0) m = fmax(m, fabs(J[S * N + S]) / cv);
  if (!(m > 0.0) || !isfinite(m)) return 1e7;
  double tau = 1.0 / m;
  return tau < 1e7 ? tau : 1e7;
}

/* ------------------------------------------------------------------------ */
/* per-cell driver                                                           */
/* ------------------------------------------------------------------------ */

static int cell_ok(const kro_net *n, const double *before, const double *y, double n_nuc) {
  for (int i = 0; i <= n->S; ++i)
    if (!isfinite(y[i])) return 0;
  for (int s = 0; s < n->S; ++s)
    if (y[s] < -1e-10 * n_nuc) return 0;
  return cell_element_residual(n, before, y) <= 1e-10;
}

/* The per-cell extras of kro_integrate_ex for one cell (pointers already
 * offset to the cell; any may be NULL). */
typedef struct {
  double *h_hint;       /* in/out */
  double *h_log;        /* [cap] with stride log_ld */
  int64_t log_ld;
  int32_t cap;
  int32_t *h_log_n;
  int32_t *post;
  kro_rad rad;          /* the cell's radiation field (F = 0: none) */
} cell_extras;

static int32_t integrate_cell(const kro_net *n, const kro_opts *o, double *nn,
                              double *T, double rho, double dt, int32_t *st,
                              const cell_extras *ex) {
  const int S = n->S;
  double y0[KRO_MAXN], y[KRO_MAXN], atol[KRO_MAXN], E0[KRO_MAXN];
  if (ex->h_log_n && o->mode != KRO_REPLAY) *ex->h_log_n = 0;
  if (ex->post) *ex->post = 0;
  /* non-finite input: leave the cell as it came */
  int bad = !isfinite(*T) || !isfinite(dt) || !(dt >= 0.0);
  for (int s = 0; s < S; ++s) bad |= !isfinite(nn[s]);
  if (bad) return 2;
  /* pre-processing (Sec. 2.2.2): floors, density floor rescale, T limits */
  for (int s = 0; s < S; ++s) y0[s] = nn[s] > 0.0 ? nn[s] : 0.0;
  if (o->rho_floor > 0.0 && rho > 0.0 && rho < o->rho_floor)
    for (int s = 0; s < S; ++s) y0[s] *= o->rho_floor / rho;
  y0[S] = fmin(fmax(*T, n->T_min), n->T_max);
  if (dt == 0.0) {
    for (int s = 0; s < S; ++s) nn[s] = y0[s];
    *T = y0[S];
    return 0;
  }
  row_totals(n, y0, E0);
  double n_nuc = nuclei(n, y0);
  for (int s = 0; s < S; ++s) atol[s] = o->floor * n_nuc;
  atol[S] = 0.0;

  /* replay: the recorded substep lengths are the input; otherwise the
   * accepted lengths are recorded (entries past the final count keep
   * whatever an earlier attempt wrote) */
  const double *replay = NULL;
  int32_t n_replay = 0;
  substep_log lg = {NULL, ex->log_ld, 0, 0, 0.0};
  if (o->mode == KRO_REPLAY) {
    if (!ex->h_log || !ex->h_log_n || *ex->h_log_n < 0 || *ex->h_log_n > ex->cap) return 2;
    n_replay = *ex->h_log_n;
    replay = ex->h_log;
  } else if (ex->h_log) {
    lg.h = ex->h_log;
    lg.cap = ex->cap;
  }

  /* attempt 0 (first substep: the caller's hint when positive, else dt),
   * then the retry with a reduced initial step and tighter step control,
   * then reversion to the pre-evolution values (Sec. 2.2.3) */
  double h0 = dt;
  if (ex->h_hint && *ex->h_hint > 0.0 && isfinite(*ex->h_hint)) h0 = *ex->h_hint;
  attempt_params ap[2] = {{h0, 0.9, 5.0}, {dt / 100.0, 0.5, 2.0}};
  int32_t status = 2;
  for (int a = 0; a < 2; ++a) {
    if (integrate_attempt(n, o, y0, atol, dt, &ex->rad, ap[a], replay, ex->log_ld, n_replay, y, st, &lg) == 0 &&
        cell_ok(n, y0, y, n_nuc)) {
      status = a;
      break;
    }
    if (o->mode != KRO_ADAPTIVE) break;   /* a given sequence has no retry */
  }
  if (status == 2) return 2;
  int flags = kro_postprocess_flags(n, E0, y);
  for (int s = 0; s < S; ++s) nn[s] = y[s];
  *T = y[S];
  if (ex->post) *ex->post = flags;
  if (o->mode != KRO_REPLAY && ex->h_log_n) *ex->h_log_n = lg.n;
  if (ex->h_hint && o->mode == KRO_ADAPTIVE) *ex->h_hint = lg.h_next;
  return status;
}

int kro_integrate_ex(const kro_net *n, int64_t n_cells, double *states, int64_t ld,
                     double *T, const double *rho, const double *dt, double dt_scalar,
                     const kro_opts *o, int32_t *status, int32_t *cell_stats,
                     const kro_extras *ex, int nthreads) {
  if (!n || !states || !T || ld < n_cells || n_cells < 0 || !o) return -1;
  if (o->mode == KRO_FIXED && o->n_fixed < 1) return -1;
  if (o->mode != KRO_ADAPTIVE && o->mode != KRO_FIXED && o->mode != KRO_REPLAY) return -1;
  kro_extras none;
  memset(&none, 0, sizeof none);
  if (!ex) ex = &none;
  if (ex->h_log && (ex->h_log_ld < n_cells || ex->h_log_cap < 0)) return -1;
  if (o->mode == KRO_REPLAY && (!ex->h_log || !ex->h_log_n)) return -1;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
#endif
  for (int64_t c = 0; c < n_cells; ++c) {
    double nn[KRO_MAXN];
    int32_t st[4] = {0, 0, 0, 0};
    for (int s = 0; s < n->S; ++s) nn[s] = states[s * ld + c];
    double Tc = T[c];
    double step = dt ? dt[c] : dt_scalar;
    cell_extras ce = {ex->h_hint ? ex->h_hint + c : NULL, ex->h_log ? ex->h_log + c : NULL,
                      ex->h_log_ld, ex->h_log_cap, ex->h_log_n ? ex->h_log_n + c : NULL,
                      ex->post ? ex->post + c : NULL,
                      {ex->photo_flux ? ex->photo_flux[c] : 0.0, ex->photo_length ? ex->photo_length[c] : 0.0}};
    int32_t code = integrate_cell(n, o, nn, &Tc, rho ? rho[c] : 0.0, step, st, &ce);
    if (code != 2) {
      for (int s = 0; s < n->S; ++s) states[s * ld + c] = nn[s];
      T[c] = Tc;
    }
    if (status) status[c] = code;
    if (cell_stats) memcpy(cell_stats + 4 * c, st, sizeof(st));
  }
  (void)nthreads;
  return 0;
}

int kro_integrate(const kro_net *n, int64_t n_cells, double *states, int64_t ld,
                  double *T, const double *rho, const double *dt, double dt_scalar,
                  const kro_opts *o, int32_t *status, int32_t *cell_stats, int nthreads) {
  return kro_integrate_ex(n, n_cells, states, ld, T, rho, dt, dt_scalar, o, status, cell_stats,
                          NULL, nthreads);
}
