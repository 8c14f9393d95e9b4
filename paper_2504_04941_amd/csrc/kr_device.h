/*
 * kr_device.h -- device code of the per-cell implicit integrator (gfx950).
 *
 * This text is compiled together with the network-specific section that the
 * network compiler generates (species count, conserved rows, heat
 * capacities, and the straight-line rate/Jacobian function kr_eval).  The
 * generated section defines:
 *   KR_S, KR_NROWS, KR_NELEM            sizes
 *   kr_comp[KR_NROWS][KR_S], kr_res[KR_NROWS], kr_cv[KR_S],
 *   kr_atoms[KR_S], kr_T_min, kr_T_max  constant tables
 *   kr_eval(y, g, J)                    g = (dn/dt, Q), J = dg/dy at
 *                                       y = (n_1..n_S, T)
 *
 * Mapping to the hardware.  One cell per lane: the Newton matrix of a cell
 * (N = S + 1 unknowns) lives in the lane's VGPRs, every index is a
 * compile-time constant, and a wave advances 64 independent cells.  Lanes
 * run a small state machine (fresh cell / start substep / Newton iteration /
 * error check / restart) whose expensive part -- rate and Jacobian
 * evaluation, assembly and the LU solve -- is the same code for every lane
 * in every loop trip, so lanes at different substeps, Newton iterations or
 * retry attempts never diverge in the heavy part.  A lane whose cell is
 * finished claims the next cell from a global atomic counter (work
 * stealing at lane granularity), so cells of very uneven stiffness keep all
 * 64 lanes busy until the queue drains.
 *
 * The method (paper Sec. 2.2): backward Euler substeps
 *   R_s = n_s - n_s^(n) - h f_s(y),  R_E = eps(y) - eps^(n) - h Q(y),
 *   eps = T sum_s c_s n_s,
 * solved by Newton iteration (M d = -R, M = dR/dy from the analytic
 * Jacobian); adaptive step size from the local error estimate
 * (h/2)|g(y_new) - g(y_old)|; pre-processing (Sec. 2.2.2: floors, density
 * floor, temperature limits), post-processing (Sec. 2.2.3, three stages) and
 * the retry-then-revert ladder (Sec. 2.2.3).
 *
 * Linear solve (paper Sec. 2.3.2 / Algorithm algo:lu-decomp computes an LU
 * with implicit row scaling and partial pivoting).  Here the elimination is
 * right-looking on the lane's registers with threshold partial pivoting: the
 * diagonal is kept unless its scaled magnitude falls below KR_PIVOT_TAU of
 * the best scaled candidate below it.  A row exchange is only executed
 * (wave-uniformly, via predicated selects) when some lane of the wave needs
 * one, since per-lane data-dependent register indexing does not exist.  The
 * solution is the same vector as the paper's LU gives, up to rounding.
 */

#define KR_N (KR_S + 1)
#ifndef KR_PIVOT_TAU
#define KR_PIVOT_TAU 0.1
#endif

enum { KR_PH_NONE = 0, KR_PH_FRESH = 1, KR_PH_START = 2, KR_PH_NEWTON = 3,
       KR_PH_CHECK = 4, KR_PH_RESTART = 5, KR_PH_GUESS = 6 };

__device__ __forceinline__ bool kr_finite(double x) { return __builtin_isfinite(x); }

/* 1/x from the hardware estimate refined by two Newton steps (within an ulp
 * or so; not correctly rounded).  Used where a value feeds a comparison or a
 * scaling, never for results that are compared bit-for-bit. */
__device__ __forceinline__ double kr_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

/* 1/x within ~1e-15 relative: the hardware estimate (relative error up to
 * 2^-24 on gfx950) refined by one Newton step (measured on gfx950: within 11
 * ulp of the quotient).  For the weights of the error and Newton norms,
 * which only feed comparisons and the step-size factor. */
__device__ __forceinline__ double kr_rcp_w(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return fma(r, fma(-x, r, 1.0), r);
}

/* 1/x of the working precision: FP64 as kr_rcp, FP32 the hardware estimate
 * (1 ulp). */
__device__ __forceinline__ double kr_rcp_r(double x) { return kr_rcp(x); }
__device__ __forceinline__ float kr_rcp_r(float x) { return __builtin_amdgcn_rcpf(x); }

/* A lane's slot in a per-wave LDS array laid out [index][lane], so that a
 * wave's 64 accesses to one index hit 64 consecutive values. */
template <typename R>
struct KrSlotT {
  R *base;
  __device__ __forceinline__ R &operator[](int i) const { return base[i * 64]; }
};
typedef KrSlotT<double> KrSlot;

/* The cell's radiation field for the photoreactions (0, 0 without one):
 * optically thin photon flux and path length; false for an invalid one
 * (negative or non-finite). */
__device__ __forceinline__ bool kr_cell_rad(const KrParams &p, long long c, double &F, double &L) {
  F = p.photo_flux ? p.photo_flux[c] : 0.0;
  L = p.photo_length ? p.photo_length[c] : 0.0;
  return F >= 0.0 && L >= 0.0 && __builtin_isfinite(F) && __builtin_isfinite(L);
}

/* c_V = sum_s c_s(T) n_s at y (kr_thermo.h) */
template <typename R>
__device__ __forceinline__ R kr_heat_capacity(const R (&y)[KR_N]) {
  R c = R(0);
#if KR_CV_POLY
#pragma unroll
  for (int s = 0; s < KR_S; ++s) {
    R es, cs;
    kr_species_thermo(s, y[KR_S], es, cs);
    c += cs * y[s];
  }
#else
#pragma unroll
  for (int s = 0; s < KR_S; ++s) c += R(kr_cv[s]) * y[s];
#endif
  return c;
}

/* thermal energy eps = sum_s n_s e_s(T) at y (T c_V for constant heat
 * capacities) */
template <typename R>
__device__ __forceinline__ R kr_thermal_energy(const R (&y)[KR_N]) {
#if KR_CV_POLY
  R e = R(0);
#pragma unroll
  for (int s = 0; s < KR_S; ++s) {
    R es, cs;
    kr_species_thermo(s, y[KR_S], es, cs);
    e += es * y[s];
  }
  return e;
#else
  return y[KR_S] * kr_heat_capacity(y);
#endif
}

/* ------------------------------------------------------------------------ */
/* dense LU in registers                                                     */
/* ------------------------------------------------------------------------ */

/* Solves a x = b in place (b <- x) for one lane's matrix, by Gaussian
 * elimination of the augmented system with threshold partial pivoting.
 * Returns false for a zero row or a zero / non-finite pivot. */
template <typename R>
__device__ __forceinline__ bool kr_lu_solve(R (&a)[KR_N][KR_N], R (&b)[KR_N],
                                            unsigned long long *swap_count) {
  /* inverse row scales only steer the pivot choice: FP32 is plenty */
  float sc[KR_N];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < KR_N; ++i) {
    R v = R(0);
#pragma unroll
    for (int k = 0; k < KR_N; ++k) v = fmax(v, fabs(a[i][k]));
    ok = ok && (v > R(0)) && kr_finite((double)v);
    sc[i] = __builtin_amdgcn_rcpf((float)v);
  }
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    /* largest scaled candidate below the diagonal; its row index is only
     * needed when some lane of the wave exchanges rows */
    float best = 0.0f;
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) best = fmaxf(best, (float)fabs(a[i][j]) * sc[i]);
    bool need = (float)fabs(a[j][j]) * sc[j] < (float)KR_PIVOT_TAU * best;
    unsigned long long mask = __ballot(need);
    if (mask) {
      int bi = j;
      float bb = 0.0f;
#pragma unroll
      for (int i = j + 1; i < KR_N; ++i) {
        float t = (float)fabs(a[i][j]) * sc[i];
        if (t > bb) { bb = t; bi = i; }
      }
      if (swap_count && __lane_id() == (int)__builtin_ctzll(__ballot(1)))
        atomicAdd(swap_count, (unsigned long long)__popcll(mask));
#pragma unroll
      for (int i = j + 1; i < KR_N; ++i) {
        bool sw = need && bi == i;
#pragma unroll
        for (int k = j; k < KR_N; ++k) {
          R u = a[j][k], w = a[i][k];
          a[j][k] = sw ? w : u;
          a[i][k] = sw ? u : w;
        }
        R u = b[j], w = b[i];
        b[j] = sw ? w : u;
        b[i] = sw ? u : w;
        float su = sc[j], sw2 = sc[i];
        sc[j] = sw ? sw2 : su;
        sc[i] = sw ? su : sw2;
      }
    }
    const R piv = a[j][j];
    ok = ok && (piv != R(0)) && kr_finite((double)piv);
    const R d = kr_rcp_r(piv);
    a[j][j] = d;                      /* reciprocal pivot kept on the diagonal */
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) {
      const R l = a[i][j] * d;
#pragma unroll
      for (int k = j + 1; k < KR_N; ++k) a[i][k] = fma(-l, a[j][k], a[i][k]);
      b[i] = fma(-l, b[j], b[i]);
    }
  }
#pragma unroll
  for (int i = KR_N - 1; i >= 0; --i) {
    R x = b[i];
#pragma unroll
    for (int k = i + 1; k < KR_N; ++k) x = fma(-a[i][k], b[k], x);
    b[i] = x * a[i][i];
  }
  return ok;
}

/* FP32 factorisation kept for several right-hand sides: L (unit, below the
 * diagonal), U (on and above, with reciprocal pivots in dinv) and the row
 * exchange taken at each column in perm. */
__device__ __forceinline__ bool kr_lu_factor32(float (&a)[KR_N][KR_N], float (&dinv)[KR_N],
                                               int (&perm)[KR_N],
                                               unsigned long long *swap_count) {
  float sc[KR_N];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < KR_N; ++i) {
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < KR_N; ++k) v = fmaxf(v, fabsf(a[i][k]));
    ok = ok && (v > 0.0f) && __builtin_isfinite(v);
    /* hardware reciprocal estimates (about an ulp) here and for the pivots:
     * the FP64 refinement corrects the factorisation's rounding anyway */
    sc[i] = __builtin_amdgcn_rcpf(v);
  }
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    float best = 0.0f;
    int bi = j;
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) {
      float t = fabsf(a[i][j]) * sc[i];
      if (t > best) { best = t; bi = i; }
    }
    bool need = fabsf(a[j][j]) * sc[j] < (float)KR_PIVOT_TAU * best;
    perm[j] = need ? bi : j;
    unsigned long long mask = __ballot(need);
    if (mask) {
      if (swap_count && __lane_id() == (int)__builtin_ctzll(__ballot(1)))
        atomicAdd(swap_count, (unsigned long long)__popcll(mask));
#pragma unroll
      for (int i = j + 1; i < KR_N; ++i) {
        bool sw = need && bi == i;
#pragma unroll
        for (int k = 0; k < KR_N; ++k) {
          float u = a[j][k], w = a[i][k];
          a[j][k] = sw ? w : u;
          a[i][k] = sw ? u : w;
        }
        float su = sc[j], sw2 = sc[i];
        sc[j] = sw ? sw2 : su;
        sc[i] = sw ? su : sw2;
      }
    }
    float piv = a[j][j];
    ok = ok && (piv != 0.0f) && __builtin_isfinite(piv);
    float d = __builtin_amdgcn_rcpf(piv);
    dinv[j] = d;
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) {
      float l = a[i][j] * d;
      a[i][j] = l;
#pragma unroll
      for (int k = j + 1; k < KR_N; ++k) a[i][k] = fmaf(-l, a[j][k], a[i][k]);
    }
  }
  return ok;
}

__device__ __forceinline__ void kr_lu_apply32(const float (&a)[KR_N][KR_N], const float (&dinv)[KR_N],
                                              const int (&perm)[KR_N], float (&b)[KR_N]) {
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) {
      bool sw = perm[j] == i;
      float u = b[j], w = b[i];
      b[j] = sw ? w : u;
      b[i] = sw ? u : w;
    }
#pragma unroll
    for (int i = j + 1; i < KR_N; ++i) b[i] = fmaf(-a[i][j], b[j], b[i]);
  }
#pragma unroll
  for (int i = KR_N - 1; i >= 0; --i) {
    float x = b[i];
#pragma unroll
    for (int k = i + 1; k < KR_N; ++k) x = fmaf(-a[i][k], b[k], x);
    b[i] = x * dinv[i];
  }
}

/* ------------------------------------------------------------------------ */
/* conservation, pre- and post-processing                                    */
/* ------------------------------------------------------------------------ */

__device__ __forceinline__ double kr_nuclei(const double (&y)[KR_N]) {
  double t = 0.0;
#pragma unroll
  for (int s = 0; s < KR_S; ++s) t += kr_atoms[s] * y[s];
  return t;
}

/* Loads the cell's input and applies the pre-processing of Sec. 2.2.2:
 * negative abundances to zero, optional density-floor rescaling, T limits.
 * Returns false for a non-finite input (the cell is then left untouched). */
__device__ __forceinline__ bool kr_load_input(const KrParams &p, long long c, double (&y0)[KR_N],
                                              double &dt) {
  bool ok = true;
#pragma unroll
  for (int s = 0; s < KR_S; ++s) {
    double v = p.states[(long long)s * p.ld + c];
    ok = ok && kr_finite(v);
    y0[s] = v > 0.0 ? v : 0.0;
  }
  double T = p.T[c];
  dt = p.dt ? p.dt[c] : p.dt_scalar;
  ok = ok && kr_finite(T) && kr_finite(dt) && dt >= 0.0;
  if (p.rho_floor > 0.0 && p.rho) {
    double rho = p.rho[c];
    if (rho > 0.0 && rho < p.rho_floor) {
      double f = p.rho_floor / rho;
#pragma unroll
      for (int s = 0; s < KR_S; ++s) y0[s] *= f;
    }
  }
  y0[KR_S] = fmin(fmax(T, kr_T_min), kr_T_max);
  return ok;
}

__device__ __forceinline__ double kr_element_resid(const double (&y0)[KR_N], const double (&y)[KR_N]) {
  const double nn = kr_nuclei(y0);
  double worst = 0.0;
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    double diff = 0.0, D = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s) {
      if (kr_comp[v][s] == 0) continue;
      diff += kr_comp[v][s] * (y[s] - y0[s]);
      D += (kr_comp[v][s] > 0 ? kr_comp[v][s] : -kr_comp[v][s]) * y0[s];
    }
    if (v >= KR_NELEM) D = nn;
    double e = fabs(diff) / fmax(D, 1e-300);
    if (!(e <= worst)) worst = e;
  }
  return worst;
}

/* Post-processing of Sec. 2.2.3: (1) negatives to zero; (2) each conserved
 * row's reservoir absorbs the difference to the initial totals E0; (3) a
 * reservoir left negative is refilled by breaking up the most abundant
 * species carrying that row (with the reservoir's sign) into the reservoirs
 * of all its rows, just enough.  All indexing is static: data-dependent
 * choices are applied through predicated updates, and the break-up loop
 * runs a wave-uniform number of trips (while any lane still has a negative
 * reservoir), each lane's trip predicated.  Returns which stages changed
 * anything: 1 a clip, 2 a break-up. */
__device__ __forceinline__ int kr_postprocess(const double (&E0)[KR_NROWS > 0 ? KR_NROWS : 1],
                                              double (&y)[KR_N]) {
  int flags = 0;
#pragma unroll
  for (int s = 0; s < KR_S; ++s) {
    flags |= y[s] < 0.0 ? 1 : 0;
    y[s] = y[s] < 0.0 ? 0.0 : y[s];
  }
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    double E = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s)
      if (kr_comp[v][s] != 0) E += kr_comp[v][s] * y[s];
    y[kr_res[v]] += (E0[v] - E) / kr_comp[v][kr_res[v]];
  }
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const int rs = kr_res[v];
    const int sr = kr_comp[v][rs] > 0 ? 1 : -1;
    unsigned long long used = 0ull;
#pragma unroll 1
    for (int it = 0; it < KR_S; ++it) {
      const bool neg = y[rs] < 0.0;
      if (!__any(neg)) break;                       /* wave-uniform exit */
      int best = -1;
      double bval = 0.0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s) {
        const int a = kr_comp[v][s];
        if (s == rs || a == 0 || (a > 0 ? 1 : -1) != sr) continue;
        bool cand = !((used >> s) & 1ull) && y[s] > 0.0 && (best < 0 || y[s] > bval);
        best = cand ? s : best;
        bval = cand ? y[s] : bval;
      }
      /* this lane's trip acts only while its reservoir is negative and a
       * species is left to break up */
      const bool act = neg && best >= 0;
      double na = 1.0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s) na = (s == best) ? (double)kr_comp[v][s] : na;
      const double need = -y[rs] * kr_comp[v][rs] / na;
      const double x = act ? (need < bval ? need : bval) : 0.0;
      used |= act ? (1ull << (best & 63)) : 0ull;
      flags |= act ? 2 : 0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s)
        if (s == best && act) y[s] -= x;
#pragma unroll
      for (int u = 0; u < KR_NROWS; ++u) {
        double au = 0.0;
#pragma unroll
        for (int s = 0; s < KR_S; ++s) au = (s == best) ? (double)kr_comp[u][s] : au;
        if (act) y[kr_res[u]] += x * au / kr_comp[u][kr_res[u]];
      }
      if (act && x == need) y[rs] = 0.0;
    }
  }
  return flags;
}

/* Weighted element projection of a Newton update (FP32 form): corrects d_S
 * so that the new iterate y + d carries the conserved totals of the substep
 * start y_n, d <- d - W N^T (N W N^T)^-1 (N d + N (y - y_n)) with W =
 * diag(max(|y_s|, atol)).  The exact Newton update of a conserving network
 * satisfies N (y + d) = N y_n (the rows of N annihilate the rates), whatever
 * the starting point -- a learned guess need not conserve; this restores it
 * after the FP32 factorisation.  (The paper's projector P = V V^T is the
 * W = I case, applied to a d whose start already conserves.) */
/* the correction of d for the conserved-row misfit r = N (y + d) - target,
 * in the working precision R: d <- d - W N^T (N W N^T)^-1 r */
template <typename R>
__device__ __forceinline__ void kr_project_core(const R (&y)[KR_N], R atol, R (&r)[KR_NROWS > 0 ? KR_NROWS : 1],
                                                R (&d)[KR_N]) {
  constexpr int V = KR_NROWS > 0 ? KR_NROWS : 1;
  constexpr R tiny = sizeof(R) == 4 ? R(1e-37) : R(1e-300);
  R W[KR_S];
#pragma unroll
  for (int s = 0; s < KR_S; ++s) W[s] = fmax(fabs(y[s]), atol);
  R G[V][V];
#pragma unroll
  for (int a = 0; a < V; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      R g = R(0);
#pragma unroll
      for (int s = 0; s < KR_S; ++s)
        if (kr_comp[a][s] != 0 && kr_comp[b][s] != 0) g += (R)(kr_comp[a][s] * kr_comp[b][s]) * W[s];
      G[a][b] = g;
    }
  }
  /* Cholesky of the SPD row Gram matrix */
#pragma unroll
  for (int a = 0; a < V; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      R t = G[a][b];
#pragma unroll
      for (int k = 0; k < b; ++k) t -= G[a][k] * G[b][k];
      if (a == b) G[a][a] = sqrt(fmax(t, tiny));
      else G[a][b] = t / G[b][b];
    }
  }
#pragma unroll
  for (int a = 0; a < V; ++a) {
    R t = r[a];
#pragma unroll
    for (int k = 0; k < a; ++k) t -= G[a][k] * r[k];
    r[a] = t / G[a][a];
  }
#pragma unroll
  for (int a = V - 1; a >= 0; --a) {
    R t = r[a];
#pragma unroll
    for (int k = a + 1; k < V; ++k) t -= G[k][a] * r[k];
    r[a] = t / G[a][a];
  }
#pragma unroll
  for (int s = 0; s < KR_S; ++s) {
    R t = R(0);
#pragma unroll
    for (int a = 0; a < V; ++a)
      if (kr_comp[a][s] != 0) t += (R)kr_comp[a][s] * r[a];
    d[s] -= W[s] * t;
  }
}

__device__ __forceinline__ void kr_project(const double (&y)[KR_N], const double (&yn)[KR_N], double atol,
                                           double (&d)[KR_N]) {
  if (KR_NROWS == 0) return;
  double r[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
  for (int a = 0; a < KR_NROWS; ++a) {
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s)
      if (kr_comp[a][s] != 0) t += kr_comp[a][s] * (d[s] + (y[s] - yn[s]));
    r[a] = t;
  }
  kr_project_core(y, atol, r, d);
}

/* The same projection onto fixed totals E (the cell's input totals), in the
 * working precision: the single- and mixed-precision integrations keep
 * every iterate within a rounding of the input's conserved totals, where a
 * projection onto the substep start would let the FP32 roundings of
 * thousands of substeps add up. */
template <typename R>
__device__ __forceinline__ void kr_project_to(const R (&y)[KR_N], const KrSlotT<R> &E, R atol, R (&d)[KR_N]) {
  if (KR_NROWS == 0) return;
  R r[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
  for (int a = 0; a < KR_NROWS; ++a) {
    R t = -E[a];
#pragma unroll
    for (int s = 0; s < KR_S; ++s)
      if (kr_comp[a][s] != 0) t += (R)kr_comp[a][s] * (y[s] + d[s]);
    r[a] = t;
  }
  kr_project_core(y, atol, r, d);
}

/* ------------------------------------------------------------------------ */
/* the integrator                                                            */
/* ------------------------------------------------------------------------ */

/* Working precision of the integrator's per-substep arithmetic (rates,
 * Jacobian, Newton matrix, LU and solve, iterate, error estimate):
 *   KR_P_FP64   plain FP64
 *   KR_P_FP32LU FP64, but the LU in FP32 with FP64 refinement and projection
 *   KR_P_SINGLE the paper's full single-precision mode: FP32 throughout the
 *               cell's integration (the substep clock h, t and the norms'
 *               weights stay FP64)
 *   KR_P_MIXED  the paper's mixed-precision mode: as KR_P_SINGLE, with the
 *               final abundance update of the call in FP64 (n_out = n_in +
 *               (y_end - y_start), the change taken in FP32)
 * The checks that send a cell to the retry scale with the working
 * precision: an element residual above 1e-10 (FP64) or 1e-5 (FP32), an
 * abundance below -1e-10 (FP64) or -1e-5 (FP32) times the nuclei density.
 * FP32 Newton iterations also stop when the update no longer moves the
 * iterate beyond 4 FP32 ulps (it cannot get smaller in that precision). */
enum { KR_P_FP64 = 0, KR_P_FP32LU = 1, KR_P_SINGLE = 2, KR_P_MIXED = 3 };

template <int PREC> struct KrReal { typedef double type; };
template <> struct KrReal<KR_P_SINGLE> { typedef float type; };
template <> struct KrReal<KR_P_MIXED> { typedef float type; };

template <typename R>
struct KrLaneT {
  long long cell;
  KrSlotT<R> y, yn, gn;         /* iterate, substep start and its rates: LDS */
  KrSlotT<R> e0;                /* FP32 modes: the input's conserved totals (LDS) */
  KrSlot hx;                    /* LDS: [0] the controller's length before the
                                   last substep was clipped to land on dt,
                                   then the proposed next length */
  double h, t, dt, atol, eps_n, prev, safety, growth;
  int phase, attempt, k, grow, attempts, fin;
  int acc0;                     /* accepted substeps before this attempt */
  int gstate;                   /* 1 guess pending, 2 Newton running from it */
  int acc, iters, rej, nfail;
#if KR_PHOTO
  double phF, phL;              /* the cell's radiation field */
#endif
};
typedef KrLaneT<double> KrLane;

template <typename R>
__device__ __forceinline__ void kr_start_attempt(const KrParams &p, KrLaneT<R> &L, const double (&y0)[KR_N]) {
  R yr[KR_N];
#pragma unroll
  for (int i = 0; i < KR_N; ++i) { yr[i] = (R)y0[i]; L.y[i] = yr[i]; L.yn[i] = yr[i]; }
  if constexpr (sizeof(R) == 4) {
#pragma unroll
    for (int v = 0; v < KR_NROWS; ++v) {
      double t = 0.0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s)
        if (kr_comp[v][s] != 0) t += kr_comp[v][s] * y0[s];
      L.e0[v] = (R)t;
    }
  }
  L.eps_n = kr_thermal_energy(yr);
  L.t = 0.0;
  if (p.mode == 1) {
    L.h = L.dt / (double)p.n_fixed;
  } else if (L.attempt == 0) {
    /* the caller's first-substep length when positive and finite (a cell
     * carries its step across calls), else dt */
    double h0 = L.dt;
    if (p.h_hint) {
      const double hh = p.h_hint[L.cell];
      h0 = (hh > 0.0 && kr_finite(hh)) ? hh : h0;
    }
    L.h = h0; L.safety = 0.9; L.growth = 5.0;
  } else {
    L.h = L.dt / 100.0; L.safety = 0.5; L.growth = 2.0;
  }
  L.attempts = 0;
  L.fin = 0;
  L.acc0 = L.acc;
  L.phase = KR_PH_FRESH;
}

/* Status, statistics, substep-log count and per-call totals of a finished
 * cell (nlog: accepted substeps of the attempt that produced the result, 0
 * for a reverted cell or one with nothing to integrate; resid: its element
 * residual after post-processing, 0 if it has none). */
template <typename R>
__device__ __forceinline__ void kr_write_outcome(const KrParams &p, const KrLaneT<R> &L, int code, int nlog,
                                                 double resid) {
  if (p.status) p.status[L.cell] = code;
  if (p.cell_stats) {
    int *st = p.cell_stats + 4 * L.cell;
    st[0] = L.acc; st[1] = L.iters; st[2] = L.rej; st[3] = L.nfail;
  }
  if (p.h_log_n) p.h_log_n[L.cell] = nlog;
  if (p.totals) {
    unsigned long long *t = p.totals;
    atomicAdd(&t[KR_TOT_CELLS], 1ull);
    atomicAdd(&t[KR_TOT_SUBSTEPS], (unsigned long long)L.acc);
    atomicAdd(&t[KR_TOT_ITERS], (unsigned long long)L.iters);
    atomicAdd(&t[KR_TOT_REJECTED], (unsigned long long)L.rej);
    atomicAdd(&t[KR_TOT_NFAIL], (unsigned long long)L.nfail);
    if (code == 1) atomicAdd(&t[KR_TOT_RETRIED], 1ull);
    if (code == 2) atomicAdd(&t[KR_TOT_REVERTED], 1ull);
    /* non-negative doubles order like their bit patterns */
    if (resid > 0.0) atomicMax(&t[KR_TOT_MAXRESID], (unsigned long long)__double_as_longlong(resid));
  }
}

/* The attempt failed: retry once with a reduced first substep and tighter
 * step control, else revert (inputs untouched, status 2). */
template <typename R>
__device__ __forceinline__ void kr_attempt_failed(const KrParams &p, KrLaneT<R> &L) {
  if (L.attempt == 0 && p.mode == 0) {
    double y0[KR_N], dt;
    kr_load_input(p, L.cell, y0, dt);
    L.attempt = 1;
    L.gstate = 0;
    kr_start_attempt(p, L, y0);
  } else {
    kr_write_outcome(p, L, 2, 0, 0.0);
    L.phase = KR_PH_NONE;
  }
}

template <int PREC, typename R>
__device__ __forceinline__ void kr_finish_cell(const KrParams &p, KrLaneT<R> &L) {
  double y0[KR_N], dt, y[KR_N];
  kr_load_input(p, L.cell, y0, dt);
#pragma unroll
  for (int i = 0; i < KR_N; ++i) {
    y[i] = (double)L.y[i];
    /* mixed precision: the change over the call, taken in the working
     * precision, added to the input in FP64 */
    if (PREC == KR_P_MIXED) y[i] = y0[i] + (y[i] - (double)(R)y0[i]);
  }
  const double nn = kr_nuclei(y0);
  constexpr double lim = sizeof(R) == 4 ? 1e-5 : 1e-10;
  bool ok = true;
#pragma unroll
  for (int i = 0; i < KR_N; ++i) ok = ok && kr_finite(y[i]);
#pragma unroll
  for (int s = 0; s < KR_S; ++s) ok = ok && !(y[s] < -lim * nn);
  ok = ok && kr_element_resid(y0, y) <= lim;
  if (!ok) { kr_attempt_failed(p, L); return; }
  double E0[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s)
      if (kr_comp[v][s] != 0) t += kr_comp[v][s] * y0[s];
    E0[v] = t;
  }
  kr_postprocess(E0, y);
#pragma unroll
  for (int s = 0; s < KR_S; ++s) p.states[(long long)s * p.ld + L.cell] = y[s];
  p.T[L.cell] = y[KR_S];
  if (p.h_hint && p.mode == 0) p.h_hint[L.cell] = L.hx[0];
  kr_write_outcome(p, L, L.attempt, L.acc - L.acc0, p.totals ? kr_element_resid(y0, y) : 0.0);
  L.phase = KR_PH_NONE;
}

/* Takes the next cell for an idle lane.  Returns false when none is left. */
template <typename R>
__device__ __forceinline__ bool kr_claim(const KrParams &p, KrLaneT<R> &L) {
  const unsigned long long c = atomicAdd(p.counter, 1ull);
  if (c >= (unsigned long long)p.n_cells) return false;
  L.cell = (long long)c;
  if (p.order) {
    const long long o = (long long)p.order[c];
    L.cell = o < p.n_cells ? o : L.cell;    /* range guard; always true */
  }
  L.acc = L.iters = L.rej = L.nfail = 0;
  L.attempt = 0;
  L.gstate = p.guess ? 1 : 0;
  double y0[KR_N], dt;
  if (!kr_load_input(p, L.cell, y0, dt)) {        /* non-finite input: revert */
    kr_write_outcome(p, L, 2, 0, 0.0);
    L.phase = KR_PH_NONE;
    return true;
  }
  L.dt = dt;
#if KR_PHOTO
  if (!kr_cell_rad(p, L.cell, L.phF, L.phL)) {      /* invalid radiation field: revert */
    kr_write_outcome(p, L, 2, 0, 0.0);
    L.phase = KR_PH_NONE;
    return true;
  }
#endif
  if (dt == 0.0) {                                  /* nothing to integrate */
#pragma unroll
    for (int s = 0; s < KR_S; ++s) p.states[(long long)s * p.ld + L.cell] = y0[s];
    p.T[L.cell] = y0[KR_S];
    kr_write_outcome(p, L, 0, 0, 0.0);
    L.phase = KR_PH_NONE;
    return true;
  }
  L.atol = p.floor * kr_nuclei(y0);
  kr_start_attempt(p, L, y0);
  return true;
}

template <typename R>
__device__ __forceinline__ double kr_weight(const KrParams &p, const KrLaneT<R> &L, int i, double yi) {
  const double a = i < KR_S ? L.atol : 0.0;
  return a + p.rtol * fmax(fabs((double)L.yn[i]), fabs(yi));
}

/* Newton failure: quarter the substep and restart it from y_n (adaptive);
 * a fixed substep sequence cannot shrink, so the attempt fails. */
template <typename R>
__device__ __forceinline__ void kr_newton_failed(const KrParams &p, KrLaneT<R> &L) {
  if (L.gstate == 2) {
    /* Newton failed from the learned guess: redo the same substep from
     * the plain starting point, without cutting the step */
    L.gstate = 0;
    if (p.counters) atomicAdd(&p.counters[1], 1ull);
#pragma unroll
    for (int i = 0; i < KR_N; ++i) L.y[i] = L.yn[i];
    L.attempts--;
    L.phase = KR_PH_RESTART;
    return;
  }
  L.nfail++;
  if (p.mode == 1) { kr_attempt_failed(p, L); return; }
  L.h *= 0.25;
#pragma unroll
  for (int i = 0; i < KR_N; ++i) L.y[i] = L.yn[i];
  L.phase = KR_PH_RESTART;
}

template <int PREC>
__device__ __forceinline__ void kr_integrate_body(const KrParams &p) {
  typedef typename KrReal<PREC>::type R;
  constexpr bool MIXED = PREC == KR_P_FP32LU;
  __shared__ R s_y[KR_N * 64], s_yn[KR_N * 64], s_gn[KR_N * 64];
  __shared__ double s_hx[64];
  __shared__ R s_e0[(sizeof(R) == 4 && KR_NROWS > 0 ? KR_NROWS : 1) * 64];
  KrLaneT<R> L;
  L.cell = -1;
  L.phase = KR_PH_NONE;
  L.y.base = s_y + threadIdx.x;
  L.yn.base = s_yn + threadIdx.x;
  L.gn.base = s_gn + threadIdx.x;
  L.hx.base = s_hx + threadIdx.x;
  L.e0.base = s_e0 + threadIdx.x;
  L.hx[0] = 0.0;
  bool exhausted = false;
#pragma unroll
  for (int i = 0; i < KR_N; ++i) { L.y[i] = R(1); L.yn[i] = R(1); L.gn[i] = R(0); }
  L.h = L.t = L.dt = L.atol = L.eps_n = L.prev = 0.0;
#if KR_PHOTO
  L.phF = L.phL = 0.0;
#endif
  L.safety = 0.9; L.growth = 5.0;
  L.attempt = L.k = L.grow = L.attempts = L.fin = L.gstate = L.acc0 = 0;
  L.acc = L.iters = L.rej = L.nfail = 0;
  unsigned long long *swaps = p.counters ? &p.counters[2] : nullptr;

  for (;;) {
    if (L.phase == KR_PH_NONE && !exhausted) exhausted = !kr_claim(p, L);
    const bool active = L.phase != KR_PH_NONE;
    if (!__any(active)) {
      if (__all(exhausted)) break;
      continue;
    }
    if (!active) continue;

    /* rates and Jacobian at the lane's current point */
    R g[KR_N], J[KR_N][KR_N], yv[KR_N];
#pragma unroll
    for (int i = 0; i < KR_N; ++i) yv[i] = L.y[i];
#if KR_PHOTO
    kr_eval(yv, g, J, (R)L.phF, (R)L.phL);
#else
    kr_eval(yv, g, J);
#endif
    /* heat capacity, thermal energy and d eps / d n_s = e_s(T) */
#if KR_CV_POLY
    R es[KR_S];
    R cv = R(0), eps = R(0);
#pragma unroll
    for (int s = 0; s < KR_S; ++s) {
      R cs;
      kr_species_thermo(s, yv[KR_S], es[s], cs);
      cv += cs * yv[s];
      eps += es[s] * yv[s];
    }
#define KR_ES(m) es[m]
#else
    const R cv = kr_heat_capacity(yv);
    const R eps = yv[KR_S] * cv;
#define KR_ES(m) (R(kr_cv[m]) * yv[KR_S])
#endif
    const R icv = kr_rcp_r(cv);
    const int ph = L.phase;

    if (ph == KR_PH_CHECK) {
      if (p.mode == 1) {                              /* fixed sequence */
#pragma unroll
        for (int i = 0; i < KR_N; ++i) L.yn[i] = yv[i];
        L.eps_n = eps;
        if (p.h_log && L.acc - L.acc0 < p.h_log_cap) p.h_log[(long long)(L.acc - L.acc0) * p.h_log_ld + L.cell] = L.h;
        L.acc++;
        if (L.acc >= p.n_fixed) kr_finish_cell<PREC>(p, L);
        else L.phase = KR_PH_START;
      } else {
        double err = 0.0;
        const R hh = (R)(0.5 * L.h);
#pragma unroll
        for (int i = 0; i < KR_N; ++i) {
          const R gi = i < KR_S ? g[i] : g[KR_S] * icv;
          const double e = (double)fabs(hh * (gi - L.gn[i])) * kr_rcp_w(kr_weight(p, L, i, (double)yv[i]));
          err = e > err ? e : err;
        }
        if (!kr_finite(err)) {
          L.rej++;
          L.h *= 0.2;
#pragma unroll
          for (int i = 0; i < KR_N; ++i) L.y[i] = L.yn[i];
          L.phase = KR_PH_RESTART;
        } else if (err <= 1.0) {
#pragma unroll
          for (int i = 0; i < KR_N; ++i) {
            L.yn[i] = yv[i];
            L.gn[i] = i < KR_S ? g[i] : g[KR_S] * icv;
          }
          L.eps_n = eps;
          if (p.h_log && L.acc - L.acc0 < p.h_log_cap) p.h_log[(long long)(L.acc - L.acc0) * p.h_log_ld + L.cell] = L.h;
          L.acc++;
          const double hnew = L.h * fmin(L.growth, fmax(0.2, L.safety / sqrt(fmax(err, 1e-10))));
          if (L.fin) {
            /* proposed next length: the controller's update of this
             * substep, or the unclipped length if that was larger */
            const double hf = L.hx[0];
            L.hx[0] = hf > hnew ? hf : hnew;
            kr_finish_cell<PREC>(p, L);
          } else {
            L.t += L.h;
            L.h = hnew;
            L.phase = KR_PH_START;
          }
        } else {
          L.rej++;
          L.h *= fmax(0.2, L.safety / sqrt(err));
#pragma unroll
          for (int i = 0; i < KR_N; ++i) L.y[i] = L.yn[i];
          L.phase = KR_PH_RESTART;
        }
      }
    } else if (ph == KR_PH_FRESH) {
#pragma unroll
      for (int i = 0; i < KR_N; ++i) L.gn[i] = i < KR_S ? g[i] : g[KR_S] * icv;
      L.phase = KR_PH_START;
    }

    if (L.phase == KR_PH_START) {                     /* y == y_n here */
      bool go = true;
      if (p.mode == 0) {
        if (L.attempts >= p.max_substeps) {
          go = false;
        } else {
          L.fin = 0;
          if (L.h >= L.dt - L.t) { L.hx[0] = L.h; L.h = L.dt - L.t; L.fin = 1; }
          else if (L.h < 1e-12 * L.dt) go = false;
        }
      }
      if (go) {
        L.attempts++;
        L.k = 0;
        L.grow = 0;
        L.prev = __builtin_inf();
        L.phase = KR_PH_NEWTON;
        if (L.gstate == 1) {
          /* first substep: start Newton from the learned guess (evaluated
           * on the next trip) */
#pragma unroll
          for (int i = 0; i < KR_N; ++i) L.y[i] = (R)p.guess[(long long)i * p.guess_ld + L.cell];
          L.gstate = 2;
          L.phase = KR_PH_GUESS;
          if (p.counters) atomicAdd(&p.counters[0], 1ull);
        }
      } else {
        kr_attempt_failed(p, L);
      }
    } else if (ph == KR_PH_GUESS) {
      L.phase = KR_PH_NEWTON;
    }

    if (L.phase == KR_PH_NEWTON) {
      /* residual and Newton matrix M = dR/dy, assembled over J in place */
      const R h = (R)L.h;
      R b[KR_N];
#pragma unroll
      for (int s = 0; s < KR_S; ++s) b[s] = -(yv[s] - L.yn[s] - h * g[s]);
      b[KR_S] = -(eps - (R)L.eps_n - h * g[KR_S]);
      if (ph == KR_PH_GUESS && L.gstate == 2) {
        /* residual gate: keep the learned starting point only if its BE
         * residual is smaller (weighted max norm) than the plain start's,
         * R(y_n) = -h (f(y_n), Q(y_n)) */
        double rg = 0.0, rp = 0.0;
#pragma unroll
        for (int s = 0; s < KR_S; ++s) {
          const double w = kr_rcp(L.atol + p.rtol * fabs((double)L.yn[s]));
          rg = fmax(rg, (double)fabs(b[s]) * w);
          rp = fmax(rp, L.h * (double)fabs(L.gn[s]) * w);
        }
        const double wE = kr_rcp(p.rtol * L.eps_n);
        rg = fmax(rg, (double)fabs(b[KR_S]) * wE);
        rp = fmax(rp, L.h * fabs((double)L.gn[KR_S] * L.eps_n / (double)L.yn[KR_S]) * wE);
        if (!(rg < rp)) {
          kr_newton_failed(p, L);   /* falls back to the plain start */
          goto kr_trip_end;
        }
      }
#pragma unroll
      for (int s = 0; s < KR_S; ++s)
#pragma unroll
        for (int m = 0; m < KR_N; ++m) J[s][m] = (s == m ? R(1) : R(0)) - h * J[s][m];
#pragma unroll
      for (int m = 0; m < KR_S; ++m) J[KR_S][m] = KR_ES(m) - h * J[KR_S][m];
      J[KR_S][KR_S] = cv - h * J[KR_S][KR_S];
      L.iters++;

      bool ok;
      if constexpr (!MIXED) {
        ok = kr_lu_solve(J, b, swaps);
        /* FP32 modes: the update lands on the input's conserved totals */
        if constexpr (sizeof(R) == 4) {
          if (ok) kr_project_to(yv, L.e0, (R)L.atol, b);
        }
      } else {
        /* FP32 LU of the row-equilibrated matrix; FP64 residual and
         * iterative refinement against the FP64 matrix; FP64 projection */
        float a32[KR_N][KR_N], dinv[KR_N];
        int perm[KR_N];
        double rs[KR_N];
#pragma unroll
        for (int i = 0; i < KR_N; ++i) {
          double v = 0.0;
#pragma unroll
          for (int k = 0; k < KR_N; ++k) v = fmax(v, fabs(J[i][k]));
          rs[i] = v > 0.0 ? 1.0 / v : 0.0;
#pragma unroll
          for (int k = 0; k < KR_N; ++k) a32[i][k] = (float)(J[i][k] * rs[i]);
        }
        bool ok32 = kr_lu_factor32(a32, dinv, perm, swaps);
        double d[KR_N];
#pragma unroll
        for (int i = 0; i < KR_N; ++i) d[i] = 0.0;
        double r[KR_N];
#pragma unroll
        for (int i = 0; i < KR_N; ++i) r[i] = b[i];
        bool conv = false;
        int sweeps = 0;
        /* the sweep loop's trip count is wave-uniform (it runs while any
         * lane still refines); each lane's sweep is predicated */
        bool live = ok32;
#pragma unroll 1
        for (int sweep = 0; sweep < 4; ++sweep) {
          if (!__any(live)) break;
          if (live) {
            sweeps = sweep + 1;
            float c32[KR_N];
#pragma unroll
            for (int i = 0; i < KR_N; ++i) c32[i] = (float)(r[i] * rs[i]);
            kr_lu_apply32(a32, dinv, perm, c32);
            double cn = 0.0;
#pragma unroll
            for (int i = 0; i < KR_N; ++i) {
              const double c = (double)c32[i];
              d[i] += c;
              const double e = fabs(c) * kr_rcp_w(kr_weight(p, L, i, L.y[i]));
              cn = e > cn ? e : cn;
            }
            if (!kr_finite(cn)) {
              ok32 = false;
              live = false;
            } else if (sweep > 0 && cn <= 1e-6) {
              conv = true;
              live = false;
            } else {
              /* r = b - M d in FP64 */
#pragma unroll
              for (int i = 0; i < KR_N; ++i) {
                double t = b[i];
#pragma unroll
                for (int k = 0; k < KR_N; ++k) t = fma(-J[i][k], d[k], t);
                r[i] = t;
              }
            }
          }
        }
        if (p.counters) atomicAdd(&p.counters[3], (unsigned long long)sweeps);
        /* an FP32 factorisation that broke down (zero, overflowing or
         * non-finite values) or a refinement that did not contract: FP64 LU
         * for those lanes */
        const bool need64 = !ok32 || !conv;
        ok = true;
        if (__any(need64)) {
          if (need64) {
            if (p.counters) atomicAdd(&p.counters[4], 1ull);
            ok = kr_lu_solve(J, b, swaps);
#pragma unroll
            for (int i = 0; i < KR_N; ++i) d[i] = b[i];
          }
        }
        double yc[KR_N], ync[KR_N];
#pragma unroll
        for (int i = 0; i < KR_N; ++i) { yc[i] = L.y[i]; ync[i] = L.yn[i]; }
        kr_project(yc, ync, L.atol, d);
#pragma unroll
        for (int i = 0; i < KR_N; ++i) b[i] = d[i];
      }

      if (!ok) {
        kr_newton_failed(p, L);
      } else {
        bool fin = true;
        double norm = 0.0;
        bool flat = true;   /* FP32: the update is within 4 ulps of the iterate */
#pragma unroll
        for (int i = 0; i < KR_N; ++i) {
          const R yo = L.y[i];
          const R yi = yo + b[i];
          L.y[i] = yi;
          fin = fin && kr_finite((double)b[i]) && kr_finite((double)yi);
          const double e = (double)fabs(b[i]) * kr_rcp_w(kr_weight(p, L, i, (double)yi));
          norm = e > norm ? e : norm;
          if (sizeof(R) == 4)
            flat = flat && (double)fabs(b[i]) <= 4.0 * 0x1p-23 * (double)fabs(yo) + (i < KR_S ? L.atol : 0.0);
        }
        if (!fin || !(L.y[KR_S] > R(0))) {
          kr_newton_failed(p, L);
        } else {
          if (norm <= p.newton_tol || (sizeof(R) == 4 && flat)) {
            L.phase = KR_PH_CHECK;
            L.gstate = 0;
          } else {
            bool failed = false;
            if (norm > L.prev) { if (++L.grow >= 2) failed = true; }
            else L.grow = 0;
            L.prev = norm;
            if (!failed && ++L.k >= p.max_newton) failed = true;
            if (failed) kr_newton_failed(p, L);
          }
        }
      }
    }

  kr_trip_end:
    if (L.phase == KR_PH_RESTART) L.phase = KR_PH_START;
  }
}
#undef KR_ES

#ifndef KR_WAVES_PER_EU
#define KR_WAVES_PER_EU 1
#endif

/* Expected-work bucket of each cell at its pre-processed input state
 * (kr_order.h): w = dt (sum_s |f_s| / sum_s n_s + |Q| / eps); cells that
 * are reverted or have nothing to integrate get bucket 0. */
__device__ __forceinline__ void kr_order_keys_body(const KrParams &p, unsigned char *bucket,
                                                   unsigned *hist) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < p.n_cells;
       c += (long long)gridDim.x * blockDim.x) {
    double y[KR_N], g[KR_N], J[KR_N][KR_N], dt;
    const bool ok = kr_load_input(p, c, y, dt);
    unsigned b = 0u;
    double F, L;
    if (ok && dt > 0.0 && kr_cell_rad(p, c, F, L)) {
      kr_eval(y, g, J, F, L);
      double sf = 0.0, sn = 0.0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s) {
        sf += fabs(g[s]);
        sn += y[s];
      }
      const double eps = kr_thermal_energy(y);
      b = kr_work_bucket(dt * (sf / sn + fabs(g[KR_S]) / eps));
    }
    bucket[c] = (unsigned char)b;
    atomicAdd(&hist[b], 1u);
  }
}

/* Fastest self-coupling timescale of each cell at its input state:
 * 1 / max(max_s |df_s/dn_s|, |dQ/dT| / c_V), capped at 1e7 s (workload set-up:
 * steps expressed in units of it). */
__device__ __forceinline__ void kr_timescale_body(const KrParams &p, double *out) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < p.n_cells;
       c += (long long)gridDim.x * blockDim.x) {
    double y[KR_N], g[KR_N], J[KR_N][KR_N], dt;
    kr_load_input(p, c, y, dt);
    double F, L;
    kr_cell_rad(p, c, F, L);
    kr_eval(y, g, J, F, L);
    double m = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s) m = fmax(m, fabs(J[s][s]));
    const double cv = kr_heat_capacity(y);
    if (cv > 0.0) m = fmax(m, fabs(J[KR_S][KR_S]) / cv);
    double tau = (m > 0.0 && kr_finite(m)) ? 1.0 / m : 1e7;
    out[c] = (kr_finite(tau) && tau < 1e7) ? tau : 1e7;
  }
}

/* Post-processing alone (Sec. 2.2.3) of the states in p.states, with the
 * conserved totals of `before` after pre-processing (negatives clipped); T
 * is not touched.  flags[c] (or null): 1 a clip, 2 a break-up.  All lanes
 * run every trip (cells past the end are predicated off). */
__device__ __forceinline__ void kr_post_body(const KrParams &p, const double *before, int *flags) {
  for (long long c0 = blockIdx.x * 64ll; c0 < p.n_cells; c0 += (long long)gridDim.x * 64ll) {
    const long long c = c0 + threadIdx.x;
    const bool in = c < p.n_cells;
    double y0[KR_N], y[KR_N];
#pragma unroll
    for (int s = 0; s < KR_S; ++s) {
      const double b = in ? before[(long long)s * p.ld + c] : 0.0;
      y0[s] = b > 0.0 ? b : 0.0;
      y[s] = in ? p.states[(long long)s * p.ld + c] : 0.0;
    }
    y0[KR_S] = y[KR_S] = 1.0;
    double E0[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
    for (int v = 0; v < KR_NROWS; ++v) {
      double t = 0.0;
#pragma unroll
      for (int s = 0; s < KR_S; ++s)
        if (kr_comp[v][s] != 0) t += kr_comp[v][s] * y0[s];
      E0[v] = t;
    }
    const int f = kr_postprocess(E0, y);
    if (in) {
#pragma unroll
      for (int s = 0; s < KR_S; ++s) p.states[(long long)s * p.ld + c] = y[s];
      if (flags) flags[c] = f;
    }
  }
}

#ifndef KR_NO_KERNELS
extern "C" __global__ void __launch_bounds__(64, 1) kr_post(KrParams p, const double *before, int *flags) {
  kr_post_body(p, before, flags);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_timescale(KrParams p, double *out) {
  kr_timescale_body(p, out);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_fp64(KrParams p) {
  kr_integrate_body<KR_P_FP64>(p);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_fp32lu(KrParams p) {
  kr_integrate_body<KR_P_FP32LU>(p);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_single(KrParams p) {
  kr_integrate_body<KR_P_SINGLE>(p);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_mixed(KrParams p) {
  kr_integrate_body<KR_P_MIXED>(p);
}

extern "C" __global__ void kr_reset_counter(unsigned long long *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_order_keys(KrParams p, unsigned char *bucket,
                                                                  unsigned *hist) {
  kr_order_keys_body(p, bucket, hist);
}
#endif /* KR_NO_KERNELS */
