/*
 * kr_group.h -- device code of the per-cell implicit integrator in the
 * lane-group layout (gfx950): one cell per group of KR_G lanes (16 or 32),
 * KR_H = 64 / KR_G cells per wavefront.
 *
 * Same method as the other two layouts (paper Sec. 2.2: backward-Euler
 * substeps solved by Newton iteration with the analytic Jacobian, adaptive
 * substeps, pre-/post-processing, retry then revert), for networks whose
 * Newton matrix fits a group with a lane to spare (N = S + 1 <= KR_G - 1):
 * between one cell per lane (whose matrix outgrows a lane's registers from
 * ~10 unknowns) and one cell per wavefront (whose LU and solves leave 64 - N
 * lanes idle).  Inside a group the data layout is the wavefront layout's
 * (kr_wide.h), on KR_G lanes:
 *
 *  - lane r of a group holds entry r of the cell's vectors and row r of its
 *    Newton matrix in registers;
 *  - rates: lane r evaluates directions r, r + KR_G, ... into the group's
 *    rate table P in LDS (the wavefront layout's direction tables, with the
 *    empty reactant slot remapped to the group's spare lane, KR_G - 1);
 *  - the rate Jacobian is gathered into the group's LDS block from
 *    contribution lists balanced over KR_G lanes (one owner per entry: no
 *    atomics, a fixed order per cell);
 *  - LU: per column a group arg-max (DPP within 16-lane rows, one swizzle
 *    across the two rows of a 32-lane group), the pivot row's entries
 *    shuffled from the pivot lane; rows are never moved.
 *
 * Control: the groups of a wavefront run different cells, so the per-cell
 * loops (attempts, substeps, Newton iterations) become a per-group state
 * machine over uniform trips of the wavefront, as in the lane layout
 * (kr_device.h): each trip evaluates rates and Jacobian once at every
 * group's current point, then each group takes its own step (error
 * estimate and acceptance, substep set-up, one Newton iteration); a group
 * whose cell is done claims the next one.  Every per-cell scalar is held
 * alike by the group's lanes (the same operations on the same values, so
 * group decisions agree lane by lane); branches are predicated per group,
 * cross-lane operations stay inside a group, and every loop trip count and
 * barrier is wavefront-uniform.
 *
 * Needs the wavefront layout's generated section and kr_wide.h (tables,
 * DPP helpers, reciprocal, per-cell kernels other than the integrator) and
 * the generated group section: KR_G, KR_GNDR (direction rounds of KR_G),
 * KR_GNC / KR_GNF (list lengths), kr_gdr (reactant slots, spare lane KR_G -
 * 1 for an empty slot), kr_gc / kr_gf (contribution lists interleaved by
 * group lane, entries as kr_wc).
 */

#define KR_H (64 / KR_G)
#define KR_GLOG (KR_G == 16 ? 4 : 5)
#define KR_GMASK (KR_G == 16 ? 0xFFFFu : 0xFFFFFFFFu)
static_assert(KR_G == 16 || KR_G == 32, "lane groups of 16 or 32 lanes");
static_assert(KR_N + 1 <= KR_G, "a group holds the N rows and one spare lane");

/* phase of a group's cell: none (idle), fresh (rates at the attempt's
 * start pending), start (substep set-up), Newton iteration, check (error
 * estimate at the converged point), restart (substep restarts from y_n) */
enum { KR_GPH_NONE = 0, KR_GPH_FRESH = 1, KR_GPH_START = 2, KR_GPH_NEWTON = 3, KR_GPH_CHECK = 4,
       KR_GPH_RESTART = 5 };

struct KrGBlock {
  double y[KR_G];                 /* published point (entries N.. are 1.0); during
                                     the gather one spare slot per lane */
  double P[5 * KR_GNDR * KR_G];   /* per direction: q, dq/dT, dq/dn (3 slots);
                                     the refinement's scratch vector after the
                                     gather */
  double J[KR_N * KR_LDJ];        /* Jacobian (as KrWave.J) */
};

__device__ __forceinline__ int kr_glane() { return (int)threadIdx.x & (KR_G - 1); }
__device__ __forceinline__ int kr_gbase() { return (int)threadIdx.x & ~(KR_G - 1); }

/* v of the group's lane src (the same src in every lane of the group) */
__device__ __forceinline__ double kr_gbc(double v, int src) { return __shfl(v, src, KR_G); }
__device__ __forceinline__ float kr_gbc(float v, int src) { return __shfl(v, src, KR_G); }
__device__ __forceinline__ int kr_gbc(int v, int src) { return __shfl(v, src, KR_G); }
__device__ __forceinline__ long long kr_gbc(long long v, int src) { return __shfl(v, src, KR_G); }

/* v of lane s of the lane's own group, s the same for every group (a
 * constant or a wavefront-uniform value): one readlane per group, no LDS
 * round trip */
template <typename F>
__device__ __forceinline__ F kr_gat(F v, int s) {
  F out = kr_wbc(v, s);
#pragma unroll
  for (int h = 1; h < KR_H; ++h) {
    const F x = kr_wbc(v, h * KR_G + s);
    out = (int)threadIdx.x >= h * KR_G ? x : out;
  }
  return out;
}

/* v of lane src of the lane's own group, src the same within each group:
 * the groups' sources are read out as scalars, then one readlane per
 * group (a short dependency chain, for the LU's and solves' critical
 * paths) */
template <typename F>
__device__ __forceinline__ F kr_gpick(F v, int src) {
  F out = kr_wbc(v, __builtin_amdgcn_readlane(src, 0));
#pragma unroll
  for (int h = 1; h < KR_H; ++h) {
    const F x = kr_wbc(v, h * KR_G + __builtin_amdgcn_readlane(src, h * KR_G));
    out = (int)threadIdx.x >= h * KR_G ? x : out;
  }
  return out;
}

/* v of the lane of the own group where c holds (its lowest such lane; lane
 * 0 of the group if none) */
template <typename F>
__device__ __forceinline__ F kr_gwhere(F v, bool c) {
  const unsigned long long bal = __ballot(c);
  F out = v;
#pragma unroll
  for (int h = 0; h < KR_H; ++h) {
    const unsigned bits = (unsigned)(bal >> (h * KR_G)) & KR_GMASK;
    const F x = kr_wbc(v, h * KR_G + (bits ? __builtin_ctz(bits) : 0));
    out = h == 0 ? x : ((int)threadIdx.x >= h * KR_G ? x : out);
  }
  return out;
}

#if KR_G == 32
/* the value of the lane 16 apart in the same 32-lane group (the other row):
 * v_permlane16_swap exchanges the odd rows of its first operand with the
 * even rows of its second, so with both operands v the first result holds
 * rows (0, 0, 2, 2) and the second rows (1, 1, 3, 3) */
__device__ __forceinline__ unsigned kr_gx16(unsigned v) {
  const auto sw = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  return (threadIdx.x & 16u) ? (unsigned)sw[0] : (unsigned)sw[1];
}
__device__ __forceinline__ double kr_gx16(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = kr_gx16((unsigned)b), hi = kr_gx16((unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
#endif

/* Group sum: quad permutes and the half-row and row mirrors leave every lane
 * of a 16-lane row with the row's sum (each pair of lanes adds the same two
 * values, so all lanes hold the same bits); a 32-lane group adds the other
 * row's sum. */
__device__ __forceinline__ double kr_gsum(double v) {
  v += kr_dpp<0xB1, 0xF>(v);
  v += kr_dpp<0x4E, 0xF>(v);
  v += kr_dpp<0x141, 0xF>(v);
  v += kr_dpp<0x140, 0xF>(v);
#if KR_G == 32
  v += kr_gx16(v);
#endif
  return v;
}

/* Group maximum of non-negative values (a NaN is skipped unless all are). */
__device__ __forceinline__ double kr_gmax(double v) {
  v = fmax(v, kr_dpp<0xB1, 0xF>(v));
  v = fmax(v, kr_dpp<0x4E, 0xF>(v));
  v = fmax(v, kr_dpp<0x141, 0xF>(v));
  v = fmax(v, kr_dpp<0x140, 0xF>(v));
#if KR_G == 32
  v = fmax(v, kr_gx16(v));
#endif
  return v;
}

/* true in every lane of the group if b holds in any of its lanes */
__device__ __forceinline__ bool kr_gany(bool b) {
  return ((unsigned)(__ballot(b) >> kr_gbase()) & KR_GMASK) != 0u;
}

/* Group lane whose key is largest (lowest lane on ties; key 0 for lanes
 * that do not compete); best = the winning packed key. */
__device__ __forceinline__ int kr_gargmax(float key, bool cand, unsigned &best) {
  const int r = kr_glane();
  unsigned k = cand ? ((__float_as_uint(key) & ~(unsigned)(KR_G - 1)) | (unsigned)(KR_G - 1 - r)) : 0u;
  k = kr_dpp_max<0xB1, 0xF>(k);
  k = kr_dpp_max<0x4E, 0xF>(k);
  k = kr_dpp_max<0x141, 0xF>(k);
  k = kr_dpp_max<0x140, 0xF>(k);
#if KR_G == 32
  {
    const unsigned o = kr_gx16(k);
    k = o > k ? o : k;
  }
#endif
  best = k;
  return KR_G - 1 - (int)(k & (unsigned)(KR_G - 1));
}

/* Lane of the group with the largest value among candidates (lowest lane on
 * ties), or -1. */
__device__ __forceinline__ int kr_gargmaxd(double v, bool cand) {
  const int r = kr_glane();
  double bv = cand ? v : -1.0;
  int bl = cand ? r : KR_G;
#pragma unroll
  for (int o = KR_G / 2; o; o >>= 1) {
    const double ov = __shfl_xor(bv, o, 64);
    const int ol = __shfl_xor(bl, o, 64);
    if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; }
  }
  return bl < KR_G ? bl : -1;
}

/* ------------------------------------------------------------------------ */
/* rates, rate Jacobian, energy row                                          */
/* ------------------------------------------------------------------------ */

__device__ __forceinline__ void kr_gpublish(KrGBlock &w, double yl) {
  const int r = kr_glane();
  w.y[r] = r < KR_N ? yl : 1.0;
  __syncthreads();
}

template <bool FULL>
__device__ __forceinline__ void kr_gdirections(KrGBlock &w) {
  const int r = kr_glane();
  const double T = w.y[KR_S];
  const double l2T = kr_log2(T);
  const double iT = 1.0 / T;
#pragma unroll
  for (int j = 0; j < KR_GNDR; ++j) {
    const int d = r + KR_G * j;
    double a2 = kr_da2[d], b = kr_db[d];
    const double E = kr_dE[d];
#if KR_NTAB > 0
    const int tb = kr_dtab[d];
    if (tb >= 0) {
      double st;
      a2 += kr_tab_log2(tb, l2T, st);
      b += st;
    }
#endif
    const unsigned rr = kr_gdr[d];
    const double n0 = w.y[rr & 31u], n1 = w.y[(rr >> 8) & 31u], n2 = w.y[(rr >> 16) & 31u];
    const double eiT = E * iT;
    const double k = kr_exp2(fma(-eiT, 0x1.71547652b82fep+0, fma(kr_db[d], l2T, a2)));
    const double q = k * n0 * n1 * n2;
    double *P = w.P + 5 * d;
    P[0] = q;
    if (FULL) {
      P[1] = q * (b + eiT) * iT;
      P[2] = k * n1 * n2;
      P[3] = k * n0 * n2;
      P[4] = k * n0 * n1;
    }
  }
  __syncthreads();
}

template <int LEN>
__device__ __forceinline__ void kr_ggather(KrGBlock &w, const unsigned *tab) {
  static_assert(LEN % 8 == 0, "contribution lists are padded to a multiple of 8");
  const int r = kr_glane();
  double acc = 0.0;
  unsigned e[8], f[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) e[u] = tab[u * KR_G + r];
#pragma unroll 1
  for (int i0 = 0; i0 < LEN; i0 += 8) {
    const int in = i0 + 8 < LEN ? i0 + 8 : i0;
#pragma unroll
    for (int u = 0; u < 8; ++u) f[u] = tab[(in + u) * KR_G + r];
    double pv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pv[u] = w.P[e[u] & 4095u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double nu = (double)((int)((e[u] >> 25) & 7u) - 4);
      acc = fma(nu, pv[u], acc);
      /* an entry that does not end its destination's group stores into
       * the lane's spare slot (the published point is dead here) */
      const bool fl = (e[u] >> 28) != 0u;
      *(fl ? &w.J[(e[u] >> 12) & 8191u] : &w.y[r]) = acc;
      acc = fl ? 0.0 : acc;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = f[u];
  }
  __syncthreads();
}

/* Energy row: row S, column m = -sum_s h_s J[s][m] (lane m, m <= S + 1). */
__device__ __forceinline__ void kr_genergy(KrGBlock &w) {
  const int m = kr_glane();
  if (m <= KR_S + 1) {
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; s += 2) t = fma(kr_hf[s], w.J[s * KR_LDJ + m], t);
    double t1 = 0.0;
#pragma unroll
    for (int s = 1; s < KR_S; s += 2) t1 = fma(kr_hf[s], w.J[s * KR_LDJ + m], t1);
    t += t1;
    w.J[KR_S * KR_LDJ + m] = -t;
  }
  __syncthreads();
}

/* This lane's species thermal energy e_r(T) and heat capacity c_r(T). */
__device__ __forceinline__ void kr_gspecies(double T, double &el, double &cl) {
  const int r = kr_glane();
  el = cl = 0.0;
#if KR_CV_POLY
  if (r < KR_S) kr_species_thermo(r, T, el, cl);
#else
  if (r < KR_S) {
    cl = kr_cv[r];
    el = cl * T;
  }
#endif
}

/* c_V and thermal energy eps of the lane-distributed point */
__device__ __forceinline__ void kr_gthermo(double yl, double &cv, double &eps, double &el) {
  const int r = kr_glane();
  const double T = kr_gat(yl, KR_S);
  double cl;
  kr_gspecies(T, el, cl);
  cv = kr_gsum(r < KR_S ? cl * yl : 0.0);
#if KR_CV_POLY
  eps = kr_gsum(r < KR_S ? el * yl : 0.0);
#else
  eps = T * cv;
#endif
}

/* ------------------------------------------------------------------------ */
/* row-per-lane LU of a group                                                */
/* ------------------------------------------------------------------------ */

/* In-place LU of the rows held by the group's lanes (lane r: row r; lanes
 * from N hold no row), as kr_wlu_impl within a group: per column the group
 * arg-max of the implicitly scaled candidates (Algorithm algo:lu-decomp's
 * scaled partial pivoting), rows never moved.  On return pc = the column at
 * which the lane's row was pivot row, a[k] the U entries for k >= pc and the
 * L multipliers for k < pc, dinv the reciprocal pivot; AUG carries b through
 * as an extra column (the forward substitution).  Returns false, alike in
 * the group's lanes, for a singular or non-finite matrix. */
template <typename F, bool AUG>
__device__ __forceinline__ bool kr_glu_impl(F (&a)[KR_N], int &pc, F &dinv, F &b) {
  const int r = kr_glane();
  F mx = F(0);
#pragma unroll
  for (int k = 0; k < KR_N; ++k) mx = fmax(mx, fabs(a[k]));
  const F sc = r < KR_N && mx > F(0) ? F(1) / mx : F(0);
  pc = r < KR_N ? KR_NOTPIV : -1;
  dinv = F(0);
  bool ok = true;
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    const bool cand = pc == KR_NOTPIV;
    const F aj = a[j];
    unsigned best;
    float key;
    if constexpr (sizeof(F) == 4) key = fabsf(aj) * sc;
    else key = fabsf((float)(fabs(aj) * sc));
    const int p = kr_gargmax(key, cand, best);
    ok = ok && (best >> KR_GLOG) != 0u;
    /* the pivot, the next column's entry (the next arg-max waits for it) and
     * the carried right-hand side by readlane; the rest of the pivot row by
     * shuffles, off the critical path */
    const F piv = kr_gpick(aj, p);
    ok = ok && piv != F(0) && kr_finite((double)piv);
    const F inv = kr_wrcp(piv);
    if (r == p) { pc = j; dinv = inv; }
    const F l = pc == KR_NOTPIV ? aj * inv : F(0);
    if (pc == KR_NOTPIV) a[j] = l;
    if (AUG) b = fma(-l, kr_gpick(b, p), b);
    if (j + 1 < KR_N) a[j + 1] = fma(-l, kr_gpick(a[j + 1], p), a[j + 1]);
#pragma unroll
    for (int k = j + 2; k < KR_N; ++k) a[k] = fma(-l, kr_gbc(a[k], p), a[k]);
  }
  return ok;
}

/* Back substitution with the factors of kr_glu_impl (b after the forward
 * substitution, by row; the solution by unknown out).  Step j reads the
 * group's pivot row of column j (found by ballot: a failed factorisation
 * has none and its solve is discarded) by readlane. */
template <typename F>
__device__ __forceinline__ F kr_gback(const F (&a)[KR_N], int pc, F dinv, F b) {
  const int r = kr_glane();
  F x = F(0);
#pragma unroll
  for (int j = KR_N - 1; j >= 0; --j) {
    const F xj = kr_gwhere(b * dinv, pc == j);
    b = fma(-(pc < j ? a[j] : F(0)), xj, b);
    x = r == j ? xj : x;
  }
  return x;
}

template <typename F>
__device__ __forceinline__ F kr_gsolve(const F (&a)[KR_N], int pc, F dinv, F b) {
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    const F yj = kr_gwhere(b, pc == j);
    b = fma(-(pc > j ? a[j] : F(0)), yj, b);
  }
  return kr_gback(a, pc, dinv, b);
}

/* ------------------------------------------------------------------------ */
/* per-group cell state                                                      */
/* ------------------------------------------------------------------------ */

struct KrGCell {
  long long c;
  double h, t, dt, atol, eps_n, prev, safety, growth, hfree;
  int phase, attempt, k, grow, attempts, fin, acc0, acc, iters, rej, nfail;
};

__device__ __forceinline__ double kr_gweight(const KrParams &p, const KrGCell &C, double yn, double y) {
  const double a = kr_glane() < KR_S ? C.atol : 0.0;
  return a + p.rtol * fmax(fabs(yn), fabs(y));
}

/* Weighted element projection of a Newton update (FP32 LU form), as
 * kr_wproject: d <- d - W N^T (N W N^T)^-1 (N d + N (y - y_n)), W =
 * diag(max(|y_s|, atol)), with group sums. */
__device__ __forceinline__ double kr_gproject(double yl, double ynl, double atol, double d) {
  if (KR_NROWS == 0) return d;
  constexpr int V = KR_NROWS > 0 ? KR_NROWS : 1;
  const int r = kr_glane();
  const double W = r < KR_S ? fmax(fabs(yl), atol) : 0.0;
  double G[V][V], q[V], Gi[V];
#pragma unroll
  for (int a = 0; a < V; ++a) {
    const double na = r < KR_S ? (double)kr_comp[a][r] : 0.0;
    q[a] = kr_gsum(na * (d + (yl - ynl)));
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const double nb = r < KR_S ? (double)kr_comp[b][r] : 0.0;
      G[a][b] = kr_gsum(na * nb * W);
    }
  }
#pragma unroll
  for (int a = 0; a < V; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      double t = G[a][b];
#pragma unroll
      for (int k = 0; k < b; ++k) t -= G[a][k] * G[b][k];
      if (a == b) {
        G[a][a] = sqrt(fmax(t, 1e-300));
        Gi[a] = 1.0 / G[a][a];
      } else {
        G[a][b] = t * Gi[b];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < V; ++a) {
    double t = q[a];
#pragma unroll
    for (int k = 0; k < a; ++k) t -= G[a][k] * q[k];
    q[a] = t * Gi[a];
  }
#pragma unroll
  for (int a = V - 1; a >= 0; --a) {
    double t = q[a];
#pragma unroll
    for (int k = a + 1; k < V; ++k) t -= G[k][a] * q[k];
    q[a] = t * Gi[a];
  }
  double t = 0.0;
#pragma unroll
  for (int a = 0; a < V; ++a) t = fma(r < KR_S ? (double)kr_comp[a][r] : 0.0, q[a], t);
  return d - W * t;
}

/* sum over the lane-distributed species of comp[v][s] * x_s */
__device__ __forceinline__ double kr_grow(int v, double x) {
  const int r = kr_glane();
  return kr_gsum(r < KR_S ? (double)kr_comp[v][r] * x : 0.0);
}

__device__ __forceinline__ double kr_gresid(double y, double y0, double nn) {
  const int r = kr_glane();
  double worst = 0.0;
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const double a = r < KR_S ? (double)kr_comp[v][r] : 0.0;
    const double diff = kr_gsum(a * (y - y0));
    const double D = v >= KR_NELEM ? nn : kr_gsum(fabs(a) * y0);
    const double e = fabs(diff) / fmax(D, 1e-300);
    if (!(e <= worst)) worst = e;
  }
  return worst;
}

/* The three post-processing stages of Sec. 2.2.3 on the group's end point
 * (as kr_wpost); the break-up trips run while any active group still has a
 * negative reservoir, each group's trip predicated. */
__device__ __forceinline__ double kr_gpost(double y, double y0, int &flags) {
  const int r = kr_glane();
  double E0[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) E0[v] = kr_grow(v, y0);
  flags = kr_gany(r < KR_S && y < 0.0) ? 1 : 0;
  if (r < KR_S && y < 0.0) y = 0.0;
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const double E = kr_grow(v, y);
    const int rs = kr_res[v];
    if (r == rs) y += (E0[v] - E) / kr_comp[v][rs];
  }
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const int rs = kr_res[v];
    const int sign_r = kr_comp[v][rs] > 0 ? 1 : -1;
    const int a = r < KR_S ? kr_comp[v][r] : 0;
    bool used = false;
#pragma unroll 1
    for (int it = 0; it < KR_S; ++it) {
      const double yr = kr_gbc(y, rs);
      const bool neg = yr < 0.0;
      if (!__any(neg)) break;                         /* uniform over the active groups */
      const bool cand = r < KR_S && r != rs && !used && a != 0 && (a > 0 ? 1 : -1) == sign_r && y > 0.0;
      const int best = kr_gargmaxd(y, cand);
      const bool act = neg && best >= 0;
      const int bi = best >= 0 ? best : 0;
      flags |= act ? 2 : 0;
      if (act && r == bi) used = true;
      const double yb = kr_gbc(y, bi);
      const double need = -yr * kr_comp[v][rs] / kr_comp[v][bi];
      const double x = need < yb ? need : yb;
      if (act && r == bi) y -= x;
#pragma unroll
      for (int u = 0; u < KR_NROWS; ++u) {
        const int au = kr_comp[u][bi];
        if (act && au != 0 && r == kr_res[u]) y += x * au / kr_comp[u][kr_res[u]];
      }
      if (act && x == need && r == rs) y = 0.0;
    }
  }
  return y;
}

/* Status, statistics, substep-log count and totals of the group's cell
 * (every lane of the group stores the same values; lane 0 adds to the
 * totals). */
__device__ __forceinline__ void kr_gstats(const KrParams &p, const KrGCell &C, int code, int nlog, double resid) {
  if (p.status) p.status[C.c] = code;
  if (p.cell_stats) {
    int *st = p.cell_stats + 4 * C.c;
    st[0] = C.acc; st[1] = C.iters; st[2] = C.rej; st[3] = C.nfail;
  }
  if (p.h_log_n) p.h_log_n[C.c] = nlog;
  if (p.totals && kr_glane() == 0) {
    unsigned long long *t = p.totals;
    atomicAdd(&t[KR_TOT_CELLS], 1ull);
    atomicAdd(&t[KR_TOT_SUBSTEPS], (unsigned long long)C.acc);
    atomicAdd(&t[KR_TOT_ITERS], (unsigned long long)C.iters);
    atomicAdd(&t[KR_TOT_REJECTED], (unsigned long long)C.rej);
    atomicAdd(&t[KR_TOT_NFAIL], (unsigned long long)C.nfail);
    if (code == 1) atomicAdd(&t[KR_TOT_RETRIED], 1ull);
    if (code == 2) atomicAdd(&t[KR_TOT_REVERTED], 1ull);
    if (resid > 0.0) atomicMax(&t[KR_TOT_MAXRESID], (unsigned long long)__double_as_longlong(resid));
  }
}

/* Pre-processing (Sec. 2.2.2) of the lane's input entry; bad = non-finite. */
__device__ __forceinline__ double kr_gload(const KrParams &p, long long c, double &dt, bool &bad) {
  const int r = kr_glane();
  double x = 0.0;
  bad = false;
  if (r < KR_S) {
    const double v = p.states[(long long)r * p.ld + c];
    bad = !kr_finite(v);
    x = v > 0.0 ? v : 0.0;
  }
  const double T = p.T[c];
  dt = p.dt ? p.dt[c] : p.dt_scalar;
  bad = bad || !kr_finite(T) || !kr_finite(dt) || !(dt >= 0.0);
  if (p.rho_floor > 0.0 && p.rho) {
    const double rho = p.rho[c];
    if (rho > 0.0 && rho < p.rho_floor) x *= p.rho_floor / rho;
  }
  if (r == KR_S) x = fmin(fmax(T, kr_T_min), kr_T_max);
  return x;
}

/* Starts attempt C.attempt from the input y0: first substep the caller's
 * hint or dt (dt / 100 with tighter control on the retry). */
__device__ __forceinline__ void kr_gstart_attempt(const KrParams &p, KrGCell &C, double y0, double &y,
                                                  double &yn) {
  y = y0;
  yn = y0;
  double cv, eps, el;
  kr_gthermo(y0, cv, eps, el);
  C.eps_n = eps;
  C.t = 0.0;
  if (p.mode == 1) {
    C.h = C.dt / (double)p.n_fixed;
  } else if (C.attempt == 0) {
    double h0 = C.dt;
    if (p.h_hint) {
      const double hh = p.h_hint[C.c];
      h0 = (hh > 0.0 && kr_finite(hh)) ? hh : h0;
    }
    C.h = h0; C.safety = 0.9; C.growth = 5.0;
  } else {
    C.h = C.dt / 100.0; C.safety = 0.5; C.growth = 2.0;
  }
  C.attempts = 0;
  C.fin = 0;
  C.acc0 = C.acc;
  C.phase = KR_GPH_FRESH;
}

/* The attempt failed: retry once (adaptive mode), else revert (status 2). */
__device__ __forceinline__ void kr_gattempt_failed(const KrParams &p, KrGCell &C, double &y, double &yn) {
  if (C.attempt == 0 && p.mode == 0) {
    double dt;
    bool bad;
    const double y0 = kr_gload(p, C.c, dt, bad);
    C.attempt = 1;
    kr_gstart_attempt(p, C, y0, y, yn);
  } else {
    kr_gstats(p, C, 2, 0, 0.0);
    C.phase = KR_GPH_NONE;
  }
}

/* The attempt reached dt: checks, post-processing, store, outcome. */
__device__ __forceinline__ void kr_gfinish(const KrParams &p, KrGCell &C, double &y, double &yn) {
  const int r = kr_glane();
  double dt;
  bool bad;
  const double y0 = kr_gload(p, C.c, dt, bad);
  const double nn = kr_gsum(r < KR_S ? kr_atoms[r] * y0 : 0.0);
  const bool badv = r < KR_N && !kr_finite(y);
  const bool neg = r < KR_S && y < -1e-10 * nn;
  const bool ok = !kr_gany(badv || neg) && kr_gresid(y, y0, nn) <= 1e-10;
  if (!ok) {
    kr_gattempt_failed(p, C, y, yn);
    return;
  }
  int flags;
  const double yp = kr_gpost(y, y0, flags);
  if (r < KR_S) p.states[(long long)r * p.ld + C.c] = yp;
  if (r == KR_S) p.T[C.c] = yp;
  if (p.h_hint && p.mode == 0) p.h_hint[C.c] = C.hfree;
  kr_gstats(p, C, C.attempt, C.acc - C.acc0, p.totals ? kr_gresid(yp, y0, nn) : 0.0);
  C.phase = KR_GPH_NONE;
}

/* Newton failure: quarter the substep and restart it from y_n (adaptive);
 * a fixed substep sequence cannot shrink, so the attempt fails. */
__device__ __forceinline__ void kr_gnewton_failed(const KrParams &p, KrGCell &C, double &y, double &yn) {
  C.nfail++;
  if (p.mode == 1) { kr_gattempt_failed(p, C, y, yn); return; }
  C.h *= 0.25;
  y = yn;
  C.phase = KR_GPH_RESTART;
}

/* Takes the next cell for the group (want: the group is idle and the queue
 * not yet found empty). */
__device__ __forceinline__ void kr_gclaim(const KrParams &p, KrGCell &C, bool want, bool &exhausted, double &y,
                                          double &yn) {
  const int r = kr_glane();
  unsigned long long c0 = 0ull;
  if (want && r == 0) c0 = atomicAdd(p.counter, 1ull);
  const unsigned long long c = (unsigned long long)kr_gbc((long long)c0, 0);
  if (!want) return;
  if (c >= (unsigned long long)p.n_cells) {
    exhausted = true;
    return;
  }
  long long cell = (long long)c;
  if (p.order) {
    const long long o = (long long)p.order[c];
    cell = o < p.n_cells ? o : cell;      /* range guard; always true */
  }
  C.c = cell;
  C.acc = C.iters = C.rej = C.nfail = 0;
  C.attempt = 0;
  double dt;
  bool bad;
  const double y0 = kr_gload(p, cell, dt, bad);
  if (kr_gany(bad)) {
    kr_gstats(p, C, 2, 0, 0.0);
    C.phase = KR_GPH_NONE;
    return;
  }
  if (dt == 0.0) {
    if (r < KR_S) p.states[(long long)r * p.ld + cell] = y0;
    if (r == KR_S) p.T[cell] = y0;
    kr_gstats(p, C, 0, 0, 0.0);
    C.phase = KR_GPH_NONE;
    return;
  }
  C.dt = dt;
  C.atol = p.floor * kr_gsum(r < KR_S ? kr_atoms[r] * y0 : 0.0);
  kr_gstart_attempt(p, C, y0, y, yn);
}

/* ------------------------------------------------------------------------ */
/* the integrator                                                            */
/* ------------------------------------------------------------------------ */

template <bool MIXED>
__device__ __forceinline__ void kr_gintegrate(const KrParams &p) {
  __shared__ KrGBlock blk[KR_H];
  const int r = kr_glane();
  KrGBlock &w = blk[threadIdx.x / KR_G];
#pragma unroll 1
  for (int k = 0; k < (KR_N * KR_LDJ + KR_G - 1) / KR_G; ++k) {
    const int i = KR_G * k + r;
    if (i < KR_N * KR_LDJ) w.J[i] = 0.0;
  }
  __syncthreads();
  KrGCell C;
  C.c = 0;
  C.h = C.t = C.dt = C.atol = C.eps_n = C.prev = C.hfree = 0.0;
  C.safety = 0.9; C.growth = 5.0;
  C.phase = KR_GPH_NONE;
  C.attempt = C.k = C.grow = C.attempts = C.fin = C.acc0 = 0;
  C.acc = C.iters = C.rej = C.nfail = 0;
  bool exhausted = false;
  /* idle groups evaluate at a harmless point (T = 1 K) */
  double y = 1.0, yn = 1.0, gn = 0.0;

  for (;;) {
    const bool want = C.phase == KR_GPH_NONE && !exhausted;
    if (__any(want)) kr_gclaim(p, C, want, exhausted, y, yn);
    const bool active = C.phase != KR_GPH_NONE;
    if (!__any(active)) {
      if (__all(exhausted)) break;
      continue;
    }

    /* rates, Jacobian and energy row at every group's current point */
    kr_gpublish(w, active ? y : 1.0);
    kr_gdirections<true>(w);
    kr_ggather<KR_GNC>(w, kr_gc);
    kr_genergy(w);
    double cv, eps, el;
    kr_gthermo(active ? y : 1.0, cv, eps, el);
    double g = 0.0;
    if (r < KR_S) g = w.J[r * KR_LDJ + KR_S + 1];
    else if (r == KR_S) g = w.J[KR_S * KR_LDJ + KR_S + 1] / cv;

    const int ph = C.phase;
    if (ph == KR_GPH_CHECK) {
      if (p.mode == 1) {                              /* fixed sequence */
        yn = y;
        C.eps_n = eps;
        if (p.h_log && C.acc - C.acc0 < p.h_log_cap) p.h_log[(long long)(C.acc - C.acc0) * p.h_log_ld + C.c] = C.h;
        C.acc++;
        if (C.acc >= p.n_fixed) kr_gfinish(p, C, y, yn);
        else C.phase = KR_GPH_START;
      } else {
        const double err = kr_gmax(r < KR_N ? fabs(0.5 * C.h * (g - gn)) / kr_gweight(p, C, yn, y) : 0.0);
        if (!kr_finite(err)) {
          C.rej++;
          C.h *= 0.2;
          y = yn;
          C.phase = KR_GPH_RESTART;
        } else if (err <= 1.0) {
          yn = y;
          gn = g;
          C.eps_n = eps;
          if (p.h_log && C.acc - C.acc0 < p.h_log_cap) p.h_log[(long long)(C.acc - C.acc0) * p.h_log_ld + C.c] = C.h;
          C.acc++;
          const double hnew = C.h * fmin(C.growth, fmax(0.2, C.safety / sqrt(fmax(err, 1e-10))));
          if (C.fin) {
            C.hfree = C.hfree > hnew ? C.hfree : hnew;
            kr_gfinish(p, C, y, yn);
          } else {
            C.t += C.h;
            C.h = hnew;
            C.phase = KR_GPH_START;
          }
        } else {
          C.rej++;
          C.h *= fmax(0.2, C.safety / sqrt(err));
          y = yn;
          C.phase = KR_GPH_RESTART;
        }
      }
    } else if (ph == KR_GPH_FRESH) {
      gn = g;
      C.phase = KR_GPH_START;
    }

    if (C.phase == KR_GPH_START) {                     /* y == y_n here */
      bool go = true;
      if (p.mode == 0) {
        if (C.attempts >= p.max_substeps) {
          go = false;
        } else {
          C.fin = 0;
          if (C.h >= C.dt - C.t) { C.hfree = C.h; C.h = C.dt - C.t; C.fin = 1; }
          else if (C.h < 1e-12 * C.dt) go = false;
        }
      }
      if (go) {
        C.attempts++;
        C.k = 0;
        C.grow = 0;
        C.prev = __builtin_inf();
        C.phase = KR_GPH_NEWTON;
      } else {
        kr_gattempt_failed(p, C, y, yn);
      }
    }

    const bool newton = C.phase == KR_GPH_NEWTON;
    if (__any(newton)) {
      /* residual and Newton matrix row of this lane (every group: the
       * factorisation runs in step across the wavefront) */
      const double h = C.h;
      double b = 0.0;
      if (r < KR_S) b = -(y - yn - h * w.J[r * KR_LDJ + KR_S + 1]);
      else if (r == KR_S) b = -(eps - C.eps_n - h * w.J[KR_S * KR_LDJ + KR_S + 1]);
      const int row = r < KR_N ? r : KR_S;
      double a[KR_N];
#pragma unroll
      for (int k = 0; k < KR_N; ++k) a[k] = w.J[row * KR_LDJ + k];
      const bool er = r == KR_S;
      const double T = kr_gat(y, KR_S);
#pragma unroll
      for (int k = 0; k < KR_S; ++k) {
#if KR_CV_POLY
        const double ek = kr_gat(el, k);
#else
        const double ek = kr_cv[k] * T;
#endif
        a[k] = (er ? ek : (r == k ? 1.0 : 0.0)) - h * a[k];
      }
      a[KR_S] = (er ? cv : 0.0) - h * a[KR_S];
      if (r >= KR_N) {
#pragma unroll
        for (int k = 0; k < KR_N; ++k) a[k] = 0.0;
      }
      if (newton) C.iters++;

      double d = 0.0;
      bool ok;
      if (!MIXED) {
        int pc;
        double dinv;
        double bf = b;
        ok = kr_glu_impl<double, true>(a, pc, dinv, bf);
        d = kr_gback(a, pc, dinv, bf);
      } else {
        /* FP32 LU of the row-equilibrated matrix; FP64 residual and
         * iterative refinement against the FP64 rows (sweeps run while any
         * group still refines); FP64 LU where FP32 breaks down or does not
         * settle; FP64 element projection */
        double mx = 0.0;
#pragma unroll
        for (int k = 0; k < KR_N; ++k) mx = fmax(mx, fabs(a[k]));
        const double rs = mx > 0.0 ? 1.0 / mx : 0.0;
        float a32[KR_N];
#pragma unroll
        for (int k = 0; k < KR_N; ++k) a32[k] = (float)(a[k] * rs);
        int pc;
        float dinv;
        float unused = 0.0f;
        bool ok32 = kr_glu_impl<float, false>(a32, pc, dinv, unused);
        double res = b;
        bool conv = false, live = ok32 && newton;
        int sweeps = 0;
        double *v = w.P;                              /* the rate table is dead here */
#pragma unroll 1
        for (int sweep = 0; sweep < 4; ++sweep) {
          if (!__any(live)) break;
          const double c = (double)kr_gsolve(a32, pc, dinv, (float)(res * rs));
          if (live) {
            sweeps = sweep + 1;
            d += c;
            const double cn = kr_gmax(r < KR_N ? fabs(c) / kr_gweight(p, C, yn, y) : 0.0);
            if (!kr_finite(cn)) { ok32 = false; live = false; }
            else if (sweep > 0 && cn <= 1e-6) { conv = true; live = false; }
          }
          /* r = b - M d in FP64 */
          v[r] = d;
          __syncthreads();
          double t = b;
#pragma unroll
          for (int k = 0; k < KR_N; k += 2) t = fma(-a[k], v[k], t);
          double t1 = 0.0;
#pragma unroll
          for (int k = 1; k < KR_N; k += 2) t1 = fma(-a[k], v[k], t1);
          t += t1;
          if (live) res = t;
          __syncthreads();
        }
        if (p.counters && newton && r == 0) atomicAdd(&p.counters[3], (unsigned long long)sweeps);
        const bool need64 = newton && (!ok32 || !conv);
        ok = true;
        if (__any(need64)) {
          if (p.counters && need64 && r == 0) atomicAdd(&p.counters[4], 1ull);
          int pc64;
          double dinv64, unused64 = 0.0;
          const bool ok64 = kr_glu_impl<double, false>(a, pc64, dinv64, unused64);
          const double d64 = kr_gsolve(a, pc64, dinv64, b);
          if (need64) { ok = ok64; d = d64; }
        }
        if (ok) d = kr_gproject(y, yn, C.atol, d);
      }

      if (newton) {
        if (!ok) {
          kr_gnewton_failed(p, C, y, yn);
        } else {
          const double yi = y + d;
          const double ynew = r < KR_N ? yi : 0.0;
          const bool bad = r < KR_N && (!kr_finite(d) || !kr_finite(yi));
          if (kr_gany(bad) || !(kr_gat(ynew, KR_S) > 0.0)) {
            kr_gnewton_failed(p, C, y, yn);
          } else {
            y = ynew;
            const double norm = kr_gmax(r < KR_N ? fabs(d) / kr_gweight(p, C, yn, y) : 0.0);
            if (norm <= p.newton_tol) {
              C.phase = KR_GPH_CHECK;
            } else {
              bool failed = false;
              if (norm > C.prev) { if (++C.grow >= 2) failed = true; }
              else C.grow = 0;
              C.prev = norm;
              if (!failed && ++C.k >= p.max_newton) failed = true;
              if (failed) kr_gnewton_failed(p, C, y, yn);
            }
          }
        }
      }
    }
    if (C.phase == KR_GPH_RESTART) C.phase = KR_GPH_START;
  }
}

#ifndef KR_NO_KERNELS
extern "C" __global__ void __launch_bounds__(64, 1) kr_post(KrParams p, const double *before, int *flags) {
  kr_wpost_cells(p, before, flags);
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_timescale(KrParams p, double *out) {
  kr_wtimescale(p, out);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_fp64(KrParams p) {
  kr_gintegrate<false>(p);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_fp32lu(KrParams p) {
  kr_gintegrate<true>(p);
}

extern "C" __global__ void kr_reset_counter(unsigned long long *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = 0ull;
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_order_keys(KrParams p, unsigned char *bucket,
                                                                  unsigned *hist) {
  kr_worder_keys(p, bucket, hist);
}
#endif /* KR_NO_KERNELS */
