/*
 * kr_wide.h -- device code of the per-cell implicit integrator for large
 * networks (gfx950): one wavefront per cell.
 *
 * Same method as the lane-per-cell integrator (paper Sec. 2.2: backward-Euler
 * substeps solved by Newton iteration with the analytic Jacobian, adaptive
 * substeps, pre-/post-processing and the retry-then-revert ladder), mapped
 * for networks whose Newton matrix (N = S + 1 unknowns, up to 63) no longer
 * fits one lane's registers:
 *
 *  - vectors of the cell (iterate y, substep start y_n, rates g_n, weights)
 *    are spread over the lanes: lane i holds entry i;
 *  - rates: lane l evaluates reaction directions l, l+64, ...: the rate
 *    coefficient k = A T^b exp(-E/T) (as a base-2 exponential, kr_math.h),
 *    the rate of progress q = k prod n,
 *    dq/dT and dq/dn per reactant slot, into an LDS table P;
 *  - the rate Jacobian is gathered into LDS (rows = species; columns =
 *    species, T and the rate f itself) from per-lane contribution lists that
 *    the network compiler builds: every matrix entry is owned by one lane,
 *    so the accumulation needs no atomics and its order is fixed (bitwise
 *    reproducible per cell); the lists are balanced over the 64 lanes;
 *  - the energy row follows from the species rows, dQ/dy = -sum_s h_s df_s/dy
 *    (heat release q_r = -sum_s nu_rs h_s), as one column sum per lane;
 *  - LU: lane i holds row i of the Newton matrix in registers; column j is
 *    eliminated by a wave-wide arg-max over the remaining rows (implicit row
 *    scaling as in the paper's Algorithm 1), the pivot row's entries read
 *    straight from the pivot lane's registers (readlane into scalar
 *    registers, no LDS round trip or barrier) and one FMA per remaining
 *    entry.  Rows are never moved:
 *    each lane records the column at which its row became pivot row, and the
 *    triangular solves walk the pivot order (found by a ballot per column).
 *
 * Control flow is wave-uniform by construction, and visibly so to the
 * compiler: every value a branch or loop depends on is moved to a scalar
 * register (read from one lane, or a ballot), and no loop has per-lane
 * exits.  Per-lane loop exits are lowered to exec-mask loops, which in
 * kernels this large (register spills) have mis-executed on gfx950.
 *
 * Generated section (network compiler) defines:
 *   KR_S, KR_NROWS, KR_NELEM, KR_LDJ (LDS row stride of the Jacobian),
 *   KR_NDR (direction rounds of 64), KR_NC / KR_NF (contribution list lengths,
 *   multiples of 8)
 *   kr_comp, kr_res, kr_cv, kr_atoms, kr_hf, kr_T_min, kr_T_max
 *   kr_da2, kr_db, kr_dE [KR_NDR * 64]  direction Arrhenius parameters (log2 A, b, E)
 *   kr_dr [KR_NDR * 64]                 reactant slots, 8 bits each (63: none, reads
 *                                       the 1.0 that lane 63 publishes)
 *   kr_wc [KR_NC * 64], kr_wf [KR_NF * 64]  contribution lists (lane-interleaved):
 *       bits 0-11 source in P, 12-24 destination in the Jacobian,
 *       25-27 stoichiometric coefficient + 4, 28 last contribution of its entry
 */

#define KR_N (KR_S + 1)
#define KR_NDP (KR_NDR * 64)

struct KrWave {
  double y[64];                 /* broadcast copy of the current point */
  double v[64];                 /* scratch vector */
  double P[5 * KR_NDP];         /* per direction: q, dq/dT, dq/dn (3 slots) */
  double J[KR_N * KR_LDJ + 64]; /* rows 0..S-1 species (cols 0..S-1 d/dn, S d/dT,
                                   S+1 f), row S energy (dQ/dn, dQ/dT, Q); then
                                   one spare slot per lane (kr_wgather) */
};

__device__ __forceinline__ bool kr_finite(double x) { return __builtin_isfinite(x); }

__device__ __forceinline__ double kr_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ float kr_bcastf(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

/* lane 0's value as a scalar (for values every lane holds alike) */
__device__ __forceinline__ double kr_u(double v) { return kr_bcast(v, 0); }
__device__ __forceinline__ int kr_ui(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ bool kr_uany(bool b) { return __ballot(b) != 0ull; }

/* v of the lane the DPP control selects; 0 in rows outside row_mask or where
 * the source lane does not exist */
template <int CTRL, int ROWS>
__device__ __forceinline__ double kr_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

/* Wave sum by DPP moves (quad permutes, half-row and row mirrors, then the
 * row broadcasts 15 and 31): lane 63 ends with the total, which every lane
 * receives as a scalar.  The order of additions is fixed. */
__device__ __forceinline__ double kr_wsum(double v) {
  v += kr_dpp<0xB1, 0xF>(v);
  v += kr_dpp<0x4E, 0xF>(v);
  v += kr_dpp<0x141, 0xF>(v);
  v += kr_dpp<0x140, 0xF>(v);
  v += kr_dpp<0x142, 0xA>(v);
  v += kr_dpp<0x143, 0xC>(v);
  return kr_bcast(v, 63);
}

/* Wave maximum of non-negative values (a NaN is skipped, as by a running
 * maximum that keeps the larger of the two), by the same DPP moves. */
__device__ __forceinline__ double kr_wmax(double v) {
  v = fmax(v, kr_dpp<0xB1, 0xF>(v));
  v = fmax(v, kr_dpp<0x4E, 0xF>(v));
  v = fmax(v, kr_dpp<0x141, 0xF>(v));
  v = fmax(v, kr_dpp<0x140, 0xF>(v));
  v = fmax(v, kr_dpp<0x142, 0xA>(v));
  v = fmax(v, kr_dpp<0x143, 0xC>(v));
  return kr_bcast(v, 63);
}

/* max(k, k of the lane the DPP control selects); lanes of rows outside
 * row_mask, or whose source lane does not exist, keep k */
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned kr_dpp_max(unsigned k) {
  const unsigned t = (unsigned)__builtin_amdgcn_update_dpp((int)k, (int)k, CTRL, ROWS, 0xF, false);
  return t > k ? t : k;
}

/* Lane holding the largest non-negative key (lowest lane on ties); key 0 for
 * lanes that do not compete.  Returns the winning lane, and its key.  The
 * wave maximum is built with DPP moves (quad permutes, half-row and row
 * mirrors, then the row broadcasts 15 and 31 into the upper rows), which
 * leaves it in lane 63: no LDS round trips. */
__device__ __forceinline__ int kr_wargmax(float key, bool cand, unsigned &best) {
  const int lane = threadIdx.x;
  unsigned k = cand ? ((__float_as_uint(key) & ~63u) | (unsigned)(63 - lane)) : 0u;
  k = kr_dpp_max<0xB1, 0xF>(k);    /* quad_perm [1,0,3,2] */
  k = kr_dpp_max<0x4E, 0xF>(k);    /* quad_perm [2,3,0,1] */
  k = kr_dpp_max<0x141, 0xF>(k);   /* row_half_mirror */
  k = kr_dpp_max<0x140, 0xF>(k);   /* row_mirror: every lane holds its row's max */
  k = kr_dpp_max<0x142, 0xA>(k);   /* row_bcast:15 into rows 1 and 3 */
  k = kr_dpp_max<0x143, 0xC>(k);   /* row_bcast:31 into rows 2 and 3: lane 63 holds the max */
  best = (unsigned)__builtin_amdgcn_readlane((int)k, 63);
  return 63 - (int)(best & 63u);
}

/* ------------------------------------------------------------------------ */
/* rates, rate Jacobian, energy row                                          */
/* ------------------------------------------------------------------------ */

/* Publishes the lane-distributed point y to LDS. */
__device__ __forceinline__ void kr_wpublish(KrWave &w, double yl) {
  /* lanes past the unknowns publish 1.0: slot 63 stands for an empty
   * reactant slot in the direction tables */
  w.y[threadIdx.x] = (int)threadIdx.x < KR_N ? yl : 1.0;
  __syncthreads();
}

/* Direction pass at the published point: P gets q, dq/dT and the slot
 * partials (full) or q only. */
template <bool FULL>
__device__ __forceinline__ void kr_wdirections(KrWave &w) {
  const int lane = threadIdx.x;
  const double T = w.y[KR_S];
  const double l2T = kr_log2(T);
  const double iT = 1.0 / T;
#pragma unroll
  for (int j = 0; j < KR_NDR; ++j) {
    const int d = lane + 64 * j;
    double a2 = kr_da2[d], b = kr_db[d];
    const double E = kr_dE[d];
#if KR_NTAB > 0
    /* a tabulated factor: its log2 joins the exponent, its log-log slope
     * the temperature derivative */
    const int tb = kr_dtab[d];
    if (tb >= 0) {
      double st;
      a2 += kr_tab_log2(tb, l2T, st);
      b += st;
    }
#endif
    const unsigned rr = kr_dr[d];
    const double n0 = w.y[rr & 63u], n1 = w.y[(rr >> 8) & 63u], n2 = w.y[(rr >> 16) & 63u];
    /* k = A T^b exp(-E/T) = 2^(log2 A + b log2 T - E log2(e) / T) */
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

/* Runs one lane's contribution list into the Jacobian workspace.  The
 * list entries are fetched eight at a time, the next eight while the
 * current ones are accumulated (the table is read from L2: a fetch per
 * entry, waited for at once, left the loop bound by load latency); an entry
 * that ends a destination's group stores the sum (entries that do not store
 * into the lane's spare slot past the matrix, so the loop has no
 * branches). */
template <int LEN>
__device__ __forceinline__ void kr_wgather(KrWave &w, const unsigned *tab) {
  static_assert(LEN % 8 == 0, "contribution lists are padded to a multiple of 8");
  const int lane = threadIdx.x;
  double acc = 0.0;
  unsigned e[8], f[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) e[u] = tab[u * 64 + lane];
#pragma unroll 1
  for (int i0 = 0; i0 < LEN; i0 += 8) {
    const int in = i0 + 8 < LEN ? i0 + 8 : i0;   /* the last pass refetches its own chunk */
#pragma unroll
    for (int u = 0; u < 8; ++u) f[u] = tab[(in + u) * 64 + lane];
    /* the eight partials first: their LDS reads overlap (stores into the
     * matrix below would otherwise keep each read behind the last store) */
    double pv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) pv[u] = w.P[e[u] & 4095u];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double nu = (double)((int)((e[u] >> 25) & 7u) - 4);
      acc = fma(nu, pv[u], acc);
      const bool fl = (e[u] >> 28) != 0u;
      w.J[fl ? ((e[u] >> 12) & 8191u) : (unsigned)(KR_N * KR_LDJ + lane)] = acc;
      acc = fl ? 0.0 : acc;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) e[u] = f[u];
  }
  __syncthreads();
}

/* Energy row: row S, column m = -sum_s h_s J[s][m] for m <= S + 1 (the last
 * column gives Q).  Lanes lo..hi each sum one column. */
__device__ __forceinline__ void kr_wenergy(KrWave &w, int lo, int hi) {
  const int m = threadIdx.x;
  if (m >= lo && m <= hi) {
    double t = 0.0;
#pragma unroll
    for (int s = 0; s < KR_S; ++s) t = fma(kr_hf[s], w.J[s * KR_LDJ + m], t);
    w.J[KR_S * KR_LDJ + m] = -t;
  }
  __syncthreads();
}

/* Rates, rate Jacobian and energy row at the lane-distributed point y. */
__device__ __forceinline__ void kr_weval(KrWave &w, double yl) {
  kr_wpublish(w, yl);
  kr_wdirections<true>(w);
  kr_wgather<KR_NC>(w, kr_wc);
  kr_wenergy(w, 0, KR_S + 1);
}

/* Rates only: f in column S+1 of the species rows, Q at (S, S+1). */
__device__ __forceinline__ void kr_wrhs(KrWave &w, double yl) {
  kr_wpublish(w, yl);
  kr_wdirections<false>(w);
  kr_wgather<KR_NF>(w, kr_wf);
  kr_wenergy(w, KR_S + 1, KR_S + 1);
}

/* This lane's species thermal energy e_l(T) and heat capacity c_l(T) (0
 * beyond the species) at the temperature T of the point. */
__device__ __forceinline__ void kr_wspecies(double T, double &el, double &cl) {
  const int lane = threadIdx.x;
  el = cl = 0.0;
#if KR_CV_POLY
  if (lane < KR_S) kr_species_thermo(lane, T, el, cl);
#else
  if (lane < KR_S) {
    cl = kr_cv[lane];
    el = cl * T;
  }
#endif
}

/* c_V = sum_s c_s(T) n_s over the lane-distributed point */
__device__ __forceinline__ double kr_wheatcap(double yl) {
  const int lane = threadIdx.x;
#if KR_CV_POLY
  double el, cl;
  kr_wspecies(kr_bcast(yl, KR_S), el, cl);
  return kr_wsum(lane < KR_S ? cl * yl : 0.0);
#else
  return kr_wsum(lane < KR_S ? kr_cv[lane] * yl : 0.0);
#endif
}

/* thermal energy eps = sum_s n_s e_s(T) of the lane-distributed point (T
 * c_V for constant heat capacities) */
__device__ __forceinline__ double kr_wenergy_of(double yl) {
#if KR_CV_POLY
  const int lane = threadIdx.x;
  double el, cl;
  kr_wspecies(kr_bcast(yl, KR_S), el, cl);
  return kr_u(kr_wsum(lane < KR_S ? el * yl : 0.0));
#else
  return kr_bcast(yl, KR_S) * kr_u(kr_wheatcap(yl));
#endif
}

/* g = (f, Q / c_V) for lane i, after kr_wrhs or kr_weval */
__device__ __forceinline__ double kr_wrate(const KrWave &w, double cv) {
  const int lane = threadIdx.x;
  if (lane < KR_S) return w.J[lane * KR_LDJ + KR_S + 1];
  if (lane == KR_S) return w.J[KR_S * KR_LDJ + KR_S + 1] / cv;
  return 0.0;
}

/* ------------------------------------------------------------------------ */
/* lane-per-row LU                                                           */
/* ------------------------------------------------------------------------ */

#define KR_NOTPIV 1000

/* In-place LU of the rows held by the lanes (lane i: row i, lanes >= N hold
 * no row).  On return: pc = column at which the lane's row was the pivot
 * row, a[k] holds U entries for k >= pc and L multipliers for k < pc, dinv
 * the reciprocal pivot.  Returns false (wave-uniform) for a singular or
 * non-finite matrix. */
template <typename F>
__device__ __forceinline__ F kr_wbc(F v, int src) {
  if constexpr (sizeof(F) == 8) return kr_bcast(v, src);
  else return kr_bcastf(v, src);
}

/* 1/x: for FP64 the hardware estimate (relative error ~2^-24) refined by
 * two Newton steps, within an ulp or so of the quotient; for FP32 (the
 * factorisation that FP64 refinement corrects) the hardware estimate alone,
 * within about an ulp, instead of the correctly rounded division's
 * ten-instruction sequence on every column's critical path */
template <typename F>
__device__ __forceinline__ F kr_wrcp(F x) {
  if constexpr (sizeof(F) == 8) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  } else {
    return __builtin_amdgcn_rcpf(x);
  }
}

template <typename F, bool AUG>
__device__ __forceinline__ bool kr_wlu_impl(F (&a)[KR_N], int &pc, F &dinv, F &b) {
  const int lane = threadIdx.x;
  F mx = F(0);
#pragma unroll
  for (int k = 0; k < KR_N; ++k) mx = fmax(mx, fabs(a[k]));
  const F sc = lane < KR_N && mx > F(0) ? F(1) / mx : F(0);
  pc = lane < KR_N ? KR_NOTPIV : -1;
  dinv = F(0);
  bool ok = true;
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    const bool cand = pc == KR_NOTPIV;
    const F aj = a[j];
    unsigned best;
    /* fabs: a -0 candidate would carry the sign bit into the key */
    const int p = kr_wargmax(fabsf((float)(fabs((double)aj) * (double)sc)), cand, best);
    ok = ok && (best >> 6) != 0u;
    const F piv = kr_wbc(aj, p);
    ok = ok && piv != F(0) && kr_finite((double)piv);
    const F inv = kr_wrcp(piv);
    if (lane == p) { pc = j; dinv = inv; }
    const F l = pc == KR_NOTPIV ? aj * inv : F(0);
    if (pc == KR_NOTPIV) a[j] = l;
    /* augmented column: the forward substitution of kr_wsolve, step j */
    if (AUG) b = fma(-l, kr_wbc(b, p), b);
    /* the pivot row's remaining entries, read from lane p's registers */
    /* two entries per step: the second readlane pair covers the first
     * pair's wait before its FMA */
#pragma unroll
    for (int k = j + 1; k < KR_N; k += 2) {
      const F u0 = kr_wbc(a[k], p);
      if (k + 1 < KR_N) {
        const F u1 = kr_wbc(a[k + 1], p);
        a[k] = fma(-l, u0, a[k]);
        a[k + 1] = fma(-l, u1, a[k + 1]);
      } else {
        a[k] = fma(-l, u0, a[k]);
      }
    }
  }
  return ok;
}

template <typename F>
__device__ __forceinline__ bool kr_wlu(F (&a)[KR_N], int &pc, F &dinv) {
  F unused = F(0);
  return kr_wlu_impl<F, false>(a, pc, dinv, unused);
}

/* kr_wlu with b (by row) carried along as an extra column: on return b has
 * been through the forward substitution (the same operations, in the same
 * order, as the first half of kr_wsolve), ready for kr_wback. */
template <typename F>
__device__ __forceinline__ bool kr_wlu_fwd(F (&a)[KR_N], int &pc, F &dinv, F &b) {
  return kr_wlu_impl<F, true>(a, pc, dinv, b);
}

/* ------------------------------------------------------------------------ */
/* FP32 LU with the trailing updates on MFMA (networks of 31+ species)      */
/* ------------------------------------------------------------------------ */

/* Blocked right-looking variant of kr_wlu<float> (same pivot choice, same
 * factor layout, different rounding): columns in panels, the first of
 * KR_PF columns, then panels of 16, so that every trailing block is a
 * multiple of 16 wide.  Inside a panel a column is eliminated as in
 * kr_wlu, but only the panel's own columns are updated.  After the panel
 * [j0, j1), with M the rows' multipliers of the panel columns (zero where a
 * row was already a pivot row) and T the rows' trailing parts (columns j1
 * and on):
 *   U = (unit lower L of the panel's pivot rows)^-1 T[pivot rows]
 *       (lanes own columns of U; a forward substitution over the panel),
 *   T -= M U  (64 x Kp times Kp x W on v_mfma_f32_16x16x4f32 tiles),
 * which leaves every row's trailing part as the unblocked elimination would.
 * M, U and T pass through LDS (the rate table P, which is dead during the
 * linear solve).  Returns false (wave-uniform) for a singular matrix. */
#ifdef KR_LU_MFMA
/* set by the network compiler only where it applies: N >= 32 and the panel
 * blocks fit into the rate table's LDS */
#define KR_USE_LU_MFMA 1
#define KR_PF (KR_N - 16 * ((KR_N - 1) / 16))
static_assert(KR_N >= 32, "blocked LU needs at least two panels");
static_assert(4 * (64 * ((KR_PF + 3) / 4 * 4) + ((KR_PF + 3) / 4 * 4) * (KR_N - KR_PF) + 64 * (KR_N - KR_PF)) <=
                  5 * KR_NDP * 8 &&
              4 * (64 * 16 + 80 * (KR_N - KR_PF - 16)) <= 5 * KR_NDP * 8,
              "panel blocks exceed the rate table's LDS");
#endif

#ifdef KR_USE_LU_MFMA
typedef float kr_v4f __attribute__((ext_vector_type(4)));

/* Trailing update after the panel [J0, J1) (see kr_wlu_blocked); pv[jj]:
 * pivot lane of column J0 + jj. */
template <int J0, int J1>
__device__ __forceinline__ void kr_wlu_trailing(float (&a)[KR_N], int pc, const int (&pv)[J1 - J0], float *lds) {
  constexpr int F = J1 - J0, KP = (F + 3) / 4 * 4, W = KR_N - J1;
  static_assert(W % 16 == 0 && W > 0, "trailing blocks are multiples of 16 wide");
  const int lane = threadIdx.x;
  float *Ml = lds, *Ul = lds + 64 * KP, *Tl = Ul + KP * W;
  /* multipliers of the panel columns (zero for pivot rows and padding) and
   * the trailing part, one row per lane */
#pragma unroll
  for (int jj = 0; jj < KP; ++jj) Ml[lane * KP + jj] = (jj < F && pc > J0 + jj) ? a[J0 + jj] : 0.0f;
#pragma unroll
  for (int k = 0; k < W; ++k) Tl[lane * W + k] = a[J1 + k];
  __syncthreads();
  /* U: lane t (columns past W repeat the last one) owns column t */
  {
    const int t = lane < W ? lane : W - 1;
    float u[KP];
#pragma unroll
    for (int jj = 0; jj < F; ++jj) {
      const int p = pv[jj];
      float x = Tl[p * W + t];
#pragma unroll
      for (int q = 0; q < jj; ++q) x = fmaf(-Ml[p * KP + q], u[q], x);
      u[jj] = x;
    }
#pragma unroll
    for (int jj = F; jj < KP; ++jj) u[jj] = 0.0f;
#pragma unroll
    for (int jj = 0; jj < KP; ++jj) Ul[jj * W + t] = u[jj];
  }
  __syncthreads();
  /* C = M U on MFMA tiles, into T's place: lane l supplies A[l%16][l/16] and
   * B[l/16][l%16] of each 16x4 / 4x16 step and receives C rows
   * 4 (l/16) .. 4 (l/16) + 3 of column l%16 */
  const int r16 = lane & 15, q4 = lane >> 4;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
    for (int nt = 0; nt < W / 16; ++nt) {
      kr_v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < KP / 4; ++kk) {
        const float av = Ml[(mt * 16 + r16) * KP + kk * 4 + q4];
        const float bv = Ul[(kk * 4 + q4) * W + nt * 16 + r16];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) Tl[(mt * 16 + 4 * q4 + r) * W + nt * 16 + r16] = acc[r];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < W; ++k) a[J1 + k] -= Tl[lane * W + k];
  __syncthreads();
}

/* Columns [J0, J1) eliminated as in kr_wlu but updating only the panel's own
 * columns, then the trailing update, then the next panel (compile-time
 * recursion, so that every loop bound is a constant). */
template <int J0, int J1>
__device__ __forceinline__ void kr_wlu_panel(float (&a)[KR_N], int &pc, float &dinv, float sc, bool &ok,
                                             float *lds) {
  const int lane = threadIdx.x;
  int pv[J1 - J0];
#pragma unroll
  for (int jj = 0; jj < J1 - J0; ++jj) {
    const int j = J0 + jj;
    const bool cand = pc == KR_NOTPIV;
    const float aj = a[j];
    unsigned best;
    const int p = kr_wargmax(fabsf(fabsf(aj) * sc), cand, best);
    ok = ok && (best >> 6) != 0u;
    pv[jj] = p;
    const float piv = kr_bcastf(aj, p);
    ok = ok && piv != 0.0f && kr_finite((double)piv);
    const float inv = kr_wrcp(piv);
    if (lane == p) { pc = j; dinv = inv; }
    const float l = pc == KR_NOTPIV ? aj * inv : 0.0f;
    if (pc == KR_NOTPIV) a[j] = l;
    /* the panel's own remaining columns, from lane p's registers */
#pragma unroll
    for (int k = j + 1; k < J1; k += 2) {
      const float u0 = kr_bcastf(a[k], p);
      if (k + 1 < J1) {
        const float u1 = kr_bcastf(a[k + 1], p);
        a[k] = fmaf(-l, u0, a[k]);
        a[k + 1] = fmaf(-l, u1, a[k + 1]);
      } else {
        a[k] = fmaf(-l, u0, a[k]);
      }
    }
  }
  if constexpr (J1 < KR_N) {
    kr_wlu_trailing<J0, J1>(a, pc, pv, lds);
    kr_wlu_panel<J1, J1 + 16>(a, pc, dinv, sc, ok, lds);
  }
}

__device__ __forceinline__ bool kr_wlu_blocked(float (&a)[KR_N], int &pc, float &dinv, float *lds) {
  const int lane = threadIdx.x;
  float mx = 0.0f;
#pragma unroll
  for (int k = 0; k < KR_N; ++k) mx = fmaxf(mx, fabsf(a[k]));
  const float sc = lane < KR_N && mx > 0.0f ? 1.0f / mx : 0.0f;
  pc = lane < KR_N ? KR_NOTPIV : -1;
  dinv = 0.0f;
  bool ok = true;
  kr_wlu_panel<0, KR_PF>(a, pc, dinv, sc, ok, lds);
  return ok;
}
#endif /* KR_USE_LU_MFMA */

/* Back substitution with the factors of kr_wlu: b after the forward
 * substitution, by row, in; the solution by unknown (lane j: x_j) out. */
template <typename F>
__device__ __forceinline__ F kr_wback(const F (&a)[KR_N], int pc, F dinv, F b) {
  const int lane = threadIdx.x;
  F x = F(0);
#pragma unroll
  for (int j = KR_N - 1; j >= 0; --j) {
    const int pj = (int)__builtin_ctzll(__ballot(pc == j));
    const F t = b * dinv;
    F xj;
    if constexpr (sizeof(F) == 8) xj = kr_bcast(t, pj);
    else xj = kr_bcastf(t, pj);
    b = fma(-(pc < j ? a[j] : F(0)), xj, b);
    x = lane == j ? xj : x;
  }
  return x;
}

/* Solves with the factors of kr_wlu: b by row (lane i: equation i) in, the
 * solution by unknown (lane j: x_j) out. */
template <typename F>
__device__ __forceinline__ F kr_wsolve(const F (&a)[KR_N], int pc, F dinv, F b) {
#pragma unroll
  for (int j = 0; j < KR_N; ++j) {
    const int pj = (int)__builtin_ctzll(__ballot(pc == j));
    F yj;
    if constexpr (sizeof(F) == 8) yj = kr_bcast(b, pj);
    else yj = kr_bcastf(b, pj);
    b = fma(-(pc > j ? a[j] : F(0)), yj, b);
  }
  return kr_wback(a, pc, dinv, b);
}

/* ------------------------------------------------------------------------ */
/* Newton substep                                                            */
/* ------------------------------------------------------------------------ */

struct KrWCell {
  long long c;
  double dt, atol, eps_n, rtol;
  int acc, iters, rej, nfail;
};

__device__ __forceinline__ double kr_wweight(const KrWCell &C, double yn, double y) {
  const int lane = threadIdx.x;
  const double a = lane < KR_S ? C.atol : 0.0;
  return a + C.rtol * fmax(fabs(yn), fabs(y));
}

/* Weighted element projection of a Newton update (FP32 form): corrects d_S
 * so that y + d carries the conserved totals of the substep start y_n,
 * d_S <- d_S - W N^T (N W N^T)^-1 (N d + N (y - y_n)) with W =
 * diag(max(|y_s|, atol)) (the exact Newton update satisfies N (y + d) =
 * N y_n from any starting point).  The row sums are wave reductions; the
 * small Gram system is solved alike in every lane. */
__device__ __forceinline__ double kr_wproject(double yl, double ynl, double atol, double d) {
  if (KR_NROWS == 0) return d;
  constexpr int V = KR_NROWS > 0 ? KR_NROWS : 1;
  const int lane = threadIdx.x;
  const double W = lane < KR_S ? fmax(fabs(yl), atol) : 0.0;
  double G[V][V], r[V];
#pragma unroll
  for (int a = 0; a < V; ++a) {
    const double na = lane < KR_S ? (double)kr_comp[a][lane] : 0.0;
    r[a] = kr_u(kr_wsum(na * (d + (yl - ynl))));
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const double nb = lane < KR_S ? (double)kr_comp[b][lane] : 0.0;
      G[a][b] = kr_u(kr_wsum(na * nb * W));
    }
  }
#pragma unroll
  for (int a = 0; a < V; ++a) {
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      double t = G[a][b];
#pragma unroll
      for (int k = 0; k < b; ++k) t -= G[a][k] * G[b][k];
      if (a == b) G[a][a] = sqrt(fmax(t, 1e-300));
      else G[a][b] = t / G[b][b];
    }
  }
#pragma unroll
  for (int a = 0; a < V; ++a) {
    double t = r[a];
#pragma unroll
    for (int k = 0; k < a; ++k) t -= G[a][k] * r[k];
    r[a] = t / G[a][a];
  }
#pragma unroll
  for (int a = V - 1; a >= 0; --a) {
    double t = r[a];
#pragma unroll
    for (int k = a + 1; k < V; ++k) t -= G[k][a] * r[k];
    r[a] = t / G[a][a];
  }
  double t = 0.0;
#pragma unroll
  for (int a = 0; a < V; ++a) t = fma(lane < KR_S ? (double)kr_comp[a][lane] : 0.0, r[a], t);
  return d - W * t;
}

/* Newton iteration for one backward-Euler substep of length h from the
 * lane-distributed y_n (plain start y = y_n).  Returns true when converged;
 * y holds the iterate either way. */
template <bool MIXED>
__device__ __forceinline__ bool kr_wnewton(const KrParams &p, KrWave &w, KrWCell &C, double yn,
                                           double h, double &y) {
  const int lane = threadIdx.x;
  y = yn;
  double prev = __builtin_inf();
  int grow = 0;
  const int max_newton = kr_ui(p.max_newton);
  for (int it = 0; it < max_newton; ++it) {
    kr_weval(w, y);
    const double T = kr_bcast(y, KR_S);
#if KR_CV_POLY
    double el, cl;
    kr_wspecies(T, el, cl);
    const double cv = kr_u(kr_wsum(lane < KR_S ? cl * y : 0.0));
    const double eps = kr_u(kr_wsum(lane < KR_S ? el * y : 0.0));
#else
    const double cv = kr_u(kr_wheatcap(y));
    const double eps = T * cv;
#endif
    /* residual (negated) and Newton matrix row of this lane */
    double b = 0.0;
    if (lane < KR_S) b = -(y - yn - h * w.J[lane * KR_LDJ + KR_S + 1]);
    else if (lane == KR_S) b = -(eps - C.eps_n - h * w.J[KR_S * KR_LDJ + KR_S + 1]);
    const int row = lane < KR_N ? lane : KR_S;
    double a[KR_N];
#pragma unroll
    for (int k = 0; k < KR_N; ++k) a[k] = w.J[row * KR_LDJ + k];
    const bool er = lane == KR_S;
#pragma unroll
    for (int k = 0; k < KR_S; ++k) {
      /* d eps / d n_k = e_k(T), from lane k */
#if KR_CV_POLY
      const double ek = kr_bcast(el, k);
#else
      const double ek = kr_cv[k] * T;
#endif
      a[k] = (er ? ek : (lane == k ? 1.0 : 0.0)) - h * a[k];
    }
    a[KR_S] = (er ? cv : 0.0) - h * a[KR_S];
    if (lane >= KR_N) {
#pragma unroll
      for (int k = 0; k < KR_N; ++k) a[k] = 0.0;
    }
    C.iters++;

    double d = 0.0;
    bool ok;
    if (!MIXED) {
      int pc;
      double dinv;
      double bf = b;
      ok = kr_wlu_fwd(a, pc, dinv, bf);
      if (ok) d = kr_wback(a, pc, dinv, bf);
    } else {
      /* FP32 LU of the row-equilibrated matrix; FP64 residual and iterative
       * refinement against the FP64 rows; FP64 LU where FP32 breaks down or
       * refinement does not settle; FP64 element projection */
      double mx = 0.0;
#pragma unroll
      for (int k = 0; k < KR_N; ++k) mx = fmax(mx, fabs(a[k]));
      const double rs = mx > 0.0 ? 1.0 / mx : 0.0;
      float a32[KR_N];
#pragma unroll
      for (int k = 0; k < KR_N; ++k) a32[k] = (float)(a[k] * rs);
      int pc;
      float dinv;
#ifdef KR_USE_LU_MFMA
      bool ok32 = kr_wlu_blocked(a32, pc, dinv, reinterpret_cast<float *>(w.P));
#else
      bool ok32 = kr_wlu(a32, pc, dinv);
#endif
      double r = b;
      bool conv = false;
      int sweeps = 0;
      for (int sweep = 0; sweep < 4; ++sweep) {
        if (!ok32) break;
        sweeps = sweep + 1;
        const double c = (double)kr_wsolve(a32, pc, dinv, (float)(r * rs));
        d += c;
        const double cn = kr_u(kr_wmax(lane < KR_N ? fabs(c) / kr_wweight(C, yn, y) : 0.0));
        if (!kr_finite(cn)) { ok32 = false; break; }
        if (sweep > 0 && cn <= 1e-6) { conv = true; break; }
        /* r = b - M d in FP64 */
        w.v[lane] = d;
        __syncthreads();
        double t = b;
#pragma unroll
        for (int k = 0; k < KR_N; ++k) t = fma(-a[k], w.v[k], t);
        r = t;
        __syncthreads();
      }
      if (p.counters) atomicAdd(&p.counters[3], lane == 0 ? (unsigned long long)sweeps : 0ull);
      ok = true;
      if (!ok32 || !conv) {
        if (p.counters) atomicAdd(&p.counters[4], lane == 0 ? 1ull : 0ull);
        int pc64;
        double dinv64;
        ok = kr_wlu(a, pc64, dinv64);
        d = ok ? kr_wsolve(a, pc64, dinv64, b) : 0.0;
      }
      if (ok) d = kr_wproject(y, yn, C.atol, d);
    }
    if (!ok) return false;
    const double yi = y + d;
    y = lane < KR_N ? yi : 0.0;
    const bool bad = lane < KR_N && (!kr_finite(d) || !kr_finite(yi));
    if (kr_uany(bad) || !(kr_bcast(y, KR_S) > 0.0)) return false;
    const double norm = kr_u(kr_wmax(lane < KR_N ? fabs(d) / kr_wweight(C, yn, y) : 0.0));
    if (norm <= p.newton_tol) return true;
    if (norm > prev) {
      if (++grow >= 2) return false;
    } else {
      grow = 0;
    }
    prev = norm;
  }
  return false;
}

/* Records the k-th accepted substep length of the running attempt (every
 * lane stores the same value). */
__device__ __forceinline__ void kr_wlog(const KrParams &p, const KrWCell &C, int k, double h) {
  if (p.h_log && k < p.h_log_cap) p.h_log[(long long)k * p.h_log_ld + C.c] = h;
}

/* One attempt over [0, dt] from y0 (lane-distributed).  Adaptive: error
 * estimate err = max_i |(h/2)(g_i(y_new) - g_i(y_old))| / w_i (a running
 * maximum that skips 0/0); accepted when err <= 1, then h *= min(growth,
 * max(0.2, safety / sqrt(max(err, 1e-10)))); rejected: h *= max(0.2, safety /
 * sqrt(err)); Newton failure: h /= 4.  The first substep is h0 (the caller's
 * hint or dt; dt/100 on the retry); the last lands on dt.  Fails when h <
 * 1e-12 dt or after max_substeps substep attempts.  On success y holds the
 * end point, nacc the accepted substeps and hnext the proposed length after
 * the last one (the controller's update, or the unclipped length if larger). */
template <bool MIXED>
__device__ __forceinline__ bool kr_wattempt(const KrParams &p, KrWave &w, KrWCell &C, double y0,
                                            int attempt, double hint, double &y, int &nacc,
                                            double &hnext) {
  const int lane = threadIdx.x;
  double yn = y0;
  nacc = 0;
  hnext = 0.0;
  C.eps_n = kr_wenergy_of(y0);
  if (kr_ui(p.mode) == 1) {
    const int nf = kr_ui(p.n_fixed);
    const double h = C.dt / (double)nf;
    for (int k = 0; k < nf; ++k) {
      if (!kr_wnewton<MIXED>(p, w, C, yn, h, y)) { C.nfail++; return false; }
      yn = y;
      C.eps_n = kr_wenergy_of(yn);
      kr_wlog(p, C, k, h);
      C.acc++;
    }
    nacc = nf;
    y = yn;
    return true;
  }
  const double h0 = attempt == 0 ? ((hint > 0.0 && kr_finite(hint)) ? hint : C.dt) : C.dt / 100.0;
  const double safety = attempt == 0 ? 0.9 : 0.5;
  const double growth = attempt == 0 ? 5.0 : 2.0;
  const int max_substeps = kr_ui(p.max_substeps);
  kr_wrhs(w, yn);
  double gn = kr_wrate(w, kr_u(kr_wheatcap(yn)));
  double t = 0.0, h = h0, hfree = 0.0;
  bool done = false;
  for (int attempts = 0; attempts < max_substeps; ++attempts) {
    bool fin = false;
    if (h >= C.dt - t) { hfree = h; h = C.dt - t; fin = true; }
    else if (h < 1e-12 * C.dt) break;
    if (!kr_wnewton<MIXED>(p, w, C, yn, h, y)) {
      C.nfail++;
      h *= 0.25;
      continue;
    }
    kr_wrhs(w, y);
    const double cv = kr_u(kr_wheatcap(y));
    const double g = kr_wrate(w, cv);
    const double err = kr_u(kr_wmax(lane < KR_N ? fabs(0.5 * h * (g - gn)) / kr_wweight(C, yn, y) : 0.0));
    if (!kr_finite(err)) { C.rej++; h *= 0.2; continue; }
    if (err <= 1.0) {
      yn = y;
      gn = g;
#if KR_CV_POLY
      C.eps_n = kr_wenergy_of(y);
#else
      C.eps_n = kr_bcast(y, KR_S) * cv;
#endif
      kr_wlog(p, C, nacc, h);
      nacc++;
      C.acc++;
      const double hnew = h * fmin(growth, fmax(0.2, safety / sqrt(fmax(err, 1e-10))));
      if (fin) { hnext = hfree > hnew ? hfree : hnew; done = true; break; }
      t += h;
      h = hnew;
    } else {
      C.rej++;
      h *= fmax(0.2, safety / sqrt(err));
    }
  }
  y = yn;
  return done;
}

/* ------------------------------------------------------------------------ */
/* one cell: pre-processing, attempts, checks, post-processing               */
/* ------------------------------------------------------------------------ */

/* sum over the lane-distributed species of comp[v][s] * x_s */
__device__ __forceinline__ double kr_wrow(int v, double x) {
  const int lane = threadIdx.x;
  return kr_u(kr_wsum(lane < KR_S ? (double)kr_comp[v][lane] * x : 0.0));
}

/* Element residual max_row |sum_s N_s (y - y0)_s| / D_row (elements: D =
 * sum |N_s| y0_s; charge-like rows: the nuclei density nn); NaN propagates. */
__device__ __forceinline__ double kr_wresid(double y, double y0, double nn) {
  const int lane = threadIdx.x;
  double worst = 0.0;
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const double a = lane < KR_S ? (double)kr_comp[v][lane] : 0.0;
    const double diff = kr_u(kr_wsum(a * (y - y0)));
    const double D = v >= KR_NELEM ? nn : kr_u(kr_wsum(fabs(a) * y0));
    const double e = fabs(diff) / fmax(D, 1e-300);
    if (!(e <= worst)) worst = e;
  }
  return worst;
}

/* Lane with the largest value among candidates (lowest lane on ties), or -1. */
__device__ __forceinline__ int kr_wargmaxd(double v, bool cand) {
  const int lane = threadIdx.x;
  double bv = cand ? v : -1.0;
  int bl = cand ? lane : 64;
#pragma unroll
  for (int o = 32; o; o >>= 1) {
    const double ov = __shfl_xor(bv, o);
    const int ol = __shfl_xor(bl, o);
    if (ov > bv || (ov == bv && ol < bl)) { bv = ov; bl = ol; }
  }
  bl = kr_ui(bl);
  return bl < 64 ? bl : -1;
}

/* The three post-processing stages of Sec. 2.2.3 on the lane-distributed
 * end point y, with the initial row totals from y0.  flags (wave-uniform):
 * 1 a clip, 2 a break-up. */
__device__ __forceinline__ double kr_wpost(double y, double y0, int &flags) {
  const int lane = threadIdx.x;
  double E0[KR_NROWS > 0 ? KR_NROWS : 1];
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) E0[v] = kr_wrow(v, y0);
  flags = kr_uany(lane < KR_S && y < 0.0) ? 1 : 0;
  if (lane < KR_S && y < 0.0) y = 0.0;
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const double E = kr_wrow(v, y);
    const int rs = kr_res[v];
    if (lane == rs) y += (E0[v] - E) / kr_comp[v][rs];
  }
#pragma unroll
  for (int v = 0; v < KR_NROWS; ++v) {
    const int rs = kr_res[v];
    const int sign_r = kr_comp[v][rs] > 0 ? 1 : -1;
    const int a = lane < KR_S ? kr_comp[v][lane] : 0;
    bool used = false;
    for (int it = 0; it < KR_S; ++it) {
      const double yr = kr_bcast(y, rs);
      if (!(yr < 0.0)) break;
      const bool cand = lane < KR_S && lane != rs && !used && a != 0 && (a > 0 ? 1 : -1) == sign_r && y > 0.0;
      const int best = kr_wargmaxd(y, cand);
      if (best < 0) break;
      flags |= 2;
      if (lane == best) used = true;
      const double yb = kr_bcast(y, best);
      const double need = -yr * kr_comp[v][rs] / kr_comp[v][best];
      const double x = need < yb ? need : yb;
      if (lane == best) y -= x;
#pragma unroll
      for (int u = 0; u < KR_NROWS; ++u) {
        const int au = kr_comp[u][best];
        if (au != 0 && lane == kr_res[u]) y += x * au / kr_comp[u][kr_res[u]];
      }
      if (x == need && lane == rs) y = 0.0;
    }
  }
  return y;
}

/* Status, statistics, substep-log count (nlog) and per-call totals of the
 * cell (resid: element residual after post-processing).  Every lane stores
 * the same (uniform) values, and every lane adds to the totals (lanes other
 * than 0 add zero): no branch on the lane index, which the optimiser would
 * otherwise thread into the loop exits and so turn the uniform loops
 * divergent. */
__device__ __forceinline__ void kr_wstats(const KrParams &p, const KrWCell &C, int code, int nlog,
                                          double resid) {
  const int lane = threadIdx.x;
  if (p.status) p.status[C.c] = code;
  if (p.cell_stats) {
    int *st = p.cell_stats + 4 * C.c;
    st[0] = C.acc; st[1] = C.iters; st[2] = C.rej; st[3] = C.nfail;
  }
  if (p.h_log_n) p.h_log_n[C.c] = nlog;
  if (p.totals) {
    unsigned long long *t = p.totals;
    const bool l0 = lane == 0;
    atomicAdd(&t[KR_TOT_CELLS], l0 ? 1ull : 0ull);
    atomicAdd(&t[KR_TOT_SUBSTEPS], l0 ? (unsigned long long)C.acc : 0ull);
    atomicAdd(&t[KR_TOT_ITERS], l0 ? (unsigned long long)C.iters : 0ull);
    atomicAdd(&t[KR_TOT_REJECTED], l0 ? (unsigned long long)C.rej : 0ull);
    atomicAdd(&t[KR_TOT_NFAIL], l0 ? (unsigned long long)C.nfail : 0ull);
    atomicAdd(&t[KR_TOT_RETRIED], l0 && code == 1 ? 1ull : 0ull);
    atomicAdd(&t[KR_TOT_REVERTED], l0 && code == 2 ? 1ull : 0ull);
    atomicMax(&t[KR_TOT_MAXRESID], l0 && resid > 0.0 ? (unsigned long long)__double_as_longlong(resid) : 0ull);
  }
}

/* Stores the lane-distributed point: lane s < S its abundance, lanes from S
 * on store T (the same value each), without a branch on the lane index. */
__device__ __forceinline__ void kr_wstore(const KrParams &p, long long c, double y) {
  const int lane = threadIdx.x;
  const double T = kr_bcast(y, KR_S);
  const double last = kr_bcast(y, KR_S - 1);
  const int s = lane < KR_S ? lane : KR_S - 1;
  const double v = lane < KR_S ? y : last;
  p.states[(long long)s * p.ld + c] = v;
  p.T[c] = T;
}

/* Pre-processing (Sec. 2.2.2) of the lane's input entry; bad = non-finite. */
__device__ __forceinline__ double kr_wload(const KrParams &p, long long c, double &dt, bool &bad) {
  const int lane = threadIdx.x;
  double x = 0.0;
  bad = false;
  if (lane < KR_S) {
    const double v = p.states[(long long)lane * p.ld + c];
    bad = !kr_finite(v);
    x = v > 0.0 ? v : 0.0;
  }
  const double T = kr_u(p.T[c]);
  dt = kr_u(p.dt ? p.dt[c] : p.dt_scalar);
  bad = bad || !kr_finite(T) || !kr_finite(dt) || !(dt >= 0.0);
  if (p.rho_floor > 0.0 && p.rho) {
    const double rho = kr_u(p.rho[c]);
    if (rho > 0.0 && rho < p.rho_floor) x *= p.rho_floor / rho;
  }
  if (lane == KR_S) x = fmin(fmax(T, kr_T_min), kr_T_max);
  return x;
}

template <bool MIXED>
__device__ __forceinline__ void kr_wcell(const KrParams &p, KrWave &w, long long c) {
  const int lane = threadIdx.x;
  KrWCell C;
  C.c = c;
  C.acc = C.iters = C.rej = C.nfail = 0;
  C.rtol = p.rtol;
  double dt;
  bool bad;
  const double y0 = kr_wload(p, c, dt, bad);
  if (kr_uany(bad)) { kr_wstats(p, C, 2, 0, 0.0); return; }
  if (dt == 0.0) {
    kr_wstore(p, c, y0);
    kr_wstats(p, C, 0, 0, 0.0);
    return;
  }
  C.dt = dt;
  const double nn = kr_u(kr_wsum(lane < KR_S ? kr_atoms[lane] * y0 : 0.0));
  C.atol = p.floor * nn;
  const int mode = kr_ui(p.mode);
  const double hint = p.h_hint ? kr_u(p.h_hint[c]) : 0.0;
  int status = 2, nacc = 0;
  double y = y0, hnext = 0.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    bool ok = kr_wattempt<MIXED>(p, w, C, y0, attempt, hint, y, nacc, hnext);
    if (ok) {
      const bool badv = lane < KR_N && !kr_finite(y);
      const bool neg = lane < KR_S && y < -1e-10 * nn;
      ok = !kr_uany(badv || neg) && kr_wresid(y, y0, nn) <= 1e-10;
    }
    if (ok) { status = attempt; break; }
    if (mode == 1) break;
  }
  if (status == 2) { kr_wstats(p, C, 2, 0, 0.0); return; }
  int flags;
  y = kr_wpost(y, y0, flags);
  kr_wstore(p, c, y);
  if (p.h_hint && mode == 0) p.h_hint[c] = hnext;
  kr_wstats(p, C, status, nacc, p.totals ? kr_wresid(y, y0, nn) : 0.0);
}

/* Claims cells one at a time for the wave; zeroes the Jacobian workspace
 * once (entries no reaction touches stay zero). */
template <bool MIXED>
__device__ __forceinline__ void kr_wintegrate(const KrParams &p) {
  __shared__ KrWave w;
  const int lane = threadIdx.x;
#pragma unroll 1
  for (int k = 0; k < (KR_N * KR_LDJ + 63) / 64; ++k) {
    const int i = 64 * k + lane;
    if (i < KR_N * KR_LDJ) w.J[i] = 0.0;
  }
  __syncthreads();
  const unsigned long long n = (unsigned long long)p.n_cells;
  for (;;) {
    /* one claim per wave: lane 0 adds 1, the others 0; lane 0's result */
    const unsigned long long c0 = atomicAdd(p.counter, lane == 0 ? 1ull : 0ull);
    const unsigned lo = (unsigned)kr_ui((int)(unsigned)c0);
    const unsigned hi = (unsigned)kr_ui((int)(unsigned)(c0 >> 32));
    const unsigned long long c = ((unsigned long long)hi << 32) | lo;
    if (c >= n) break;
    long long cell = (long long)c;
    if (p.order) {   /* range guard on the ordered index; always true */
      const long long o = (long long)(unsigned)kr_ui((int)p.order[c]);
      cell = o < p.n_cells ? o : cell;
    }
    kr_wcell<MIXED>(p, w, cell);
  }
}

/* Fastest self-coupling timescale 1 / max(max_s |df_s/dn_s|, |dQ/dT| / c_V)
 * of each cell's input state, capped at 1e7 s (workload set-up). */
__device__ __forceinline__ void kr_wtimescale(const KrParams &p, double *out) {
  __shared__ KrWave w;
  const int lane = threadIdx.x;
#pragma unroll 1
  for (int k = 0; k < (KR_N * KR_LDJ + 63) / 64; ++k) {
    const int i = 64 * k + lane;
    if (i < KR_N * KR_LDJ) w.J[i] = 0.0;
  }
  __syncthreads();
  for (long long c = blockIdx.x; c < p.n_cells; c += gridDim.x) {
    double dt;
    bool bad;
    const double y = kr_wload(p, c, dt, bad);
    kr_weval(w, y);
    const double cv = kr_u(kr_wheatcap(y));
    double m = 0.0;
    if (lane < KR_S) m = fabs(w.J[lane * KR_LDJ + lane]);
    if (lane == KR_S && cv > 0.0) m = fabs(w.J[KR_S * KR_LDJ + KR_S]) / cv;
    m = kr_u(kr_wmax(m));
    const double tau = (m > 0.0 && kr_finite(m)) ? 1.0 / m : 1e7;
    out[c] = (kr_finite(tau) && tau < 1e7) ? tau : 1e7;
  }
}

/* Expected-work bucket of each cell (kr_order.h), one cell per wave:
 * w = dt (sum_s |f_s| / sum_s n_s + |Q| / eps) at the input state. */
__device__ __forceinline__ void kr_worder_keys(const KrParams &p, unsigned char *bucket, unsigned *hist) {
  __shared__ KrWave w;
  const int lane = threadIdx.x;
#pragma unroll 1
  for (int k = 0; k < (KR_N * KR_LDJ + 63) / 64; ++k) {
    const int i = 64 * k + lane;
    if (i < KR_N * KR_LDJ) w.J[i] = 0.0;
  }
  __syncthreads();
  for (long long c = blockIdx.x; c < p.n_cells; c += gridDim.x) {
    double dt;
    bool bad;
    const double y = kr_wload(p, c, dt, bad);
    unsigned b = 0u;
    if (!kr_uany(bad) && dt > 0.0) {
      kr_wrhs(w, y);
      const double eps = kr_wenergy_of(y);
      const double sf = kr_u(kr_wsum(lane < KR_S ? fabs(w.J[lane * KR_LDJ + KR_S + 1]) : 0.0));
      const double sn = kr_u(kr_wsum(lane < KR_S ? y : 0.0));
      const double Q = w.J[KR_S * KR_LDJ + KR_S + 1];
      b = kr_work_bucket(dt * (sf / sn + fabs(Q) / eps));
    }
    b = (unsigned)kr_ui((int)b);
    bucket[c] = (unsigned char)b;
    atomicAdd(&hist[b], lane == 0 ? 1u : 0u);
    __syncthreads();
  }
}

#ifndef KR_WAVES_PER_EU
#define KR_WAVES_PER_EU 1
#endif

/* Post-processing alone (Sec. 2.2.3) of the states in p.states, one cell per
 * wave, with the conserved totals of `before` after pre-processing
 * (negatives clipped); T is not touched.  flags[c] (or null): 1 a clip, 2 a
 * break-up. */
__device__ __forceinline__ void kr_wpost_cells(const KrParams &p, const double *before, int *flags) {
  const int lane = threadIdx.x;
  for (long long c = blockIdx.x; c < p.n_cells; c += gridDim.x) {
    const int sl = lane < KR_S ? lane : KR_S - 1;
    const double b = before[(long long)sl * p.ld + c];
    const double y0 = lane < KR_S && b > 0.0 ? b : 0.0;
    double y = lane < KR_S ? p.states[(long long)sl * p.ld + c] : 0.0;
    int f;
    y = kr_wpost(y, y0, f);
    const double last = kr_bcast(y, KR_S - 1);
    p.states[(long long)sl * p.ld + c] = lane < KR_S ? y : last;
    if (flags) flags[c] = f;
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
  kr_wintegrate<false>(p);
}

extern "C" __global__ void __launch_bounds__(64, KR_WAVES_PER_EU) kr_integrate_fp32lu(KrParams p) {
  kr_wintegrate<true>(p);
}

extern "C" __global__ void kr_reset_counter(unsigned long long *c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) c[0] = 0ull;
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_order_keys(KrParams p, unsigned char *bucket,
                                                                  unsigned *hist) {
  kr_worder_keys(p, bucket, hist);
}
#endif /* KR_NO_KERNELS */
