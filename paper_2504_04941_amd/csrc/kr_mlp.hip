/*
 * kr_mlp.hip -- the learned Newton guess: a small MLP trained and evaluated
 * with hand-written BF16 MFMA kernels (gfx950).
 *
 * Model: x (n_in features, standardised) -> [Linear -> GELU] x layers ->
 * Linear -> n_out outputs.  Weights and activations enter every product in
 * BF16, products accumulate in FP32, biases, pre-activations and gradients
 * are FP32, and Adam keeps FP32 master weights from which the BF16 copies
 * are re-rounded after every step.  Rounding points (shared with the CPU
 * reference used by the tests): a0 = bf16(x); z_l = a_{l-1} W_l^T + b_l;
 * a_l = bf16(gelu(z_l)); out = a_L W_out^T + b_out; d_out = 2 (out - t) /
 * (B n_out); the gradient that enters each product is bf16-rounded; dW_l =
 * bf16(dz_l)^T a_{l-1}, db_l = sum_b dz_l, da_{l-1} = bf16(dz_l) W_l,
 * dz_{l-1} = da_{l-1} * gelu'(z_{l-1}).  GELU is the tanh form.
 *
 * The paper notes that a learned solver (DeepODE) wins on highly stiff
 * phases and loses on slow ones (Sec. 5); here the network only supplies
 * the starting point of Newton's method, and the Newton residual decides.
 *
 * GEMM: 64x64 output tile per 256-thread workgroup, 4 waves of 32x32, K in
 * steps of 32 through LDS, v_mfma_f32_16x16x32_bf16 (gfx950; 2x2 per wave and
 * step), operands staged with 16-byte loads where the layout allows.
 * Operand layouts: A(m,k) and B(n,k) are read either k-contiguous or
 * transposed, so forward (X W^T), input gradient (dZ W) and weight gradient
 * (dZ^T X) share one kernel.
 */
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

typedef uint16_t kr_bf16;
typedef float kr_v4f32 __attribute__((ext_vector_type(4)));

__host__ __device__ static inline kr_bf16 kr_f2bf(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (kr_bf16)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u); /* round to nearest, ties to even */
  return (kr_bf16)(u >> 16);
}

__host__ __device__ static inline float kr_bf2f(kr_bf16 b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

__device__ static inline float kr_gelu(float z) {
  const float c = 0.7978845608028654f; /* sqrt(2/pi) */
  const float t = tanhf(c * (z + 0.044715f * z * z * z));
  return 0.5f * z * (1.0f + t);
}

__device__ static inline float kr_gelu_grad(float z) {
  const float c = 0.7978845608028654f;
  const float t = tanhf(c * (z + 0.044715f * z * z * z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

/* epilogues: pre-activation and its BF16 GELU (training), bias only, GELU
 * derivative, plain store, BF16 GELU only (inference: no pre-activation to
 * keep for a backward pass) */
enum { KR_EPI_BIAS_GELU = 0, KR_EPI_BIAS = 1, KR_EPI_DGELU = 2, KR_EPI_STORE = 3, KR_EPI_GELU = 4 };

struct KrEpi {
  const float *bias;   /* [N] (BIAS_GELU, BIAS) */
  float *outf;         /* [M][ldc] FP32 result (z, out, dz or dW) */
  kr_bf16 *outb;       /* [M][ldc] BF16 copy (gelu(z) or dz), or null */
  const float *zprev;  /* [M][ldc] pre-activation for DGELU */
  int ldc;
  long long zstride;   /* STORE with a split K: slice z writes outf + z * zstride */
};

#define KR_SPLITS 16 /* batch slices of the weight-gradient products */
#define KR_BM 64
#define KR_BN 64
#define KR_BK 32
#define KR_LDS_K (KR_BK + 8)

typedef __bf16 kr_v8bf16 __attribute__((ext_vector_type(8)));
typedef unsigned short kr_v8u16 __attribute__((ext_vector_type(8)));

/* Stages one operand's 64 x 32 tile into s[row][k] (zero outside the
 * matrix).  Element (r, k) of the tile is X(r0 + r, k0 + k) with X(r, k) =
 * TX ? X[k * ld + r] : X[r * ld + k].  VEC: 16-byte loads of 8 elements
 * along the contiguous dimension (its extent and ld are multiples of 8). */
template <bool TX, bool VEC>
__device__ __forceinline__ void kr_stage_tile(kr_bf16 (*s)[KR_LDS_K], const kr_bf16 *__restrict__ X, int ld,
                                              int R, int K, int r0, int k0, int tid) {
  if (VEC) {
    if (!TX) {
      /* 64 rows x 4 chunks of 8 k: one chunk per thread */
      const int r = tid >> 2, kc = (tid & 3) * 8;
      const int gr = r0 + r, gk = k0 + kc;
      kr_v8u16 v = (kr_v8u16){0, 0, 0, 0, 0, 0, 0, 0};
      if (gr < R && gk < K) v = *reinterpret_cast<const kr_v8u16 *>(X + (size_t)gr * ld + gk);
      *reinterpret_cast<kr_v8u16 *>(&s[r][kc]) = v;
    } else {
      /* 32 k x 8 chunks of 8 rows: one chunk per thread, stored transposed */
      const int k = tid >> 3, rc = (tid & 7) * 8;
      const int gk = k0 + k, gr = r0 + rc;
      kr_v8u16 v = (kr_v8u16){0, 0, 0, 0, 0, 0, 0, 0};
      if (gk < K && gr < R) v = *reinterpret_cast<const kr_v8u16 *>(X + (size_t)gk * ld + gr);
#pragma unroll
      for (int e = 0; e < 8; ++e) s[rc + e][k] = v[e];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;                  /* 0..2047 */
      int r, kk;
      if (!TX) { r = idx / KR_BK; kk = idx % KR_BK; } else { kk = idx / KR_BM; r = idx % KR_BM; }
      const int gr = r0 + r, gk = k0 + kk;
      kr_bf16 v = 0;
      if (gr < R && gk < K) v = TX ? X[(size_t)gk * ld + gr] : X[(size_t)gr * ld + gk];
      s[r][kk] = v;
    }
  }
}

/* C(m, n) = sum_k A(m, k) B(n, k), A(m,k) = TA ? A[k*lda+m] : A[m*lda+k],
 * B(n,k) = TB ? B[k*ldb+n] : B[n*ldb+k].  64 x 64 output tile per 256-thread
 * workgroup (4 waves of 32 x 32), K in steps of 32 through LDS, each wave
 * 2 x 2 v_mfma_f32_16x16x32_bf16 per step (lane l supplies A rows l%16,
 * k = 8 (l/16) .. +7, and receives C rows 4 (l/16) .. +3 of column l%16).
 * VA / VB: 16-byte operand loads (see kr_stage_tile). */
template <bool TA, bool TB, int EPI, bool VA, bool VB>
__global__ void __launch_bounds__(256) kr_gemm_bf16(int M, int N, int K, const kr_bf16 *__restrict__ A,
                                                    int lda, const kr_bf16 *__restrict__ B, int ldb,
                                                    KrEpi ep, int kchunk) {
  __shared__ __attribute__((aligned(16))) kr_bf16 sA[KR_BM][KR_LDS_K];
  __shared__ __attribute__((aligned(16))) kr_bf16 sB[KR_BN][KR_LDS_K];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * KR_BM, n0 = blockIdx.x * KR_BN;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  kr_v4f32 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (kr_v4f32){0.f, 0.f, 0.f, 0.f};

  /* split K: slice blockIdx.z covers [kb, ke) (kchunk a multiple of 32) */
  const int kb = blockIdx.z * kchunk;
  const int ke = min(K, kb + kchunk);
  if (EPI == KR_EPI_STORE) ep.outf += (size_t)blockIdx.z * ep.zstride;
  for (int k0 = kb; k0 < ke; k0 += KR_BK) {
    kr_stage_tile<TA, VA>(sA, A, lda, M, ke, m0, k0, tid);
    kr_stage_tile<TB, VB>(sB, B, ldb, N, ke, n0, k0, tid);
    __syncthreads();
    const int kq = 8 * (lane >> 4);
    kr_v8bf16 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      af[i] = __builtin_bit_cast(kr_v8bf16, *reinterpret_cast<const kr_v8u16 *>(&sA[wm + i * 16 + (lane & 15)][kq]));
      bfr[i] = __builtin_bit_cast(kr_v8bf16, *reinterpret_cast<const kr_v8u16 *>(&sB[wn + i * 16 + (lane & 15)][kq]));
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }
  /* epilogue: lane holds rows 4*(lane/16)+r of column lane%16 of each 16x16 block */
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row >= M || col >= N) continue;
        const size_t o = (size_t)row * ep.ldc + col;
        const float v = acc[i][j][r];
        if (EPI == KR_EPI_BIAS_GELU) {
          const float z = v + ep.bias[col];
          ep.outf[o] = z;
          ep.outb[o] = kr_f2bf(kr_gelu(z));
        } else if (EPI == KR_EPI_GELU) {
          ep.outb[o] = kr_f2bf(kr_gelu(v + ep.bias[col]));
        } else if (EPI == KR_EPI_BIAS) {
          ep.outf[o] = v + ep.bias[col];
        } else if (EPI == KR_EPI_DGELU) {
          const float dz = v * kr_gelu_grad(ep.zprev[o]);
          ep.outf[o] = dz;
          ep.outb[o] = kr_f2bf(dz);
        } else {
          ep.outf[o] = v;
        }
      }
}

/* Launches kr_gemm_bf16 with 16-byte operand loads where the contiguous
 * dimension and the leading dimension allow them.  splits > 1 (STORE only):
 * K is cut into that many slices of whole 32-steps, slice z writing its
 * partial product at ep.outf + z * ep.zstride (summed by kr_sum_slices). */
template <bool TA, bool TB, int EPI>
static hipError_t kr_gemm(int M, int N, int K, const kr_bf16 *A, int lda, const kr_bf16 *B, int ldb, const KrEpi &ep,
                          hipStream_t st, int splits = 1) {
  const int kchunk = ((K + splits - 1) / splits + KR_BK - 1) / KR_BK * KR_BK;
  const int nz = kchunk > 0 ? (K + kchunk - 1) / kchunk : 1;
  const dim3 grid((N + KR_BN - 1) / KR_BN, (M + KR_BM - 1) / KR_BM, nz > 0 ? nz : 1);
  const bool va = lda % 8 == 0 && (TA ? M : K) % 8 == 0 && (((uintptr_t)A) & 15) == 0;
  const bool vb = ldb % 8 == 0 && (TB ? N : K) % 8 == 0 && (((uintptr_t)B) & 15) == 0;
  if (va && vb)
    hipLaunchKernelGGL((kr_gemm_bf16<TA, TB, EPI, true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, ep,
                       kchunk);
  else if (va)
    hipLaunchKernelGGL((kr_gemm_bf16<TA, TB, EPI, true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, ep,
                       kchunk);
  else if (vb)
    hipLaunchKernelGGL((kr_gemm_bf16<TA, TB, EPI, false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, ep,
                       kchunk);
  else
    hipLaunchKernelGGL((kr_gemm_bf16<TA, TB, EPI, false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb,
                       ep, kchunk);
  return hipGetLastError();
}

/* dst[i] = sum over z of src[z * n + i], z in order (deterministic) */
__global__ void kr_sum_slices(long n, int nz, const float *__restrict__ src, float *__restrict__ dst) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int z = 0; z < nz; ++z) s += src[(size_t)z * n + i];
    dst[i] = s;
  }
}

/* ------------------------------------------------------------------------ */
/* elementwise kernels                                                       */
/* ------------------------------------------------------------------------ */

/* loss partial sums and d_out = 2 (out - t) / (B n_out), in FP32 and BF16 */
__global__ void kr_mse_grad(int B, int n_out, int ld, const float *__restrict__ out,
                            const float *__restrict__ tgt, float *__restrict__ dout,
                            kr_bf16 *__restrict__ doutb, double *__restrict__ loss) {
  double local = 0.0;
  const float scale = 2.0f / ((float)B * (float)n_out);
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (long)B * n_out;
       i += (long)gridDim.x * blockDim.x) {
    const int b = (int)(i / n_out), c = (int)(i % n_out);
    const float d = out[(size_t)b * ld + c] - tgt[i];
    local += (double)d * d;
    const float g = scale * d;
    dout[(size_t)b * ld + c] = g;
    doutb[(size_t)b * ld + c] = kr_f2bf(g);
  }
  for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(loss, local);
}

/* Column sums of dz [B][ld] over row slices: workgroup (x, y) sums the 64
 * columns 64 x .. 64 x + 63 over rows [y rows_per, (y + 1) rows_per) into
 * part[y][c] (4 row groups of 4 partial sums each, added in a fixed order;
 * kr_sum_slices then adds the slices in order: deterministic). */
__global__ void __launch_bounds__(256) kr_col_sum(int B, int N, int ld, int rows_per, const float *__restrict__ dz,
                                                  float *__restrict__ part) {
  __shared__ float sp[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rows_per, r1 = min(B, r0 + rows_per);
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  if (c < N) {
    int b = r0 + g;
    for (; b + 12 < r1; b += 16) {
      s0 += dz[(size_t)b * ld + c];
      s1 += dz[(size_t)(b + 4) * ld + c];
      s2 += dz[(size_t)(b + 8) * ld + c];
      s3 += dz[(size_t)(b + 12) * ld + c];
    }
    for (; b < r1; b += 4) s0 += dz[(size_t)b * ld + c];
  }
  sp[g][threadIdx.x & 63] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (g == 0 && c < N)
    part[(size_t)blockIdx.y * N + c] = (sp[0][threadIdx.x] + sp[1][threadIdx.x]) + (sp[2][threadIdx.x] + sp[3][threadIdx.x]);
}

/* Adam on FP32 master weights, re-rounding the BF16 copy (n elements) */
__global__ void kr_adam(long n, float *__restrict__ w, kr_bf16 *__restrict__ wb,
                        const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                        float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = kr_f2bf(wi);
  }
}

__global__ void kr_round_bf16(long n, const float *__restrict__ src, kr_bf16 *__restrict__ dst) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    dst[i] = kr_f2bf(src[i]);
}

/* ------------------------------------------------------------------------ */
/* features, targets, normalisation, batches                                 */
/* ------------------------------------------------------------------------ */

/* x = (log10 max(n_s / n_nuc, 1e-20) for each species, log10 T, log10 h) */
__global__ void kr_guess_features_kernel(int S, const double *__restrict__ atoms, long n,
                                         const double *__restrict__ states, long ld,
                                         const double *__restrict__ T, const double *__restrict__ dt,
                                         double dt_scalar, float *__restrict__ X) {
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
    double nn = 0.0;
    for (int s = 0; s < S; ++s) nn += atoms[s] * states[(size_t)s * ld + c];
    float *x = X + (size_t)c * (S + 2);
    for (int s = 0; s < S; ++s) x[s] = (float)log10(fmax(states[(size_t)s * ld + c] / nn, 1e-20));
    x[S] = (float)log10(T[c]);
    x[S + 1] = (float)log10(dt ? dt[c] : dt_scalar);
  }
}

/* y = change of (log10 max(n_s/n_nuc, 1e-20), log10 T) over the step */
__global__ void kr_guess_targets_kernel(int S, const double *__restrict__ atoms, long n,
                                        const double *__restrict__ before, const double *__restrict__ Tb,
                                        const double *__restrict__ after, const double *__restrict__ Ta,
                                        long ld, float *__restrict__ Y) {
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
    double nb = 0.0, na = 0.0;
    for (int s = 0; s < S; ++s) {
      nb += atoms[s] * before[(size_t)s * ld + c];
      na += atoms[s] * after[(size_t)s * ld + c];
    }
    float *y = Y + (size_t)c * (S + 1);
    for (int s = 0; s < S; ++s)
      y[s] = (float)(log10(fmax(after[(size_t)s * ld + c] / na, 1e-20)) -
                     log10(fmax(before[(size_t)s * ld + c] / nb, 1e-20)));
    y[S] = (float)(log10(Ta[c]) - log10(Tb[c]));
  }
}

/* per-column sums of x and x^2 (double accumulators) for n rows of width w */
__global__ void kr_col_moments(long n, int w, const float *__restrict__ X, double *__restrict__ acc) {
  double s[16], q[16];
  for (int j = 0; j < w; ++j) { s[j] = 0.0; q[j] = 0.0; }
  for (long r = blockIdx.x * (long)blockDim.x + threadIdx.x; r < n; r += (long)gridDim.x * blockDim.x)
    for (int j = 0; j < w; ++j) {
      const double v = X[(size_t)r * w + j];
      s[j] += v;
      q[j] += v * v;
    }
  for (int j = 0; j < w; ++j) {
    double a = s[j], b = q[j];
    for (int off = 32; off > 0; off >>= 1) { a += __shfl_xor(a, off); b += __shfl_xor(b, off); }
    if ((threadIdx.x & 63) == 0) { atomicAdd(&acc[j], a); atomicAdd(&acc[16 + j], b); }
  }
}

__global__ void kr_finish_moments(long n, int w, const double *__restrict__ acc, float *__restrict__ mu,
                                  float *__restrict__ sd) {
  const int j = threadIdx.x;
  if (j >= w) return;
  const double m = acc[j] / (double)n;
  const double var = fmax(acc[16 + j] / (double)n - m * m, 0.0);
  mu[j] = (float)m;
  sd[j] = (float)fmax(sqrt(var), 1e-6);
}

/* splitmix64: the row index of batch entry b at step t */
__device__ static inline unsigned long long kr_mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/* standardised BF16 inputs and FP32 targets of one batch; rows drawn
 * uniformly (with replacement) when sample != 0, else rows row0.. */
__global__ void kr_guess_batch_kernel(int nin, int nout, int B, long n, int sample,
                                      unsigned long long seed, long row0,
                                      const float *__restrict__ X, const float *__restrict__ Y,
                                      const float *__restrict__ mu_in, const float *__restrict__ sd_in,
                                      const float *__restrict__ mu_out, const float *__restrict__ sd_out,
                                      kr_bf16 *__restrict__ a0, float *__restrict__ tgt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const long r = sample ? (long)(kr_mix64(seed ^ (unsigned long long)b * 0x2545f4914f6cdd1dull) % (unsigned long long)n)
                        : row0 + b;
  for (int j = 0; j < nin; ++j) a0[(size_t)b * nin + j] = kr_f2bf((X[(size_t)r * nin + j] - mu_in[j]) / sd_in[j]);
  if (Y)
    for (int j = 0; j < nout; ++j) tgt[(size_t)b * nout + j] = (Y[(size_t)r * nout + j] - mu_out[j]) / sd_out[j];
}

/* Newton starting point from the network's output: fractions and T moved
 * by the predicted change of their logarithms. */
__global__ void kr_guess_apply_kernel(int S, const double *__restrict__ atoms, long n, long row0,
                                      const double *__restrict__ states, long ld, const double *__restrict__ T,
                                      const float *__restrict__ out, const float *__restrict__ mu_out,
                                      const float *__restrict__ sd_out, double *__restrict__ guess, long gld) {
  const long b = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long c = row0 + b;
  if (c >= n) return;
  double nn = 0.0;
  for (int s = 0; s < S; ++s) nn += atoms[s] * states[(size_t)s * ld + c];
  const float *o = out + (size_t)b * (S + 1);
  for (int s = 0; s < S; ++s) {
    const double lf = log10(fmax(states[(size_t)s * ld + c] / nn, 1e-20));
    const double d = (double)o[s] * sd_out[s] + mu_out[s];
    guess[(size_t)s * gld + c] = nn * exp10(lf + d);
  }
  const double dT = (double)o[S] * sd_out[S] + mu_out[S];
  guess[(size_t)S * gld + c] = T[c] * exp10(dT);
}

/* ------------------------------------------------------------------------ */
/* the model object                                                          */
/* ------------------------------------------------------------------------ */

struct kr_guess {
  int S = 0, nin = 0, nout = 0, hidden = 0, layers = 0, device = -1;
  long nparams = 0;
  std::vector<long> w_off, b_off, fan_in, fan_out; /* per linear layer */
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr; /* FP32 */
  kr_bf16 *wb = nullptr;
  float *norm = nullptr;         /* mu_in[16], sd_in[16], mu_out[16], sd_out[16] */
  double *atoms = nullptr;       /* [S] */
  double *dacc = nullptr;        /* moments / loss accumulators [64] */
  long step = 0;
  int bcap = 0;                  /* activation buffers sized for bcap rows */
  kr_bf16 *a_in = nullptr, *act[2] = {nullptr, nullptr}, *dzb[2] = {nullptr, nullptr};
  float *zbuf = nullptr, *out = nullptr, *tgt = nullptr, *dzf[2] = {nullptr, nullptr};
  float *part = nullptr;         /* split-K partial weight gradients [KR_SPLITS][max layer size] */
  std::vector<float *> zl;       /* per hidden layer pre-activations (training) */
  std::vector<kr_bf16 *> al;     /* per hidden layer BF16 activations (training) */
};

static void guess_free_buffers(kr_guess *q) {
  for (auto p : q->zl) (void)hipFree(p);
  for (auto p : q->al) (void)hipFree(p);
  q->zl.clear();
  q->al.clear();
  void *bufs[] = {q->a_in, q->out, q->tgt, q->dzf[0], q->dzf[1], q->dzb[0], q->dzb[1], q->part};
  for (void *p : bufs)
    if (p) (void)hipFree(p);
  q->a_in = nullptr; q->out = q->tgt = nullptr; q->part = nullptr;
  q->dzf[0] = q->dzf[1] = nullptr; q->dzb[0] = q->dzb[1] = nullptr;
  q->bcap = 0;
}

static int guess_reserve(kr_guess *q, int B) {
  if (B <= q->bcap) return KR_OK;
  guess_free_buffers(q);
  const size_t H = (size_t)q->hidden;
  const size_t HD = std::max<size_t>(H, (size_t)q->nout); /* gradient rows hold either width */
  HIP_TRY(hipMalloc(&q->a_in, sizeof(kr_bf16) * B * q->nin));
  HIP_TRY(hipMalloc(&q->out, sizeof(float) * B * q->nout));
  HIP_TRY(hipMalloc(&q->tgt, sizeof(float) * B * q->nout));
  for (int k = 0; k < 2; ++k) {
    HIP_TRY(hipMalloc(&q->dzf[k], sizeof(float) * B * HD));
    HIP_TRY(hipMalloc(&q->dzb[k], sizeof(kr_bf16) * B * HD));
  }
  long maxw = 0;
  for (int l = 0; l <= q->layers; ++l) maxw = std::max(maxw, q->fan_in[l] * q->fan_out[l]);
  HIP_TRY(hipMalloc(&q->part, sizeof(float) * KR_SPLITS * (size_t)maxw));
  q->zl.assign(q->layers, nullptr);
  q->al.assign(q->layers, nullptr);
  for (int l = 0; l < q->layers; ++l) {
    HIP_TRY(hipMalloc(&q->zl[l], sizeof(float) * B * H));
    HIP_TRY(hipMalloc(&q->al[l], sizeof(kr_bf16) * B * H));
  }
  q->bcap = B;
  return KR_OK;
}

/* forward pass of B standardised rows already in a_in; out <- outputs.
 * keep_z: store the hidden layers' FP32 pre-activations for a backward pass
 * (training); inference writes only the BF16 activations. */
static int guess_forward(kr_guess *q, int B, hipStream_t st, bool keep_z = true) {
  const kr_bf16 *a = q->a_in;
  int K = q->nin;
  for (int l = 0; l <= q->layers; ++l) {
    const int N = l < q->layers ? q->hidden : q->nout;
    KrEpi ep{};
    ep.bias = q->w + q->b_off[l];
    ep.ldc = N;
    const kr_bf16 *W = q->wb + q->w_off[l];
    if (l < q->layers) {
      ep.outf = q->zl[l];
      ep.outb = q->al[l];
      if (keep_z)
        HIP_TRY((kr_gemm<false, false, KR_EPI_BIAS_GELU>(B, N, K, a, K, W, K, ep, st)));
      else
        HIP_TRY((kr_gemm<false, false, KR_EPI_GELU>(B, N, K, a, K, W, K, ep, st)));
      a = q->al[l];
    } else {
      ep.outf = q->out;
      HIP_TRY((kr_gemm<false, false, KR_EPI_BIAS>(B, N, K, a, K, W, K, ep, st)));
    }
    HIP_TRY(hipGetLastError());
    K = N;
  }
  return KR_OK;
}

/* loss and gradients of the batch in a_in / tgt into q->g */
static int guess_backward(kr_guess *q, int B, hipStream_t st) {
  const int H = q->hidden, L = q->layers, O = q->nout;
  hipLaunchKernelGGL(kr_zero_u64, dim3(1), dim3(64), 0, st, (unsigned long long *)(q->dacc + 40));
  hipLaunchKernelGGL(kr_mse_grad, dim3(std::min(1024, (B * O + 255) / 256)), dim3(256), 0, st, B, O, O, q->out,
                     q->tgt, q->dzf[0], q->dzb[0], q->dacc + 40);
  HIP_TRY(hipGetLastError());
  /* dzf/dzb[cur] holds the gradient at the output of linear layer l */
  int cur = 0;
  for (int l = L; l >= 0; --l) {
    const int N = l < L ? H : O;           /* outputs of layer l */
    const int K = l > 0 ? H : q->nin;      /* inputs of layer l */
    const kr_bf16 *ain = l > 0 ? q->al[l - 1] : q->a_in;
    KrEpi ep{};
    ep.outf = q->g + q->w_off[l];
    ep.ldc = K;
    /* dW_l[n][k] = sum_b dz[b][n] a[b][k] */
    /* dW over KR_SPLITS slices of the batch, then summed in order */
    KrEpi ep_s = ep;
    ep_s.outf = q->part;
    ep_s.zstride = (long long)N * K;
    HIP_TRY((kr_gemm<true, true, KR_EPI_STORE>(N, K, B, q->dzb[cur], N, ain, K, ep_s, st, KR_SPLITS)));
    const int kchunk = ((B + KR_SPLITS - 1) / KR_SPLITS + KR_BK - 1) / KR_BK * KR_BK;
    const int nz = (B + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(kr_sum_slices, dim3((N * K + 255) / 256), dim3(256), 0, st, (long)N * K, nz, q->part,
                       q->g + q->w_off[l]);
    HIP_TRY(hipGetLastError());
    /* db the same way: column sums over row slices, then the slices in order */
    const int rows_per = (B + KR_SPLITS - 1) / KR_SPLITS;
    const int ny = (B + rows_per - 1) / rows_per;
    hipLaunchKernelGGL(kr_col_sum, dim3((N + 63) / 64, ny), dim3(256), 0, st, B, N, N, rows_per, q->dzf[cur],
                       q->part);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(kr_sum_slices, dim3((N + 255) / 256), dim3(256), 0, st, (long)N, ny, q->part,
                       q->g + q->b_off[l]);
    HIP_TRY(hipGetLastError());
    if (l > 0) {
      /* dz_{l-1}[b][k] = (sum_n dz[b][n] W[n][k]) gelu'(z_{l-1}[b][k]) */
      KrEpi e2{};
      e2.outf = q->dzf[cur ^ 1];
      e2.outb = q->dzb[cur ^ 1];
      e2.zprev = q->zl[l - 1];
      e2.ldc = K;
      HIP_TRY((kr_gemm<false, true, KR_EPI_DGELU>(B, K, N, q->dzb[cur], N, q->wb + q->w_off[l], K, e2, st)));
      cur ^= 1;
    }
  }
  return KR_OK;
}

static int guess_make_batch(kr_guess *q, int B, long n, int sample, unsigned long long seed, long row0,
                            const float *X, const float *Y, hipStream_t st) {
  const float *nm = q->norm;
  hipLaunchKernelGGL(kr_guess_batch_kernel, dim3((B + 255) / 256), dim3(256), 0, st, q->nin, q->nout, B, n,
                     sample, seed, row0, X, Y, nm, nm + 16, nm + 32, nm + 48, q->a_in, q->tgt);
  HIP_TRY(hipGetLastError());
  return KR_OK;
}

extern "C" int kr_guess_create(const kr_network *net, int32_t hidden, int32_t layers, uint64_t seed,
                               kr_guess **out) {
  try {
    if (!net || !out || hidden < 1 || hidden > 4096 || layers < 1 || layers > 16)
      return fail(KR_EINVAL, "bad guess model arguments");
    if (net->S + 2 > 16) return fail(KR_EINVAL, "the guess model supports at most 14 species");
    *out = nullptr;
    kr_guess *q = new (std::nothrow) kr_guess;
    if (!q) return fail(KR_ENOMEM, "out of host memory");
    q->S = net->S; q->nin = net->S + 2; q->nout = net->S + 1; q->hidden = hidden; q->layers = layers;
    q->device = net->device;
    long off = 0;
    for (int l = 0; l <= layers; ++l) {
      const long fi = l == 0 ? q->nin : hidden, fo = l == layers ? q->nout : hidden;
      q->w_off.push_back(off); off += fi * fo;
      q->b_off.push_back(off); off += fo;
      q->fan_in.push_back(fi); q->fan_out.push_back(fo);
    }
    q->nparams = off;
    /* PyTorch-Linear-style uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a
     * splitmix64 stream of the seed */
    std::vector<float> w0(off);
    unsigned long long st = seed;
    for (int l = 0; l <= layers; ++l) {
      const double bound = 1.0 / std::sqrt((double)q->fan_in[l]);
      for (long i = q->w_off[l]; i < q->b_off[l] + q->fan_out[l]; ++i) {
        st += 0x9e3779b97f4a7c15ull;
        unsigned long long z = st;
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        const double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        w0[i] = (float)((2.0 * u - 1.0) * bound);
      }
    }
    std::vector<float> nm(64, 0.0f);
    for (int j = 0; j < 16; ++j) { nm[16 + j] = 1.0f; nm[48 + j] = 1.0f; }
    std::vector<double> atoms(q->S, 0.0);
    for (int s = 0; s < q->S; ++s)
      for (int v = 0; v < net->n_elem; ++v) atoms[s] += net->comp[(size_t)v * net->S + s];
    int rc = KR_OK;
    hipError_t e = hipSuccess;
    if ((e = hipSetDevice(q->device)) != hipSuccess ||
        (e = hipMalloc(&q->w, sizeof(float) * off)) != hipSuccess ||
        (e = hipMalloc(&q->g, sizeof(float) * off)) != hipSuccess ||
        (e = hipMalloc(&q->m, sizeof(float) * off)) != hipSuccess ||
        (e = hipMalloc(&q->v, sizeof(float) * off)) != hipSuccess ||
        (e = hipMalloc(&q->wb, sizeof(kr_bf16) * off)) != hipSuccess ||
        (e = hipMalloc(&q->norm, sizeof(float) * 64)) != hipSuccess ||
        (e = hipMalloc(&q->atoms, sizeof(double) * q->S)) != hipSuccess ||
        (e = hipMalloc(&q->dacc, sizeof(double) * 64)) != hipSuccess ||
        (e = hipMemcpy(q->w, w0.data(), sizeof(float) * off, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(q->m, 0, sizeof(float) * off)) != hipSuccess ||
        (e = hipMemset(q->v, 0, sizeof(float) * off)) != hipSuccess ||
        (e = hipMemcpy(q->norm, nm.data(), sizeof(float) * 64, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(q->atoms, atoms.data(), sizeof(double) * q->S, hipMemcpyHostToDevice)) != hipSuccess)
      rc = fail(KR_EDEVICE, "guess model allocation: %s", hipGetErrorString(e));
    if (rc == KR_OK) {
      hipLaunchKernelGGL(kr_round_bf16, dim3(256), dim3(256), 0, 0, (long)off, q->w, q->wb);
      if ((e = hipDeviceSynchronize()) != hipSuccess) rc = fail(KR_EDEVICE, "guess init: %s", hipGetErrorString(e));
    }
    if (rc != KR_OK) {
      kr_guess_destroy(q);
      return rc;
    }
    *out = q;
    return KR_OK;
  } KR_CATCH
}

extern "C" void kr_guess_destroy(kr_guess *q) {
  try {
    if (!q) return;
    guess_free_buffers(q);
    void *bufs[] = {q->w, q->g, q->m, q->v, q->wb, q->norm, q->atoms, q->dacc};
    for (void *p : bufs)
      if (p) (void)hipFree(p);
    delete q;
  } catch (...) {
  }
}

extern "C" int64_t kr_guess_num_params(const kr_guess *q) {
  try {
    return q ? q->nparams : KR_EINVAL;
  } KR_CATCH
}

extern "C" int kr_guess_get_params(const kr_guess *q, float *host) {
  try {
    if (!q || !host) return fail(KR_EINVAL, "null argument");
    HIP_TRY(hipMemcpy(host, q->w, sizeof(float) * q->nparams, hipMemcpyDeviceToHost));
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_set_params(kr_guess *q, const float *host) {
  try {
    if (!q || !host) return fail(KR_EINVAL, "null argument");
    HIP_TRY(hipMemcpy(q->w, host, sizeof(float) * q->nparams, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(kr_round_bf16, dim3(256), dim3(256), 0, 0, q->nparams, q->w, q->wb);
    HIP_TRY(hipDeviceSynchronize());
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_get_normalization(const kr_guess *q, float *norm64) {
  try {
    if (!q || !norm64) return fail(KR_EINVAL, "null argument");
    HIP_TRY(hipMemcpy(norm64, q->norm, sizeof(float) * 64, hipMemcpyDeviceToHost));
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_set_normalization(kr_guess *q, const float *norm64) {
  try {
    if (!q || !norm64) return fail(KR_EINVAL, "null argument");
    for (int j = 0; j < 16; ++j)
      if (!(norm64[16 + j] > 0.0f) || !(norm64[48 + j] > 0.0f)) return fail(KR_EINVAL, "standard deviations must be > 0");
    HIP_TRY(hipMemcpy(q->norm, norm64, sizeof(float) * 64, hipMemcpyHostToDevice));
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_features(const kr_guess *q, int64_t n, const double *states, int64_t ld, const double *T,
                                 const double *dt, double dt_scalar, float *X, kr_stream_t stream) {
  try {
    if (!q || n < 0 || ld < n || (n && (!states || !T || !X))) return fail(KR_EINVAL, "bad feature arguments");
    if (!n) return KR_OK;
    long blocks = std::min<long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(kr_guess_features_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, q->S, q->atoms,
                       (long)n, states, (long)ld, T, dt, dt_scalar, X);
    HIP_TRY(hipGetLastError());
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_targets(const kr_guess *q, int64_t n, const double *before, const double *T_before,
                                const double *after, const double *T_after, int64_t ld, float *Y,
                                kr_stream_t stream) {
  try {
    if (!q || n < 0 || ld < n || (n && (!before || !after || !T_before || !T_after || !Y)))
      return fail(KR_EINVAL, "bad target arguments");
    if (!n) return KR_OK;
    long blocks = std::min<long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(kr_guess_targets_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, q->S, q->atoms,
                       (long)n, before, T_before, after, T_after, (long)ld, Y);
    HIP_TRY(hipGetLastError());
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_fit_normalization(kr_guess *q, int64_t n, const float *X, const float *Y,
                                          kr_stream_t stream) {
  try {
    if (!q || n < 2 || !X || !Y) return fail(KR_EINVAL, "bad normalisation arguments");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(q->device));
    const float *src[2] = {X, Y};
    const int wid[2] = {q->nin, q->nout};
    for (int t = 0; t < 2; ++t) {
      hipLaunchKernelGGL(kr_zero_doubles, dim3(1), dim3(64), 0, st, q->dacc, 32);
      hipLaunchKernelGGL(kr_col_moments, dim3(1024), dim3(256), 0, st, (long)n, wid[t], src[t], q->dacc);
      hipLaunchKernelGGL(kr_finish_moments, dim3(1), dim3(64), 0, st, (long)n, wid[t], q->dacc,
                         q->norm + 32 * t, q->norm + 32 * t + 16);
      HIP_TRY(hipGetLastError());
    }
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_gradients(kr_guess *q, int32_t B, const float *X, const float *Y, float *grads,
                                  double *loss, kr_stream_t stream) {
  try {
    if (!q || B < 1 || !X || !Y) return fail(KR_EINVAL, "bad gradient arguments");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(q->device));
    int rc = guess_reserve(q, B);
    if (rc) return rc;
    if ((rc = guess_make_batch(q, B, B, 0, 0, 0, X, Y, st))) return rc;
    if ((rc = guess_forward(q, B, st))) return rc;
    if ((rc = guess_backward(q, B, st))) return rc;
    if (grads) HIP_TRY(hipMemcpyAsync(grads, q->g, sizeof(float) * q->nparams, hipMemcpyDeviceToDevice, st));
    if (loss) {
      double s = 0.0;
      HIP_TRY(hipMemcpyAsync(&s, q->dacc + 40, sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      *loss = s / ((double)B * q->nout);
    }
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_train(kr_guess *q, int64_t n, const float *X, const float *Y, const kr_train_opts *o,
                              double *last_loss, kr_stream_t stream) {
  try {
    if (!q || !o || n < 1 || !X || !Y || o->batch < 1 || o->steps < 0 || !(o->lr > 0.0f))
      return fail(KR_EINVAL, "bad training arguments");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(q->device));
    int rc = guess_reserve(q, o->batch);
    if (rc) return rc;
    const double pi = 3.14159265358979323846;
    for (int64_t t = 0; t < o->steps; ++t) {
      /* seed 0: consecutive blocks of rows (deterministic, for checks);
       * otherwise rows drawn uniformly with replacement */
      const unsigned long long seed = o->seed * 0x9e3779b97f4a7c15ull + (unsigned long long)(q->step + 1);
      long row0 = 0;
      if (o->seed == 0 && n >= o->batch) row0 = (long)((q->step * (int64_t)o->batch) % (n - o->batch + 1));
      if (o->seed == 0 && n < o->batch) return fail(KR_EINVAL, "sequential batches need n >= batch");
      if ((rc = guess_make_batch(q, o->batch, n, o->seed != 0, seed, row0, X, Y, st))) return rc;
      if ((rc = guess_forward(q, o->batch, st))) return rc;
      if ((rc = guess_backward(q, o->batch, st))) return rc;
      q->step++;
      /* cosine decay from lr to lr_min over this call's steps */
      const double frac = o->steps > 1 ? (double)t / (double)(o->steps - 1) : 1.0;
      const float lr = (float)(o->lr_min + 0.5 * (o->lr - o->lr_min) * (1.0 + std::cos(pi * frac)));
      const float c1 = (float)(1.0 - std::pow((double)o->beta1, (double)q->step));
      const float c2 = (float)(1.0 - std::pow((double)o->beta2, (double)q->step));
      hipLaunchKernelGGL(kr_adam, dim3(512), dim3(256), 0, st, q->nparams, q->w, q->wb, q->g, q->m, q->v, lr,
                         o->beta1, o->beta2, o->eps, c1, c2);
      HIP_TRY(hipGetLastError());
    }
    if (last_loss) {
      double s = 0.0;
      HIP_TRY(hipMemcpyAsync(&s, q->dacc + 40, sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
      *last_loss = s / ((double)o->batch * q->nout);
    }
    return KR_OK;
  } KR_CATCH
}

/* outputs (standardised) for n rows of raw features */
extern "C" int kr_guess_forward(kr_guess *q, int64_t n, const float *X, float *out, kr_stream_t stream) {
  try {
    if (!q || n < 0 || (n && (!X || !out))) return fail(KR_EINVAL, "bad forward arguments");
    hipStream_t st = (hipStream_t)stream;
    HIP_TRY(hipSetDevice(q->device));
    const int chunk = 65536;
    int rc = guess_reserve(q, (int)std::min<int64_t>(n, chunk));
    if (rc) return rc;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
      const int B = (int)std::min<int64_t>(chunk, n - r0);
      if ((rc = guess_make_batch(q, B, n, 0, 0, r0, X, nullptr, st))) return rc;
      if ((rc = guess_forward(q, B, st, false))) return rc;
      HIP_TRY(hipMemcpyAsync(out + (size_t)r0 * q->nout, q->out, sizeof(float) * B * q->nout,
                             hipMemcpyDeviceToDevice, st));
    }
    return KR_OK;
  } KR_CATCH
}

extern "C" int kr_guess_predict(kr_guess *q, int64_t n, const double *states, int64_t ld, const double *T,
                                const double *dt, double dt_scalar, float *X_scratch, double *guess,
                                int64_t guess_ld, kr_stream_t stream) {
  try {
    if (!q || n < 0 || ld < n || guess_ld < n || (n && (!states || !T || !X_scratch || !guess)))
      return fail(KR_EINVAL, "bad predict arguments");
    if (!n) return KR_OK;
    hipStream_t st = (hipStream_t)stream;
    int rc = kr_guess_features(q, n, states, ld, T, dt, dt_scalar, X_scratch, stream);
    if (rc) return rc;
    const int chunk = 65536;
    if ((rc = guess_reserve(q, (int)std::min<int64_t>(n, chunk)))) return rc;
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
      const int B = (int)std::min<int64_t>(chunk, n - r0);
      if ((rc = guess_make_batch(q, B, n, 0, 0, r0, X_scratch, nullptr, st))) return rc;
      if ((rc = guess_forward(q, B, st, false))) return rc;
      hipLaunchKernelGGL(kr_guess_apply_kernel, dim3((B + 255) / 256), dim3(256), 0, st, q->S, q->atoms, (long)n,
                         (long)r0, states, (long)ld, T, q->out, q->norm + 32, q->norm + 48, guess, (long)guess_ld);
      HIP_TRY(hipGetLastError());
    }
    return KR_OK;
  } KR_CATCH
}
