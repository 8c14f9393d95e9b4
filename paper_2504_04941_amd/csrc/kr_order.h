/*
 * kr_order.h -- largest-expected-work-first order of a batch's cells for the
 * persistent integrator (gfx950).
 *
 * The integrator hands cells out through one atomic counter: a lane (lane
 * layout) or a wave (wave layout) that finishes a cell takes the next one.
 * Cells of one batch can differ in cost by orders of magnitude (substep
 * counts from 1 to 1e4 and more), and a wave is only done when its slowest
 * lane is: cells that start late and run long leave the other 63 lanes, and
 * in the end the other SIMDs, idle.  Handing out the expensive cells first
 * (longest-processing-time-first list scheduling) leaves only cheap cells
 * for the tail.
 *
 * Expected work of a cell: w = dt (sum_s |f_s| / sum_s n_s + |Q| / eps) at
 * its pre-processed input state, the relative change of the composition and
 * of the internal energy eps = T sum_s c_s n_s that the rates would cause
 * over the step if they stayed constant (the number of substeps an adaptive
 * BE integration needs grows with it).  Cells are sorted by a counting sort
 * on half-octaves of w (256 buckets, the largest first; order within a
 * bucket is arbitrary).  Each cell's result does not depend on the order.
 *
 * Passes (one stream): per-layout key kernel (kr_order_keys: bucket of each
 * cell, histogram) -> kr_order_scan (bucket start offsets, histogram cleared
 * for the next call) -> kr_order_scatter (order[position] = cell).
 */

#ifndef KR_ORDER_H
#define KR_ORDER_H

#define KR_ORDER_BUCKETS 256

/* Bucket of the expected work w: 2 log2 w + 128 clamped to [0, 255];
 * w <= 0 or NaN gives 0 (least work first-served last). */
__device__ __forceinline__ unsigned kr_work_bucket(double w) {
  if (!(w > 0.0)) return 0u;
  const double b = __builtin_floor(2.0 * kr_log2(w)) + 128.0;
  return (unsigned)__builtin_fmin(__builtin_fmax(b, 0.0), 255.0);
}

/* start[b] = number of cells in buckets above b (descending order); the
 * histogram is cleared for the next batch.  One wave: lane l owns buckets
 * 4l..4l+3. */
__device__ __forceinline__ void kr_order_scan_body(unsigned *hist, unsigned *start) {
  const int lane = threadIdx.x;
  unsigned h[4], t = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    h[k] = hist[4 * lane + k];
    t += h[k];
  }
  /* exclusive suffix sum of the lane totals over higher lanes */
  unsigned above = 0;
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const unsigned tl = (unsigned)__shfl((int)t, l);
    above += l > lane ? tl : 0u;
  }
  unsigned s = above;
#pragma unroll
  for (int k = 3; k >= 0; --k) {
    start[4 * lane + k] = s;
    s += h[k];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) hist[4 * lane + k] = 0u;
}

/* order[start[bucket[c]]++] = c.  Positions stay below n when the
 * histogram counted exactly this batch (the host serialises the passes);
 * the bound check only keeps a broken sequence from writing out of range. */
__device__ __forceinline__ void kr_order_scatter_body(long long n, const unsigned char *bucket,
                                                      unsigned *start, unsigned *order) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const unsigned pos = atomicAdd(&start[bucket[c]], 1u);
    if ((long long)pos < n) order[pos] = (unsigned)c;
  }
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_order_scan(unsigned *hist, unsigned *start) {
  kr_order_scan_body(hist, start);
}

extern "C" __global__ void __launch_bounds__(64, 1) kr_order_scatter(long long n, const unsigned char *bucket,
                                                                     unsigned *start, unsigned *order) {
  kr_order_scatter_body(n, bucket, start, order);
}

#endif /* KR_ORDER_H */
