// Host build of the device rate-coefficient math (kr_math.h) for tests: the
// reciprocal estimate is a single-precision one (about 24 bits, like the
// hardware's), so the two Newton steps are exercised too.
#define KR_MATH_QUAL static inline
#define KR_MATH_RCP_ESTIMATE(x) ((double)(1.0f / (float)(x)))
#include "../paper_2504_04941_amd/csrc/kr_math.h"

extern "C" void kr_exp2_host(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = kr_exp2(x[i]);
}
extern "C" void kr_log2_host(const double *x, double *y, long n) {
  for (long i = 0; i < n; ++i) y[i] = kr_log2(x[i]);
}
