// Shared device/host helpers of libmercergp (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gp.h"

namespace mgp {

// MFMA operand / accumulator vector types.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short i16x8 __attribute__((ext_vector_type(8)));

// Per-dimension constants of the 1-D SE eigenpairs (Sec. 2.3, eqs. 14-16),
// stored as 4 doubles per input dimension in device memory:
//   [0] alpha*beta   (argument scale of H_{i-1}, eq. 15)
//   [1] delta^2      (Gaussian factor exp(-delta^2 x^2), eq. 15)
//   [2] sqrt(beta)   (gamma_1; the normalised recurrence carries the rest)
//   [3] unused
constexpr int kDimStride = 4;

// Largest dynamic LDS request of any kernel (160 KB per work-group on gfx950,
// less 1 KB kept for static __shared__ variables).
constexpr int kMaxDynLds = 159 * 1024;

// Layout of the per-model constant table (device, float64):
//   dimc[GP_MAX_P * 4]       per-dimension constants above
//   rc1[GP_MAX_N], rc2[GP_MAX_N]  normalised Hermite recurrence coefficients
//   lam1d[GP_MAX_P * GP_MAX_N]   1-D eigenvalues lambda_{j,k}
constexpr int kTabDim = 0;
constexpr int kTabRc1 = GP_MAX_P * kDimStride;
constexpr int kTabRc2 = kTabRc1 + GP_MAX_N;
constexpr int kTabLam1 = kTabRc2 + GP_MAX_N;
constexpr int kTabSize = kTabLam1 + GP_MAX_P * GP_MAX_N;

// 1-D eigenfunctions phi_1..phi_n at one x (eq. 15) through the normalised
// Hermite functions h_k = H_k / sqrt(2^k k!):
//   h_0 = 1, h_1 = sqrt(2) t, h_{k+1} = sqrt(2/(k+1)) t h_k - sqrt(k/(k+1)) h_{k-1}
//   phi_{k+1}(x) = sqrt(beta) exp(-delta^2 x^2) h_k(alpha beta x)
// which equals gamma_{k+1} exp(-delta^2 x^2) H_k(alpha beta x) and stays in
// range where H_k and gamma_k alone would not.  out[k*stride] = phi_{k+1}.
template <typename T, typename O>
__device__ __forceinline__ void phi_1d(T x, T ab, T d2, T sb, const T* __restrict__ rc1,
                                       const T* __restrict__ rc2, int n, O* out, int stride) {
  const T t = ab * x;
  const T e = sb * exp(-d2 * x * x);
  T h0 = T(1);
  T h1 = T(1.4142135623730951) * t;
  out[0] = (O)e;
  if (n > 1) out[stride] = (O)(e * h1);
  for (int k = 1; k + 1 < n; ++k) {
    const T h2 = rc1[k] * t * h1 - rc2[k] * h0;
    out[(k + 1) * stride] = (O)(e * h2);
    h0 = h1;
    h1 = h2;
  }
}

// Mixed-radix digits of column m (C order: last dimension fastest).
__device__ __forceinline__ void digits_of(int m, int p, int n, int* k) {
  for (int j = p - 1; j >= 0; --j) {
    k[j] = m % n;
    m /= n;
  }
}

// Optional per-phase event timing (phases: GP_PH_* of gp.h); p may be null.
struct Prof;
void prof_mark(Prof* p, int phase, bool begin, hipStream_t s);

__host__ __device__ __forceinline__ int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace mgp
