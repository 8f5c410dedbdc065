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

// Per-dimension constants of the 1-D eigenpairs, stored as 4 doubles per
// input dimension in device memory.  SE kernel (Sec. 2.3, eqs. 14-16):
//   [0] alpha*beta   (argument scale of H_{i-1}, eq. 15)
//   [1] delta^2      (Gaussian factor exp(-delta^2 x^2), eq. 15)
//   [2] sqrt(beta)   (gamma_1; the normalised recurrence carries the rest)
//   [3] 0            (the kernel family, gp_kernel)
// periodic kernel: [0] alpha (angular frequency), [1] 0, [2] 1, [3] 1.
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

// 1-D eigenfunctions phi_1..phi_n at one x, out[k*stride] = phi_{k+1}; dc
// the dimension's 4 constants above.  SE (eq. 15), through the normalised
// Hermite functions h_k = H_k / sqrt(2^k k!):
//   h_0 = 1, h_1 = sqrt(2) t, h_{k+1} = sqrt(2/(k+1)) t h_k - sqrt(k/(k+1)) h_{k-1}
//   phi_{k+1}(x) = sqrt(beta) exp(-delta^2 x^2) h_k(alpha beta x)
// which equals gamma_{k+1} exp(-delta^2 x^2) H_k(alpha beta x) and stays in
// range where H_k and gamma_k alone would not.  Periodic: phi_1 = 1,
// phi_{2k} = sqrt2 cos(k theta), phi_{2k+1} = sqrt2 sin(k theta), theta =
// alpha x, the harmonics by rotation from (cos theta, sin theta).
template <typename T, typename O>
__device__ __forceinline__ void phi_1d(T x, const T* __restrict__ dc, const T* __restrict__ rc1,
                                       const T* __restrict__ rc2, int n, O* out, int stride) {
  if (dc[3] != T(0)) {
    T s1, c1;
    sincos(dc[0] * x, &s1, &c1);
    T c = c1, s = s1;
    out[0] = (O)1;
    for (int k = 1; 2 * k - 1 < n; ++k) {
      out[(2 * k - 1) * stride] = (O)(T(1.4142135623730951) * c);
      if (2 * k < n) out[2 * k * stride] = (O)(T(1.4142135623730951) * s);
      const T cn = c * c1 - s * s1;
      s = s * c1 + c * s1;
      c = cn;
    }
    return;
  }
  const T ab = dc[0], d2 = dc[1], sb = dc[2];
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
