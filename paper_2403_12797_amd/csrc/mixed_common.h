// Device helpers shared by the mixed-precision kernels: split of FP32
// values into BF16 / FP16 terms, the MFMA wrappers, and the layout of the
// FP32 1-D eigenfunction tables that the Gram kernels stream.
#pragma once

#include "kernels.h"

namespace mgp {

__device__ __forceinline__ f32x16 mfma_bf16(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Round-to-nearest-even FP32 -> BF16 of two values, packed (lo half = a).
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
  typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
  bf16x2_t v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// The same with the packed word kept opaque to the compiler (an empty asm):
// otherwise it re-derives each unpacked half with a second conversion of
// one value, which costs a VALU instruction per half.
__device__ __forceinline__ uint32_t pack_bf16x2_opaque(float a, float b) {
  uint32_t w = pack_bf16x2(a, b);
  asm volatile("" : "+v"(w));
  return w;
}
__device__ __forceinline__ float bf16lo_f(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi_f(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Three-term BF16 split of a pair of FP32 values; returns packed (hi, mid, lo).
__device__ __forceinline__ void split3(float a, float b, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = pack_bf16x2_opaque(a, b);
  const float ra = a - bf16lo_f(h), rb = b - bf16hi_f(h);
  m = pack_bf16x2_opaque(ra, rb);
  const float sa = ra - bf16lo_f(m), sb = rb - bf16hi_f(m);
  l = pack_bf16x2(sa, sb);
}
__device__ __forceinline__ void split2(float a, float b, uint32_t& h, uint32_t& l) {
  h = pack_bf16x2(a, b);
  l = pack_bf16x2(a - bf16lo_f(h), b - bf16hi_f(h));
}

typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f32x16 mfma_f16(const f16x8& a, const f16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}
// Round-to-nearest-even FP32 -> FP16 of two values, packed (lo half = a).
__device__ __forceinline__ uint32_t pack_f16x2(float a, float b) {
  f16x2 v = {(_Float16)a, (_Float16)b};
  return __builtin_bit_cast(uint32_t, v);
}
// Two-term FP16 split of a pair of FP32 values; returns packed (hi, lo).
__device__ __forceinline__ void split2h(float a, float b, uint32_t& h, uint32_t& l) {
  h = pack_f16x2(a, b);
  asm volatile("" : "+v"(h));
  const f16x2 hv = __builtin_bit_cast(f16x2, h);
  l = pack_f16x2(a - (float)hv[0], b - (float)hv[1]);
}

// Layout of the FP32 1-D tables (written by phi1d_table_kernel):
//   tab32[s][j*n + k][16]  (s = sample / 16), zero for samples >= N,
// followed by kGmMaxWords words: the largest |value| of each row j*n + k
// over all samples (FP32 bits, which order like the magnitudes).
constexpr int kGmKC = 16;
constexpr int kGmMaxWords = GP_MAX_P * GP_MAX_N;
// Zero stages past the end let the kernel prefetch without bounds tests: a
// work-group reads at most four stages past its last one.
constexpr int kGmTabPad = 4;
__host__ __device__ inline int64_t gm_max_offset(int64_t N, int p, int n) {
  return (ceil_div(N, kGmKC) + kGmTabPad) * p * n * kGmKC;
}
// Exponent e(j,k) of a row's scale: the power of two that brings the row's
// largest magnitude into [0.5, 1) (zero rows: 0), raised by `top`; bounded
// so that 2^e stays a normal FP32 number.
__device__ __forceinline__ int gm_row_exp(unsigned maxbits, int top) {
  int e = 0;
  if (maxbits) {
    int E;
    frexpf(__uint_as_float(maxbits), &E);
    e = -E;
  }
  e += top;
  return min(max(e, -120), 100);
}

}  // namespace mgp
