// Mixed-precision kernels: fused Phi-generation + split-FP16 MFMA Gram (a3)
// and the split-BF16 predictive variance with the fused FP64 mean (a5).
//
// Gram scaling.  Every 1-D table row (dimension j, order k) is scaled by a
// power of two 2^e(j,k) that brings its largest magnitude over the samples
// into [0.5, 1), the last dimension's rows by a further 2^15, so each scaled
// Phi value lies below 2^15 (inside the FP16 range) and a column's scale is
// 2^(sum of its rows' exponents); the finished tile is unscaled by the exact
// power of two of its row and column.  Two Gram schemes, FP32 accumulation:
//  * split-FP16: v = hi + lo with hi = f16(v), lo = f16(v - hi), both
//    round-to-nearest-even (the subtraction is exact in FP32), about 22
//    significant bits; a*b as the three products ah*bh + ah*bl + al*bh.
//  * split-BF16: v = hi + mid + lo, each term bf16 of the remainder; a*b as
//    the six products of relative order >= 2^-16:
//    ah*bh + ah*bm + am*bh + ah*bl + al*bh + am*bm.
//
// Split-BF16 arithmetic (variance).  v = hi + lo with hi = bf16(v), lo =
// bf16(v - hi); a product is taken as ah*bh + ah*bl + al*bh.
//
// MFMA v_mfma_f32_32x32x16_{f16,bf16} operand layout (lane l of a wave64):
//   A (32 x 16): lane l holds A[l % 32][8*(l/32) .. 8*(l/32)+7]
//   B (16 x 32): lane l holds B[8*(l/32) .. +7][l % 32]
//   D (32 x 32): element r of the lane's float16 is
//                D[8*(r/4) + 4*(l/32) + (r%4)][l % 32]
#include <stdlib.h>
#include <string.h>

#include "mixed_common.h"

namespace mgp {

// ================================================================ a3 mixed Gram
// Pre-pass: the 1-D eigenfunctions of every sample, computed in FP64 and
// stored as FP32 in stage-contiguous blocks of 16 samples, with the row
// maxima (layout in mixed_common.h).
constexpr int kGmTableBlocks = 1024;

// Grid-stride over (stage, dimension, sample-in-stage); the 16 lanes of one
// (stage, dimension) are consecutive and reduce their maxima by shuffles,
// the work-group through LDS, then one atomic per row and work-group.
__global__ void __launch_bounds__(256) phi1d_table_kernel(const double* __restrict__ x, int64_t N, int p, int n,
                                                          const double* __restrict__ tab, float* __restrict__ out,
                                                          int64_t nstage, unsigned* __restrict__ tmax) {
  __shared__ unsigned smax[kGmMaxWords];
  for (int r = threadIdx.x; r < p * n; r += blockDim.x) smax[r] = 0u;
  __syncthreads();
  const int64_t total = nstage * p * kGmKC;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < total; u += stride) {
    const int i = (int)(u % kGmKC);
    const int j = (int)((u / kGmKC) % p);
    const int64_t st = u / ((int64_t)kGmKC * p);
    const int64_t row = st * kGmKC + i;
    float* o = out + (st * p * n + (int64_t)j * n) * kGmKC + i;
    // SE: phi_{k+1}(x) = sqrt(beta) exp(-delta^2 x^2) h_k(alpha beta x), h_k
    // the normalised Hermite recurrence (eq. 15); periodic: 1, then sqrt2 cos
    // and sqrt2 sin of each harmonic of alpha x (as phi_1d); zero past the
    // last sample
    const double* dc = tab + kTabDim + j * kDimStride;
    const double* rc1 = tab + kTabRc1;
    const double* rc2 = tab + kTabRc2;
    const bool live = row < N;
    const bool per = dc[3] != 0.0;
    const double xv = live ? x[row * p + j] : 0.0;
    const double t = dc[0] * xv;
    const double e = live ? (per ? 1.0 : dc[2] * exp(-dc[1] * xv * xv)) : 0.0;
    double h0 = 1.0, h1 = 1.4142135623730951 * t;
    double s1 = 0.0, c1 = 1.0;
    if (per) sincos(t, &s1, &c1);
    double hc = c1, hs = s1;   // periodic: cos and sin of the current harmonic
    for (int k = 0; k < n; ++k) {
      double hk;
      if (k == 0) {
        hk = 1.0;
      } else if (per) {
        if (k & 1) {
          hk = 1.4142135623730951 * hc;
        } else {
          hk = 1.4142135623730951 * hs;
          const double cn = hc * c1 - hs * s1;
          hs = hs * c1 + hc * s1;
          hc = cn;
        }
      } else if (k == 1) {
        hk = h1;
      } else {
        hk = rc1[k - 1] * t * h1 - rc2[k - 1] * h0;
        h0 = h1;
        h1 = hk;
      }
      const float v = (float)(e * hk);
      o[k * kGmKC] = v;
      unsigned m = __float_as_uint(fabsf(v));
#pragma unroll
      for (int off = 1; off < kGmKC; off <<= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, kGmKC));
      if (i == 0 && m) atomicMax(&smax[j * n + k], m);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < p * n; r += blockDim.x)
    if (smax[r]) atomicMax(&tmax[r], smax[r]);
}

// Last dimension's rows are raised by a further 2^15 (see the scaling note).
constexpr int kGmF16Top = 15;

// Gram work-group: rows I*256..+256 and columns J*256 + h*128..+128 (half h
// of the J-block) of Phi^T Phi, I <= J, over one chunk of samples.  512
// threads = 8 waves in a 4 (rows) x 2 (cols) grid, each owning 64 x 64
// outputs = 2 x 2 MFMA 32x32 blocks (two waves per SIMD).
// Stage = 16 samples.  A column c = hi*n + k (k its last digit) has
// Phi[i, c] = PRE[hi][i] * phi_{p-1,k}(x_i), where PRE is the product of the
// leading p-1 factors.  Per stage the work-group forms PRE once per column
// prefix it needs, then every thread generates 8 samples of one I-block
// column and 4 samples of one J-half column with one multiply each, splits
// them into the scheme's terms (two FP16 or three BF16) and stores them in
// LDS as [term][column slot][16 samples] (slot pitch padded against bank
// conflicts).  Pipeline (one barrier per stage): while the MFMAs of stage t
// run, the work-group generates stage t+1, forms PRE of stage t+2 and
// streams the 1-D tables of stage t+3 from memory.
// Accumulation: the MFMAs accumulate into a fresh FP32 register block for
// kG2Flush stages, which is then added into the running FP32 sum with
// round-to-nearest VALU adds.  Long MFMA accumulation chains drift
// systematically (the hardware's FP32 accumulation is not round-to-nearest);
// short chains plus rounded adds keep the Gram error unbiased.
constexpr int kGmT = 256;                                   // tile edge of the partial layout
constexpr int kG2H = 128;                                   // columns per work-group
constexpr int kG2Threads = 512;
constexpr int kG2Flush = 16;                                // stages per MFMA chain
constexpr int kG2Slots = kGmT + kG2H;                       // 384 column slots per stage
constexpr int kG2SlotPitch = kGmKC + 8;                     // f16 per slot (16 samples + pad)
constexpr int kG2TabPitch = kGmKC + 4;                      // floats per table / prefix row (16 + pad)
constexpr int kGmChunk = 32768;                             // samples per FP32 partial
constexpr int64_t kGmPartCap = 8ll << 30;                   // bytes of partials per pass
// 16-bit elements per stage buffer: [term][slot][sample]
__host__ __device__ constexpr int gm_stage_elems(bool f16) { return (f16 ? 2 : 3) * kG2Slots * kG2SlotPitch; }

// Paired layout where pair_plan accepts it, unless MGP_GRAM_LAYOUT=direct.
static bool pair_allowed() {
  const char* v = getenv("MGP_GRAM_LAYOUT");
  return !(v && strcmp(v, "direct") == 0);
}

GramPlan gram_mixed_plan(int64_t N, int p, int n, int M, bool f16, int chunk) {
  GramPlan g{};
  g.T = (int)ceil_div(M, kGmT);
  if (pair_allowed() && pair_plan(p, n, M, f16, g)) {
    pair_plan_splits(N, g, chunk);
    return g;
  }
  g.ntiles = g.T * (g.T + 1) / 2;
  if (chunk <= 0) {
    // enough work items to fill the GPU several times over: chunks of 1024..32768 samples
    const int64_t want = ceil_div(N * 2 * g.ntiles, 1024);
    chunk = (int)std::min<int64_t>(kGmChunk, std::max<int64_t>(1024, ceil_div(want, kGmKC) * kGmKC));
  }
  g.chunk = (int)ceil_div(chunk, kGmKC) * kGmKC;
  g.splits_total = (int)ceil_div(N, g.chunk);
  const int64_t per_split = (int64_t)g.ntiles * kGmT * kGmT * sizeof(float);
  int64_t sp = kGmPartCap / per_split;
  if (sp < 1) sp = 1;
  if (sp > g.splits_total) sp = g.splits_total;
  g.splits_per_pass = (int)sp;
  g.passes = (int)ceil_div(g.splits_total, sp);
  return g;
}

int64_t gram_mixed_part_elems(const GramPlan& g) {
  return (int64_t)g.splits_per_pass * g.ntiles * (g.pair ? kGmT * kG2H : kGmT * kGmT);
}
int64_t gram_mixed_hbuf_elems(const GramPlan& g) { return g.pair ? (int64_t)g.S1 * g.S2 : 0; }

int64_t gram_mixed_table_elems(int64_t N, int p, int n) { return gm_max_offset(N, p, n) + kGmMaxWords; }

// Prefix rows per stage: I-block prefixes then J-half prefixes (L consecutive
// columns hold at most L/n + 2 distinct prefixes).
__host__ __device__ inline int gm_pre_rows_i(int n, int M) { return min(kGmT, M) / n + 2; }
__host__ __device__ inline int gm_pre_rows(int n, int M) { return gm_pre_rows_i(n, M) + min(kG2H, M) / n + 2; }

static size_t gram_lds_bytes(int p, int n, int M, bool f16) {
  return 2 * (size_t)gm_stage_elems(f16) * 2 + 3 * (size_t)p * n * kG2TabPitch * sizeof(float) +
         2 * (size_t)(gm_pre_rows(n, M) + 1) * kG2TabPitch * sizeof(float) + kG2Slots * sizeof(int) +
         (size_t)gm_pre_rows(n, M) * GP_MAX_P * sizeof(uint16_t) + 16;
}

// Split NS values into the scheme's terms and store them at [term][slot][s_off..].
template <bool F16, int NS, typename E>
__device__ __forceinline__ void gm_store(const float* v, E* __restrict__ stage, int slot, int s_off) {
  constexpr int NT = F16 ? 2 : 3;
  uint32_t w[NT][NS / 2];
#pragma unroll
  for (int q = 0; q < NS / 2; ++q) {
    if constexpr (F16)
      split2h(v[2 * q], v[2 * q + 1], w[0][q], w[1][q]);
    else
      split3(v[2 * q], v[2 * q + 1], w[0][q], w[1][q], w[2][q]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    E* d = stage + (t * kG2Slots + slot) * kG2SlotPitch + s_off;
    if constexpr (NS == 8)
      *reinterpret_cast<uint4*>(d) = uint4{w[t][0], w[t][1], w[t][2], w[t][3]};
    else
      *reinterpret_cast<uint2*>(d) = uint2{w[t][0], w[t][1]};
  }
}

// One work item: tile `tile` (upper-triangle index), half h, samples
// [r0, r0 + chunk) of a problem; writes the item's FP32 partial 256x256 tile
// (half h) at `out`.
template <bool F16>
__device__ __forceinline__ void gram_item(unsigned char* smraw, const float* __restrict__ tab32, int64_t N, int P,
                                          int n, int M, int T, int tile, int h, int64_t r0, int chunk,
                                          float* __restrict__ out) {
  // LDS: two stage buffers of split Phi, three 1-D table buffers, two prefix
  // buffers.  Addressed as base + offset so the compiler keeps them in LDS.
  using E = std::conditional_t<F16, _Float16, __bf16>;
  using V8 = std::conditional_t<F16, f16x8, bf16x8>;
  constexpr int NT = F16 ? 2 : 3;                 // terms per value
  constexpr int SE = gm_stage_elems(F16);
  E* const stg0 = reinterpret_cast<E*>(smraw);
  float* const tb0 = reinterpret_cast<float*>(smraw + 2 * SE * sizeof(E));
  const int rows = P * n;                       // 1-D table rows per stage
  const int tbs = rows * kG2TabPitch;           // floats per table buffer
  float* const pr0 = tb0 + 3 * tbs;
  // prefix buffers: gm_pre_rows prefix rows, then a zero row that invalid
  // columns use as their prefix, so they generate zeros
  const int zrow = gm_pre_rows(n, M);
  const int prs = (zrow + 1) * kG2TabPitch;     // floats per prefix buffer
  // per column slot: the exponent of its scale (sum over its table rows)
  int* const csc = reinterpret_cast<int*>(pr0 + 2 * prs);
  // per prefix row: the 1-D table rows of its leading digits (rows with no
  // prefix take row 0 and are never referenced)
  uint16_t* const pre_off = reinterpret_cast<uint16_t*>(csc + kG2Slots);
  const unsigned* const tmax = reinterpret_cast<const unsigned*>(tab32 + gm_max_offset(N, P, n));
  const int tchunks = rows * (kGmKC / 4);       // float4 per stage of the table

  int I = 0;
  while (tile >= T - I) {
    tile -= T - I;
    ++I;
  }
  const int J = I + tile;
  const bool diag = (I == J);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;

  // column ranges and their first prefixes
  const int cI0 = I * kGmT, cJ0 = J * kGmT + h * kG2H;
  const int hiI0 = cI0 / n, hiJ0 = cJ0 / n;
  const int nhiI = (min(cI0 + kGmT, M) - 1) / n - hiI0 + 1;   // prefixes used by the I-block
  const int nhiJ = diag ? 0 : (min(cJ0 + kG2H, M) - 1) / n - hiJ0 + 1;

  // generation roles (consecutive lanes take consecutive columns, so the
  // table reads of a wave fall in distinct LDS banks):
  //   I-block column tid & 255, samples (tid >> 8)*8 .. +8;
  //   J-half column tid & 127, samples (tid >> 7)*4 .. +4 (off-diagonal tiles only)
  const int sI = (tid >> 8) * 8, sJ = (tid >> 7) * 4;
  const int colI = cI0 + (tid & 255);
  const bool validI = colI < M;
  const int preI = (validI ? colI / n - hiI0 : zrow) * kG2TabPitch + sI;
  const int lastI = ((P - 1) * n + (validI ? colI % n : 0)) * kG2TabPitch + sI;
  const int colJ = cJ0 + (tid & 127);
  const bool genJ = !diag;
  const bool validJ = genJ && colJ < M;
  const int preJ = (validJ ? gm_pre_rows_i(n, M) + colJ / n - hiJ0 : zrow) * kG2TabPitch + sJ;
  const int lastJ = ((P - 1) * n + (validJ ? colJ % n : 0)) * kG2TabPitch + sJ;
  const int jslot = diag ? h * kG2H : kGmT;  // B operand columns start here in a stage

  f32x16 acc[2][2], sum[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[a][b][r] = 0.0f;
        sum[a][b][r] = 0.0f;
      }

  int64_t r1 = r0 + chunk;
  if (r1 > N) r1 = N;
  const int nst = (int)ceil_div(r1 - r0, kGmKC);
  const int64_t st0 = r0 / kGmKC;

  // 1-D tables of one stage: at most 128 rows x 16 floats = 512 float4, one per thread
  // (requested two stages before they are stored, alternating between two
  // registers, so the global latency is hidden behind two stages of work)
  // (each thread stores one table row's 4 samples, scaled by the row's 2^e)
  float4 treg0, treg1;
  const int trow = tid / (kGmKC / 4);
  const float tsc = tid < tchunks ? ldexpf(1.0f, gm_row_exp(tmax[trow], trow >= (P - 1) * n ? kGmF16Top : 0)) : 0.0f;
  auto load_tab = [&](int64_t gst, float4& r) {
    if (tid < tchunks) r = reinterpret_cast<const float4*>(tab32 + gst * rows * kGmKC)[tid];
  };
  auto store_tab = [&](float* dst, const float4& r) {
    if (tid < tchunks) {
      const int c4 = tid % (kGmKC / 4);
      *reinterpret_cast<float4*>(dst + trow * kG2TabPitch + c4 * 4) =
          float4{r.x * tsc, r.y * tsc, r.z * tsc, r.w * tsc};
    }
  };
  // prefix rows of one stage from its 1-D tables, in items of (row, 4
  // samples).  Item tid's table-row offsets are held in registers for the
  // whole work item; items past 512 (only when n <= 2) read them from
  // pre_off in LDS.
  const int npre = gm_pre_rows(n, M);
  int mp_off[GP_MAX_P - 1];
  const bool mp_own = tid < npre * 4;
  const int mp_dst = (tid >> 2) * kG2TabPitch + (tid & 3) * 4;
  // (one unrolled body per factor count, so all reads issue before the products)
  auto make_pre_k = [&](auto kc, const float* Tb, float* dst) {
    constexpr int K = decltype(kc)::value;
    float4 f[K > 0 ? K : 1];
#pragma unroll
    for (int j = 0; j < K; ++j) f[j] = *reinterpret_cast<const float4*>(Tb + mp_off[j]);
    float4 v = float4{1.f, 1.f, 1.f, 1.f};
#pragma unroll
    for (int j = 0; j < K; ++j) {
      v.x *= f[j].x;
      v.y *= f[j].y;
      v.z *= f[j].z;
      v.w *= f[j].w;
    }
    *reinterpret_cast<float4*>(dst + mp_dst) = v;
  };
  auto make_pre = [&](const float* Tb, float* dst) {
    if (mp_own) {
      switch (P - 1) {
        case 0: make_pre_k(std::integral_constant<int, 0>{}, Tb, dst); break;
        case 1: make_pre_k(std::integral_constant<int, 1>{}, Tb, dst); break;
        case 2: make_pre_k(std::integral_constant<int, 2>{}, Tb, dst); break;
        case 3: make_pre_k(std::integral_constant<int, 3>{}, Tb, dst); break;
        case 4: make_pre_k(std::integral_constant<int, 4>{}, Tb, dst); break;
        case 5: make_pre_k(std::integral_constant<int, 5>{}, Tb, dst); break;
        case 6: make_pre_k(std::integral_constant<int, 6>{}, Tb, dst); break;
        default: make_pre_k(std::integral_constant<int, 7>{}, Tb, dst); break;
      }
    }
    if (npre * 4 > kG2Threads) {
      for (int u = tid + kG2Threads; u < npre * 4; u += kG2Threads) {
        const int pr = u >> 2, q4 = (u & 3) * 4;
        const uint16_t* po = pre_off + pr * GP_MAX_P;
        float4 v = float4{1.f, 1.f, 1.f, 1.f};
        for (int j = 0; j < P - 1; ++j) {
          const float4 f = *reinterpret_cast<const float4*>(Tb + po[j] * kG2TabPitch + q4);
          v.x *= f.x;
          v.y *= f.y;
          v.z *= f.z;
          v.w *= f.w;
        }
        *reinterpret_cast<float4*>(dst + pr * kG2TabPitch + q4) = v;
      }
    }
  };
  // generation inputs of one stage (prefix and last-factor values) into
  // registers, then products, split and store
  struct GenIn {
    float4 pa[2], la[2], pj, lj;
  };
  auto gen_read = [&](const float* Tb, const float* Pr, GenIn& g) {
    const float4* pa = reinterpret_cast<const float4*>(Pr + preI);
    const float4* la = reinterpret_cast<const float4*>(Tb + lastI);
    g.pa[0] = pa[0];
    g.pa[1] = pa[1];
    g.la[0] = la[0];
    g.la[1] = la[1];
    g.pj = *reinterpret_cast<const float4*>(Pr + preJ);
    g.lj = *reinterpret_cast<const float4*>(Tb + lastJ);
  };
  auto gen_store = [&](const GenIn& g, E* D) {
    {
      float v[8];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        v[4 * q] = g.pa[q].x * g.la[q].x;
        v[4 * q + 1] = g.pa[q].y * g.la[q].y;
        v[4 * q + 2] = g.pa[q].z * g.la[q].z;
        v[4 * q + 3] = g.pa[q].w * g.la[q].w;
      }
      gm_store<F16, 8>(v, D, tid & 255, sI);
    }
    {
      // J half (on diagonal tiles these slots are unused and get zeros)
      // (invalid columns read the zero prefix row)
      float v[4];
      v[0] = g.pj.x * g.lj.x;
      v[1] = g.pj.y * g.lj.y;
      v[2] = g.pj.z * g.lj.z;
      v[3] = g.pj.w * g.lj.w;
      gm_store<F16, 4>(v, D, kGmT + (tid & 127), sJ);
    }
  };
  auto generate = [&](const float* Tb, const float* Pr, E* D) {
    GenIn g;
    gen_read(Tb, Pr, g);
    gen_store(g, D);
  };

  for (int pr = tid; pr < gm_pre_rows(n, M); pr += kG2Threads) {
    int hi = -1;
    if (pr < nhiI) hi = hiI0 + pr;
    else if (pr >= gm_pre_rows_i(n, M) && pr - gm_pre_rows_i(n, M) < nhiJ) hi = hiJ0 + pr - gm_pre_rows_i(n, M);
    uint16_t* po = pre_off + pr * GP_MAX_P;
    int rem = hi < 0 ? 0 : hi;
    for (int j = P - 2; j >= 0; --j) {
      po[j] = (uint16_t)(j * n + rem % n);
      rem /= n;
    }
  }
  {
    // the same rows for item tid, in registers
    const int pr = tid >> 2;
    int hi = -1;
    if (pr < nhiI) hi = hiI0 + pr;
    else if (pr >= gm_pre_rows_i(n, M) && pr - gm_pre_rows_i(n, M) < nhiJ) hi = hiJ0 + pr - gm_pre_rows_i(n, M);
    int rem = hi < 0 ? 0 : hi;
#pragma unroll
    for (int j = GP_MAX_P - 2; j >= 0; --j) {
      mp_off[j] = 0;
      if (j < P - 1) {
        mp_off[j] = (j * n + rem % n) * kG2TabPitch + (tid & 3) * 4;
        rem /= n;
      }
    }
  }
  // zero rows of both prefix buffers
  if (tid < kG2TabPitch) {
    pr0[zrow * kG2TabPitch + tid] = 0.0f;
    pr0[prs + zrow * kG2TabPitch + tid] = 0.0f;
  }
  for (int sl = tid; sl < kG2Slots; sl += kG2Threads) {
    const int c = sl < kGmT ? cI0 + sl : cJ0 + sl - kGmT;
    int e = 0;
    if (c < M && (sl < kGmT || genJ)) {
      int rem = c;
      for (int j = P - 1; j >= 0; --j) {
        e += gm_row_exp(tmax[j * n + rem % n], j == P - 1 ? kGmF16Top : 0);
        rem /= n;
      }
    }
    csc[sl] = e;
  }
  // (pre_off is read after the prologue's first barrier)
  // prologue: tables of stages 0..2, prefixes of stages 0..1, Phi of stage 0
  load_tab(st0, treg0);
  store_tab(tb0, treg0);
  load_tab(st0 + 1, treg0);
  store_tab(tb0 + tbs, treg0);
  load_tab(st0 + 2, treg0);
  store_tab(tb0 + 2 * tbs, treg0);
  load_tab(st0 + 3, treg1);
  __syncthreads();
  make_pre(tb0, pr0);
  make_pre(tb0 + tbs, pr0 + prs);
  __syncthreads();
  generate(tb0, pr0, stg0);
  __syncthreads();

  // one stage: MFMAs on stage st, generation of st+1, prefixes of st+2,
  // tables of st+3 stored (from Rstore, requested one stage earlier) and
  // tables of st+4 requested into Rload.  Stages alternate the registers.
  auto stage = [&](int st, float4& Rload, const float4& Rstore) {
    load_tab(st0 + st + 4, Rload);
    // inputs of stage st+1 (past the chunk end they produce unused values)
    GenIn gin;
    gen_read(tb0 + ((st + 1) % 3) * tbs, pr0 + ((st + 1) & 1) * prs, gin);
    const E* S = stg0 + (st & 1) * SE;
    V8 aop[2][NT], bop[2][NT];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int q = 0; q < NT; ++q)
        bop[cb][q] = *reinterpret_cast<const V8*>(
            S + (q * kG2Slots + jslot + wc * 64 + cb * 32 + (lane & 31)) * kG2SlotPitch + (lane >> 5) * 8);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < NT; ++q)
        aop[rb][q] = *reinterpret_cast<const V8*>(
            S + (q * kG2Slots + wr * 64 + rb * 32 + (lane & 31)) * kG2SlotPitch + (lane >> 5) * 8);
    // the scheme's products (smallest first), interleaved over the four accumulators
    auto prod = [&](int qa, int qb) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          if constexpr (F16)
            acc[rb][cb] = mfma_f16(aop[rb][qa], bop[cb][qb], acc[rb][cb]);
          else
            acc[rb][cb] = mfma_bf16(aop[rb][qa], bop[cb][qb], acc[rb][cb]);
        }
    };
    if constexpr (!F16) {
      prod(1, 1);   // mid*mid
      prod(2, 0);   // lo*hi
      prod(0, 2);   // hi*lo
      prod(1, 0);   // mid*hi
      prod(0, 1);   // hi*mid
    } else {
      prod(1, 0);   // lo*hi
      prod(0, 1);   // hi*lo
    }
    prod(0, 0);     // hi*hi
    gen_store(gin, stg0 + ((st + 1) & 1) * SE);
    make_pre(tb0 + ((st + 2) % 3) * tbs, pr0 + (st & 1) * prs);
    store_tab(tb0 + (st % 3) * tbs, Rstore);
    __syncthreads();
  };

  for (int g0 = 0; g0 < nst; g0 += kG2Flush) {
    const int gend = min(g0 + kG2Flush, nst);
    for (int st = g0; st < gend; st += 2) {
      stage(st, treg0, treg1);
      if (st + 1 < gend) stage(st + 1, treg1, treg0);
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          sum[a][b][r] += acc[a][b][r];
          acc[a][b][r] = 0.0f;
        }
  }

#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 64 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int cl = h * kG2H + wc * 64 + cb * 32 + (lane & 31);
        const int cs = jslot + wc * 64 + cb * 32 + (lane & 31);   // the column's slot
        out[row * kGmT + cl] = ldexpf(sum[rb][cb][r], -(csc[row] + csc[cs]));
      }
}

// A (+)= sum of the pass's FP32 partials in split order (FP64); the first pass
// also adds reg on the diagonal.  Writes both triangles.
// Single problem: grid (2 * ntiles, splits of this pass).
template <bool F16>
__global__ void __launch_bounds__(kG2Threads) gram_mixed_kernel(const float* __restrict__ tab32, int64_t N, int p,
                                                                int n, int M, int T, int split0, int chunk,
                                                                float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  const int ntiles = T * (T + 1) / 2;
  const int tile = blockIdx.x >> 1;
  float* out = part + ((int64_t)blockIdx.y * ntiles + tile) * (kGmT * kGmT);
  gram_item<F16>(smraw, tab32, N, p, n, M, T, tile, blockIdx.x & 1, (int64_t)(split0 + blockIdx.y) * chunk, chunk, out);
}

// Many problems in one persistent launch: work-groups take items from a
// longest-first list through an atomic counter until it runs out.
template <bool F16>
__global__ void __launch_bounds__(kG2Threads) gram_mixed_batch_kernel(const GramProb* __restrict__ probs,
                                                                      const GramItem* __restrict__ items, int nitems,
                                                                      int* __restrict__ counter) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  __shared__ int next;
  while (true) {
    __syncthreads();
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = next;
    if (it >= nitems) break;
    const GramItem wi = items[it];
    const GramProb pr = probs[wi.prob];
    const int ntiles = pr.T * (pr.T + 1) / 2;
    float* out = pr.part + ((int64_t)wi.split * ntiles + wi.tile) * (kGmT * kGmT);
    gram_item<F16>(smraw, pr.tab32, pr.N, pr.p, pr.n, pr.M, pr.T, wi.tile, wi.h, (int64_t)wi.split * pr.chunk, pr.chunk,
              out);
  }
}

__global__ void reset_counter_kernel(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// One 64x64 tile of the upper triangle per work-group: each element sums
// its splits in split order in FP64 (256 threads, 16 elements each), then
// the tile is written to A and, transposed through LDS, to its mirror
// image, both with row-contiguous stores.
__global__ void __launch_bounds__(256) gram_mixed_reduce_kernel(const float* __restrict__ part, int splits, int T,
                                                                int M, const double* __restrict__ reg, int first,
                                                                double* __restrict__ A) {
  __shared__ double tr[64][65];
  const int T64 = (M + 63) / 64;
  int t = blockIdx.x, R = 0;                 // upper-triangle 64-tile (R, C), C >= R
  while (t >= T64 - R) {
    t -= T64 - R;
    ++R;
  }
  const int C = R + t;
  const int g0 = R * 64, h0 = C * 64;
  const int I = g0 / kGmT, J = h0 / kGmT;    // the 256-tile holding this 64-tile
  const int ti = I * T - I * (I - 1) / 2 + (J - I);
  const int64_t ntile = (int64_t)(T * (T + 1) / 2) * kGmT * kGmT;
  const int c = threadIdx.x & 63, r0 = threadIdx.x >> 6;
  const int h = h0 + c;
  double s[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int g = g0 + r0 + 4 * q;
    s[q] = first ? ((g == h && g < M) ? reg[g] : 0.0) : ((g < M && h < M) ? A[(int64_t)g * M + h] : 0.0);
  }
  const int64_t base = (int64_t)ti * kGmT * kGmT + (int64_t)(g0 - I * kGmT) * kGmT + (h0 - J * kGmT) + c;
  for (int k = 0; k < splits; ++k) {
    const float* pk = part + (int64_t)k * ntile + base;
#pragma unroll
    for (int q = 0; q < 16; ++q) s[q] += (double)pk[(int64_t)(r0 + 4 * q) * kGmT];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int g = g0 + r0 + 4 * q;
    if (g < M && h < M && h >= g) A[(int64_t)g * M + h] = s[q];
    tr[r0 + 4 * q][c] = s[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int hh = h0 + r0 + 4 * q, gg = g0 + c;   // A[hh][gg] = A[gg][hh]
    if (hh < M && gg < M && hh > gg) A[(int64_t)hh * M + gg] = tr[c][r0 + 4 * q];
  }
}

size_t gram_mixed_lds_bytes(int p, int n, int M, const GramPlan& g, bool f16) {
  return g.pair ? pair_gram_lds_bytes(p, n, g, f16) : gram_lds_bytes(p, n, M, f16);
}

void launch_gram_mixed_table(const double* x, int64_t N, int p, int n, const double* tab, float* tab32,
                             hipStream_t s) {
  const int64_t nstage = ceil_div(N, kGmKC) + kGmTabPad;
  unsigned* tmax = reinterpret_cast<unsigned*>(tab32 + gm_max_offset(N, p, n));
  launch_fill_zero_int(reinterpret_cast<int*>(tmax), p * n, s);
  const int blocks = (int)std::min<int64_t>(kGmTableBlocks, ceil_div(nstage * p * kGmKC, 256));
  hipLaunchKernelGGL(phi1d_table_kernel, dim3(blocks), dim3(256), 0, s, x, N, p, n, tab, tab32, nstage, tmax);
}

void launch_gram_mixed(const double* x, int64_t N, int p, int n, int M, const GramPlan& g, bool f16,
                       const double* tab, const double* reg, float* part, float* tab32, double* hbuf, double* A,
                       hipStream_t s, Prof* prof) {
  if (g.pair) {
    launch_gram_pair(N, p, n, M, g, f16, reg, part, tab32, hbuf, A, s, prof);
    return;
  }
  for (int ps = 0; ps < g.passes; ++ps) {
    const int split0 = ps * g.splits_per_pass;
    const int cnt = std::min(g.splits_per_pass, g.splits_total - split0);
    prof_mark(prof, GP_PH_GRAM, true, s);
    hipLaunchKernelGGL(f16 ? gram_mixed_kernel<true> : gram_mixed_kernel<false>, dim3(2 * g.ntiles, cnt),
                       dim3(kG2Threads), gram_lds_bytes(p, n, M, f16), s, tab32, N, p, n, M, g.T, split0, g.chunk,
                       part);
    prof_mark(prof, GP_PH_GRAM, false, s);
    prof_mark(prof, GP_PH_GRAM_REDUCE, true, s);
    launch_gram_mixed_reduce(part, cnt, p, n, M, g, reg, ps == 0, ps == g.passes - 1, hbuf, A, s);
    prof_mark(prof, GP_PH_GRAM_REDUCE, false, s);
  }
}

void launch_gram_mixed_reduce(const float* part, int splits, int p, int n, int M, const GramPlan& g,
                              const double* reg, bool first, bool last, double* hbuf, double* A, hipStream_t s) {
  if (g.pair) {
    launch_pair_reduce(part, splits, p, n, M, g, reg, first, last, hbuf, A, s);
    return;
  }
  const int T = g.T;
  const int T64 = (int)ceil_div(M, 64);
  hipLaunchKernelGGL(gram_mixed_reduce_kernel, dim3(T64 * (T64 + 1) / 2), dim3(256), 0, s, part, splits, T, M, reg,
                     first ? 1 : 0, A);
}

void launch_gram_mixed_batch(const GramProb* probs_dev, const GramItem* items_dev, int nitems, bool f16,
                             int* counter, size_t lds, hipStream_t s, Prof* prof) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = std::max(1, std::min(nitems, cus));
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
  prof_mark(prof, GP_PH_GRAM, true, s);
  hipLaunchKernelGGL(f16 ? gram_mixed_batch_kernel<true> : gram_mixed_batch_kernel<false>, dim3(grid),
                     dim3(kG2Threads), lds, s, probs_dev, items_dev, nitems, counter);
  prof_mark(prof, GP_PH_GRAM, false, s);
}

// ================================================================ multi-index table
// midx[c][j] = j*n + k_j(c): the 1-D table row of column c's factor in
// dimension j (C order), zero past p.  8 uint16 per column.
__global__ void midx_kernel(int p, int n, int M, uint16_t* __restrict__ midx) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  uint16_t d[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int rem = c;
  for (int j = p - 1; j >= 0; --j) {
    d[j] = (uint16_t)(j * n + rem % n);
    rem /= n;
  }
  uint4 v;
  v.x = d[0] | ((uint32_t)d[1] << 16);
  v.y = d[2] | ((uint32_t)d[3] << 16);
  v.z = d[4] | ((uint32_t)d[5] << 16);
  v.w = d[6] | ((uint32_t)d[7] << 16);
  reinterpret_cast<uint4*>(midx)[c] = v;
}

void launch_midx(int p, int n, int M, uint16_t* midx, hipStream_t s) {
  hipLaunchKernelGGL(midx_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, p, n, M, midx);
}

// ================================================================ L^-1 split
// pieces[0] = hi, pieces[1] = lo of L^-1 (row pitch P, padding zero), each
// element first rounded to FP32.  One thread per pair of columns.
__global__ void split_linv_kernel(const double* __restrict__ Li, __bf16* __restrict__ pieces, int M, int P) {
  const int r = blockIdx.y;   // 0 .. linv_rows(M) - 1; rows past M are zero
  const int c = (blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (c >= P) return;
  const float a = (r < M && c < M) ? (float)Li[(int64_t)r * M + c] : 0.0f;
  const float b = (r < M && c + 1 < M) ? (float)Li[(int64_t)r * M + c + 1] : 0.0f;
  uint32_t h, l;
  split2(a, b, h, l);
  const int64_t PP = (int64_t)linv_rows(M) * P;
  *reinterpret_cast<uint32_t*>(pieces + (int64_t)r * P + c) = h;
  *reinterpret_cast<uint32_t*>(pieces + PP + (int64_t)r * P + c) = l;
}

void launch_split_linv(const double* Linv, __bf16* pieces, int M, hipStream_t s) {
  const int P = linv_pitch(M);
  hipLaunchKernelGGL(split_linv_kernel, dim3(ceil_div(P / 2, 256), linv_rows(M)), dim3(256), 0, s, Linv, pieces, M,
                     P);
}

// ================================================================ a5 mixed predict
// Variance part of the prediction: Z = Phi_* L^-T for a tile of TN test
// points x 256 columns r, over the columns c <= r of L^-1 in stages of 16;
// var = sigma^2 * sum_r Z^2.  512 threads = 8 waves in a WP (points) x WR (r)
// grid; each wave owns 64 points x 256/WR columns.
//
// Phi_* is formed per stage from the work-group's FP32 1-D tables through
// the prefix factorisation Phi_*[i][hi*n + k] = PRE[i][hi] * phi_{p-1,k}(x_i):
// the prefixes of a stage's 16 columns (at most 15/n + 2 of them) are formed
// one stage ahead into a small LDS table, and every value is then one
// product of two LDS reads whose rows come from a per-column descriptor
// (wave-uniform, read through the scalar cache).  Values are split in two
// BF16 terms into LDS; the matching slab of the two L^-1 terms (256 rows x 16
// columns) is prefetched into registers one stage ahead.  LDS is
// double-buffered (one barrier per stage).  After the last stage of a column
// block the squares of Z are summed per point.  (The mean is formed by the
// FP64 Phi w kernel.)
constexpr int kPmTR = 256;
constexpr int kPmKC = 16;
constexpr int kPmThreads = 512;
// Stage buffers hold 16 columns of R rows per term as [term][column / 8][row][8]:
// the 8 consecutive columns an MFMA lane reads are one contiguous 16-byte
// word, and a wave's 64 reads are two contiguous 512-byte runs (no bank
// conflicts, no padding).
__host__ __device__ constexpr int pm_at(int q, int R, int x, int c) { return ((q * 2 + (c >> 3)) * R + x) * 8 + (c & 7); }

// distinct prefixes among 16 consecutive columns
__host__ __device__ inline int pm_pre_rows(int n) { return 15 / n + 2; }

template <int TN>
struct PmCfg {
  static constexpr int WP = TN / 64;               // waves along points
  static constexpr int WR = 8 / WP;                // waves along r
  static constexpr int CB = kPmTR / WR / 32;       // 32x32 column blocks per wave
  static constexpr int CPT = kPmKC * TN / kPmThreads;  // columns generated per thread per stage
  static constexpr int PHI = 2 * kPmKC * TN;       // bf16 in one Phi_* stage buffer
  static constexpr int LIN = 2 * kPmKC * kPmTR;    // bf16 in one L^-1 stage buffer
};

int64_t predict_mixed_part_elems(int64_t Ns, int M, int* groups_out) {
  const int64_t ib = ceil_div(Ns, 128);
  const int64_t RB = ceil_div(M, kPmTR);
  int64_t g = ceil_div(1024, ib);
  if (g > RB) g = RB;
  if (g < 1) g = 1;
  if (groups_out) *groups_out = (int)g;
  return g * Ns;
}

// Per-column descriptor of the prediction, as LDS byte offsets for a
// work-group of TN test points: .x the prefix row relative to the first
// prefix of the column's stage of 16 (times TN*4), .y the 1-D table row of
// the last factor, (p-1)*n + k (times TN*4).  Columns M .. ceil16(M)-1 take
// prefix row 0 and last-factor row (p-1)*n: finite values, multiplied by the
// zero padding columns of L^-1.
__global__ void pdesc_kernel(int p, int n, int M, int TN, uint2* __restrict__ pdesc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int Mp = (int)ceil_div(M, kPmKC) * kPmKC;
  if (c >= Mp) return;
  const uint32_t rb = (uint32_t)TN * 4;
  if (c >= M) {
    pdesc[c] = uint2{0u, (uint32_t)((p - 1) * n) * rb};
    return;
  }
  const int hrel = c / n - (c - c % kPmKC) / n;
  pdesc[c] = uint2{(uint32_t)hrel * rb, (uint32_t)((p - 1) * n + c % n) * rb};
}

static int predict_tn(int p, int n);
void launch_pdesc(int p, int n, int M, uint32_t* pdesc, hipStream_t s) {
  const int Mp = (int)ceil_div(M, kPmKC) * kPmKC;
  hipLaunchKernelGGL(pdesc_kernel, dim3(ceil_div(Mp, 256)), dim3(256), 0, s, p, n, M, predict_tn(p, n),
                     reinterpret_cast<uint2*>(pdesc));
}
int64_t pdesc_elems(int M) { return 2 * ceil_div(M, kPmKC) * kPmKC; }

// Prefix digit table kept in LDS when it has at most this many entries: for
// every prefix hi and leading dimension j, the byte offset of its 1-D table
// row (j*n + digit_j) in a TN-point table.
constexpr int kPdigMax = 2048;
__host__ __device__ inline int pm_pdig_entries(int p, int n, int M) {
  const int e = (M / n) * (p - 1);
  return e <= kPdigMax ? e : 0;
}

// Instruction-scheduling pattern of a stage (SCH): 0 leaves it to the
// compiler; 1..3 interleave the MFMAs with the stage's LDS reads and vector
// work through scheduling-group barriers.
template <int SCH>
__device__ __forceinline__ void pm_sched() {
  if constexpr (SCH == 1) {
    __builtin_amdgcn_sched_group_barrier(0x100, 12, 0);   // operand reads
#pragma unroll
    for (int i = 0; i < 24; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 2, 0);  // two vector instructions
    }
  } else if constexpr (SCH == 2) {
    __builtin_amdgcn_sched_group_barrier(0x100, 6, 0);    // operands of the first product
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);  // the remaining reads
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // LDS stores among them
    }
  } else if constexpr (SCH == 3) {
    __builtin_amdgcn_iglp_opt(0);
  }
}

template <int TN, int P, bool G, int SCH = 0>
__global__ void __launch_bounds__(kPmThreads) predict_var_mixed_kernel(
    const double* __restrict__ xs, int64_t Ns, int n, int M, const double* __restrict__ tab,
    const uint16_t* __restrict__ midx, const uint32_t* __restrict__ pdesc_words, const __bf16* __restrict__ lpieces,
    int groups, double* __restrict__ part) {
  const uint2* __restrict__ pdesc = reinterpret_cast<const uint2*>(pdesc_words);
  using C = PmCfg<TN>;
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  const int npr = pm_pre_rows(n);
  float* const Tf = reinterpret_cast<float*>(smraw);                       // [P*n + 1][TN], row P*n zero
  float* const pre0 = Tf + (P * n + 1) * TN;                                // [2][npr][TN]
  __bf16* const buf0 = reinterpret_cast<__bf16*>(pre0 + 2 * npr * TN);      // [2][PHI + LIN]
  double* const ssw = reinterpret_cast<double*>(buf0 + 2 * (C::PHI + C::LIN));  // [WR][TN]
  uint32_t* const pdig = reinterpret_cast<uint32_t*>(ssw + C::WR * TN);     // [M/n][P-1] or empty
  const int npd = pm_pdig_entries(P, n, M);
  const int64_t i0 = (int64_t)blockIdx.x * TN;
  const int RB = (M + kPmTR - 1) / kPmTR;
  // Row blocks [rb0, rb1) of this group: the groups split the column stages
  // evenly (row block rb has min((rb + 1) * 16, ceil(M / 16)) of them, the
  // triangle of L^-1), not the row blocks, which would leave the last group
  // with most of the work.
  int rb0 = RB, rb1 = RB;
  {
    const int mcs = (M + kPmKC - 1) / kPmKC;
    int total = 0;
    for (int r = 0; r < RB; ++r) total += min((r + 1) * (kPmTR / kPmKC), mcs);
    const int g = blockIdx.y;
    int cum = 0;
    for (int r = 0; r < RB; ++r) {
      if (rb0 == RB && cum * groups >= g * total) rb0 = r;
      if (cum * groups >= (g + 1) * total) {
        rb1 = r;
        break;
      }
      cum += min((r + 1) * (kPmTR / kPmKC), mcs);
    }
  }
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wp = wv % C::WP, wr = wv / C::WP;
  const int LP = linv_pitch(M);
  const int64_t PP = (int64_t)linv_rows(M) * LP;

  for (int u = t; u < TN * P; u += kPmThreads) {
    const int i = u % TN, j = u / TN;
    float* o = Tf + (j * n) * TN + i;
    if (i0 + i < Ns) {
      const double* dc = tab + kTabDim + j * kDimStride;
      phi_1d<double, float>(xs[(i0 + i) * P + j], dc, tab + kTabRc1, tab + kTabRc2, n, o, TN);
    } else {
      for (int k = 0; k < n; ++k) o[k * TN] = 0.0f;
    }
  }
  for (int u = t; u < TN; u += kPmThreads) Tf[P * n * TN + u] = 0.0f;
  for (int u = t; u < C::WR * TN; u += kPmThreads) ssw[u] = 0.0;
  for (int u = t; u < npd; u += kPmThreads) {
    const int hi = u / (P > 1 ? P - 1 : 1), j = u - hi * (P > 1 ? P - 1 : 1);
    pdig[u] = (uint32_t)midx[(int64_t)hi * n * 8 + j] * (TN * 4);
  }

  const int Mc = (M + kPmKC - 1) / kPmKC;   // stages of the whole column range
  auto nstages = [&](int rb) { return min((rb + 1) * (kPmTR / kPmKC), Mc); };
  auto advance = [&](int& rb, int& k) {
    if (++k == nstages(rb)) {
      ++rb;
      k = 0;
    }
  };
  // product of the leading factors j < jend of prefix hi at point i
  auto pre_prod = [&](int hi, int i, int jend) {
    float v = 1.0f;
    if (npd) {
      const char* tfi = reinterpret_cast<const char*>(Tf + i);
#pragma unroll
      for (int j = 0; j < P - 1; ++j)
        if (j < jend) v *= *reinterpret_cast<const float*>(tfi + pdig[hi * (P - 1) + j]);
    } else {
      const uint4 dq = reinterpret_cast<const uint4*>(midx)[hi * n];
      const uint32_t d[4] = {dq.x, dq.y, dq.z, dq.w};
#pragma unroll
      for (int j = 0; j < P - 1; ++j) {
        const int row = (d[j >> 1] >> ((j & 1) * 16)) & 0xffff;
        if (j < jend) v *= Tf[row * TN + i];
      }
    }
    return v;
  };
  // G: one (row, point) item per thread (the stage's prefix rows times TN
  // points fit in 512), and PRE[hi] = PRE2[hi / n] * phi_{p-2, hi % n}, with
  // the product PRE2 of the factors before the last prefix digit kept in a
  // register and formed again only when hi / n changes (uniform per wave).
  int mp_q = -1;
  float mp_pre2 = 1.0f;
  // (divisions by n as a multiply-high by floor((2^32 - 1) / n) + 1: exact
  // for the numerators here, all below 2^20, since n <= 64; n = 1 divides
  // trivially)
  const uint32_t n_magic = n > 1 ? 0xffffffffu / (uint32_t)n + 1u : 0u;
  auto div_n = [&](int a) { return n > 1 ? (int)__umulhi((uint32_t)a, n_magic) : a; };
  auto make_pre_g = [&](int k, float* dst) {
    const int hi0 = div_n(k * kPmKC);
    const int nrow = div_n(k * kPmKC + kPmKC - 1) - hi0 + 1;
    const int r = __builtin_amdgcn_readfirstlane(t / TN);
    const int i = t % TN;
    if (r < nrow) {
      int hi = hi0 + r;
      if (hi * n >= M) hi = 0;   // past the last column: never referenced
      float v = 1.0f;
      if constexpr (P > 1) {
        const int q = div_n(hi);
        if (q != mp_q) {
          mp_q = q;
          mp_pre2 = pre_prod(hi, i, P - 2);
        }
        v = mp_pre2 * Tf[((P - 2) * n + (hi - q * n)) * TN + i];
      }
      dst[r * TN + i] = v;
    }
  };
  // prefixes of stage k (columns 16k .. 16k+15): PRE[r][i] for hi = 16k/n + r,
  // r over the stage's own prefixes only
  auto make_pre = [&](int k, float* dst) {
    if constexpr (G) {
      make_pre_g(k, dst);
      return;
    }
    const int hi0 = div_n(k * kPmKC);
    const int nrow = div_n(k * kPmKC + kPmKC - 1) - hi0 + 1;
    for (int u = t; u < nrow * TN; u += kPmThreads) {
      const int r = __builtin_amdgcn_readfirstlane(u / TN);
      const int i = u % TN;
      int hi = hi0 + r;
      if (hi * n >= M) hi = 0;   // past the last column: never referenced
      float v = 1.0f;
      if (npd) {
        const char* tfi = reinterpret_cast<const char*>(Tf + i);
#pragma unroll
        for (int j = 0; j < P - 1; ++j) v *= *reinterpret_cast<const float*>(tfi + pdig[hi * (P - 1) + j]);
      } else {
        const uint4 dq = reinterpret_cast<const uint4*>(midx)[hi * n];
        const uint32_t d[4] = {dq.x, dq.y, dq.z, dq.w};
#pragma unroll
        for (int j = 0; j < P - 1; ++j) {
          const int row = (d[j >> 1] >> ((j & 1) * 16)) & 0xffff;
          v *= Tf[row * TN + i];
        }
      }
      dst[r * TN + i] = v;
    }
  };
  // Phi_* of stage k: point gp, columns gq*CPT .. +CPT (gq wave-uniform)
  const int gp = t % TN;
  const int gq = __builtin_amdgcn_readfirstlane(t / TN);
  const char* const tf_gp = reinterpret_cast<const char*>(Tf + gp);
  // G (CPT divides n): a thread's CPT columns share one prefix and take
  // consecutive last-factor rows (CPT-aligned groups never cross a prefix),
  // so one descriptor serves the group.  (Columns past M generate finite
  // values that meet the zero columns of the padded L^-1.)
  // The descriptors of a stage are loaded one stage before they are used,
  // by a vector load (lane u takes the stage's descriptor u), and moved to
  // scalar registers when used: a scalar load would share the wait counter
  // of the LDS operand reads and hold up the MFMAs until it returned.
  constexpr int ND = G ? 1 : C::CPT;
  auto load_desc = [&](int k) {
    const int c0 = __builtin_amdgcn_readfirstlane(k * kPmKC + gq * C::CPT);
    return pdesc[c0 + (lane & (C::CPT - 1))];   // c0 + CPT - 1 < ceil16(M)
  };
  auto take_desc = [&](const uint2& dv, uint2* d) {
#pragma unroll
    for (int u = 0; u < ND; ++u)
      d[u] = uint2{(uint32_t)__builtin_amdgcn_readlane((int)dv.x, u), (uint32_t)__builtin_amdgcn_readlane((int)dv.y, u)};
  };
  auto gen_read = [&](const uint2* d, const float* pre, float* ga, float* gb) {
    const char* pre_gp = reinterpret_cast<const char*>(pre + gp);
    if constexpr (G) {
      const float pv = *reinterpret_cast<const float*>(pre_gp + d[0].x);
      const float* lp = reinterpret_cast<const float*>(tf_gp + d[0].y);
#pragma unroll
      for (int u = 0; u < C::CPT; ++u) {
        ga[u] = pv;
        gb[u] = lp[u * TN];
      }
    } else {
#pragma unroll
      for (int u = 0; u < C::CPT; ++u) {
        ga[u] = *reinterpret_cast<const float*>(pre_gp + d[u].x);
        gb[u] = *reinterpret_cast<const float*>(tf_gp + d[u].y);
      }
    }
  };
  auto gen_store = [&](const float* ga, const float* gb, __bf16* phi) {
    float v[C::CPT];
#pragma unroll
    for (int u = 0; u < C::CPT; ++u) v[u] = ga[u] * gb[u];
    uint32_t hh[C::CPT / 2], ll[C::CPT / 2];
#pragma unroll
    for (int q = 0; q < C::CPT / 2; ++q) split2(v[2 * q], v[2 * q + 1], hh[q], ll[q]);
    __bf16* dh = phi + pm_at(0, TN, gp, gq * C::CPT);
    __bf16* dl = phi + pm_at(1, TN, gp, gq * C::CPT);
    if constexpr (C::CPT == 8) {
      *reinterpret_cast<uint4*>(dh) = uint4{hh[0], hh[1], hh[2], hh[3]};
      *reinterpret_cast<uint4*>(dl) = uint4{ll[0], ll[1], ll[2], ll[3]};
    } else {
      *reinterpret_cast<uint2*>(dh) = uint2{hh[0], hh[1]};
      *reinterpret_cast<uint2*>(dl) = uint2{ll[0], ll[1]};
    }
  };
  auto gen = [&](int k, const float* pre, __bf16* phi) {
    uint2 d[ND];
    take_desc(load_desc(k), d);
    float ga[C::CPT], gb[C::CPT];
    gen_read(d, pre, ga, gb);
    gen_store(ga, gb, phi);
  };
  // L^-1 slab (rows r0..r0+255, columns c0..c0+15, both terms): 1024 uint4,
  // two per thread.  Rows past M read as zero; padding columns are zero.
  // (stage columns stay inside the pitch LP, a multiple of 16 >= M)
  // thread t holds row lr_r, columns 8 lr_h .. +8: 16 consecutive lanes take
  // 16 rows of one half, so their LDS stores fall on 16 distinct 16-byte bank
  // groups (a wave still reads 32 whole rows)
  const int lr_r = ((t >> 5) << 4) | (t & 15), lr_h = (t >> 4) & 1;
  const __bf16* const lbase0 = lpieces + (int64_t)lr_r * LP + lr_h * 8;   // term 0 (t < 512)
  const __bf16* const lbase1 = lbase0 + PP;                                   // term 1
  // (rows are padded to a multiple of 256 with zeros; a look-ahead past the
  // last row block re-reads the last one)
  auto lin_load = [&](int rb, int k, uint4& r0, uint4& r1) {
    const int64_t off = (int64_t)min(rb, RB - 1) * kPmTR * LP + k * kPmKC;
    r0 = *reinterpret_cast<const uint4*>(lbase0 + off);
    r1 = *reinterpret_cast<const uint4*>(lbase1 + off);
  };
  // thread t stores its two uint4 at row lr_r, columns 8 lr_h .. +8 of term 0
  // and the same place of term 1
  auto lin_store = [&](__bf16* lin, const uint4& r0, const uint4& r1) {
    *reinterpret_cast<uint4*>(lin + pm_at(0, kPmTR, lr_r, lr_h * 8)) = r0;
    *reinterpret_cast<uint4*>(lin + pm_at(1, kPmTR, lr_r, lr_h * 8)) = r1;
  };

  __syncthreads();  // tables ready
  if (rb0 < rb1) {
    // Stage iterator (rb, k): column stage k of row block rb.  Past the last
    // stage it keeps to valid descriptors, prefixes and (clamped) L^-1 rows.
    struct It {
      int rb, k, ns;
    };
    auto adv = [&](It& a) {
      if (++a.k == a.ns) {
        ++a.rb;
        a.k = 0;
        a.ns = nstages(a.rb);
      }
    };
    int S = 0;
    for (int rb = rb0; rb < rb1; ++rb) S += nstages(rb);
    It s0{rb0, 0, nstages(rb0)};
    It s1 = s0;
    adv(s1);
    It s2 = s1;
    adv(s2);
    It s3 = s2;
    adv(s3);
    // prologue: prefixes of stages 0 and 1, Phi_* and L^-1 slab of stage 0 in
    // buffer 0, the slabs of stages 1 and 2 in registers
    uint4 la0, la1, lb0, lb1;
    make_pre(s0.k, pre0);
    lin_load(s0.rb, s0.k, la0, la1);
    __syncthreads();
    gen(s0.k, pre0, buf0);
    lin_store(buf0 + C::PHI, la0, la1);
    // (loads in the steady state's order: slab of s1, descriptors of s1,
    // slab of s2)
    lin_load(s1.rb, s1.k, lb0, lb1);
    __builtin_amdgcn_sched_barrier(0);
    uint2 dcur = load_desc(s1.k);   // descriptors of stage s1 (lane u: descriptor u)
    __builtin_amdgcn_sched_barrier(0);
    lin_load(s2.rb, s2.k, la0, la1);
    if (s1.rb < rb1) make_pre(s1.k, pre0 + npr * TN);
    __syncthreads();
    f32x16 acc[2][C::CB];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int cb = 0; cb < C::CB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][cb][r] = 0.0f;
    float vs[2][16];     // per lane: running sums of squares of its column over the row blocks
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) vs[a][r] = 0.0f;
    int b = 0, pb = 1;   // stage buffer of the current stage; prefix buffer of the next
    // One stage: MFMAs on stage s0 (buffer b), Phi_* of s1 generated into
    // buffer b^1 with the L^-1 slab of s1 (from R, which is then refilled with
    // the slab of s3, two stages ahead), prefixes of s2.
    auto stage = [&](uint4& R0, uint4& R1) __attribute__((always_inline)) {
      const bool pre_next = s2.rb < rb1;
      float* const pdst = pre0 + (pb ^ 1) * npr * TN;
      const uint2 dnext = load_desc(s2.k);
      float ga[C::CPT], gb[C::CPT];
      {
        uint2 d[ND];
        take_desc(dcur, d);
        gen_read(d, pre0 + pb * npr * TN, ga, gb);
      }
      const __bf16* PHs = buf0 + b * (C::PHI + C::LIN);
      const __bf16* LNs = PHs + C::PHI;
      bf16x8 aop[2][2], bop[C::CB][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          aop[a][q] = *reinterpret_cast<const bf16x8*>(
              PHs + pm_at(q, TN, wp * 64 + a * 32 + (lane & 31), (lane >> 5) * 8));
#pragma unroll
      for (int cb = 0; cb < C::CB; ++cb)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          bop[cb][q] = *reinterpret_cast<const bf16x8*>(
              LNs + pm_at(q, kPmTR, wr * (kPmTR / C::WR) + cb * 32 + (lane & 31), (lane >> 5) * 8));
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) acc[a][cb] = mfma_bf16(aop[a][1], bop[cb][0], acc[a][cb]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) acc[a][cb] = mfma_bf16(aop[a][0], bop[cb][1], acc[a][cb]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int cb = 0; cb < C::CB; ++cb) acc[a][cb] = mfma_bf16(aop[a][0], bop[cb][0], acc[a][cb]);
      {
        __bf16* nb = buf0 + (b ^ 1) * (C::PHI + C::LIN);
        gen_store(ga, gb, nb);
        lin_store(nb + C::PHI, R0, R1);
        lin_load(s3.rb, s3.k, R0, R1);
      }
      pm_sched<SCH>();
      if (pre_next) make_pre(s2.k, pdst);
      if (s0.k == s0.ns - 1) {
        // squares of this column block, summed over the lane's column
        // blocks into its running FP32 sums (16 row blocks at most)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            float s2v = 0.0f;
#pragma unroll
            for (int cb = 0; cb < C::CB; ++cb) s2v = fmaf(acc[a][cb][r], acc[a][cb][r], s2v);
            vs[a][r] += s2v;
          }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int cb = 0; cb < C::CB; ++cb)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][cb][r] = 0.0f;
      }
      __syncthreads();
      b ^= 1;
      pb ^= 1;
      s0 = s1;
      s1 = s2;
      s2 = s3;
      adv(s3);
      dcur = dnext;
    };
    // stages alternate the two slab registers
    for (int q = 0; q + 1 < S; q += 2) {
      stage(lb0, lb1);
      stage(la0, la1);
    }
    if (S & 1) stage(lb0, lb1);
    // per point, the sum over the wave's 32 column lanes, in FP64
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        double v = (double)vs[a][r];
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        v += __shfl_xor(v, 8);
        v += __shfl_xor(v, 16);
        if ((lane & 31) == 0) ssw[wr * TN + wp * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] += v;
      }
  }
  __syncthreads();
  if (t < TN && i0 + t < Ns) {
    double v = 0.0;
    for (int q = 0; q < C::WR; ++q) v += ssw[q * TN + t];
    part[(int64_t)blockIdx.y * Ns + i0 + t] = v;
  }
}

__global__ void predict_mixed_reduce_kernel(const double* __restrict__ part, int groups, int64_t Ns, double sigma2,
                                            double* __restrict__ var) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ns) return;
  double v = 0.0;
  for (int g = 0; g < groups; ++g) v += part[(int64_t)g * Ns + i];
  var[i] = sigma2 * v;
}

template <int TN>
static size_t predict_lds_bytes(int p, int n) {
  using C = PmCfg<TN>;
  return ((size_t)(p * n + 1) + 2 * (size_t)pm_pre_rows(n)) * TN * sizeof(float) +
         2 * (C::PHI + C::LIN) * sizeof(__bf16) + (size_t)C::WR * TN * sizeof(double) +
         (size_t)kPdigMax * sizeof(uint32_t);
}

// TN = 256 test points per work-group when its tables fit, else 128.
static int predict_tn(int p, int n) { return predict_lds_bytes<256>(p, n) <= (size_t)kMaxDynLds ? 256 : 128; }

typedef void (*PredictKernel)(const double*, int64_t, int, int, const double*, const uint16_t*, const uint32_t*,
                              const __bf16*, int, double*);
template <int TN, bool G>
static PredictKernel predict_kernel_p(int p) {
  switch (p) {
    case 1: return predict_var_mixed_kernel<TN, 1, G>;
    case 2: return predict_var_mixed_kernel<TN, 2, G>;
    case 3: return predict_var_mixed_kernel<TN, 3, G>;
    case 4: return predict_var_mixed_kernel<TN, 4, G>;
    case 5: return predict_var_mixed_kernel<TN, 5, G>;
    case 6: return predict_var_mixed_kernel<TN, 6, G>;
    case 7: return predict_var_mixed_kernel<TN, 7, G>;
    default: return predict_var_mixed_kernel<TN, 8, G>;
  }
}
// G: the thread's column group (CPT = 16 TN / 512 columns) divides n
// (MGP_VAR_SCHED = 1..3 selects a scheduling pattern for TN = 256, p = 4
// with grouped descriptors; a tuning knob, default 0)
static int var_sched() {
  const char* v = getenv("MGP_VAR_SCHED");
  return v ? atoi(v) : 0;
}
static PredictKernel predict_kernel_for(int TN, int p, bool G) {
  if (TN == 256 && p == 4 && G) {
    switch (var_sched()) {
      case 1: return predict_var_mixed_kernel<256, 4, true, 1>;
      case 2: return predict_var_mixed_kernel<256, 4, true, 2>;
      case 3: return predict_var_mixed_kernel<256, 4, true, 3>;
      default: break;
    }
  }
  if (TN == 256) return G ? predict_kernel_p<256, true>(p) : predict_kernel_p<256, false>(p);
  return G ? predict_kernel_p<128, true>(p) : predict_kernel_p<128, false>(p);
}

void launch_predict_mixed(const double* xs, int64_t Ns, int p, int n, int M, const double* tab,
                          const uint16_t* midx, const uint32_t* pdesc, const __bf16* linv_pieces, const double* w,
                          double sigma2, double* part, double* mean, double* var, hipStream_t s, Prof* prof) {
  if (Ns <= 0) return;
  if (mean) {
    prof_mark(prof, GP_PH_PREDICT_MEAN, true, s);
    launch_phi_matvec(xs, Ns, p, n, M, tab, midx, w, nullptr, mean, s);
    prof_mark(prof, GP_PH_PREDICT_MEAN, false, s);
  }
  if (!var) return;
  const int TN = predict_tn(p, n);
  const int64_t ib = ceil_div(Ns, TN);
  const int RB = (int)ceil_div(M, kPmTR);
  int groups = 1;
  predict_mixed_part_elems(Ns, M, &groups);   // upper bound of the partial buffer
  int want = (int)ceil_div(1024, ib);
  if (want > groups) want = groups;
  if (want < 1) want = 1;
  groups = want < RB ? want : RB;
  prof_mark(prof, GP_PH_PREDICT, true, s);
  const bool G = n % (kPmKC * TN / kPmThreads) == 0;
  predict_kernel_for(TN, p, G)<<<dim3(ib, groups), dim3(kPmThreads), TN == 256 ? predict_lds_bytes<256>(p, n)
                                                                             : predict_lds_bytes<128>(p, n), s>>>(
      xs, Ns, n, M, tab, midx, pdesc, linv_pieces, groups, part);
  prof_mark(prof, GP_PH_PREDICT, false, s);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, true, s);
  hipLaunchKernelGGL(predict_mixed_reduce_kernel, dim3(ceil_div(Ns, 256)), dim3(256), 0, s, part, groups, Ns,
                     sigma2, var);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, false, s);
}


}  // namespace mgp

namespace mgp {
hipError_t configure_kernels() {
  // dynamic LDS limit: 160 KB per work-group minus room for small static arrays
  const int big = kMaxDynLds;
  hipError_t e = hipSuccess;
  for (const void* k : {(const void*)gram_mixed_kernel<true>, (const void*)gram_mixed_kernel<false>,
                        (const void*)gram_mixed_batch_kernel<true>, (const void*)gram_mixed_batch_kernel<false>}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  e = configure_pair_kernels();
  if (e != hipSuccess) return e;
  for (const void* k : {(const void*)predict_var_mixed_kernel<256, 4, true, 1>,
                        (const void*)predict_var_mixed_kernel<256, 4, true, 2>,
                        (const void*)predict_var_mixed_kernel<256, 4, true, 3>}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  for (int p = 1; p <= GP_MAX_P; ++p)
    for (int tn : {128, 256}) {
      for (bool G : {false, true}) {
        e = hipFuncSetAttribute((const void*)predict_kernel_for(tn, p, G), hipFuncAttributeMaxDynamicSharedMemorySize,
                                big);
        if (e != hipSuccess) return e;
      }
    }
  return e;
}
}  // namespace mgp
