// Paired Gram (a3): Phi^T Phi through the pair symmetry of the
// tensor-product expansion (eqs. 18-19).
//
// A column m of Phi is a product of 1-D eigenfunctions over the input
// dimensions, Phi[i,m] = prod_j phi_{j,k_j(m)}(x_ij), so an entry of the Gram
//   G[m,m'] = sum_i prod_j phi_{j,k_j(m)}(x_ij) phi_{j,k_j(m')}(x_ij)
// depends on (m, m') only through the unordered pair {k_j(m), k_j(m')} of
// every dimension.  With the s = n(n+1)/2 pairs t = (a <= b), numbered
// t = b(b+1)/2 + a, and the pair tables Q_j[t](x) = phi_{j,a}(x) phi_{j,b}(x),
// the dimensions are split into a leading group j < p1 = floor(p/2) and a
// trailing group j >= p1:
//   Psi1[i,u] = prod_{j<p1}  Q_j[t_j(u)](x_ij),   u over the s^p1 pair tuples,
//   Psi2[i,v] = prod_{j>=p1} Q_j[t_j(v)](x_ij),   v over the s^p2 pair tuples,
//   H = Psi1^T Psi2,                              (s^p1 x s^p2)
// (tuples in C order, last dimension fastest) and G[m,m'] = H[u(m,m'),
// v(m,m')].  H holds (n(n+1)/2)^p values against the n^p (n^p + 1)/2 of the
// Gram's upper triangle (5.0x fewer at p = 4, n = 8; 7.4x at p = 5, n = 6),
// and it is a dense product of two generated operands, each formed like Phi
// in the direct scheme: u = hi*s + t has Psi1[i,u] = PRE1[hi](x_i) *
// Q_{p1-1}[t](x_i), PRE1 the product of the group's leading pair tables.
//
// Work item: rows u0..u0+255 of H and columns v0..v0+127, over one chunk of
// samples; 512 threads = 8 waves in a 4 x 2 grid, 64 x 64 outputs per wave
// (2 x 2 MFMA 32x32 blocks).  Per 16-sample stage the work-group streams the
// FP32 1-D tables (scaled by the power of two of each row, as in the direct
// scheme; the last dimension of each group is raised by a further 2^7, so
// every scaled Psi value is below 2^14, inside the FP16 range), forms the
// "derived" rows -- the pair tables of the two groups' last dimensions and
// the prefix rows of the item -- each a product of table rows, then
// generates and splits the operands into LDS.  Pipeline, split arithmetic,
// FP32 accumulation (chains of 16 stages folded into running FP32 sums) and
// the FP32 partial per chunk are those of the direct scheme; partials are
// summed in FP64 in split order into H, from which A = G + sigma^2 Lambda^-1
// is gathered.
#include <stdlib.h>

#include "mixed_common.h"

namespace mgp {

constexpr int kPgT = 256;                      // rows of H per work item
constexpr int kPgH = 128;                      // columns of H per work item
constexpr int kPgThreads = 512;
constexpr int kPgSlots = kPgT + kPgH;          // operand slots per stage
constexpr int kPgTabPitch = kGmKC + 4;         // floats per table / derived row
constexpr int kPgFlush = 16;                   // stages per MFMA accumulation chain
constexpr int kPgTop = 7;                      // extra exponent of each group's last dimension
constexpr int kPgMaxF = 6;                     // table factors per derived row, 2 * max(1, p2 - 1)
constexpr int kPgChunk = 32768;                // samples per FP32 partial
constexpr int64_t kPgPartCap = 8ll << 30;      // bytes of partials per pass
constexpr int kPgAsmMax = 1024;                // n^p1, n^p2 tabulated by the assembly

__host__ __device__ inline int pg_s(int n) { return n * (n + 1) / 2; }
__host__ __device__ inline int pg_npre1(int p1, int s, int S1) { return p1 > 1 ? (S1 < kPgT ? S1 : kPgT) / s + 2 : 0; }
__host__ __device__ inline int pg_npre2(int p2, int s, int S2) { return p2 > 1 ? (S2 < kPgH ? S2 : kPgH) / s + 2 : 0; }
__host__ __device__ constexpr int pg_stage_elems(bool f16) { return (f16 ? 2 : 3) * kPgSlots * kGmKC; }
// Stage buffers hold 16 samples of each operand slot per term as
// [term][sample / 8][slot][8]: the 8 consecutive samples an MFMA lane reads
// are one contiguous 16-byte word, and a wave's 64 reads are two contiguous
// 512-byte runs.
__host__ __device__ constexpr int pg_at(int t, int slot, int smp) {
  return ((t * 2 + (smp >> 3)) * kPgSlots + slot) * 8 + (smp & 7);
}

// (a, b), a <= b, of pair number t = b(b+1)/2 + a
__host__ __device__ inline void pg_pair(int t, int& a, int& b) {
  b = 0;
  while ((b + 1) * (b + 2) / 2 <= t) ++b;
  a = t - b * (b + 1) / 2;
}

static size_t pair_lds_bytes(int p, int n, int p1, int S1, int S2, bool f16) {
  const int s = pg_s(n), ndi = 2 * s + pg_npre1(p1, s, S1) + pg_npre2(p - p1, s, S2);
  return 2 * (size_t)pg_stage_elems(f16) * 2 + 3 * (size_t)(p * n + 1) * kPgTabPitch * sizeof(float) +
         2 * (size_t)(ndi + 2) * kPgTabPitch * sizeof(float) + kPgSlots * sizeof(int) +
         (size_t)ndi * kPgMaxF * sizeof(uint16_t) + 16;
}

// Paired plan when p >= 2, its LDS fits and it issues fewer 256 x 128 items
// per chunk than the direct scheme's upper triangle.
bool pair_plan(int p, int n, int M, bool f16, GramPlan& g) {
  if (p < 2) return false;
  const int s = pg_s(n), p1 = p / 2;
  int64_t S1 = 1, S2 = 1;
  for (int j = 0; j < p; ++j) (j < p1 ? S1 : S2) *= s;
  if (S1 * S2 > (int64_t)1 << 30) return false;
  int64_t NP1 = 1, NP2 = 1;   // values of the leading / trailing digits of a column
  for (int j = 0; j < p; ++j) (j < p1 ? NP1 : NP2) *= n;
  if (NP1 > kPgAsmMax || NP2 > kPgAsmMax) return false;
  if (pair_lds_bytes(p, n, p1, (int)S1, (int)S2, f16) > (size_t)kMaxDynLds) return false;
  const int64_t T1 = ceil_div(S1, kPgT), T2 = ceil_div(S2, kPgH);
  const int64_t T = ceil_div(M, 256);
  if (T1 * T2 >= T * (T + 1)) return false;
  g.pair = 1;
  g.p1 = p1;
  g.s = s;
  g.S1 = (int)S1;
  g.S2 = (int)S2;
  g.T1 = (int)T1;
  g.T2 = (int)T2;
  g.ntiles = (int)(T1 * T2);
  return true;
}

void pair_plan_splits(int64_t N, GramPlan& g, int chunk) {
  if (chunk <= 0) {
    const int64_t want = ceil_div(N * g.ntiles, 1024);
    chunk = (int)std::min<int64_t>(kPgChunk, std::max<int64_t>(1024, ceil_div(want, kGmKC) * kGmKC));
  }
  g.chunk = (int)ceil_div(chunk, kGmKC) * kGmKC;
  g.splits_total = (int)ceil_div(N, g.chunk);
  const int64_t per_split = (int64_t)g.ntiles * kPgT * kPgH * sizeof(float);
  int64_t sp = kPgPartCap / per_split;
  if (sp < 1) sp = 1;
  if (sp > g.splits_total) sp = g.splits_total;
  g.splits_per_pass = (int)sp;
  g.passes = (int)ceil_div(g.splits_total, sp);
}

size_t pair_gram_lds_bytes(int p, int n, const GramPlan& g, bool f16) {
  return pair_lds_bytes(p, n, g.p1, g.S1, g.S2, f16);
}

// Instruction-scheduling pattern of a stage (SCH): 0 leaves it to the
// compiler; 1, 2 interleave the MFMAs with the stage's LDS traffic and
// vector work through scheduling-group barriers.
template <int SCH, int NMF>
__device__ __forceinline__ void pg_sched() {
  if constexpr (SCH == 1) {
    __builtin_amdgcn_sched_group_barrier(0x100, 8, 0);    // operand reads
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one MFMA
      __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // four vector instructions
    }
  } else if constexpr (SCH == 2) {
#pragma unroll
    for (int i = 0; i < NMF; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // an LDS read
      __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);  // an LDS store
    }
  }
}

// One work item: tile = I * T2 + J (rows I*256.., columns J*128..), samples
// [r0, r0 + chunk); writes the item's FP32 partial [256][128] at `out`.
template <bool F16, int F, int SCH = 0>
__device__ __forceinline__ void pair_item(unsigned char* smraw, const float* __restrict__ tab32, int64_t N, int P,
                                          int n, int p1, int S1, int S2, int T2, int tile, int64_t r0, int chunk,
                                          float* __restrict__ out) {
  using E = std::conditional_t<F16, _Float16, __bf16>;
  using V8 = std::conditional_t<F16, f16x8, bf16x8>;
  constexpr int NT = F16 ? 2 : 3;
  constexpr int SE = pg_stage_elems(F16);
  const int s = pg_s(n), p2 = P - p1;
  const int npre1 = pg_npre1(p1, s, S1), npre2 = pg_npre2(p2, s, S2);
  const int ndi = 2 * s + npre1 + npre2;            // derived rows formed per stage
  const int ONES = ndi, ZERO = ndi + 1;             // constant derived rows
  const int rows = P * n;                           // 1-D table rows; row `rows` is all ones
  const int tbs = (rows + 1) * kPgTabPitch;         // floats per table buffer
  const int drs = (ndi + 2) * kPgTabPitch;          // floats per derived buffer

  E* const stg0 = reinterpret_cast<E*>(smraw);
  float* const tb0 = reinterpret_cast<float*>(smraw + 2 * SE * sizeof(E));
  float* const dr0 = tb0 + 3 * tbs;
  int* const csc = reinterpret_cast<int*>(dr0 + 2 * drs);
  uint16_t* const dfac = reinterpret_cast<uint16_t*>(csc + kPgSlots);
  const unsigned* const tmax = reinterpret_cast<const unsigned*>(tab32 + gm_max_offset(N, P, n));
  const int tchunks = rows * (kGmKC / 4);

  const int I = tile / T2, J = tile - (tile / T2) * T2;
  const int u0 = I * kPgT, v0 = J * kPgH;
  const int hiI0 = u0 / s, hiJ0 = v0 / s;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;

  // table-row exponent: 2^e(j,k) brings the row's maximum into [0.5, 1);
  // each group's last dimension is raised by kPgTop more
  auto rexp = [&](int j, int k) { return gm_row_exp(tmax[j * n + k], (j == p1 - 1 || j == P - 1) ? kPgTop : 0); };

  // factors (1-D table rows) of derived row r; unused factors take the ones row
  auto der_factors = [&](int r, int* f) {
#pragma unroll
    for (int q = 0; q < kPgMaxF; ++q) f[q] = rows;
    if (r < 2 * s) {
      const int j = r < s ? p1 - 1 : P - 1;
      int a, b;
      pg_pair(r < s ? r : r - s, a, b);
      f[0] = j * n + a;
      f[1] = j * n + b;
    } else if (r < ndi) {
      const bool g1 = r < 2 * s + npre1;
      const int hi = g1 ? hiI0 + (r - 2 * s) : hiJ0 + (r - 2 * s - npre1);
      const int jb = g1 ? 0 : p1, je = g1 ? p1 - 1 : P - 1;   // the prefix's dimensions jb..je-1
      const int lim = (g1 ? S1 : S2) / s;                      // number of prefixes of the group
      if (hi < lim) {
        int rem = hi;
        for (int j = je - 1; j >= jb; --j) {
          int a, b;
          pg_pair(rem % s, a, b);
          rem /= s;
          f[2 * (j - jb)] = j * n + a;
          f[2 * (j - jb) + 1] = j * n + b;
        }
      }
    }
  };

  // generation roles (consecutive lanes take consecutive slots):
  //   row slot tid & 255, samples (tid >> 8)*8 .. +8;
  //   column slot 256 + (tid & 127), samples (tid >> 7)*4 .. +4
  const int sI = (tid >> 8) * 8, sJ = (tid >> 7) * 4;
  const int uI = u0 + (tid & 255);
  const bool okI = uI < S1;
  const int preI = (okI ? (p1 > 1 ? 2 * s + uI / s - hiI0 : ONES) : ZERO) * kPgTabPitch + sI;
  const int lastI = (okI ? uI % s : 0) * kPgTabPitch + sI;
  const int vJ = v0 + (tid & 127);
  const bool okJ = vJ < S2;
  const int preJ = (okJ ? (p2 > 1 ? 2 * s + npre1 + vJ / s - hiJ0 : ONES) : ZERO) * kPgTabPitch + sJ;
  const int lastJ = (s + (okJ ? vJ % s : 0)) * kPgTabPitch + sJ;

  // MFMA blocks that hold at least one valid row and column (wave-uniform)
  bool rv[2], cv[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    rv[q] = __builtin_amdgcn_readfirstlane(u0 + wr * 64 + q * 32 < S1 ? 1 : 0) != 0;
    cv[q] = __builtin_amdgcn_readfirstlane(v0 + wc * 64 + q * 32 < S2 ? 1 : 0) != 0;
  }

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

  // 1-D tables of one stage: rows x 16 floats, one float4 per thread,
  // requested two stages before they are stored
  float4 treg0, treg1;
  const int trow = tid / (kGmKC / 4);
  const float tsc = tid < tchunks ? ldexpf(1.0f, rexp(trow / n, trow % n)) : 0.0f;
  auto load_tab = [&](int64_t gst, float4& r) {
    if (tid < tchunks) r = reinterpret_cast<const float4*>(tab32 + gst * rows * kGmKC)[tid];
  };
  auto store_tab = [&](float* dst, const float4& r) {
    if (tid < tchunks) {
      const int c4 = tid % (kGmKC / 4);
      *reinterpret_cast<float4*>(dst + trow * kPgTabPitch + c4 * 4) =
          float4{r.x * tsc, r.y * tsc, r.z * tsc, r.w * tsc};
    }
  };

  // derived rows of one stage, in items of (row, 4 samples): item tid's
  // factor offsets are held in registers, items past 512 read the factor
  // table dfac in LDS
  const int nitem = ndi * 4;
  const bool own = tid < nitem;
  int doff[F];
  {
    int f[kPgMaxF];
    der_factors(own ? (tid >> 2) : ndi, f);
#pragma unroll
    for (int q = 0; q < F; ++q) doff[q] = f[q] * kPgTabPitch + (tid & 3) * 4;
  }
  const int ddst = (tid >> 2) * kPgTabPitch + (tid & 3) * 4;
  auto make_der = [&](const float* Tb, float* dst) {
    if (own) {
      float4 f[F];
#pragma unroll
      for (int q = 0; q < F; ++q) f[q] = *reinterpret_cast<const float4*>(Tb + doff[q]);
      float4 v = f[0];
#pragma unroll
      for (int q = 1; q < F; ++q) {
        v.x *= f[q].x;
        v.y *= f[q].y;
        v.z *= f[q].z;
        v.w *= f[q].w;
      }
      *reinterpret_cast<float4*>(dst + ddst) = v;
    }
    for (int u = tid + kPgThreads; u < nitem; u += kPgThreads) {
      const int r = u >> 2, q4 = (u & 3) * 4;
      const uint16_t* fr = dfac + r * kPgMaxF;
      float4 v = float4{1.f, 1.f, 1.f, 1.f};
      for (int q = 0; q < F; ++q) {
        const float4 f = *reinterpret_cast<const float4*>(Tb + fr[q] * kPgTabPitch + q4);
        v.x *= f.x;
        v.y *= f.y;
        v.z *= f.z;
        v.w *= f.w;
      }
      *reinterpret_cast<float4*>(dst + r * kPgTabPitch + q4) = v;
    }
  };

  // operands of one stage: values into registers, then products, split, store
  struct GenIn {
    float4 pa[2], la[2], pj, lj;
  };
  auto gen_read = [&](const float* Dr, GenIn& g) {
    const float4* pa = reinterpret_cast<const float4*>(Dr + preI);
    const float4* la = reinterpret_cast<const float4*>(Dr + lastI);
    g.pa[0] = pa[0];
    g.pa[1] = pa[1];
    g.la[0] = la[0];
    g.la[1] = la[1];
    g.pj = *reinterpret_cast<const float4*>(Dr + preJ);
    g.lj = *reinterpret_cast<const float4*>(Dr + lastJ);
  };
  auto store_terms = [&](auto ns, const float* v, E* D, int slot, int s_off) {
    constexpr int NS = decltype(ns)::value;
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
      E* d = D + pg_at(t, slot, s_off);
      if constexpr (NS == 8)
        *reinterpret_cast<uint4*>(d) = uint4{w[t][0], w[t][1], w[t][2], w[t][3]};
      else
        *reinterpret_cast<uint2*>(d) = uint2{w[t][0], w[t][1]};
    }
  };
  auto gen_store = [&](const GenIn& g, E* D) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      v[4 * q] = g.pa[q].x * g.la[q].x;
      v[4 * q + 1] = g.pa[q].y * g.la[q].y;
      v[4 * q + 2] = g.pa[q].z * g.la[q].z;
      v[4 * q + 3] = g.pa[q].w * g.la[q].w;
    }
    store_terms(std::integral_constant<int, 8>{}, v, D, tid & 255, sI);
    float w[4] = {g.pj.x * g.lj.x, g.pj.y * g.lj.y, g.pj.z * g.lj.z, g.pj.w * g.lj.w};
    store_terms(std::integral_constant<int, 4>{}, w, D, kPgT + (tid & 127), sJ);
  };

  // prologue state: factor table, constant rows, operand scale exponents
  for (int r = tid; r < ndi; r += kPgThreads) {
    int f[kPgMaxF];
    der_factors(r, f);
#pragma unroll
    for (int q = 0; q < kPgMaxF; ++q) dfac[r * kPgMaxF + q] = (uint16_t)f[q];
  }
  if (tid < kPgTabPitch) {
    for (int b = 0; b < 3; ++b) tb0[b * tbs + rows * kPgTabPitch + tid] = 1.0f;
    for (int b = 0; b < 2; ++b) {
      dr0[b * drs + ONES * kPgTabPitch + tid] = 1.0f;
      dr0[b * drs + ZERO * kPgTabPitch + tid] = 0.0f;
    }
  }
  for (int sl = tid; sl < kPgSlots; sl += kPgThreads) {
    const bool row = sl < kPgT;
    const int f = row ? u0 + sl : v0 + sl - kPgT;
    int e = 0;
    if (f < (row ? S1 : S2)) {
      int rem = f;
      const int jb = row ? 0 : p1, je = row ? p1 : P;
      for (int j = je - 1; j >= jb; --j) {
        int a, b;
        pg_pair(rem % s, a, b);
        rem /= s;
        e += rexp(j, a) + rexp(j, b);
      }
    }
    csc[sl] = e;
  }
  // prologue: tables of stages 0..2, derived rows of stages 0..1, operands of stage 0
  load_tab(st0, treg0);
  store_tab(tb0, treg0);
  load_tab(st0 + 1, treg0);
  store_tab(tb0 + tbs, treg0);
  load_tab(st0 + 2, treg0);
  store_tab(tb0 + 2 * tbs, treg0);
  load_tab(st0 + 3, treg1);
  __syncthreads();
  make_der(tb0, dr0);
  make_der(tb0 + tbs, dr0 + drs);
  __syncthreads();
  {
    GenIn g;
    gen_read(dr0, g);
    gen_store(g, stg0);
  }
  __syncthreads();

  // one stage: MFMAs on stage st, operands of st+1, derived rows of st+2,
  // tables of st+3 stored (requested one stage earlier) and of st+4 requested
  auto stage = [&](int st, float4& Rload, const float4& Rstore) {
    load_tab(st0 + st + 4, Rload);
    GenIn gin;
    gen_read(dr0 + ((st + 1) & 1) * drs, gin);
    const E* S = stg0 + (st & 1) * SE;
    V8 aop[2][NT], bop[2][NT];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int q = 0; q < NT; ++q)
        bop[cb][q] = *reinterpret_cast<const V8*>(
            S + pg_at(q, kPgT + wc * 64 + cb * 32 + (lane & 31), (lane >> 5) * 8));
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int q = 0; q < NT; ++q)
        aop[rb][q] = *reinterpret_cast<const V8*>(
            S + pg_at(q, wr * 64 + rb * 32 + (lane & 31), (lane >> 5) * 8));
    auto prod = [&](int qa, int qb) {
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          if (rv[rb] && cv[cb]) {
            if constexpr (F16)
              acc[rb][cb] = mfma_f16(aop[rb][qa], bop[cb][qb], acc[rb][cb]);
            else
              acc[rb][cb] = mfma_bf16(aop[rb][qa], bop[cb][qb], acc[rb][cb]);
          }
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
    make_der(tb0 + ((st + 2) % 3) * tbs, dr0 + (st & 1) * drs);
    store_tab(tb0 + (st % 3) * tbs, Rstore);
    pg_sched<SCH, F16 ? 12 : 24>();
    __syncthreads();
  };

  for (int g0 = 0; g0 < nst; g0 += kPgFlush) {
    const int gend = min(g0 + kPgFlush, nst);
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
        const int col = wc * 64 + cb * 32 + (lane & 31);
        out[row * kPgH + col] = ldexpf(sum[rb][cb][r], -(csc[row] + csc[kPgT + col]));
      }
}

// Single problem: grid (T1 * T2 items, splits of this pass).
template <bool F16, int F, int SCH = 0>
__global__ void __launch_bounds__(kPgThreads) gram_pair_kernel(const float* __restrict__ tab32, int64_t N, int p, int n,
                                                               int p1, int S1, int S2, int T2, int ntiles, int split0,
                                                               int chunk, float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  float* out = part + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (kPgT * kPgH);
  pair_item<F16, F, SCH>(smraw, tab32, N, p, n, p1, S1, S2, T2, blockIdx.x, (int64_t)(split0 + blockIdx.y) * chunk,
                         chunk, out);
}

// Many problems in one persistent launch (see gram_mixed_batch_kernel).
template <bool F16, int F>
__global__ void __launch_bounds__(kPgThreads) gram_pair_batch_kernel(const GramProb* __restrict__ probs,
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
    float* out = pr.part + ((int64_t)wi.split * pr.ntiles + wi.tile) * (kPgT * kPgH);
    pair_item<F16, F>(smraw, pr.tab32, pr.N, pr.p, pr.n, pr.p1, pr.S1, pr.S2, pr.T2, wi.tile,
                      (int64_t)wi.split * pr.chunk, pr.chunk, out);
  }
}

// H (+)= sum of the pass's partials in split order (FP64); H is s^p1 x s^p2
// row-major.
__global__ void __launch_bounds__(256) pair_reduce_kernel(const float* __restrict__ part, int splits, int ntiles,
                                                          int T2, int S1, int S2, int first, double* __restrict__ H) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)S1 * S2) return;
  const int u = (int)(e / S2), v = (int)(e - (e / S2) * S2);
  const int64_t off = ((int64_t)(u / kPgT) * T2 + v / kPgH) * (kPgT * kPgH) + (u % kPgT) * kPgH + (v % kPgH);
  const int64_t stride = (int64_t)ntiles * kPgT * kPgH;
  double acc = first ? 0.0 : H[e];
  for (int k = 0; k < splits; ++k) acc += (double)part[k * stride + off];
  H[e] = acc;
}

// A[m][m'] = H[u(m,m')][v(m,m')] + (m == m' ? reg[m] : 0), both triangles.
// One work-group per row m: the leading-group part of the pair index is a
// function of m' / n^p2 and the trailing part of m' % n^p2 (each a table of
// values, at most kPgAsmMax), tabulated in LDS first.
__global__ void __launch_bounds__(256) pair_assemble_kernel(const double* __restrict__ H, int p, int n, int p1, int M,
                                                            const double* __restrict__ reg, double* __restrict__ A) {
  __shared__ int uoff[kPgAsmMax], voff[kPgAsmMax];
  const int m = blockIdx.x;
  const int s = pg_s(n);
  int NP1 = 1, NP2 = 1, S2 = 1;
  for (int j = 0; j < p; ++j) {
    if (j < p1) NP1 *= n;
    else {
      NP2 *= n;
      S2 *= s;
    }
  }
  const int mu = m / NP2, mv = m - (m / NP2) * NP2;
  auto pidx = [](int a, int b) {
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    return hi * (hi + 1) / 2 + lo;
  };
  for (int c = threadIdx.x; c < NP1; c += blockDim.x) {
    int ra = mu, rb = c, u = 0, w = 1;
    for (int j = p1 - 1; j >= 0; --j) {
      u += pidx(ra % n, rb % n) * w;
      w *= s;
      ra /= n;
      rb /= n;
    }
    uoff[c] = u;
  }
  for (int c = threadIdx.x; c < NP2; c += blockDim.x) {
    int ra = mv, rb = c, v = 0, w = 1;
    for (int j = p - 1; j >= p1; --j) {
      v += pidx(ra % n, rb % n) * w;
      w *= s;
      ra /= n;
      rb /= n;
    }
    voff[c] = v;
  }
  __syncthreads();
  double* row = A + (int64_t)m * M;
  for (int c = threadIdx.x; c < M; c += blockDim.x) {
    const int cu = c / NP2, cv = c - (c / NP2) * NP2;
    double a = H[(int64_t)uoff[cu] * S2 + voff[cv]];
    if (c == m) a += reg[m];
    row[c] = a;
  }
}

typedef void (*PairKernel)(const float*, int64_t, int, int, int, int, int, int, int, int, int, float*);
template <bool F16>
static PairKernel pair_kernel_f(int F) {
  switch (F) {
    case 2: return gram_pair_kernel<F16, 2>;
    case 4: return gram_pair_kernel<F16, 4>;
    default: return gram_pair_kernel<F16, 6>;
  }
}
// (MGP_GRAM_SCHED = 1, 2 selects a scheduling pattern for the FP16 scheme
// with two factors per derived row; a tuning knob, default 0)
static int gram_sched() {
  const char* v = getenv("MGP_GRAM_SCHED");
  return v ? atoi(v) : 0;
}
static PairKernel pair_kernel_for(bool f16, int F) {
  if (f16 && F == 2) {
    switch (gram_sched()) {
      case 1: return gram_pair_kernel<true, 2, 1>;
      case 2: return gram_pair_kernel<true, 2, 2>;
      default: break;
    }
  }
  return f16 ? pair_kernel_f<true>(F) : pair_kernel_f<false>(F);
}

typedef void (*PairBatchKernel)(const GramProb*, const GramItem*, int, int*);
template <bool F16>
static PairBatchKernel pair_batch_kernel_f(int F) {
  switch (F) {
    case 2: return gram_pair_batch_kernel<F16, 2>;
    case 4: return gram_pair_batch_kernel<F16, 4>;
    default: return gram_pair_batch_kernel<F16, 6>;
  }
}
static PairBatchKernel pair_batch_kernel_for(bool f16, int F) {
  return f16 ? pair_batch_kernel_f<true>(F) : pair_batch_kernel_f<false>(F);
}

// factors per derived row of a plan: the pair tables of the last dimensions
// (2) and the prefixes of the larger group (2 (p2 - 1))
int pair_factors(int p, const GramPlan& g) {
  const int p2 = p - g.p1;
  return 2 * (p2 - 1 > 1 ? p2 - 1 : 1);
}

void launch_gram_pair(int64_t N, int p, int n, int M, const GramPlan& g, bool f16, const double* reg, float* part,
                      const float* tab32, double* H, double* A, hipStream_t s, Prof* prof) {
  const int F = pair_factors(p, g);
  const size_t lds = pair_lds_bytes(p, n, g.p1, g.S1, g.S2, f16);
  for (int ps = 0; ps < g.passes; ++ps) {
    const int split0 = ps * g.splits_per_pass;
    const int cnt = std::min(g.splits_per_pass, g.splits_total - split0);
    prof_mark(prof, GP_PH_GRAM, true, s);
    hipLaunchKernelGGL(pair_kernel_for(f16, F), dim3(g.ntiles, cnt), dim3(kPgThreads), lds, s, tab32, N, p, n, g.p1,
                       g.S1, g.S2, g.T2, g.ntiles, split0, g.chunk, part);
    prof_mark(prof, GP_PH_GRAM, false, s);
    prof_mark(prof, GP_PH_GRAM_REDUCE, true, s);
    launch_pair_reduce(part, cnt, p, n, M, g, reg, ps == 0, ps == g.passes - 1, H, A, s);
    prof_mark(prof, GP_PH_GRAM_REDUCE, false, s);
  }
}

void launch_pair_reduce(const float* part, int splits, int p, int n, int M, const GramPlan& g, const double* reg,
                        bool first, bool last, double* H, double* A, hipStream_t s) {
  const int64_t HE = (int64_t)g.S1 * g.S2;
  hipLaunchKernelGGL(pair_reduce_kernel, dim3(ceil_div(HE, 256)), dim3(256), 0, s, part, splits, g.ntiles, g.T2, g.S1,
                     g.S2, first ? 1 : 0, H);
  if (last) hipLaunchKernelGGL(pair_assemble_kernel, dim3(M), dim3(256), 0, s, H, p, n, g.p1, M, reg, A);
}

void launch_gram_pair_batch(const GramProb* probs_dev, const GramItem* items_dev, int nitems, bool f16, int F,
                            int* counter, size_t lds, hipStream_t s, Prof* prof) {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int grid = std::max(1, std::min(nitems, cus));
  launch_fill_zero_int(counter, 1, s);
  prof_mark(prof, GP_PH_GRAM, true, s);
  hipLaunchKernelGGL(pair_batch_kernel_for(f16, F), dim3(grid), dim3(kPgThreads), lds, s, probs_dev, items_dev, nitems,
                     counter);
  prof_mark(prof, GP_PH_GRAM, false, s);
}

hipError_t configure_pair_kernels() {
  hipError_t e = hipSuccess;
  for (const void* k : {(const void*)gram_pair_kernel<true, 2, 1>, (const void*)gram_pair_kernel<true, 2, 2>}) {
    e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
    if (e != hipSuccess) return e;
  }
  for (bool f16 : {false, true})
    for (int F : {2, 4, 6}) {
      e = hipFuncSetAttribute((const void*)pair_kernel_for(f16, F), hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxDynLds);
      if (e != hipSuccess) return e;
      e = hipFuncSetAttribute((const void*)pair_batch_kernel_for(f16, F), hipFuncAttributeMaxDynamicSharedMemorySize,
                              kMaxDynLds);
      if (e != hipSuccess) return e;
    }
  return e;
}

}  // namespace mgp
