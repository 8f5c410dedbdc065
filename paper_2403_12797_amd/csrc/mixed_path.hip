// Mixed-precision kernels: fused Phi-generation + split-BF16 MFMA Gram (a3)
// and the split-BF16 predictive variance with the fused FP64 mean (a5).
//
// Split-BF16 arithmetic.  A value v (first rounded once to FP32) is written
// as v = hi + mid + lo with hi = bf16(v), mid = bf16(v - hi), lo = bf16(v -
// hi - mid), every bf16() round-to-nearest-even; each subtraction is exact in
// FP32, so the three terms carry the FP32 value.  A product a*b is taken as
// the six MFMA products of relative order >= 2^-16:
//   ah*bh + ah*bm + am*bh + ah*bl + al*bh + am*bm
// with FP32 accumulation.  The variance contraction uses two terms (hi, lo)
// and three products (ah*bh + ah*bl + al*bh).
//
// MFMA v_mfma_f32_32x32x16_bf16 operand layout (lane l of a wave64):
//   A (32 x 16): lane l holds A[l % 32][8*(l/32) .. 8*(l/32)+7]
//   B (16 x 32): lane l holds B[8*(l/32) .. +7][l % 32]
//   D (32 x 32): element r of the lane's float16 is
//                D[8*(r/4) + 4*(l/32) + (r%4)][l % 32]
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
__device__ __forceinline__ float bf16lo_f(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16hi_f(uint32_t w) { return __uint_as_float(w & 0xffff0000u); }

// Three-term split of a pair of FP32 values; returns packed (hi, mid, lo).
__device__ __forceinline__ void split3(float a, float b, uint32_t& h, uint32_t& m, uint32_t& l) {
  h = pack_bf16x2(a, b);
  const float ra = a - bf16lo_f(h), rb = b - bf16hi_f(h);
  m = pack_bf16x2(ra, rb);
  const float sa = ra - bf16lo_f(m), sb = rb - bf16hi_f(m);
  l = pack_bf16x2(sa, sb);
}
__device__ __forceinline__ void split2(float a, float b, uint32_t& h, uint32_t& l) {
  h = pack_bf16x2(a, b);
  l = pack_bf16x2(a - bf16lo_f(h), b - bf16hi_f(h));
}

// ================================================================ a3 mixed Gram
// Pre-pass: the 1-D eigenfunctions of every sample, computed in FP64 and
// stored as FP32 in stage-contiguous blocks of 16 samples:
//   tab32[s][j*n + k][16]  (s = sample / 16), zero for samples >= N.
constexpr int kGmKC = 16;

__global__ void phi1d_table_kernel(const double* __restrict__ x, int64_t N, int p, int n,
                                   const double* __restrict__ tab, float* __restrict__ out, int64_t nstage) {
  const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (stage, dim, sample-in-stage)
  if (u >= nstage * p * kGmKC) return;
  const int i = (int)(u % kGmKC);
  const int j = (int)((u / kGmKC) % p);
  const int64_t st = u / ((int64_t)kGmKC * p);
  const int64_t row = st * kGmKC + i;
  float* o = out + (st * p * n + (int64_t)j * n) * kGmKC + i;
  if (row < N) {
    const double* dc = tab + kTabDim + j * kDimStride;
    phi_1d<double, float>(x[row * p + j], dc[0], dc[1], dc[2], tab + kTabRc1, tab + kTabRc2, n, o, kGmKC);
  } else {
    for (int k = 0; k < n; ++k) o[k * kGmKC] = 0.0f;
  }
}

// Gram work-group: rows I*256..+256 and columns J*256 + h*128..+128 (half h
// of the J-block) of Phi^T Phi, I <= J, over one chunk of samples.  256
// threads = 4 waves in a 2 (rows) x 2 (cols) grid, each owning 128 x 64
// outputs = 4 x 2 MFMA 32x32 blocks.
// Stage = 16 samples.  Per stage every thread generates one I-block column
// for the 16 samples and (off-diagonal tiles) half of one J-half column: the
// product of the P FP32 1-D table values, split into three BF16 terms and
// stored in LDS as [term][column slot][16 samples] (slot pitch padded against
// bank conflicts).  LDS is double-buffered and the MFMAs of stage t sit in
// the same straight-line block as the generation of stage t+1, so the
// hardware overlaps matrix and vector work.  The 1-D tables of stage t+2 are
// streamed from memory meanwhile.
// Accumulation: the MFMAs accumulate into a fresh FP32 register block for
// kG2Flush stages, which is then added into the running FP32 sum with
// round-to-nearest VALU adds.  Long MFMA accumulation chains drift
// systematically (the hardware's FP32 accumulation is not round-to-nearest);
// short chains plus rounded adds keep the Gram error unbiased.
constexpr int kGmT = 256;                                   // tile edge of the partial layout
constexpr int kG2H = 128;                                   // columns per work-group
constexpr int kG2Threads = 256;
constexpr int kG2Flush = 16;                                // stages per MFMA chain
constexpr int kG2Slots = kGmT + kG2H;                       // 384 column slots per stage
constexpr int kG2SlotPitch = kGmKC + 8;                     // bf16 per slot (16 samples + pad)
constexpr int kG2TabPitch = kGmKC + 4;                      // floats per 1-D table row (16 + pad)
constexpr int kGmChunk = 8192;                              // samples per FP32 partial
constexpr int64_t kGmPartCap = 4ll << 30;                   // bytes of partials per pass
constexpr int kGmStageElems = 3 * kG2Slots * kG2SlotPitch;  // bf16 per stage buffer

struct GramPlan {
  int T, ntiles, splits_total, splits_per_pass, passes;
};

static GramPlan gram_mixed_plan(int64_t N, int M) {
  GramPlan g;
  g.T = (int)ceil_div(M, kGmT);
  g.ntiles = g.T * (g.T + 1) / 2;
  g.splits_total = (int)ceil_div(N, kGmChunk);
  const int64_t per_split = (int64_t)g.ntiles * kGmT * kGmT * sizeof(float);
  int64_t sp = kGmPartCap / per_split;
  if (sp < 1) sp = 1;
  if (sp > g.splits_total) sp = g.splits_total;
  g.splits_per_pass = (int)sp;
  g.passes = (int)ceil_div(g.splits_total, sp);
  return g;
}

int64_t gram_mixed_part_elems(int64_t N, int M, int* splitk_out) {
  const GramPlan g = gram_mixed_plan(N, M);
  if (splitk_out) *splitk_out = g.splits_per_pass;
  return (int64_t)g.splits_per_pass * g.ntiles * kGmT * kGmT;
}

// Two zero stages past the end let the kernels prefetch without bounds tests.
int64_t gram_mixed_table_elems(int64_t N, int p, int n) { return (ceil_div(N, kGmKC) + 2) * p * n * kGmKC; }

// Generate NS samples (from sample s_off of the stage) of one column from
// the stage's FP32 tables and store its three BF16 terms.
template <int P, int NS>
__device__ __forceinline__ void gm_generate(const float* __restrict__ Tb, const int* off, bool valid,
                                            __bf16* __restrict__ stage, int slot, int s_off) {
  float v[NS];
  {
    const float4* r0 = reinterpret_cast<const float4*>(Tb + off[0] * kG2TabPitch + s_off);
#pragma unroll
    for (int q = 0; q < NS / 4; ++q) {
      const float4 u = r0[q];
      v[4 * q] = u.x;
      v[4 * q + 1] = u.y;
      v[4 * q + 2] = u.z;
      v[4 * q + 3] = u.w;
    }
  }
#pragma unroll
  for (int j = 1; j < P; ++j) {
    const float4* rj = reinterpret_cast<const float4*>(Tb + off[j] * kG2TabPitch + s_off);
#pragma unroll
    for (int q = 0; q < NS / 4; ++q) {
      const float4 u = rj[q];
      v[4 * q] *= u.x;
      v[4 * q + 1] *= u.y;
      v[4 * q + 2] *= u.z;
      v[4 * q + 3] *= u.w;
    }
  }
  if (!valid) {
#pragma unroll
    for (int i = 0; i < NS; ++i) v[i] = 0.0f;
  }
  uint32_t h[NS / 2], m[NS / 2], l[NS / 2];
#pragma unroll
  for (int q = 0; q < NS / 2; ++q) split3(v[2 * q], v[2 * q + 1], h[q], m[q], l[q]);
  uint4* dh = reinterpret_cast<uint4*>(stage + (0 * kG2Slots + slot) * kG2SlotPitch + s_off);
  uint4* dm = reinterpret_cast<uint4*>(stage + (1 * kG2Slots + slot) * kG2SlotPitch + s_off);
  uint4* dl = reinterpret_cast<uint4*>(stage + (2 * kG2Slots + slot) * kG2SlotPitch + s_off);
#pragma unroll
  for (int q = 0; q < NS / 8; ++q) {
    dh[q] = uint4{h[4 * q], h[4 * q + 1], h[4 * q + 2], h[4 * q + 3]};
    dm[q] = uint4{m[4 * q], m[4 * q + 1], m[4 * q + 2], m[4 * q + 3]};
    dl[q] = uint4{l[4 * q], l[4 * q + 1], l[4 * q + 2], l[4 * q + 3]};
  }
}

template <int P>
__global__ void __launch_bounds__(kG2Threads) gram_mixed_kernel(const float* __restrict__ tab32, int64_t N, int n,
                                                                int M, int T, int split0, float* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  // LDS: two stage buffers of split Phi, then two stage buffers of 1-D
  // tables.  Addressed as base + offset so the compiler keeps them in LDS.
  __bf16* const stg0 = reinterpret_cast<__bf16*>(smraw);
  float* const tb0 = reinterpret_cast<float*>(smraw + 2 * kGmStageElems * sizeof(__bf16));
  const int rows = P * n;                       // 1-D table rows per stage
  const int tbs = rows * kG2TabPitch;           // floats per table buffer
  const int tchunks = rows * (kGmKC / 4);       // float4 per stage of the table

  int tile = blockIdx.x >> 1, I = 0;
  const int h = blockIdx.x & 1;
  while (tile >= T - I) {
    tile -= T - I;
    ++I;
  }
  const int J = I + tile;
  const bool diag = (I == J);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;

  const int colI = I * kGmT + tid;
  const bool validI = colI < M;
  const int colJ = J * kGmT + h * kG2H + (tid >> 1);
  const bool genJ = !diag;
  const bool validJ = genJ && colJ < M;
  int offI[P], offJ[P];
  {
    int rem = validI ? colI : 0;
#pragma unroll
    for (int j = P - 1; j >= 0; --j) {
      offI[j] = j * n + rem % n;
      rem /= n;
    }
    rem = validJ ? colJ : 0;
#pragma unroll
    for (int j = P - 1; j >= 0; --j) {
      offJ[j] = j * n + rem % n;
      rem /= n;
    }
  }
  const int jslot = diag ? h * kG2H : kGmT;  // B operand columns start here in a stage

  f32x16 acc[4][2], sum[4][2];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[a][b][r] = 0.0f;
        sum[a][b][r] = 0.0f;
      }

  const int64_t r0 = (int64_t)(split0 + blockIdx.y) * kGmChunk;
  int64_t r1 = r0 + kGmChunk;
  if (r1 > N) r1 = N;
  const int nst = (int)ceil_div(r1 - r0, kGmKC);
  const int64_t st0 = r0 / kGmKC;
  // table stage loader: thread t moves float4 number t and t + 256 (P*n <= 128
  // rows of 16 floats = at most 512 float4).  The table carries two zero
  // stages past the last sample, so stage st0 + st + 2 is always readable.
  auto load_tab = [&](int64_t gst, float4* reg) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + u * kG2Threads;
      if (q < tchunks) reg[u] = reinterpret_cast<const float4*>(tab32 + gst * rows * kGmKC)[q];
    }
  };
  auto store_tab = [&](float* dst, const float4* reg) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int q = tid + u * kG2Threads;
      if (q < tchunks) {
        const int row = q / (kGmKC / 4), c4 = q % (kGmKC / 4);
        *reinterpret_cast<float4*>(dst + row * kG2TabPitch + c4 * 4) = reg[u];
      }
    }
  };
  // Rows of stages past the chunk end must not enter the sum: stages st >= nst
  // are never multiplied, and the chunk's own last stage is zero-padded by the
  // table (samples >= N) or ends exactly at a chunk boundary (chunks are
  // multiples of 16).
  float4 treg[2];
  load_tab(st0, treg);
  store_tab(tb0, treg);
  load_tab(st0 + 1, treg);
  store_tab(tb0 + tbs, treg);
  __syncthreads();
  gm_generate<P, 16>(tb0, offI, validI, stg0, tid, 0);
  if (genJ) gm_generate<P, 8>(tb0, offJ, validJ, stg0, kGmT + (tid >> 1), (tid & 1) * 8);
  __syncthreads();

  for (int g0 = 0; g0 < nst; g0 += kG2Flush) {
    const int gend = min(g0 + kG2Flush, nst);
    for (int st = g0; st < gend; ++st) {
      // stream the tables of stage st+2 while this stage computes
      load_tab(st0 + st + 2, treg);
      const __bf16* S = stg0 + (st & 1) * kGmStageElems;
      bf16x8 bop[2][3];
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int q = 0; q < 3; ++q)
          bop[cb][q] = *reinterpret_cast<const bf16x8*>(
              S + (q * kG2Slots + jslot + wc * 64 + cb * 32 + (lane & 31)) * kG2SlotPitch + (lane >> 5) * 8);
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        bf16x8 aop[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          aop[q] = *reinterpret_cast<const bf16x8*>(
              S + (q * kG2Slots + wr * 128 + rb * 32 + (lane & 31)) * kG2SlotPitch + (lane >> 5) * 8);
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          f32x16 c = acc[rb][cb];
          c = mfma_bf16(aop[1], bop[cb][1], c);  // mid*mid
          c = mfma_bf16(aop[2], bop[cb][0], c);  // lo*hi
          c = mfma_bf16(aop[0], bop[cb][2], c);  // hi*lo
          c = mfma_bf16(aop[1], bop[cb][0], c);  // mid*hi
          c = mfma_bf16(aop[0], bop[cb][1], c);  // hi*mid
          c = mfma_bf16(aop[0], bop[cb][0], c);  // hi*hi
          acc[rb][cb] = c;
        }
      }
      // generate stage st+1 (past the chunk end this produces unused zeros)
      {
        __bf16* D = stg0 + ((st + 1) & 1) * kGmStageElems;
        const float* Tn = tb0 + ((st + 1) & 1) * tbs;
        gm_generate<P, 16>(Tn, offI, validI, D, tid, 0);
        if (genJ) gm_generate<P, 8>(Tn, offJ, validJ, D, kGmT + (tid >> 1), (tid & 1) * 8);
      }
      store_tab(tb0 + (st & 1) * tbs, treg);
      __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          sum[a][b][r] += acc[a][b][r];
          acc[a][b][r] = 0.0f;
        }
  }

  const int ntiles = T * (T + 1) / 2;
  float* out = part + ((int64_t)blockIdx.y * ntiles + (blockIdx.x >> 1)) * (kGmT * kGmT);
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr * 128 + rb * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int cl = h * kG2H + wc * 64 + cb * 32 + (lane & 31);
        out[row * kGmT + cl] = sum[rb][cb][r];
      }
}

typedef void (*GramKernel)(const float*, int64_t, int, int, int, int, float*);
static GramKernel gram_kernel_for(int p) {
  switch (p) {
    case 1: return gram_mixed_kernel<1>;
    case 2: return gram_mixed_kernel<2>;
    case 3: return gram_mixed_kernel<3>;
    case 4: return gram_mixed_kernel<4>;
    case 5: return gram_mixed_kernel<5>;
    case 6: return gram_mixed_kernel<6>;
    case 7: return gram_mixed_kernel<7>;
    default: return gram_mixed_kernel<8>;
  }
}

// A (+)= sum of the pass's FP32 partials in split order (FP64); the first pass
// also adds reg on the diagonal.  Writes both triangles.
__global__ void gram_mixed_reduce_kernel(const float* __restrict__ part, int splits, int T, int M,
                                         const double* __restrict__ reg, int first, double* __restrict__ A) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (h >= M || h < g) return;
  const int I = g / kGmT, J = h / kGmT;
  const int ti = I * T - I * (I - 1) / 2 + (J - I);
  const int ntiles = T * (T + 1) / 2;
  const int64_t off = (int64_t)ti * kGmT * kGmT + (int64_t)(g - I * kGmT) * kGmT + (h - J * kGmT);
  double s = first ? (g == h ? reg[g] : 0.0) : A[(int64_t)g * M + h];
  for (int k = 0; k < splits; ++k) s += (double)part[(int64_t)k * ntiles * kGmT * kGmT + off];
  A[(int64_t)g * M + h] = s;
  A[(int64_t)h * M + g] = s;
}

void launch_gram_mixed(const double* x, int64_t N, int p, int n, int M, const double* tab, const double* reg,
                       float* part, float* tab32, double* A, hipStream_t s, Prof* prof) {
  const GramPlan g = gram_mixed_plan(N, M);
  const int64_t nstage = ceil_div(N, kGmKC) + 2;
  const size_t lds = 2 * kGmStageElems * sizeof(__bf16) + 2 * (size_t)p * n * kG2TabPitch * sizeof(float);
  prof_mark(prof, GP_PH_GRAM, true, s);
  hipLaunchKernelGGL(phi1d_table_kernel, dim3(ceil_div(nstage * p * kGmKC, 256)), dim3(256), 0, s, x, N, p, n, tab,
                     tab32, nstage);
  prof_mark(prof, GP_PH_GRAM, false, s);
  for (int ps = 0; ps < g.passes; ++ps) {
    const int split0 = ps * g.splits_per_pass;
    const int cnt = std::min(g.splits_per_pass, g.splits_total - split0);
    prof_mark(prof, GP_PH_GRAM, true, s);
    hipLaunchKernelGGL(gram_kernel_for(p), dim3(2 * g.ntiles, cnt), dim3(kG2Threads), lds, s, tab32, N, n, M, g.T,
                       split0, part);
    prof_mark(prof, GP_PH_GRAM, false, s);
    prof_mark(prof, GP_PH_GRAM_REDUCE, true, s);
    hipLaunchKernelGGL(gram_mixed_reduce_kernel, dim3(ceil_div(M, 256), M), dim3(256), 0, s, part, cnt, g.T, M,
                       reg, ps == 0 ? 1 : 0, A);
    prof_mark(prof, GP_PH_GRAM_REDUCE, false, s);
  }
}

// ================================================================ L^-1 split
// pieces[0] = hi, pieces[1] = lo of L^-1 (row pitch P, padding zero), each
// element first rounded to FP32.  One thread per pair of columns.
__global__ void split_linv_kernel(const double* __restrict__ Li, __bf16* __restrict__ pieces, int M, int P) {
  const int r = blockIdx.y;
  const int c = (blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (c >= P) return;
  const float a = c < M ? (float)Li[(int64_t)r * M + c] : 0.0f;
  const float b = c + 1 < M ? (float)Li[(int64_t)r * M + c + 1] : 0.0f;
  uint32_t h, l;
  split2(a, b, h, l);
  const int64_t PP = (int64_t)M * P;
  *reinterpret_cast<uint32_t*>(pieces + (int64_t)r * P + c) = h;
  *reinterpret_cast<uint32_t*>(pieces + PP + (int64_t)r * P + c) = l;
}

void launch_split_linv(const double* Linv, __bf16* pieces, int M, hipStream_t s) {
  const int P = linv_pitch(M);
  hipLaunchKernelGGL(split_linv_kernel, dim3(ceil_div(P / 2, 256), M), dim3(256), 0, s, Linv, pieces, M, P);
}

// ================================================================ a5 mixed predict
// Work-group: 128 test points x a group of 256-wide column blocks r of
// Z = Phi_* L^-T.  8 waves in a 2 (points) x 4 (r) grid, each 64 x 64 =
// 2 x 2 MFMA 32x32 blocks.  Per stage of 16 columns c, Phi_* (128 x 16) is
// generated from the work-group's FP32 1-D tables and split in two terms;
// the matching 256 x 16 slab of the L^-1 terms is copied from memory.  Squares
// of Z are summed per point across all r of the group.  The mean partial
// sum_c Phi_*[i][c] w[c] (FP64) is accumulated for the columns c of each
// r-block while that block's diagonal stages are generated.
constexpr int kPmTn = 128;
constexpr int kPmTr = 256;
constexpr int kPmKC = 16;
constexpr int kPmThreads = 512;
constexpr int kPmPhiElems = 2 * kPmTn * kPmKC;   // bf16 per stage (2 terms)
constexpr int kPmLinvElems = 2 * kPmTr * kPmKC;

int64_t predict_mixed_part_elems(int64_t Ns, int M, int* groups_out) {
  const int64_t ib = ceil_div(Ns, kPmTn);
  const int64_t RB = ceil_div(M, kPmTr);
  int64_t g = ceil_div(1024, ib);
  if (g > RB) g = RB;
  if (g < 1) g = 1;
  if (groups_out) *groups_out = (int)g;
  return 2 * g * Ns;
}

__global__ void __launch_bounds__(kPmThreads) predict_var_mixed_kernel(
    const double* __restrict__ xs, int64_t Ns, int p, int n, int M, const double* __restrict__ tab,
    const __bf16* __restrict__ lpieces, const double* __restrict__ w, int rpg, double* __restrict__ part) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smraw[];
  float* Tf = reinterpret_cast<float*>(smraw);                                   // [p*n][128]
  __bf16* PS = reinterpret_cast<__bf16*>(smraw + (size_t)p * n * kPmTn * sizeof(float));  // [2][128][16]
  __bf16* LS = PS + kPmPhiElems;                                                  // [2][256][16]
  double* red = reinterpret_cast<double*>(LS + kPmLinvElems);                     // [4][128] + [4][128]
  const int64_t i0 = (int64_t)blockIdx.x * kPmTn;
  const int RB = (M + kPmTr - 1) / kPmTr;
  const int rb0 = blockIdx.y * rpg, rb1 = min(rb0 + rpg, RB);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wi = wv >> 2, wr = wv & 3;
  const int P = linv_pitch(M);
  const int64_t PP = (int64_t)M * P;

  {
    const double* rc1 = tab + kTabRc1;
    const double* rc2 = tab + kTabRc2;
    for (int u = t; u < kPmTn * p; u += kPmThreads) {
      const int i = u % kPmTn, j = u / kPmTn;
      float* o = Tf + (j * n) * kPmTn + i;
      if (i0 + i < Ns) {
        const double* dc = tab + kTabDim + j * kDimStride;
        phi_1d<double, float>(xs[(i0 + i) * p + j], dc[0], dc[1], dc[2], rc1, rc2, n, o, kPmTn);
      } else {
        for (int k = 0; k < n; ++k) o[k * kPmTn] = 0.0f;
      }
    }
  }
  // generation role: thread -> (point gi, 4 consecutive columns gq*4..+3)
  const int gi = t & (kPmTn - 1), gq = t >> 7;   // gq in 0..3
  double mean_acc = 0.0;
  float ss[2][16];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) ss[a][r] = 0.0f;

  for (int rb = rb0; rb < rb1; ++rb) {
    const int r0 = rb * kPmTr;
    const int cend = min(r0 + kPmTr, M);
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
    for (int c0 = 0; c0 < cend; c0 += kPmKC) {
      __syncthreads();
      // Phi_* stage: 4 columns for point gi
      {
        float v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + gq * 4 + u;
          float ph = 0.0f;
          if (c < M) {
            int rem = c;
            ph = 1.0f;
            for (int j = p - 1; j >= 0; --j) {
              ph *= Tf[(j * n + rem % n) * kPmTn + gi];
              rem /= n;
            }
            if (c >= r0 && w) mean_acc = fma((double)ph, w[c], mean_acc);
          }
          v[u] = ph;
        }
        uint32_t h0, l0, h1, l1;
        split2(v[0], v[1], h0, l0);
        split2(v[2], v[3], h1, l1);
        *reinterpret_cast<uint2*>(PS + (0 * kPmTn + gi) * kPmKC + gq * 4) = uint2{h0, h1};
        *reinterpret_cast<uint2*>(PS + (1 * kPmTn + gi) * kPmKC + gq * 4) = uint2{l0, l1};
      }
      // L^-1 slab: rows r0..r0+255, columns c0..c0+15, both terms (16 B per load)
      for (int u = t; u < 2 * kPmTr * 2; u += kPmThreads) {
        const int q = u / (2 * kPmTr);          // term
        const int rem = u % (2 * kPmTr);
        const int r = rem >> 1, half = rem & 1;
        uint4 val = uint4{0u, 0u, 0u, 0u};
        const int row = r0 + r, c = c0 + half * 8;
        if (row < M && c < P) val = *reinterpret_cast<const uint4*>(lpieces + q * PP + (int64_t)row * P + c);
        *reinterpret_cast<uint4*>(LS + (q * kPmTr + r) * kPmKC + half * 8) = val;
      }
      __syncthreads();
      bf16x8 aop[2][2], bop[2][2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          aop[a][q] = *reinterpret_cast<const bf16x8*>(PS + (q * kPmTn + wi * 64 + a * 32 + (lane & 31)) * kPmKC +
                                                       (lane >> 5) * 8);
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          bop[b][q] = *reinterpret_cast<const bf16x8*>(LS + (q * kPmTr + wr * 64 + b * 32 + (lane & 31)) * kPmKC +
                                                       (lane >> 5) * 8);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          f32x16 c = acc[a][b];
          c = mfma_bf16(aop[a][1], bop[b][0], c);
          c = mfma_bf16(aop[a][0], bop[b][1], c);
          c = mfma_bf16(aop[a][0], bop[b][0], c);
          acc[a][b] = c;
        }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) ss[a][r] = fmaf(acc[a][b][r], acc[a][b][r], ss[a][r]);
  }
  // reduce squares over the 32 lanes that hold one row's columns, then over wr
  __syncthreads();
  double* vred = red;               // [4][128]
  double* mred = red + 4 * kPmTn;   // [4][128]
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      double v = (double)ss[a][r];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      v += __shfl_xor(v, 16);
      if ((lane & 31) == 0) vred[wr * kPmTn + wi * 64 + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3)] = v;
    }
  mred[gq * kPmTn + gi] = mean_acc;
  __syncthreads();
  if (t < kPmTn && i0 + t < Ns) {
    const double v = ((vred[t] + vred[kPmTn + t]) + vred[2 * kPmTn + t]) + vred[3 * kPmTn + t];
    const double mu = ((mred[t] + mred[kPmTn + t]) + mred[2 * kPmTn + t]) + mred[3 * kPmTn + t];
    part[(int64_t)blockIdx.y * 2 * Ns + i0 + t] = v;
    part[(int64_t)blockIdx.y * 2 * Ns + Ns + i0 + t] = mu;
  }
}

__global__ void predict_mixed_reduce_kernel(const double* __restrict__ part, int groups, int64_t Ns, double sigma2,
                                            double* __restrict__ mean, double* __restrict__ var) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ns) return;
  double v = 0.0, mu = 0.0;
  for (int g = 0; g < groups; ++g) {
    v += part[(int64_t)g * 2 * Ns + i];
    mu += part[(int64_t)g * 2 * Ns + Ns + i];
  }
  if (var) var[i] = sigma2 * v;
  if (mean) mean[i] = mu;
}

void launch_predict_mixed(const double* xs, int64_t Ns, int p, int n, int M, const double* tab,
                          const __bf16* linv_pieces, const double* w, double sigma2, double* part, double* mean,
                          double* var, hipStream_t s, Prof* prof) {
  if (Ns <= 0) return;
  int groups = 1;
  predict_mixed_part_elems(Ns, M, &groups);
  const int RB = (int)ceil_div(M, kPmTr);
  const int rpg = (int)ceil_div(RB, groups);
  groups = (int)ceil_div(RB, rpg);
  const size_t lds = (size_t)p * n * kPmTn * sizeof(float) + (kPmPhiElems + kPmLinvElems) * sizeof(__bf16) +
                     8 * kPmTn * sizeof(double);
  prof_mark(prof, GP_PH_PREDICT, true, s);
  hipLaunchKernelGGL(predict_var_mixed_kernel, dim3(ceil_div(Ns, kPmTn), groups), dim3(kPmThreads), lds, s, xs, Ns,
                     p, n, M, tab, linv_pieces, w, rpg, part);
  prof_mark(prof, GP_PH_PREDICT, false, s);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, true, s);
  hipLaunchKernelGGL(predict_mixed_reduce_kernel, dim3(ceil_div(Ns, 256)), dim3(256), 0, s, part, groups, Ns,
                     sigma2, mean, var);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, false, s);
}

}  // namespace mgp

namespace mgp {
hipError_t configure_kernels() {
  const int big = 160 * 1024;
  hipError_t e = hipSuccess;
  for (int p = 1; p <= GP_MAX_P; ++p) {
    e = hipFuncSetAttribute((const void*)gram_kernel_for(p), hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
  }
  e = hipFuncSetAttribute((const void*)predict_var_mixed_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, big);
  return e;
}
}  // namespace mgp
