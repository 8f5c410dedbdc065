// FP64 kernels: fused Phi-generation + FP64-MFMA Gram (a3), blocked
// Cholesky / triangular inverse / triangular mat-vecs (a4) and the FP64
// predictive variance (a5).
//
// MFMA v_mfma_f64_16x16x4_f64 operand layout (lane l of a wave64):
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): element q of the lane's double4 is D[4*q + l/16][l % 16]
#include <stdlib.h>
#include <algorithm>
#include <utility>
#include <string.h>

#include "kernels.h"

namespace mgp {

__device__ __forceinline__ f64x4 mfma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Column-fastest 1-D table fill, shared with the vector kernels' layout:
// T[i * ld + j*n + k] = phi_{j,k+1}(x_{s0+i, j}), zero past N.
__device__ __forceinline__ void fill_tab_cf64(const double* __restrict__ x, int64_t N, int p, int n,
                                              int64_t s0, int cnt, int ld, const double* __restrict__ tab,
                                              double* __restrict__ out) {
  const double* rc1 = tab + kTabRc1;
  const double* rc2 = tab + kTabRc2;
  for (int t = threadIdx.x; t < cnt * p; t += blockDim.x) {
    const int i = t % cnt, j = t / cnt;
    const int64_t row = s0 + i;
    double* o = out + i * ld + j * n;
    if (row < N) {
      const double* dc = tab + kTabDim + j * kDimStride;
      phi_1d<double, double>(x[row * p + j], dc, rc1, rc2, n, o, 1);
    } else {
      for (int k = 0; k < n; ++k) o[k] = 0.0;
    }
  }
}

// ================================================================ a3 FP64 Gram
// One work-group computes the 128 x 128 tile (I, J), I <= J, of Phi^T Phi over
// a contiguous range of samples (split-K).  Per stage of 16 samples it builds
// the 1-D tables, generates Phi[:, I-block] and Phi[:, J-block] into LDS
// (one column per thread), then 4 waves (2 x 2) run 4 x 4 FP64 MFMA blocks.
constexpr int kG64T = 128;
constexpr int kG64KC = 16;
constexpr int kG64LD = kG64T + 2;  // LDS row pitch (doubles) of the Phi stages

__host__ __device__ inline int upper_tile_index(int I, int J, int T) { return I * T - I * (I - 1) / 2 + (J - I); }

int64_t gram_f64_part_elems(int64_t N, int M, int* splitk_out) {
  const int T = (int)ceil_div(M, kG64T);
  const int ntiles = T * (T + 1) / 2;
  int64_t sk = ceil_div(2048, ntiles);
  const int64_t maxsk = ceil_div(N, 64 * kG64KC);
  if (sk > maxsk) sk = maxsk;
  if (sk < 1) sk = 1;
  if (splitk_out) *splitk_out = (int)sk;
  return sk * ntiles * (int64_t)kG64T * kG64T;
}

__global__ void __launch_bounds__(256) gram_f64_kernel(const double* __restrict__ x, int64_t N, int p, int n,
                                                       int M, const double* __restrict__ tab, int T,
                                                       int64_t rows_per_split, double* __restrict__ part) {
  extern __shared__ double sm[];
  const int ld = p * n + 1;
  double* Tb = sm;                           // [KC][ld]
  double* PI = Tb + kG64KC * ld;             // [KC][kG64LD]
  double* PJ = PI + kG64KC * kG64LD;         // [KC][kG64LD]

  // tile (I, J) from the linear upper-triangle index
  int tile = blockIdx.x, I = 0;
  while (tile >= T - I) {
    tile -= T - I;
    ++I;
  }
  const int J = I + tile;
  const bool diag = (I == J);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;

  const int col = (tid < kG64T) ? I * kG64T + tid : J * kG64T + (tid - kG64T);
  const bool gen = !diag || tid < kG64T;
  const bool valid = gen && col < M;
  int off[GP_MAX_P];
  {
    int rem = valid ? col : 0;
    for (int j = p - 1; j >= 0; --j) {
      off[j] = j * n + rem % n;
      rem /= n;
    }
  }
  double* dst = (tid < kG64T) ? PI + tid : PJ + (tid - kG64T);
  const double* B = diag ? PI : PJ;

  f64x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
  int64_t r1 = r0 + rows_per_split;
  if (r1 > N) r1 = N;
  for (int64_t s0 = r0; s0 < r1; s0 += kG64KC) {
    __syncthreads();
    fill_tab_cf64(x, r1, p, n, s0, kG64KC, ld, tab, Tb);
    __syncthreads();
    if (gen) {
      for (int i = 0; i < kG64KC; ++i) {
        double ph = 0.0;
        if (valid) {
          const double* Ti = Tb + i * ld;
          ph = Ti[off[0]];
          for (int j = 1; j < p; ++j) ph *= Ti[off[j]];
        }
        dst[i * kG64LD] = ph;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kG64KC / 4; ++kk) {
      const int srow = (kk * 4 + (lane >> 4)) * kG64LD;
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = PI[srow + wr * 64 + q * 16 + (lane & 15)];
        b[q] = B[srow + wc * 64 + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int ra = 0; ra < 4; ++ra)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) acc[ra][cb] = mfma64(a[ra], b[cb], acc[ra][cb]);
    }
  }
  const int ntiles = T * (T + 1) / 2;
  double* out = part + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * (kG64T * kG64T);
#pragma unroll
  for (int ra = 0; ra < 4; ++ra)
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = wr * 64 + ra * 16 + 4 * q + (lane >> 4);
        const int cl = wc * 64 + cb * 16 + (lane & 15);
        out[row * kG64T + cl] = acc[ra][cb][q];
      }
}

// A[g][h] = A[h][g] = sum_split part + (g == h ? reg[g] : 0), fixed order.
template <typename P>
__global__ void gram_reduce_kernel(const P* __restrict__ part, int splitk, int T, int tileDim, int M,
                                   const double* __restrict__ reg, double* __restrict__ A) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  const int g = blockIdx.y;
  if (h >= M || h < g) return;
  const int I = g / tileDim, J = h / tileDim;
  const int ti = upper_tile_index(I, J, T);
  const int ntiles = T * (T + 1) / 2;
  const int64_t off = (int64_t)ti * tileDim * tileDim + (int64_t)(g - I * tileDim) * tileDim + (h - J * tileDim);
  double s = 0.0;
  for (int k = 0; k < splitk; ++k) s += (double)part[(int64_t)k * ntiles * tileDim * tileDim + off];
  if (g == h) s += reg[g];
  A[(int64_t)g * M + h] = s;
  A[(int64_t)h * M + g] = s;
}

void launch_gram_f64(const double* x, int64_t N, int p, int n, int M, const double* tab, const double* reg,
                     double* part, double* A, hipStream_t s, Prof* prof) {
  int sk = 1;
  gram_f64_part_elems(N, M, &sk);
  const int T = (int)ceil_div(M, kG64T);
  const int ntiles = T * (T + 1) / 2;
  const int64_t rps = ceil_div(ceil_div(N, sk), kG64KC) * kG64KC;
  const size_t lds = (size_t)(kG64KC * (p * n + 1) + 2 * kG64KC * kG64LD) * sizeof(double);
  prof_mark(prof, GP_PH_GRAM, true, s);
  hipLaunchKernelGGL(gram_f64_kernel, dim3(ntiles, sk), dim3(256), lds, s, x, N, p, n, M, tab, T, rps, part);
  prof_mark(prof, GP_PH_GRAM, false, s);
  prof_mark(prof, GP_PH_GRAM_REDUCE, true, s);
  hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(ceil_div(M, 256), M), dim3(256), 0, s, part, sk, T, kG64T,
                     M, reg, A);
  prof_mark(prof, GP_PH_GRAM_REDUCE, false, s);
}

// ================================================================ a4 Cholesky
// Right-looking blocked Cholesky, block 64: factor the diagonal block in LDS
// (and invert it), scale the panel below by L_kk^-T, update the trailing
// lower triangle with FP64 MFMA.  A non-positive pivot stores its column + 1
// in *info and every later kernel returns at once.
constexpr int kNb = kCholNb;
constexpr int kNbLd = kNb + 1;

constexpr int kPfThreads = 512;
constexpr int kPfTpr = 8;                      // threads per row of W
constexpr int kPfCols = 2 * kNb / kPfTpr;      // 16 consecutive columns of W per thread
constexpr int kPfPitch = kPfCols + 2;          // padded so the 8 column groups hit distinct banks

__global__ void __launch_bounds__(kPfThreads) potrf_diag_kernel(double* __restrict__ A, int M, int k0,
                                                                double* __restrict__ Dinv, int* __restrict__ info) {
  // Factor the diagonal block B = L L^T and form X = L^-1 together, by row
  // elimination on W = [B | I] (64 x 128): step j takes the pivot
  // sqrt(W[j][j]), then every row i > j subtracts l_ij / piv times the
  // pivot row (l_ij = W[i][j] / piv = L[i][j]) and row j is divided by the
  // pivot.  The trailing part of B stays symmetric, so the pivot row also
  // supplies column j, and only the pivot row is exchanged (through LDS,
  // double-buffered, column groups padded).  Afterwards the right half of W
  // is X.  Thread t owns row i = t/8 and the 16 consecutive columns
  // 16 (t%8) .. +16 of W in registers (groups 0-3 in B, 4-7 in I).  Rows and
  // columns past the matrix are the identity.
  __shared__ double prow[2][kPfTpr * kPfPitch];
  __shared__ double Ls[kNb * kNbLd];
  if (*info) return;
  const int t = threadIdx.x, wv = t >> 6;
  const int nb = min(kNb, M - k0);
  const int i = t / kPfTpr, g = t % kPfTpr;
  const bool inB = g < kPfTpr / 2;
  auto pidx = [](int c) { return (c / kPfCols) * kPfPitch + c % kPfCols; };
  double w[kPfCols];
#pragma unroll
  for (int m = 0; m < kPfCols; ++m) {
    const int c = g * kPfCols + m;                    // column of W
    if (inB) {
      const int r = i > c ? i : c, cc = i > c ? c : i;  // lower triangle of the block
      w[m] = (i < nb && c < nb) ? A[(int64_t)(k0 + r) * M + k0 + cc] : (i == c ? 1.0 : 0.0);
    } else {
      w[m] = (i == c - kNb) ? 1.0 : 0.0;
    }
  }
  if (i == 0) {
#pragma unroll
    for (int m = 0; m < kPfCols; ++m) prow[0][g * kPfPitch + m] = w[m];
  }
  for (int j = 0; j < kNb; ++j) {
    __syncthreads();
    const int bs = j & 1;
    const double d = prow[bs][pidx(j)];
    if (!(d > 0.0) || !isfinite(d)) {   // same value in every thread
      if (t == 0) *info = k0 + j + 1;
      return;
    }
    const double piv = sqrt(d), rp = 1.0 / piv;
    if (wv * (64 / kPfTpr) + (64 / kPfTpr) - 1 >= j) {   // waves whose rows are all above j are done
      if (i == j) {
#pragma unroll
        for (int m = 0; m < kPfCols; ++m) w[m] *= rp;
      } else {
        const double l = (i > j) ? prow[bs][pidx(i)] * rp : 0.0;
        const double lr = l * rp;
        const double* pr = &prow[bs][g * kPfPitch];
#pragma unroll
        for (int m = 0; m < kPfCols; ++m) w[m] = fma(-lr, pr[m], w[m]);
        if (g == 0 && i > j) Ls[i * kNbLd + j] = l;
      }
      if (i == j && g == 0) Ls[j * kNbLd + j] = piv;
      if (i == j + 1) {
#pragma unroll
        for (int m = 0; m < kPfCols; ++m) prow[bs ^ 1][g * kPfPitch + m] = w[m];
      }
    }
  }
  __syncthreads();
  double* D = Dinv + (int64_t)(k0 / kNb) * kNb * kNb;
#pragma unroll
  for (int m = 0; m < kPfCols; ++m) {
    if (inB) {
      const int c = g * kPfCols + m;
      if (i < nb && c < nb) A[(int64_t)(k0 + i) * M + k0 + c] = (c <= i) ? Ls[i * kNbLd + c] : 0.0;
    } else {
      const int c = g * kPfCols + m - kNb;
      D[i * kNb + c] = (i < nb && c < nb && c <= i) ? w[m] : 0.0;
    }
  }
}

// The same factor and inverse with W waves (launched with 4).
// Lane i of wave H holds row i of the block, columns C H .. C H + C - 1
// (C = 64 / W), in registers, and the same rows of the identity that
// become X = L^-1 (X[r][i] in lane i, rows C H .. C H + C - 1); wave H
// owns those columns and factors them while the waves right of it apply
// their updates.  The owner works in blocks of 8 steps whose body is
// unrolled, shifting its registers down by 8 after each block, so the pivot
// column of step 8b + k is always register k.  Step K keeps the pivot chain
// in registers: column K of L, l (lane i: B[i][K] r with r = 1/sqrt(B[K][K]),
// L[K][K] = d r, zero above), was formed at the end of the previous step; it
// is stored in LDS (transposed: Lt[K][i]), column K+1 gets its update from l
// and l_{K+1} (read from lane K+1), and its pivot is read from lane K+1 and
// turned into the next l.  Row K of X is the forward-substitution row
// (e_K - sum_{j<K} L[K][j] X_j) / L[K][K]: its last term, from row K-1, is
// taken here, the others were applied before.  Meanwhile every register
// takes the rank-1 update of the previous step, l_j read back from LDS (the
// wave's own writes, in order, stored a step earlier), so the LDS round trip
// stays off the pivot chain; the same multipliers L[j][K-1] update the rows
// of X with row K-1 of X.  Registers of columns already factored, or past
// the wave's columns, collect values that are never read.  The waves right
// of the owner apply a block's 8 updates of both after the block's barrier.
// Column K of L and row K of X leave for global memory as soon as they are
// formed.  r comes from the hardware estimate and two Newton steps.  A
// failing pivot is recorded and replaced by 1 so the loop runs to the end
// (what was written is then meaningless; info says so).  Rows and columns
// past the matrix are the identity; 8-step blocks wholly past it are skipped.
constexpr int kPdNone = kNb + 1;
constexpr int kD2Blk = 8;    // steps per unrolled block
// Lt pitch for W waves of 64 / W columns: the owner's shifted registers reach
// column 56 + 64 / W - 1; even (16-byte rows), 2 * pitch = 4 mod 8 words
// (transposed reads at most 4-way bank conflicts)
template <int W> constexpr int kD2Ld = W == 2 ? 90 : 74;

// 1/sqrt(d) from the hardware estimate and two Newton steps
// r <- r (3 - d r^2) / 2, each doubling the correct bits.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
  r = r * fma(-0.5 * d * r, r, 1.5);
  r = r * fma(-0.5 * d * r, r, 1.5);
  return r;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Column `col` of L from the fully updated column c (lane i: B[i][col]):
// l and rk = 1/L[col][col]; a failing pivot sets bad (1-based) when `real`.
__device__ __forceinline__ void d2_pivot(double c, int col, int i, bool real, double& l, double& rk, int& bad) {
  double d = readlane_f64(c, min(col, kNb - 1));   // same value in every lane
  const bool ok = d > 0.0 && isfinite(d);
  if (real && !ok && !bad) bad = col + 1;
  d = ok ? d : 1.0;
  rk = rsqrt_nr(d);
  l = i > col ? c * rk : (i == col ? d * rk : 0.0);
}

template <int W>
__global__ void __launch_bounds__(64 * W) potrf_diag2_kernel(double* __restrict__ A, int M, int k0,
                                                             double* __restrict__ Dinv, int* __restrict__ info) {
  constexpr int C = kNb / W;          // columns (rows in the inverse) per wave
  constexpr int BPW = C / kD2Blk;     // 8-step blocks per wave
  constexpr int Ld = kD2Ld<W>;
  static_assert(C % kD2Blk == 0 && C % 4 == 0, "wave columns");
  __shared__ double Lt[kNb * Ld];   // Lt[j][i] = L[i][j]
  __shared__ double Xs[kNb * kNb];     // X[r][c]
  __shared__ int sbad;
  if (*info) return;
  const int t = threadIdx.x, i = t & 63;
  const int H = __builtin_amdgcn_readfirstlane(t >> 6);
  const int nb = min(kNb, M - k0);
  double* D = Dinv + (int64_t)(k0 / kNb) * kNb * kNb;
  for (int e = t; e < kNb * (Ld - kNb); e += 64 * W) Lt[(e / (Ld - kNb)) * Ld + kNb + e % (Ld - kNb)] = 0.0;
  if (t == 0) sbad = kPdNone;
  double a[C], x[C];
  // row j of the (symmetric) block, read coalesced: lane i takes B[j][i] = B[i][j]
#pragma unroll
  for (int jl = 0; jl < C; ++jl) {
    const int j = C * H + jl;
    a[jl] = (i < nb && j < nb) ? A[(int64_t)(k0 + j) * M + k0 + i] : (i == j ? 1.0 : 0.0);
    x[jl] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  int bad = 0;
  double l = 0.0, rk = 1.0;   // the owner's next column of L and its 1/L[K][K]
  double lp = 0.0;            // the owner's previous column, whose rank-1 update is pending
  double xp = 0.0;            // the owner's previous row of X, whose update is pending
  // blocks of 8 steps holding columns of the matrix; the rest of the block
  // is the identity, nothing to factor (its rows of X are zero below)
  const int nbb = (nb + kD2Blk - 1) / kD2Blk;
#pragma unroll 1
  for (int b = 0; b < nbb; ++b) {
    const int K0 = kD2Blk * b;
    if (b / BPW == H) {
      const bool first_blk = b % BPW == 0;
      if (first_blk) {
        d2_pivot(a[0], K0, i, true, l, rk, bad);
        lp = 0.0;
        xp = 0.0;
      }
      const bool last_blk = b % BPW == BPW - 1;
#pragma unroll
      for (int kl = 0; kl < kD2Blk; ++kl) {
        const int K = K0 + kl;
        Lt[K * Ld + i] = l;
        // The rank-1 update of step K is applied one step late, from the row
        // stored a step earlier (its LDS round trip off the pivot chain); the
        // next column takes the pending update and this step's from lanes
        // K + 1 of lp and l, in the same order.  Register jl holds column
        // K0 + jl (after a block's shift the pending row lines up with the
        // next block's columns).  The first step of the wave has none pending.
        const bool pend = kl > 0 || !first_blk;
        double lv[C];
        if (pend) {
          const double* lr = Lt + (K - 1) * Ld + K0;
#pragma unroll
          for (int jl = 0; jl < C; ++jl) lv[jl] = lr[jl];
        } else {
#pragma unroll
          for (int jl = 0; jl < C; ++jl) lv[jl] = 0.0;
        }
        // the pivot chain of the next column in segments, each followed by a
        // quarter of the pending rank-1 updates, so that its latency hides
        // under them
        const int k1 = min(K + 1, kNb - 1);
        const double c = fma(-l, readlane_f64(l, k1), fma(-lp, readlane_f64(lp, k1), a[kl + 1]));
        double d = readlane_f64(c, min(K + 1, kNb - 1));
        const bool ok = d > 0.0 && isfinite(d);
        if ((kl + 1 < kD2Blk || !last_blk) && !ok && !bad) bad = K + 2;
        d = ok ? d : 1.0;
        double r = __builtin_amdgcn_rsq(d);
        const double hd = -0.5 * d;
        __builtin_amdgcn_sched_barrier(0);
        // row K of X (its update from row K - 1 pending until now), kept for
        // the later waves and written out with column K of L
        const double xk = fma(-readlane_f64(lp, K), xp, x[kl]) * rk;
        Xs[K * kNb + i] = xk;
        D[K * kNb + i] = (K < nb && i < nb && i <= K) ? xk : 0.0;
        if (K < nb && i < nb) A[(int64_t)(k0 + i) * M + k0 + K] = l;
#pragma unroll
        for (int jl = 0; jl < C / 4; ++jl) {
          a[jl] = fma(-lp, lv[jl], a[jl]);
          x[jl] = fma(-xp, lv[jl], x[jl]);
        }
        __builtin_amdgcn_sched_barrier(0);
        r = r * fma(hd * r, r, 1.5);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jl = C / 4; jl < C / 2; ++jl) {
          a[jl] = fma(-lp, lv[jl], a[jl]);
          x[jl] = fma(-xp, lv[jl], x[jl]);
        }
        __builtin_amdgcn_sched_barrier(0);
        r = r * fma(hd * r, r, 1.5);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jl = C / 2; jl < 3 * C / 4; ++jl) {
          a[jl] = fma(-lp, lv[jl], a[jl]);
          x[jl] = fma(-xp, lv[jl], x[jl]);
        }
        __builtin_amdgcn_sched_barrier(0);
        const double ln = i > K + 1 ? c * r : (i == K + 1 ? d * r : 0.0);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int jl = 3 * C / 4; jl < C; ++jl) {
          a[jl] = fma(-lp, lv[jl], a[jl]);
          x[jl] = fma(-xp, lv[jl], x[jl]);
        }
        lp = l;
        l = ln;
        rk = r;
        xp = xk;
      }
#pragma unroll
      for (int j = 0; j < C - kD2Blk; ++j) {
        a[j] = a[j + kD2Blk];
        x[j] = x[j + kD2Blk];
      }
    }
    __syncthreads();
    if (b / BPW < H) {
#pragma unroll
      for (int kl = 0; kl < kD2Blk; ++kl) {
        const int K = K0 + kl;
        const double li = Lt[K * Ld + i];
        const double xk = Xs[K * kNb + i];
        const double* lr = Lt + K * Ld + C * H;
#pragma unroll
        for (int jl = 0; jl < C; ++jl) {
          const double m = lr[jl];
          a[jl] = fma(-li, m, a[jl]);
          x[jl] = fma(-xk, m, x[jl]);
        }
      }
    }
  }
  for (int r = kD2Blk * nbb + H; r < kNb; r += W) D[r * kNb + i] = 0.0;
  if (bad && i == 0) atomicMin(&sbad, bad);
  __syncthreads();
  if (sbad != kPdNone && t == 0) *info = k0 + sbad;
}

// One 64x64 output tile of C = sum_k A[m][k] B[k][n] with A, B row-major in
// global memory (lda, ldb), k in [kb, ke), rows m >= mv / columns n >= nv and
// k >= kv read as zero.  4 waves, each a 32x32 quarter (2x2 MFMA blocks).
// BT: B is given transposed, as Bt[n][k] = B[k][n] with row pitch ldb.
// K steps of 32: each thread fetches four pairs of consecutive A values and
// four of B into registers while the previous step is multiplied, and stores
// them to LDS as 16-byte writes, A as As[m][k] and Bt as Bs[n][k] (pitch 34),
// a [k][n] B as Bs[k][n] (pitch 66).  In MFMA s (0..7) of a step, the lanes
// of K-slot q (lane / 16) take k = 8 q + s (the sum over k in another order),
// so a lane's eight A (and Bt) values of a step are contiguous in LDS and
// come in 16-byte reads.  Full tiles (all rows and columns inside, the K
// range whole steps) skip the per-element bounds checks.
constexpr int kTgK = 32;                // K per step
constexpr int kTgP = kTgK + 2;          // pitch of the [row][k] tiles
constexpr int kTgPn = 64 + 2;           // pitch of the [k][n] tile
constexpr int kTgLds = 64 * kTgP;       // LDS doubles per operand tile
static_assert(kTgK * kTgPn <= kTgLds, "B tile");

template <bool BT, bool FULL>
__device__ __forceinline__ void tile_gemm64_run(const double* __restrict__ A, int64_t lda,
                                                const double* __restrict__ B, int64_t ldb, int kb, int ke, int mv,
                                                int nv, int kv, double* As, double* Bs, f64x4 (&acc)[2][2]) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int i16 = lane & 15, kq = lane >> 4;
  const int kend = min(ke, kv);
  double2 ra[4], rb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = t + r * 256;
      const int m = u >> 4, k = k0 + (u & 15) * 2;   // [row][k] tiles: row u / 16, k pair u % 16
      const double* pa = A + (int64_t)m * lda + k;
      if constexpr (FULL) {
        ra[r].x = pa[0];
        ra[r].y = pa[1];
      } else {
        ra[r].x = (m < mv && k < kend) ? pa[0] : 0.0;
        ra[r].y = (m < mv && k + 1 < kend) ? pa[1] : 0.0;
      }
      if constexpr (BT) {
        const double* pb = B + (int64_t)m * ldb + k;
        if constexpr (FULL) {
          rb[r].x = pb[0];
          rb[r].y = pb[1];
        } else {
          rb[r].x = (m < nv && k < kend) ? pb[0] : 0.0;
          rb[r].y = (m < nv && k + 1 < kend) ? pb[1] : 0.0;
        }
      } else {
        const int kk = k0 + (u >> 5), n = (u & 31) * 2;   // [k][n] tile: k u / 32, n pair u % 32
        const double* pb = B + (int64_t)kk * ldb + n;
        if constexpr (FULL) {
          rb[r].x = pb[0];
          rb[r].y = pb[1];
        } else {
          rb[r].x = (n < nv && kk < kend) ? pb[0] : 0.0;
          rb[r].y = (n + 1 < nv && kk < kend) ? pb[1] : 0.0;
        }
      }
    }
  };
  fetch(kb);
  for (int k0 = kb; k0 < ke; k0 += kTgK) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int u = t + r * 256;
      *reinterpret_cast<double2*>(As + (u >> 4) * kTgP + (u & 15) * 2) = ra[r];
      if constexpr (BT)
        *reinterpret_cast<double2*>(Bs + (u >> 4) * kTgP + (u & 15) * 2) = rb[r];
      else
        *reinterpret_cast<double2*>(Bs + (u >> 5) * kTgPn + (u & 31) * 2) = rb[r];
    }
    __syncthreads();
    if (k0 + kTgK < ke) fetch(k0 + kTgK);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      // MFMAs s = 4 h .. 4 h + 3: lane values k = 8 kq + s
      double av[2][4], bv[2][4];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const double* pa = As + (wr * 32 + q * 16 + i16) * kTgP + 8 * kq + 4 * h;
        const double2 a0 = *reinterpret_cast<const double2*>(pa), a1 = *reinterpret_cast<const double2*>(pa + 2);
        av[q][0] = a0.x;
        av[q][1] = a0.y;
        av[q][2] = a1.x;
        av[q][3] = a1.y;
        if constexpr (BT) {
          const double* pb = Bs + (wc * 32 + q * 16 + i16) * kTgP + 8 * kq + 4 * h;
          const double2 b0 = *reinterpret_cast<const double2*>(pb), b1 = *reinterpret_cast<const double2*>(pb + 2);
          bv[q][0] = b0.x;
          bv[q][1] = b0.y;
          bv[q][2] = b1.x;
          bv[q][3] = b1.y;
        } else {
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) bv[q][s4] = Bs[(8 * kq + 4 * h + s4) * kTgPn + wc * 32 + q * 16 + i16];
        }
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a][s4], bv[b][s4], acc[a][b]);
    }
  }
}

template <bool BT = false>
__device__ __forceinline__ void tile_gemm64(const double* __restrict__ A, int64_t lda, const double* __restrict__ B,
                                            int64_t ldb, int kb, int ke, int mv, int nv, int kv, double* As,
                                            double* Bs, f64x4 (&acc)[2][2]) {
  if (kb >= ke) return;
  if (mv >= 64 && nv >= 64 && kv >= ke && (ke - kb) % kTgK == 0)
    tile_gemm64_run<BT, true>(A, lda, B, ldb, kb, ke, mv, nv, kv, As, Bs, acc);
  else
    tile_gemm64_run<BT, false>(A, lda, B, ldb, kb, ke, mv, nv, kv, As, Bs, acc);
}

// C = alpha A B^T (A: m x k, B: n x k, both row-major; C: m x n, pitch ldc),
// one 64x64 tile of C per work-group on the pipelined FP64-MFMA tile
// product.  b_lower: B is lower triangular (B[r][c] = 0 for c > r), so the
// tile of columns n0.. needs k < n0 + 64 only.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) gemm_nt_f64_kernel(const double* __restrict__ A, int64_t lda,
                                                          const double* __restrict__ B, int64_t ldb,
                                                          double* __restrict__ C, int64_t ldc, int m, int n, int k,
                                                          double alpha, int b_lower) {
  __shared__ __align__(16) double As[kTgLds];
  __shared__ __align__(16) double Bs[kTgLds];
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int ke = b_lower ? min(k, n0 + 64) : k;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  tile_gemm64<true>(A + (int64_t)m0 * lda, lda, B + (int64_t)n0 * ldb, ldb, 0, ke, m - m0, n - n0, k, As, Bs, acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wr = wv >> 1, wc = wv & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = m0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int col = n0 + wc * 32 + b * 16 + (lane & 15);
        if (row < m && col < n) C[(int64_t)row * ldc + col] = alpha * acc[a][b][q];
      }
}

void launch_gemm_nt_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int m,
                        int n, int k, double alpha, bool b_lower, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  hipLaunchKernelGGL(gemm_nt_f64_kernel, dim3(ceil_div(n, 64), ceil_div(m, 64)), dim3(256), 0, s, A, lda, B, ldb, C,
                     ldc, m, n, k, alpha, b_lower ? 1 : 0);
}

// Panel below the diagonal block: L21 = B21 L11^-T = B21 X^T as one 64x64x64
// FP64-MFMA product per 64-row block (X lower, zero above the diagonal).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) trsm_panel_kernel(double* __restrict__ A, int M, int k0,
                                                         const double* __restrict__ Dinv,
                                                         const int* __restrict__ info) {
  __shared__ __align__(16) double As[kTgLds];
  __shared__ __align__(16) double Bs[kTgLds];
  if (*info) return;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int R0 = k0 + kNb + blockIdx.x * kNb;
  const double* Dk = Dinv + (int64_t)(k0 / kNb) * kNb * kNb;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // B21 X^T: X (row-major, lower) is the transposed B operand
  tile_gemm64<true>(A + (int64_t)R0 * M + k0, M, Dk, kNb, 0, kNb, M - R0, kNb, kNb, As, Bs, acc);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = R0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int col = k0 + wc * 32 + b * 16 + (lane & 15);
        if (row < M) A[(int64_t)row * M + col] = acc[a][b][q];
      }
}

// Update of 64-tiles (R, C) of the lower part below / right of the
// factored columns [k0, k0 + kw): A[R][C] -= L_R L_C^T, L_R and L_C the kw
// factored columns of the tiles' rows, on the pipelined 64x64 FP64-MFMA tile
// product (L_C read transposed).  Tiles are counted from row/column `base`:
// tile columns cb <= C < ce, rows C <= R < T (the diagonal tiles whole).
// Tile j of the lower-triangle tile set {0 <= C <= R < T} in bands of 8
// columns: band by band, row by row, the band's columns of each row.  A run
// of consecutive tiles shares its 8 column panels and each row panel 8 times.
__device__ __forceinline__ void band_tile(int j, int T, int& R, int& C) {
  int g0 = 0;
  for (;;) {
    const int w = min(8, T - g0);
    const int n = w * (w + 1) / 2 + (T - g0 - w) * w;
    if (j < n) {
      if (j < w * (w + 1) / 2) {
        int r = 0;
        while ((r + 1) * (r + 2) / 2 <= j) ++r;
        R = g0 + r;
        C = g0 + j - r * (r + 1) / 2;
      } else {
        j -= w * (w + 1) / 2;
        R = g0 + w + j / w;
        C = g0 + j % w;
      }
      return;
    }
    j -= n;
    g0 += 8;
  }
}

// XCD-aware order (banded = 1): blocks are dealt round-robin to the 8 XCDs,
// so block b is given tile (b % 8) q + b / 8 (q = tiles / 8, the rest in
// order) and each XCD runs one contiguous stretch of the banded order, its
// panels shared in its own L2.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) syrk_update_kernel(double* __restrict__ A, int M, int k0, int kw, int base,
                                                          int cb, int T, int banded, const int* __restrict__ info) {
  __shared__ __align__(16) double As[kTgLds];
  __shared__ __align__(16) double Bs[kTgLds];
  if (*info) return;
  int R, C;
  if (banded) {
    const int nt = gridDim.x, q = nt / 8, b = blockIdx.x;
    band_tile(b < 8 * q ? (b % 8) * q + b / 8 : b, T, R, C);
  } else {
    int t = blockIdx.x;
    C = cb;
    while (t >= T - C) {
      t -= T - C;
      ++C;
    }
    R = C + t;
  }
  const int R0 = base + R * kNb, C0 = base + C * kNb;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  tile_gemm64<true>(A + (int64_t)R0 * M + k0, M, A + (int64_t)C0 * M + k0, M, 0, kw, M - R0, M - C0, kw, As, Bs,
                    acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wr = wv >> 1, wc = wv & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = R0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int col = C0 + wc * 32 + b * 16 + (lane & 15);
        if (row < M && col < M) A[(int64_t)row * M + col] -= acc[a][b][q];
      }
}

// tiles of syrk_update_kernel's set {cb <= C < ce, C <= R < T}
static int64_t update_tiles(int cb, int ce, int T) {
  int64_t n = 0;
  for (int C = cb; C < ce; ++C) n += T - C;
  return n;
}

// The register-resident diagonal factor on four waves of 16 columns (two
// waves of 32 would need a, x and the broadcast row in 192 registers).
static void launch_diag2(double* A, int M, int k0, double* Dinv, int* info, hipStream_t s) {
  hipLaunchKernelGGL(potrf_diag2_kernel<4>, dim3(1), dim3(256), 0, s, A, M, k0, Dinv, info);
}

// (MGP_CHOL_DIAG=block selects the 512-thread diagonal factor; a tuning
// knob, the register-resident four-wave factor is the default)
static bool chol_diag_block() {
  const char* v = getenv("MGP_CHOL_DIAG");
  return v && strcmp(v, "block") == 0;
}

// The trailing update in the XCD-aware banded tile order (MGP_SYRK_ORDER=0
// selects the plain column order; a tuning knob).
static bool syrk_banded() {
  const char* v = getenv("MGP_SYRK_ORDER");
  return !(v && atoi(v) == 0);
}

// Two-level blocking: outer panels of kCholOuter columns, factored in
// 64-column steps (diagonal block, panel solve below it, update of the
// panel's remaining columns only); the trailing matrix right of an outer
// panel is updated once, with all its columns (rank kCholOuter), so the
// trailing matrix is read and written once per outer panel instead of once
// per 64 columns.
constexpr int kCholOuter = 256;

void launch_cholesky(double* A, int M, double* Dinv, int* info, hipStream_t s) {
  const bool blk = chol_diag_block();
  for (int K0 = 0; K0 < M; K0 += kCholOuter) {
    const int kend = std::min(M, K0 + kCholOuter);
    for (int k0 = K0; k0 < kend; k0 += kNb) {
      if (blk)
        hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(kPfThreads), 0, s, A, M, k0, Dinv, info);
      else
        launch_diag2(A, M, k0, Dinv, info, s);
      const int rest = M - k0 - kNb;
      if (rest <= 0) break;
      const int tb = (int)ceil_div(rest, kNb);
      hipLaunchKernelGGL(trsm_panel_kernel, dim3(tb), dim3(256), 0, s, A, M, k0, Dinv, info);
      // the outer panel's remaining columns
      const int ce = (int)ceil_div(kend - k0 - kNb, kNb);
      if (ce > 0)
        hipLaunchKernelGGL(syrk_update_kernel, dim3(update_tiles(0, ce, tb)), dim3(256), 0, s, A, M, k0, kNb,
                           k0 + kNb, 0, tb, 0, info);
    }
    const int rest = M - kend;
    if (rest > 0) {
      const int T = (int)ceil_div(rest, kNb);
      hipLaunchKernelGGL(syrk_update_kernel, dim3(update_tiles(0, T, T)), dim3(256), 0, s, A, M, K0, kend - K0,
                         kend, 0, T, syrk_banded() ? 1 : 0, info);
    }
  }
}

// ---------------------------------------------------------------- L^-1
// Bottom-up recursive inversion.  The diagonal 64-blocks of X = L^-1 are the
// inverses formed during the factorisation.  Level l merges pairs of
// diagonal blocks of width b = 64*2^l: for the pair starting at row o,
//   X21 = -X22 (L21 X11),  L21 = L[o+b.., o..o+b), X11, X22 its diagonal blocks,
// as two batched FP64-MFMA GEMMs over all pairs of the level (T holds L21 X11).
// Triangularity skips zero products: X11 is lower (k >= n), X22 is lower
// (k <= m).  Rows and columns past M are zero.
__global__ void trtri_diag_kernel(const double* __restrict__ Dinv, double* __restrict__ X, int M) {
  const int blk = blockIdx.x;
  const int o = blk * kNb;
  for (int idx = threadIdx.x; idx < kNb * kNb; idx += blockDim.x) {
    const int i = idx / kNb, c = idx % kNb;
    if (o + i < M && o + c < M) X[(int64_t)(o + i) * M + o + c] = Dinv[(int64_t)blk * kNb * kNb + idx];
  }
}

// T[g] = L21 X11 for pair g of width b (T is b x b, row-major, per pair).
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) trtri_merge_t_kernel(const double* __restrict__ L,
                                                            const double* __restrict__ X, double* __restrict__ T,
                                                            int M, int b, const int* __restrict__ info) {
  __shared__ __align__(16) double As[kTgLds];
  __shared__ __align__(16) double Bs[kTgLds];
  if (*info) return;
  const int g = blockIdx.z;
  const int o = 2 * g * b;          // first row/column of the pair
  const int r0 = o + b;             // first row of L21 / X22
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (r0 >= M) return;
  const int mrows = min(b, M - r0);
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (m0 < mrows) {
    // k runs over the columns of L21 = rows of X11; X11 lower: k >= n0
    tile_gemm64(L + (int64_t)(r0 + m0) * M + o, M, X + (int64_t)o * M + o + n0, M, n0 & ~15, b, mrows - m0, b - n0,
                b, As, Bs, acc);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wr = wv >> 1, wc = wv & 1;
  double* Tg = T + (int64_t)g * b * b;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int n = n0 + wc * 32 + c * 16 + (lane & 15);
        if (m < b && n < b) Tg[(int64_t)m * b + n] = acc[a][c][q];
      }
}

// X21 = -X22 T[g].
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) trtri_merge_x_kernel(double* __restrict__ X, const double* __restrict__ T,
                                                            int M, int b, const int* __restrict__ info) {
  __shared__ __align__(16) double As[kTgLds];
  __shared__ __align__(16) double Bs[kTgLds];
  if (*info) return;
  const int g = blockIdx.z;
  const int o = 2 * g * b;
  const int r0 = o + b;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (r0 >= M) return;
  const int mrows = min(b, M - r0);
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0.0, 0.0, 0.0, 0.0};
  if (m0 < mrows) {
    // X22 lower: k <= m, so k < m0 + 64
    tile_gemm64(X + (int64_t)(r0 + m0) * M + r0, M, T + (int64_t)g * b * b + n0, b, 0, min(m0 + 64, mrows),
                mrows - m0, b - n0, mrows, As, Bs, acc);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, wr = wv >> 1, wc = wv & 1;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = m0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int n = n0 + wc * 32 + c * 16 + (lane & 15);
        if (m < mrows && n < b) X[(int64_t)(r0 + m) * M + o + n] = -acc[a][c][q];
      }
}

size_t trtri_workspace_elems(int M) {
  size_t mx = 64 * 64;
  for (int b = kNb; b < M; b *= 2) {
    const size_t need = (size_t)ceil_div(M, 2 * b) * b * b;
    if (need > mx) mx = need;
  }
  return mx;
}

void launch_trtri(const double* L, const double* Dinv, double* Linv, double* ws, int M, const int* info,
                  hipStream_t s) {
  // (one diagonal block writes every entry, zeros above the diagonal included)
  if (M > kNb) launch_fill_zero_f64(Linv, (int64_t)M * M, s);
  const int nblk = (int)ceil_div(M, kNb);
  hipLaunchKernelGGL(trtri_diag_kernel, dim3(nblk), dim3(256), 0, s, Dinv, Linv, M);
  for (int b = kNb; b < M; b *= 2) {
    const int pairs = (int)ceil_div(M, 2 * b);
    const int tiles = (int)ceil_div(b, 64);
    hipLaunchKernelGGL(trtri_merge_t_kernel, dim3(tiles, tiles, pairs), dim3(256), 0, s, L, Linv, ws, M, b, info);
    hipLaunchKernelGGL(trtri_merge_x_kernel, dim3(tiles, tiles, pairs), dim3(256), 0, s, Linv, ws, M, b, info);
  }
}

// ---------------------------------------------------------------- triangular mat-vecs
// z[r] = sum_{c<=r} Linv[r][c] b[c]; one wave per row.
__global__ void __launch_bounds__(256) lower_matvec_kernel(const double* __restrict__ Li,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ z, int M) {
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= M) return;
  double s = 0.0;
  const double* row = Li + (int64_t)r * M;
  for (int c = lane; c <= r; c += 64) s = fma(row[c], b[c], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) z[r] = s;
}

// w[c] = sum_{r>=c} Linv[r][c] z[r]; thread = column, row chunks of 256
// reduced in order.
constexpr int kLtChunk = 256;
__global__ void __launch_bounds__(256) lower_t_part_kernel(const double* __restrict__ Li,
                                                           const double* __restrict__ z,
                                                           double* part, int M, const double* add) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int rc = blockIdx.y;
  if (c >= M) return;
  double s = 0.0;
  const int rs = max(rc * kLtChunk, c), re = min((rc + 1) * kLtChunk, M);
  for (int r = rs; r < re; ++r) s = fma(Li[(int64_t)r * M + c], z[r], s);
  part[(int64_t)rc * M + c] = add ? add[c] + s : s;
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int chunks, int M, double* w, const double* add) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += part[(int64_t)k * M + c];
  w[c] = add ? add[c] + s : s;
}

void launch_lower_matvec(const double* Linv, const double* b, double* z, int M, hipStream_t s) {
  hipLaunchKernelGGL(lower_matvec_kernel, dim3(ceil_div(M, 4)), dim3(256), 0, s, Linv, b, z, M);
}

void launch_lower_t_matvec(const double* Linv, const double* z, double* w, double* part, int M, hipStream_t s,
                           const double* add) {
  const int chunks = (int)ceil_div(M, kLtChunk);
  // one row chunk: its partial is the result (no second launch)
  hipLaunchKernelGGL(lower_t_part_kernel, dim3(ceil_div(M, 256), chunks), dim3(256), 0, s, Linv, z,
                     chunks == 1 ? w : part, M, chunks == 1 ? add : nullptr);
  if (chunks > 1)
    hipLaunchKernelGGL(sum_parts_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, part, chunks, M, w, add);
}

// ================================================================ a5 FP64 variance
// Work-group: 64 test points x a group of 64-wide column blocks r of
// Z = Phi_* L^-T.  Phi_* (64 x 16 per stage) is regenerated from the
// work-group's 1-D tables (built once); L^-1 stages come from memory.
// var partial = sum over the group's r of Z^2.
constexpr int kPvTn = 64;
constexpr int kPvTr = 64;
constexpr int kPvKC = 16;
constexpr int kPvLd = 64 + 2;

int64_t predict_part_elems(int64_t Ns, int M, int* groups_out) {
  const int64_t ib = ceil_div(Ns, kPvTn);
  const int64_t RB = ceil_div(M, kPvTr);
  int64_t g = ceil_div(2048, ib);
  if (g > RB) g = RB;
  if (g < 1) g = 1;
  if (groups_out) *groups_out = (int)g;
  return g * Ns;
}

__global__ void __launch_bounds__(256) predict_var_f64_kernel(const double* __restrict__ xs, int64_t Ns,
                                                              int p, int n, int M,
                                                              const double* __restrict__ tab,
                                                              const double* __restrict__ Linv, int rpg,
                                                              double* __restrict__ part) {
  extern __shared__ double sm[];
  double* T = sm;                        // [p*n][64]  (test point fastest)
  double* PS = T + p * n * kPvTn;        // [KC][kPvLd]
  double* LT = PS + kPvKC * kPvLd;       // [KC][kPvLd]
  double* red = LT + kPvKC * kPvLd;      // [2][64]
  const int64_t i0 = (int64_t)blockIdx.x * kPvTn;
  const int RB = (M + kPvTr - 1) / kPvTr;
  const int rb0 = blockIdx.y * rpg, rb1 = min(rb0 + rpg, RB);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wi = wv >> 1, wr = wv & 1;

  // 1-D tables of the 64 test points, test point fastest
  {
    const double* rc1 = tab + kTabRc1;
    const double* rc2 = tab + kTabRc2;
    for (int u = t; u < kPvTn * p; u += 256) {
      const int i = u % kPvTn, j = u / kPvTn;
      double* o = T + (j * n) * kPvTn + i;
      if (i0 + i < Ns) {
        const double* dc = tab + kTabDim + j * kDimStride;
        phi_1d<double, double>(xs[(i0 + i) * p + j], dc, rc1, rc2, n, o, kPvTn);
      } else {
        for (int k = 0; k < n; ++k) o[k * kPvTn] = 0.0;
      }
    }
  }
  double ss[2][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) ss[a][q] = 0.0;

  for (int rb = rb0; rb < rb1; ++rb) {
    const int r0 = rb * kPvTr;
    const int cend = min(r0 + kPvTr, M);
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int c0 = 0; c0 < cend; c0 += kPvKC) {
      __syncthreads();
      // Phi_* stage: wave wv makes columns c0 + 4*wv .. +3 for its lane's point
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kk = wv * 4 + u;
        const int c = c0 + kk;
        double ph = 0.0;
        if (c < M) {
          int rem = c;
          ph = 1.0;
          for (int j = p - 1; j >= 0; --j) {
            ph *= T[(j * n + rem % n) * kPvTn + lane];
            rem /= n;
          }
        }
        PS[kk * kPvLd + lane] = ph;
      }
      // L^-1 stage transposed: LT[kk][r] = Linv[r0 + r][c0 + kk]
      {
        const int r = t >> 2, kq = (t & 3) * 4;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + kq + u;
          LT[(kq + u) * kPvLd + r] = (r0 + r < M && c < M) ? Linv[(int64_t)(r0 + r) * M + c] : 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int kk = 0; kk < kPvKC / 4; ++kk) {
        const int srow = (kk * 4 + (lane >> 4)) * kPvLd;
        double av[2], bv[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          av[q] = PS[srow + wi * 32 + q * 16 + (lane & 15)];
          bv[q] = LT[srow + wr * 32 + q * 16 + (lane & 15)];
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) ss[a][q] = fma(acc[a][b][q], acc[a][b][q], ss[a][q]);
  }
  // sum over the 16 lanes holding the columns of one row, then over wr
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = ss[a][q];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      ss[a][q] = v;
    }
  __syncthreads();
  if ((lane & 15) == 0) {
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int q = 0; q < 4; ++q) red[wr * 64 + wi * 32 + a * 16 + 4 * q + (lane >> 4)] = ss[a][q];
  }
  __syncthreads();
  if (t < kPvTn && i0 + t < Ns) part[(int64_t)blockIdx.y * Ns + i0 + t] = red[t] + red[64 + t];
}

__global__ void var_reduce_kernel(const double* __restrict__ part, int groups, int64_t Ns, double sigma2,
                                  double* __restrict__ var) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Ns) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * Ns + i];
  var[i] = sigma2 * s;
}

void launch_predict_var_f64(const double* xs, int64_t Ns, int p, int n, int M, const double* tab,
                            const double* Linv, double sigma2, double* part, double* var, hipStream_t s,
                            Prof* prof) {
  if (Ns <= 0) return;
  int groups = 1;
  predict_part_elems(Ns, M, &groups);
  const int RB = (int)ceil_div(M, kPvTr);
  const int rpg = (int)ceil_div(RB, groups);
  groups = (int)ceil_div(RB, rpg);
  const size_t lds = (size_t)(p * n * kPvTn + 2 * kPvKC * kPvLd + 2 * 64) * sizeof(double);
  prof_mark(prof, GP_PH_PREDICT, true, s);
  hipLaunchKernelGGL(predict_var_f64_kernel, dim3(ceil_div(Ns, kPvTn), groups), dim3(256), lds, s, xs, Ns, p, n,
                     M, tab, Linv, rpg, part);
  prof_mark(prof, GP_PH_PREDICT, false, s);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, true, s);
  hipLaunchKernelGGL(var_reduce_kernel, dim3(ceil_div(Ns, 256)), dim3(256), 0, s, part, groups, Ns, sigma2, var);
  prof_mark(prof, GP_PH_PREDICT_REDUCE, false, s);
}

}  // namespace mgp
