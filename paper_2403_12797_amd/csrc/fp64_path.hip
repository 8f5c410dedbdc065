// FP64 kernels: fused Phi-generation + FP64-MFMA Gram (a3), blocked
// Cholesky / triangular inverse / triangular mat-vecs (a4) and the FP64
// predictive variance (a5).
//
// MFMA v_mfma_f64_16x16x4_f64 operand layout (lane l of a wave64):
//   A (16 x 4):  A[l % 16][l / 16]
//   B (4 x 16):  B[l / 16][l % 16]
//   D (16 x 16): element q of the lane's double4 is D[4*q + l/16][l % 16]
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
      phi_1d<double, double>(x[row * p + j], dc[0], dc[1], dc[2], rc1, rc2, n, o, 1);
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

__global__ void __launch_bounds__(256) potrf_diag_kernel(double* __restrict__ A, int M, int k0,
                                                         double* __restrict__ Dinv, int* __restrict__ info) {
  __shared__ double a[kNb * kNbLd];
  __shared__ double inv[kNb * kNbLd];
  __shared__ int bad;
  if (*info) return;
  const int t = threadIdx.x;
  const int nb = min(kNb, M - k0);
  for (int idx = t; idx < kNb * kNb; idx += 256) {
    const int i = idx / kNb, c = idx % kNb;
    a[i * kNbLd + c] = (i < nb && c < nb && c <= i) ? A[(int64_t)(k0 + i) * M + k0 + c] : 0.0;
  }
  if (t == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t == 0) {
      const double d = a[j * kNbLd + j];
      if (!(d > 0.0) || !isfinite(d))
        bad = k0 + j + 1;
      else
        a[j * kNbLd + j] = sqrt(d);
    }
    __syncthreads();
    if (bad) break;
    const double piv = a[j * kNbLd + j];
    for (int i = j + 1 + t; i < nb; i += 256) a[i * kNbLd + j] /= piv;
    __syncthreads();
    const int w = nb - j - 1;
    for (int idx = t; idx < w * w; idx += 256) {
      const int i = j + 1 + idx / w, c = j + 1 + idx % w;
      if (c <= i) a[i * kNbLd + c] -= a[i * kNbLd + j] * a[c * kNbLd + j];
    }
    __syncthreads();
  }
  if (bad) {
    if (t == 0) *info = bad;
    return;
  }
  // inverse of the lower-triangular block, one column per thread
  if (t < kNb) {
    const int c = t;
    for (int i = 0; i < kNb; ++i) inv[i * kNbLd + c] = 0.0;
    if (c < nb) {
      inv[c * kNbLd + c] = 1.0 / a[c * kNbLd + c];
      for (int i = c + 1; i < nb; ++i) {
        double s = 0.0;
        for (int q = c; q < i; ++q) s = fma(a[i * kNbLd + q], inv[q * kNbLd + c], s);
        inv[i * kNbLd + c] = -s / a[i * kNbLd + i];
      }
    }
  }
  __syncthreads();
  double* D = Dinv + (int64_t)(k0 / kNb) * kNb * kNb;
  for (int idx = t; idx < kNb * kNb; idx += 256) {
    const int i = idx / kNb, c = idx % kNb;
    D[idx] = inv[i * kNbLd + c];
    if (i < nb && c < nb) A[(int64_t)(k0 + i) * M + k0 + c] = (c <= i) ? a[i * kNbLd + c] : 0.0;
  }
}

// Panel rows below the diagonal block: L_rk = A_rk L_kk^-T.
__global__ void __launch_bounds__(256) trsm_panel_kernel(double* __restrict__ A, int M, int k0,
                                                         const double* __restrict__ Dinv,
                                                         const int* __restrict__ info) {
  __shared__ double X[kNb * kNbLd];
  __shared__ double D[kNb * kNbLd];
  if (*info) return;
  const int t = threadIdx.x;
  const int R0 = k0 + kNb + blockIdx.x * kNb;
  const double* Dk = Dinv + (int64_t)(k0 / kNb) * kNb * kNb;
  for (int idx = t; idx < kNb * kNb; idx += 256) {
    const int i = idx / kNb, c = idx % kNb;
    X[i * kNbLd + c] = (R0 + i < M) ? A[(int64_t)(R0 + i) * M + k0 + c] : 0.0;
    D[i * kNbLd + c] = Dk[idx];
  }
  __syncthreads();
  const int i = t >> 2, cbase = (t & 3) * 16;
  if (R0 + i >= M) return;
  for (int cc = 0; cc < 16; ++cc) {
    const int c = cbase + cc;
    double s = 0.0;
    for (int q = 0; q <= c; ++q) s = fma(X[i * kNbLd + q], D[c * kNbLd + q], s);
    A[(int64_t)(R0 + i) * M + k0 + c] = s;
  }
}

// Trailing update of lower tiles (R >= C) of the region past the panel:
// A_RC -= P_R P_C^T, P = A[:, k0:k0+64].
__global__ void __launch_bounds__(256) syrk_trailing_kernel(double* __restrict__ A, int M, int k0,
                                                            const int* __restrict__ info) {
  __shared__ double PR[kNb * kNbLd];
  __shared__ double PC[kNb * kNbLd];
  if (*info) return;
  int tile = blockIdx.x, R = 0;
  while (tile > R) {
    tile -= R + 1;
    ++R;
  }
  const int C = tile;
  const int base = k0 + kNb;
  const int R0 = base + R * kNb, C0 = base + C * kNb;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int idx = t; idx < kNb * kNb; idx += 256) {
    const int i = idx / kNb, c = idx % kNb;
    PR[i * kNbLd + c] = (R0 + i < M) ? A[(int64_t)(R0 + i) * M + k0 + c] : 0.0;
    PC[i * kNbLd + c] = (C0 + i < M) ? A[(int64_t)(C0 + i) * M + k0 + c] : 0.0;
  }
  __syncthreads();
  const int wr = wv >> 1, wc = wv & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNb / 4; ++kk) {
    const int k = kk * 4 + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = PR[(wr * 32 + q * 16 + (lane & 15)) * kNbLd + k];
      bv[q] = PC[(wc * 32 + q * 16 + (lane & 15)) * kNbLd + k];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
  }
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

void launch_cholesky(double* A, int M, double* Dinv, int* info, hipStream_t s) {
  for (int k0 = 0; k0 < M; k0 += kNb) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, A, M, k0, Dinv, info);
    const int rest = M - k0 - kNb;
    if (rest <= 0) break;
    const int tb = (int)ceil_div(rest, kNb);
    hipLaunchKernelGGL(trsm_panel_kernel, dim3(tb), dim3(256), 0, s, A, M, k0, Dinv, info);
    hipLaunchKernelGGL(syrk_trailing_kernel, dim3(tb * (tb + 1) / 2), dim3(256), 0, s, A, M, k0, info);
  }
}

// ---------------------------------------------------------------- L^-1
// Block row ib of X = L^-1:  X_ib,cb = -Dinv_ib * sum_{q=cb}^{ib-1} L_ib,q X_q,cb,
// X_ib,ib = Dinv_ib.  One work-group per block column cb <= ib.
__global__ void __launch_bounds__(256) trtri_row_kernel(const double* __restrict__ L,
                                                        const double* __restrict__ Dinv,
                                                        double* __restrict__ X, int M, int ib,
                                                        const int* __restrict__ info) {
  __shared__ double Ls[kNb * kNbLd];
  __shared__ double Xs[kNb * kNbLd];
  if (*info) return;
  const int cb = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int R0 = ib * kNb, C0 = cb * kNb;
  const double* Di = Dinv + (int64_t)ib * kNb * kNb;
  if (cb == ib) {
    for (int idx = t; idx < kNb * kNb; idx += 256) {
      const int i = idx / kNb, c = idx % kNb;
      if (R0 + i < M && C0 + c < M) X[(int64_t)(R0 + i) * M + C0 + c] = Di[idx];
    }
    return;
  }
  const int wr = wv >> 1, wc = wv & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  // Y = sum_q L[R-block][q-block] * X[q-block][C-block]
  for (int qb = cb; qb < ib; ++qb) {
    const int Q0 = qb * kNb;
    __syncthreads();
    for (int idx = t; idx < kNb * kNb; idx += 256) {
      const int i = idx / kNb, c = idx % kNb;
      Ls[i * kNbLd + c] = (R0 + i < M) ? L[(int64_t)(R0 + i) * M + Q0 + c] : 0.0;
      Xs[i * kNbLd + c] = X[(int64_t)(Q0 + i) * M + C0 + c];  // rows Q0+i < R0 <= M-1
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kNb / 4; ++kk) {
      const int k = kk * 4 + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        av[q] = Ls[(wr * 32 + q * 16 + (lane & 15)) * kNbLd + k];
        bv[q] = Xs[k * kNbLd + wc * 32 + q * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
  }
  // Y -> Xs, then X_ib,cb = -Dinv_ib * Y  (Dinv in Ls)
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        Xs[(wr * 32 + a * 16 + 4 * q + (lane >> 4)) * kNbLd + wc * 32 + b * 16 + (lane & 15)] = acc[a][b][q];
  for (int idx = t; idx < kNb * kNb; idx += 256) Ls[(idx / kNb) * kNbLd + idx % kNb] = Di[idx];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < kNb / 4; ++kk) {
    const int k = kk * 4 + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      av[q] = Ls[(wr * 32 + q * 16 + (lane & 15)) * kNbLd + k];
      bv[q] = Xs[k * kNbLd + wc * 32 + q * 16 + (lane & 15)];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = R0 + wr * 32 + a * 16 + 4 * q + (lane >> 4);
        const int col = C0 + wc * 32 + b * 16 + (lane & 15);
        if (row < M) X[(int64_t)row * M + col] = -acc[a][b][q];
      }
}

void launch_trtri(const double* L, const double* Dinv, double* Linv, int M, const int* info, hipStream_t s) {
  hipMemsetAsync(Linv, 0, (size_t)M * M * sizeof(double), s);
  const int T = (int)ceil_div(M, kNb);
  for (int ib = 0; ib < T; ++ib)
    hipLaunchKernelGGL(trtri_row_kernel, dim3(ib + 1), dim3(256), 0, s, L, Dinv, Linv, M, ib, info);
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
                                                           double* __restrict__ part, int M) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  const int rc = blockIdx.y;
  if (c >= M) return;
  double s = 0.0;
  const int rs = max(rc * kLtChunk, c), re = min((rc + 1) * kLtChunk, M);
  for (int r = rs; r < re; ++r) s = fma(Li[(int64_t)r * M + c], z[r], s);
  part[(int64_t)rc * M + c] = s;
}

__global__ void sum_parts_kernel(const double* __restrict__ part, int chunks, int M, double* __restrict__ w) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  double s = 0.0;
  for (int k = 0; k < chunks; ++k) s += part[(int64_t)k * M + c];
  w[c] = s;
}

void launch_lower_matvec(const double* Linv, const double* b, double* z, int M, hipStream_t s) {
  hipLaunchKernelGGL(lower_matvec_kernel, dim3(ceil_div(M, 4)), dim3(256), 0, s, Linv, b, z, M);
}

void launch_lower_t_matvec(const double* Linv, const double* z, double* w, double* part, int M, hipStream_t s) {
  const int chunks = (int)ceil_div(M, kLtChunk);
  hipLaunchKernelGGL(lower_t_part_kernel, dim3(ceil_div(M, 256), chunks), dim3(256), 0, s, Linv, z, part, M);
  hipLaunchKernelGGL(sum_parts_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, part, chunks, M, w);
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
        phi_1d<double, double>(xs[(i0 + i) * p + j], dc[0], dc[1], dc[2], rc1, rc2, n, o, kPvTn);
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
