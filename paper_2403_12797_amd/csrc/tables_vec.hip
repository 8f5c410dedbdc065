// a1 eigen tables and the FP64 matrix-free Phi / Phi^T vector products.
#include "kernels.h"

namespace mgp {

// ---------------------------------------------------------------- a1
// e^-a I_k(a) (the periodic kernel's eigenvalues, a = eps^2 <= 256) by its
// power series sum_m e^-a (a/2)^(2m+k) / (m! (m+k)!): positive terms, the
// first in logarithms, the rest by their ratio (a/2)^2 / ((m+1)(m+k+1)),
// summed until past the largest term and below 1e-18 of the sum.
__device__ double bessel_i_scaled(int k, double a) {
  if (a == 0.0) return k == 0 ? 1.0 : 0.0;
  const double h = 0.5 * a, h2 = h * h;
  double term = exp(k * log(h) - lgamma(k + 1.0) - a), sum = 0.0;
  for (int m = 0; m < 4096; ++m) {
    sum += term;
    if (m > h && term < 1e-18 * sum) break;
    term *= h2 / ((m + 1.0) * (m + k + 1.0));
  }
  return sum;
}

// Per-dimension scalars of eq. 14 (delta^2 = alpha^2/2 (beta^2-1)), the
// eigenvalues of eq. 16 and the normalised Hermite recurrence coefficients
// (SE); for the periodic kernel the angular frequencies and the Bessel
// eigenvalues, one thread per (dimension, column).
__global__ void eig_dim_kernel(EigArgs a, double* __restrict__ tab) {
  const int t = threadIdx.x;
  if (a.kind == GP_KERNEL_PERIODIC) {
    const int j = t / GP_MAX_N, k = t % GP_MAX_N;
    if (j < a.p && k < a.n) {
      if (k == 0) {
        double* dc = tab + kTabDim + j * kDimStride;
        dc[0] = a.alpha[j];
        dc[1] = 0.0;
        dc[2] = 1.0;
        dc[3] = 1.0;
      }
      tab[kTabLam1 + j * GP_MAX_N + k] = bessel_i_scaled((k + 1) / 2, a.eps[j] * a.eps[j]);
    }
  } else if (t < a.p) {
    const double eps = a.eps[t], al = a.alpha[t];
    const double r = 2.0 * eps / al;
    const double beta = sqrt(sqrt(1.0 + r * r));
    const double d2 = al * al * 0.5 * (beta * beta - 1.0);
    double* dc = tab + kTabDim + t * kDimStride;
    dc[0] = al * beta;
    dc[1] = d2;
    dc[2] = sqrt(beta);
    dc[3] = 0.0;
    const double D = al * al + d2 + eps * eps;
    const double q = eps * eps / D;
    double lam = sqrt(al * al / D);
    for (int k = 0; k < a.n; ++k) {
      tab[kTabLam1 + t * GP_MAX_N + k] = lam;
      lam *= q;
    }
  }
  if (t < GP_MAX_N) {
    tab[kTabRc1 + t] = t > 0 ? sqrt(2.0 / (t + 1.0)) : 0.0;
    tab[kTabRc2 + t] = t > 0 ? sqrt((double)t / (t + 1.0)) : 0.0;
  }
}

// Lambda_m = prod_j lambda_{j,k_j(m)} (eq. 20) and the ridge sigma^2/Lambda_m.
__global__ void eig_lambda_kernel(int p, int n, int M, double sigma2, const double* __restrict__ tab,
                                  double* __restrict__ lam, double* __restrict__ reg) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  int rem = m;
  double v = 1.0;
  for (int j = p - 1; j >= 0; --j) {
    v *= tab[kTabLam1 + j * GP_MAX_N + rem % n];
    rem /= n;
  }
  lam[m] = v;
  reg[m] = sigma2 / v;
}

void launch_eig_tables(const EigArgs& a, double* tab, double* lam, double* reg, int M, hipStream_t s) {
  hipLaunchKernelGGL(eig_dim_kernel, dim3(1), dim3(GP_MAX_P * GP_MAX_N), 0, s, a, tab);
  hipLaunchKernelGGL(eig_lambda_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, a.p, a.n, M,
                     a.sigma * a.sigma, tab, lam, reg);
}

// ---------------------------------------------------------------- helpers
// Fill the 1-D eigenfunction table of `cnt` samples starting at s0 into LDS.
// Layout "sample-fastest": T[(j*n + k) * ld + i] = phi_{j,k+1}(x_{s0+i, j}).
// Rows past N are zero.  Called by the whole block; caller syncs.
template <typename T>
__device__ __forceinline__ void fill_tab_sf(const double* __restrict__ x, int64_t N, int p, int n,
                                            int64_t s0, int cnt, int ld, const double* __restrict__ tab,
                                            T* __restrict__ out) {
  const double* rc1 = tab + kTabRc1;
  const double* rc2 = tab + kTabRc2;
  for (int t = threadIdx.x; t < cnt * p; t += blockDim.x) {
    const int i = t % cnt, j = t / cnt;
    const int64_t row = s0 + i;
    T* o = out + (j * n) * ld + i;
    if (row < N) {
      const double* dc = tab + kTabDim + j * kDimStride;
      phi_1d<double, T>(x[row * p + j], dc, rc1, rc2, n, o, ld);
    } else {
      for (int k = 0; k < n; ++k) o[k * ld] = (T)0;
    }
  }
}

// Same table, "column-fastest": T[i * ld + j*n + k].
__device__ __forceinline__ void fill_tab_cf(const double* __restrict__ x, int64_t N, int p, int n,
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

// ---------------------------------------------------------------- Phi w
// Block = 4 waves, 64 samples (one per lane).  Wave q walks the column
// prefixes m_hi = m / n with m_hi % 4 == q; the last digit loops inside, so
// each element costs one multiply and one FMA.  Wave partials are summed in
// fixed order.
constexpr int kMvRows = 64;
constexpr int kMvLd = kMvRows + 2;   // table row pitch: 16 rows x 2 samples hit distinct LDS banks

__device__ __forceinline__ f64x4 mfma64m(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Phi w (or y - Phi w) for a block of 64 samples, on FP64 MFMA.  With
// m = hi*n + k (k the last digit) Phi[i, m] = PRE[i][hi] * phi_{p-1,k}(x_i), so
//   (Phi w)[i] = sum_hi PRE[i][hi] * U[i][hi],  U = Lt Wm,
// Lt[i][k] = phi_{p-1,k}(x_i) (64 x n), Wm[k][hi] = w[hi*n + k] (n x M/n).
// Each wave takes prefix tiles of 16 (tile wv, wv+4, ...) against all 64
// samples (four 16-row MFMA tiles, k padded to 4), scales U by the prefix
// products of its lanes' (sample, prefix) pairs and accumulates per sample;
// the 16 lanes of a sample and then the four waves are summed at the end.
// The w block of a wave's next tile (16 n contiguous values) and its lanes'
// prefix digit rows are fetched while the current tile is computed (the w
// block through a per-wave double buffer in LDS).
__global__ void __launch_bounds__(256) phi_matvec_kernel(const double* __restrict__ x, int64_t N, int p,
                                                         int n, int M, const double* __restrict__ tab,
                                                         const uint16_t* __restrict__ midx,
                                                         const double* __restrict__ w,
                                                         const double* __restrict__ y,
                                                         double* __restrict__ out) {
  extern __shared__ double sm[];
  double* T = sm;                                 // [p*n][64]
  double* red = sm + p * n * kMvLd;               // [4][64]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int wblk = 16 * n;                        // w values of one prefix tile
  double* wb = red + 4 * kMvRows + wv * 2 * wblk; // this wave's [2][16 n] w buffers
  const int64_t s0 = (int64_t)blockIdx.x * kMvRows;
  fill_tab_sf<double>(x, N, p, n, s0, kMvRows, kMvLd, tab, T);
  const int H = M / n, nk = (n + 3) / 4;
  const double* Tl = T + (p - 1) * n * kMvLd;     // rows of the last factor
  // fetch tile ht's w block (zero past M) into buffer bf, and the digit rows
  // of this lane's prefix in tile ht
  auto fetch_w = [&](int ht, int bf) {
    const int64_t base = (int64_t)ht * wblk;
    for (int u = lane; u < wblk; u += 64) wb[bf * wblk + u] = base + u < M ? w[base + u] : 0.0;
  };
  auto fetch_dig = [&](int ht) {
    const int hi = ht * 16 + (lane & 15);
    return reinterpret_cast<const uint4*>(midx)[hi < H ? hi * n : 0];
  };
  double acc[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[rt][q] = 0.0;
  int bf = 0;
  uint4 dq_next = fetch_dig(wv);
  if (wv * 16 < H) fetch_w(wv, 0);
  __syncthreads();
  for (int ht = wv; ht * 16 < H; ht += 4) {
    const uint4 dq = dq_next;
    if ((ht + 4) * 16 < H) {
      dq_next = fetch_dig(ht + 4);
      fetch_w(ht + 4, bf ^ 1);
    }
    const int hi = ht * 16 + (lane & 15);
    const bool hv = hi < H;
    const double* wt = wb + bf * wblk;
    f64x4 d[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) d[rt] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int ks = 0; ks < nk; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const bool kv = k < n;
      const double b = kv ? wt[(lane & 15) * n + k] : 0.0;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt) {
        const double a = kv ? Tl[k * kMvLd + rt * 16 + (lane & 15)] : 0.0;
        d[rt] = mfma64m(a, b, d[rt]);
      }
    }
    // 1-D table rows of the leading digits of this lane's prefix, then
    // PRE * U per (sample, prefix) with one unrolled body per factor count
    int rows[GP_MAX_P];
    {
      const uint32_t dd[4] = {dq.x, dq.y, dq.z, dq.w};
#pragma unroll
      for (int j = 0; j < GP_MAX_P; ++j) rows[j] = ((dd[j >> 1] >> ((j & 1) * 16)) & 0xffff) * kMvLd;
    }
    auto scale_acc = [&](auto kc) {
      constexpr int K = decltype(kc)::value;
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int sm_i = rt * 16 + 4 * q + (lane >> 4);
          double pre = hv ? 1.0 : 0.0;
#pragma unroll
          for (int j = 0; j < K; ++j) pre *= T[rows[j] + sm_i];
          acc[rt][q] = fma(pre, d[rt][q], acc[rt][q]);
        }
    };
    switch (p - 1) {
      case 0: scale_acc(std::integral_constant<int, 0>{}); break;
      case 1: scale_acc(std::integral_constant<int, 1>{}); break;
      case 2: scale_acc(std::integral_constant<int, 2>{}); break;
      case 3: scale_acc(std::integral_constant<int, 3>{}); break;
      case 4: scale_acc(std::integral_constant<int, 4>{}); break;
      case 5: scale_acc(std::integral_constant<int, 5>{}); break;
      case 6: scale_acc(std::integral_constant<int, 6>{}); break;
      default: scale_acc(std::integral_constant<int, 7>{}); break;
    }
    bf ^= 1;
  }
  // sum over the 16 lanes that share a sample, then over the waves
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = acc[rt][q];
      v += __shfl_xor(v, 1);
      v += __shfl_xor(v, 2);
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if ((lane & 15) == 0) red[wv * kMvRows + rt * 16 + 4 * q + (lane >> 4)] = v;
    }
  __syncthreads();
  if (wv == 0) {
    const double sum = ((red[lane] + red[64 + lane]) + red[128 + lane]) + red[192 + lane];
    const int64_t row = s0 + lane;
    if (row < N) out[row] = y ? y[row] - sum : sum;
  }
}

void launch_phi_matvec(const double* x, int64_t N, int p, int n, int M, const double* tab, const uint16_t* midx,
                       const double* w, const double* y, double* out, hipStream_t s) {
  if (N <= 0) return;
  const size_t lds = (size_t)(p * n * kMvLd + 4 * kMvRows + 4 * 2 * 16 * n) * sizeof(double);
  hipLaunchKernelGGL(phi_matvec_kernel, dim3(ceil_div(N, kMvRows)), dim3(256), lds, s, x, N, p, n, M, tab, midx,
                     w, y, out);
}

// ---------------------------------------------------------------- Phi^T v
// With m = hi*n + k (k the last digit), Phi[i, m] = PRE[i][hi] * phi_{p-1,k}(x_i)
// where PRE is the product of the leading p-1 factors, so
//   (Phi^T v)[hi*n + k] = sum_i PRE[i][hi] * (phi_{p-1,k}(x_i) v_i),
// an (M/n x N) by (N x n) product.  Work-group: 256 prefixes hi x all n
// last digits over a chunk of samples, FP64 MFMA (16x16x4) on per-stage
// tiles of 16 samples built in LDS: PRE^T [16 samples][256 hi] and
// W [16 samples][n padded to 16]; the samples (x, v) of the next stage are
// loaded while the current one is processed.  The chunk (a multiple of 16,
// 64 .. 1024) is sized so that about 256 work-groups share the samples: a
// small problem is not left to a few work-groups walking long chunks.
// Partials part[chunk][M] are reduced in chunk order.
constexpr int kTvChunkMax = 1024;
static int64_t phiT_chunk(int64_t N) {
  int64_t c = (ceil_div(N, 256) + 15) / 16 * 16;
  return c < 64 ? 64 : c > kTvChunkMax ? kTvChunkMax : c;
}
constexpr int kTvKC = 16;
constexpr int kTvLd = kTvKC + 1;     // table row pitch: rows of consecutive digits hit distinct LDS banks
constexpr int kTvH = 256;

__device__ __forceinline__ f64x4 mfma64v(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Partials are reduced in two passes: kTvGroups groups of consecutive
// chunks (one work-group column each), then the group sums in order.
constexpr int64_t kTvGroups = 64;
static int64_t phiT_groups(int64_t chunks) { return chunks < kTvGroups ? chunks : kTvGroups; }
int64_t phiT_part_elems(int64_t N, int M) {
  const int64_t chunks = ceil_div(N, phiT_chunk(N));
  return (chunks + phiT_groups(chunks)) * (int64_t)M;
}

template <int NB>   // NB = ceil(n / 16) column blocks of the last digit
__global__ void __launch_bounds__(256) phiT_gemm_kernel(const double* __restrict__ x, const double* __restrict__ v,
                                                        int64_t N, int p, int n, int M, int64_t chunk,
                                                        const double* __restrict__ tab, double* __restrict__ part) {
  extern __shared__ double sm[];
  double* T = sm;                                 // [p*n][17] 1-D tables of the stage
  double* PR = T + p * n * kTvLd;                 // [16][kTvH + 2]
  double* W = PR + kTvKC * (kTvH + 2);            // [16][NB*16 + 2]
  double* VS = W + kTvKC * (NB * 16 + 2);         // [16] v of the stage
  const int WP = NB * 16 + 2;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int H = M / n;
  const int h0 = blockIdx.y * kTvH;
  const int64_t c0 = (int64_t)blockIdx.x * chunk;
  const int64_t c1 = min(c0 + chunk, N);
  // prefix digits of this thread's hi (one per thread)
  const int hi = h0 + t;
  int dig[GP_MAX_P];
  {
    int rem = hi < H ? hi : 0;
#pragma unroll
    for (int j = GP_MAX_P - 2; j >= 0; --j) {
      dig[j] = 0;
      if (j <= p - 2) {
        dig[j] = rem % n;
        rem /= n;
      }
    }
  }
  f64x4 acc[4][NB];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};

  // the stage's samples: thread (i, j), i < 16, j < p, holds x[s0 + i][j];
  // thread i < 16 holds v[s0 + i]
  const int xi = t % kTvKC, xj = t / kTvKC;
  auto load_x = [&](int64_t s) { return (xj < p && s + xi < c1) ? x[(s + xi) * p + xj] : 0.0; };
  auto load_v = [&](int64_t s) { return (t < kTvKC && s + t < c1) ? v[s + t] : 0.0; };
  double xn = load_x(c0), vn = load_v(c0);
  for (int64_t s0 = c0; s0 < c1; s0 += kTvKC) {
    const double xc = xn, vc = vn;
    xn = load_x(s0 + kTvKC);
    vn = load_v(s0 + kTvKC);
    __syncthreads();
    // 1-D tables: thread (i, j) for i < 16, j < p
    if (xj < p) {
      const int64_t row = s0 + xi;
      double* o = T + (xj * n) * kTvLd + xi;
      if (row < c1) {
        const double* dc = tab + kTabDim + xj * kDimStride;
        phi_1d<double, double>(xc, dc, tab + kTabRc1, tab + kTabRc2, n, o, kTvLd);
      } else {
        for (int k = 0; k < n; ++k) o[k * kTvLd] = 0.0;
      }
    }
    if (t < kTvKC) VS[t] = vc;
    __syncthreads();
    // PRE^T: thread = prefix, 16 samples (one unrolled body per factor count)
    {
      double pr[kTvKC];
#pragma unroll
      for (int i = 0; i < kTvKC; ++i) pr[i] = (hi < H) ? 1.0 : 0.0;
      auto mul_rows = [&](auto kc) {
        constexpr int K = decltype(kc)::value;
#pragma unroll
        for (int j = 0; j < K; ++j) {
          const double* Tj = T + (j * n + dig[j]) * kTvLd;
#pragma unroll
          for (int i = 0; i < kTvKC; ++i) pr[i] *= Tj[i];
        }
      };
      switch (p - 1) {
        case 0: break;
        case 1: mul_rows(std::integral_constant<int, 1>{}); break;
        case 2: mul_rows(std::integral_constant<int, 2>{}); break;
        case 3: mul_rows(std::integral_constant<int, 3>{}); break;
        case 4: mul_rows(std::integral_constant<int, 4>{}); break;
        case 5: mul_rows(std::integral_constant<int, 5>{}); break;
        case 6: mul_rows(std::integral_constant<int, 6>{}); break;
        default: mul_rows(std::integral_constant<int, 7>{}); break;
      }
#pragma unroll
      for (int i = 0; i < kTvKC; ++i) PR[i * (kTvH + 2) + t] = pr[i];
    }
    // W = last-dimension factor times v: [16][NB*16]
    for (int u = t; u < kTvKC * NB * 16; u += 256) {
      const int i = u / (NB * 16), k = u % (NB * 16);
      const int64_t row = s0 + i;
      W[i * WP + k] = (k < n && row < c1) ? T[((p - 1) * n + k) * kTvLd + i] * VS[i] : 0.0;
    }
    __syncthreads();
    // MFMA: wave wv owns prefixes wv*64 .. +64 (4 blocks of 16)
#pragma unroll
    for (int kk = 0; kk < kTvKC / 4; ++kk) {
      const int i = kk * 4 + (lane >> 4);
      double av[4], bv[NB];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = PR[i * (kTvH + 2) + wv * 64 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < NB; ++b) bv[b] = W[i * WP + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[a][b] = mfma64v(av[a], bv[b], acc[a][b]);
    }
  }
  // D[hi][k]: element q of acc[a][b] is row 4q + lane/16, column lane%16
  double* out = part + (int64_t)blockIdx.x * M;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int h = h0 + wv * 64 + a * 16 + 4 * q + (lane >> 4);
        const int k = b * 16 + (lane & 15);
        if (h < H && k < n) out[(int64_t)h * n + k] = acc[a][b][q];
      }
}

// Group g of G sums the chunks [g*per, (g+1)*per) of column m in order into
// row chunks + g of part; then the G group rows are summed in order.
__global__ void reduce_cols_group_kernel(double* __restrict__ part, int64_t chunks, int64_t per, int M) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const int64_t c0 = (int64_t)blockIdx.y * per, c1 = min(c0 + per, chunks);
  double s = 0.0;
  for (int64_t c = c0; c < c1; ++c) s += part[c * M + m];
  part[(chunks + blockIdx.y) * M + m] = s;
}

__global__ void reduce_cols_kernel(const double* __restrict__ part, int64_t rows, int M,
                                   const double* __restrict__ sub, const double* __restrict__ wsub,
                                   double* __restrict__ out) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double s = 0.0;
  for (int64_t c = 0; c < rows; ++c) s += part[c * M + m];
  if (sub) s -= sub[m] * wsub[m];
  out[m] = s;
}

void launch_phiT_vec(const double* x, const double* v, int64_t N, int p, int n, int M, const double* tab,
                     double* part, const double* sub, const double* wsub, double* out, hipStream_t s) {
  const int64_t chunk = phiT_chunk(N);
  const int64_t chunks = ceil_div(N, chunk);
  const int H = M / n;
  const int NB = (int)ceil_div(n, 16);
  const size_t lds =
      (size_t)(p * n * kTvLd + kTvKC * (kTvH + 2) + kTvKC * (NB * 16 + 2) + kTvKC) * sizeof(double);
  const dim3 grid(chunks, ceil_div(H, kTvH));
  switch (NB) {
    case 1: hipLaunchKernelGGL(phiT_gemm_kernel<1>, grid, dim3(256), lds, s, x, v, N, p, n, M, chunk, tab, part); break;
    case 2: hipLaunchKernelGGL(phiT_gemm_kernel<2>, grid, dim3(256), lds, s, x, v, N, p, n, M, chunk, tab, part); break;
    case 3: hipLaunchKernelGGL(phiT_gemm_kernel<3>, grid, dim3(256), lds, s, x, v, N, p, n, M, chunk, tab, part); break;
    default: hipLaunchKernelGGL(phiT_gemm_kernel<4>, grid, dim3(256), lds, s, x, v, N, p, n, M, chunk, tab, part); break;
  }
  const int64_t G = phiT_groups(chunks), per = ceil_div(chunks, G);
  if (per == 1) {
    // groups of one chunk: the group pass would only copy the rows
    hipLaunchKernelGGL(reduce_cols_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, part, chunks, M, sub, wsub, out);
    return;
  }
  hipLaunchKernelGGL(reduce_cols_group_kernel, dim3(ceil_div(M, 256), ceil_div(chunks, per)), dim3(256), 0, s, part,
                     chunks, per, M);
  hipLaunchKernelGGL(reduce_cols_kernel, dim3(ceil_div(M, 256)), dim3(256), 0, s, part + chunks * (int64_t)M,
                     ceil_div(chunks, per), M, sub, wsub, out);
}

// ---------------------------------------------------------------- input checks
__global__ void check_finite_kernel(const double* __restrict__ a, int64_t na, const double* __restrict__ b,
                                    int64_t nb, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < na + nb; i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(i < na ? a[i] : b[i - na]);
  if (__any(bad) && (threadIdx.x & 63) == 0) *flag = 1;
}

void launch_check_finite(const double* a, int64_t na, const double* b, int64_t nb, int* flag, hipStream_t s) {
  const int64_t count = na + nb;
  if (count <= 0) return;
  int64_t blocks = ceil_div(count, 256);
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(check_finite_kernel, dim3(blocks), dim3(256), 0, s, a, na, b, nb, flag);
}

// ---------------------------------------------------------------- fills (kernels, not memset nodes)
__global__ void fill_zero_int_kernel(int* __restrict__ p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}
__global__ void fill_zero_f64_kernel(double* __restrict__ p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}
void launch_fill_zero_int(int* p, int count, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_int_kernel, dim3(ceil_div(count, 256)), dim3(256), 0, s, p, count);
}
void launch_fill_zero_f64(double* p, int64_t count, hipStream_t s) {
  int64_t blocks = ceil_div(count, 256);
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(fill_zero_f64_kernel, dim3(blocks), dim3(256), 0, s, p, count);
}

}  // namespace mgp
