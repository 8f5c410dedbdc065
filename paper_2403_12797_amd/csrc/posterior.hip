// Beyond the diagonal of the posterior: the materialised Phi_* of a block of
// test points (for the full predictive covariance of eq. 12), and the fit
// statistics that give the log marginal likelihood of the truncated-kernel
// GP (the quantity hyperparameter learning maximises).
#include "kernels.h"

namespace mgp {

// Phi_*[i][m] = prod_j phi_{j, k_j(m)}(x_ij) (eqs. 15, 19): one work-group
// per 32 points; their 1-D tables are formed in LDS in FP64, then each thread
// takes columns of its point row through the multi-index table.
constexpr int kPdPts = 32;
__global__ void __launch_bounds__(256) phi_dense_kernel(const double* __restrict__ xs, int64_t Ns, int p, int n, int M,
                                                        const double* __restrict__ tab,
                                                        const uint16_t* __restrict__ midx, double* __restrict__ out) {
  extern __shared__ double T[];   // [kPdPts][p*n]
  const int64_t i0 = (int64_t)blockIdx.x * kPdPts;
  const int rows = p * n;
  for (int u = threadIdx.x; u < kPdPts * p; u += blockDim.x) {
    const int i = u / p, j = u % p;
    double* o = T + i * rows + j * n;
    if (i0 + i < Ns) {
      const double* dc = tab + kTabDim + j * kDimStride;
      phi_1d<double, double>(xs[(i0 + i) * p + j], dc, tab + kTabRc1, tab + kTabRc2, n, o, 1);
    } else {
      for (int k = 0; k < n; ++k) o[k] = 0.0;
    }
  }
  __syncthreads();
  const int np = (int)min<int64_t>(kPdPts, Ns - i0);
  for (int64_t u = threadIdx.x; u < (int64_t)np * M; u += blockDim.x) {
    const int i = (int)(u / M), m = (int)(u - (u / M) * M);
    const uint4 dq = reinterpret_cast<const uint4*>(midx)[m];
    const uint32_t d[4] = {dq.x, dq.y, dq.z, dq.w};
    double v = 1.0;
    for (int j = 0; j < p; ++j) v *= T[i * rows + ((d[j >> 1] >> ((j & 1) * 16)) & 0xffff)];
    out[(i0 + i) * M + m] = v;
  }
}

void launch_phi_dense(const double* xs, int64_t Ns, int p, int n, int M, const double* tab, const uint16_t* midx,
                      double* out, hipStream_t s) {
  if (Ns <= 0) return;
  const size_t lds = (size_t)kPdPts * p * n * sizeof(double);
  hipLaunchKernelGGL(phi_dense_kernel, dim3(ceil_div(Ns, kPdPts)), dim3(256), lds, s, xs, Ns, p, n, M, tab, midx,
                     out);
}

// Deterministic sum of squares of y: kLmlParts work-groups, each a fixed
// grid-stride range and a fixed tree in LDS.
__global__ void __launch_bounds__(256) sumsq_part_kernel(const double* __restrict__ y, int64_t N,
                                                         double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)kLmlParts * 256) acc += y[i] * y[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One work-group: y^T y from the parts, sum log L_ii, sum log Lambda_m and
// b^T w over the M columns (fixed trees), then
//   log p(y) = -(y^T y - b^T w) / (2 sigma^2)
//              - ((N - M) log sigma^2 + sum log Lambda + 2 sum log L_ii) / 2
//              - N log(2 pi) / 2,
// the Gaussian log-density of y under K~ + sigma^2 I (eqs. 7-8) written with
// the M x M system: Woodbury for the quadratic form (as in eq. 10) and the
// determinant lemma with A = Phi^T Phi + sigma^2 Lambda^-1 = L L^T.
__global__ void __launch_bounds__(256) lml_kernel(const double* __restrict__ part, int64_t N,
                                                  const double* __restrict__ b, const double* __restrict__ w,
                                                  const double* __restrict__ L, const double* __restrict__ lam, int M,
                                                  double sigma, double* __restrict__ stats) {
  __shared__ double red[4][256];
  const int t = threadIdx.x;
  double yy = 0.0, ld = 0.0, ll = 0.0, bw = 0.0;
  for (int i = t; i < kLmlParts; i += 256) yy += part[i];
  for (int m = t; m < M; m += 256) {
    ld += log(L[(int64_t)m * M + m]);
    ll += log(lam[m]);
    bw += b[m] * w[m];
  }
  red[0][t] = yy;
  red[1][t] = ld;
  red[2][t] = ll;
  red[3][t] = bw;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s)
      for (int q = 0; q < 4; ++q) red[q][t] += red[q][t + s];
    __syncthreads();
  }
  if (t == 0) {
    const double s2 = sigma * sigma;
    const double Nd = (double)N;
    const double logdet_S = (Nd - M) * log(s2) + red[2][0] + 2.0 * red[1][0];
    stats[0] = red[0][0];
    stats[1] = red[1][0];
    stats[2] = red[2][0];
    stats[3] = red[3][0];
    stats[4] = -0.5 * (red[0][0] - red[3][0]) / s2 - 0.5 * logdet_S - 0.5 * Nd * log(2.0 * 3.14159265358979323846);
    stats[5] = Nd;
  }
}

void launch_fit_stats(const double* y, int64_t N, const double* b, const double* w, const double* L,
                      const double* lam, int M, double sigma, double* part, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_part_kernel, dim3(kLmlParts), dim3(256), 0, s, y, N, part);
  hipLaunchKernelGGL(lml_kernel, dim3(1), dim3(256), 0, s, part, N, b, w, L, lam, M, sigma, stats);
}

}  // namespace mgp
