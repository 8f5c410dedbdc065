// Launchers of the libmercergp device kernels (all asynchronous on `s`).
#pragma once

#include "common.h"

namespace mgp {

struct EigArgs {
  int p, n;
  int kind;   // gp_kernel
  double sigma;
  double eps[GP_MAX_P];
  double alpha[GP_MAX_P];
};

// a1: per-dimension constants, recurrence coefficients and 1-D eigenvalues
// into tab[kTabSize]; Lambda[M] (eq. 20) and reg[M] = sigma^2 / Lambda.
void launch_eig_tables(const EigArgs& a, double* tab, double* lam, double* reg, int M, hipStream_t s);

// out[i] = y ? y[i] - (Phi w)_i : (Phi w)_i, Phi generated on the fly from x
// (the mean Phi_* w and the residual y - Phi w); midx is the multi-index table.
void launch_phi_matvec(const double* x, int64_t N, int p, int n, int M, const double* tab,
                       const uint16_t* midx, const double* w, const double* y, double* out, hipStream_t s);

// out[m] = sum_i Phi[i,m] v[i] - (sub ? sub[m] * wsub[m] : 0), deterministic
// two-pass reduction through `part` (see phiT_part_elems).
int64_t phiT_part_elems(int64_t N, int M);
void launch_phiT_vec(const double* x, const double* v, int64_t N, int p, int n, int M,
                     const double* tab, double* part, const double* sub, const double* wsub,
                     double* out, hipStream_t s);

// a3 (FP64): A = Phi^T Phi + diag(reg), full symmetric M x M row-major.
int64_t gram_f64_part_elems(int64_t N, int M, int* splitk_out);
void launch_gram_f64(const double* x, int64_t N, int p, int n, int M, const double* tab,
                     const double* reg, double* part, double* A, hipStream_t s, Prof* prof = nullptr);

// a3 (mixed): split MFMA Gram on scaled Phi (f16: two FP16 terms, three
// products; else three BF16 terms, six products), FP32 accumulate, FP64
// split-K reduce.  Samples are processed in chunks of `chunk` (a multiple of
// 16); each (upper tile, chunk) writes an FP32 partial, at most 8 GiB of
// partials per pass.  tab32 holds gram_mixed_table_elems() floats: the 1-D
// tables and their per-row maxima, written by launch_gram_mixed_table(),
// which must run before launch_gram_mixed() on the same stream.
// Two layouts of the work:
//  * direct: upper 256 x 256 tiles of Phi^T Phi, each in two 128-column halves;
//  * paired (pair = 1, pair_gram.hip): H = Psi1^T Psi2 over the pair tuples of
//    two groups of dimensions (s = n(n+1)/2 pairs per dimension, p1 = p / 2
//    leading dimensions, S1 = s^p1, S2 = s^(p - p1)), in T1 x T2 items of
//    256 x 128; A is gathered from H (hbuf, S1 x S2 FP64).
struct GramPlan {
  int T, ntiles, chunk, splits_total, splits_per_pass, passes;
  int pair, p1, s, S1, S2, T1, T2;
};
GramPlan gram_mixed_plan(int64_t N, int p, int n, int M, bool f16, int chunk /* <= 0: default */);
int64_t gram_mixed_part_elems(const GramPlan& g);
int64_t gram_mixed_hbuf_elems(const GramPlan& g);
int64_t gram_mixed_table_elems(int64_t N, int p, int n);
size_t gram_mixed_lds_bytes(int p, int n, int M, const GramPlan& g, bool f16);
void launch_gram_mixed_table(const double* x, int64_t N, int p, int n, const double* tab, float* tab32,
                             hipStream_t s);
void launch_gram_mixed(const double* x, int64_t N, int p, int n, int M, const GramPlan& g, bool f16,
                       const double* tab, const double* reg, float* part, float* tab32, double* hbuf, double* A,
                       hipStream_t s, Prof* prof = nullptr);
// Sum `splits` partials into A (first: A = reg on the diagonal + sum; else
// A += sum); paired plans sum into hbuf and gather A on the last pass.
void launch_gram_mixed_reduce(const float* part, int splits, int p, int n, int M, const GramPlan& g,
                              const double* reg, bool first, bool last, double* hbuf, double* A, hipStream_t s);
// Batched: one persistent launch over the work items of many problems that
// share a Gram scheme and layout.
struct GramProb {
  const float* tab32;
  float* part;
  int64_t N;
  int p, n, M, T, chunk, ntiles;
  int p1, S1, S2, T2;   // paired layout
};
struct GramItem {
  int prob, tile, h, split;
};
void launch_gram_mixed_batch(const GramProb* probs_dev, const GramItem* items_dev, int nitems, bool f16,
                             int* counter, size_t lds, hipStream_t s, Prof* prof = nullptr);
// paired layout (pair_gram.hip): plan, kernels and reduction
bool pair_plan(int p, int n, int M, bool f16, GramPlan& g);
void pair_plan_splits(int64_t N, GramPlan& g, int chunk);
size_t pair_gram_lds_bytes(int p, int n, const GramPlan& g, bool f16);
int pair_factors(int p, const GramPlan& g);
void launch_gram_pair(int64_t N, int p, int n, int M, const GramPlan& g, bool f16, const double* reg, float* part,
                      const float* tab32, double* H, double* A, hipStream_t s, Prof* prof);
void launch_pair_reduce(const float* part, int splits, int p, int n, int M, const GramPlan& g, const double* reg,
                        bool first, bool last, double* H, double* A, hipStream_t s);
void launch_gram_pair_batch(const GramProb* probs_dev, const GramItem* items_dev, int nitems, bool f16, int F,
                            int* counter, size_t lds, hipStream_t s, Prof* prof);
hipError_t configure_pair_kernels();

// a4: blocked Cholesky in place (lower), block inverses Dinv[M/64][64*64],
// info (device int, 0 = ok, else failing column + 1).
constexpr int kCholNb = 64;
void launch_cholesky(double* A, int M, double* Dinv, int* info, hipStream_t s);
// L^-1 (lower, upper part zero) from L and Dinv; ws holds
// trtri_workspace_elems(M) doubles.
size_t trtri_workspace_elems(int M);
void launch_trtri(const double* L, const double* Dinv, double* Linv, double* ws, int M,
                  const int* info, hipStream_t s);
// z = Linv b ; w = Linv^T z  (both through `tmp`, M doubles)
void launch_lower_matvec(const double* Linv, const double* b, double* z, int M, hipStream_t s);
// (w = add + Linv^T z when add is given; add may be w itself)
void launch_lower_t_matvec(const double* Linv, const double* z, double* w, double* part, int M,
                           hipStream_t s, const double* add = nullptr);
// Split of L^-1 into two bf16 terms (mixed predict): pieces[q][M][P] with
// row pitch P = linv_pitch(M) (multiple of 16, padding columns zero).
__host__ __device__ inline int linv_pitch(int M) { return (M + 15) & ~15; }
// Rows of each L^-1 term: M rounded up to 256 (padding rows zero), so that
// 256-row slabs read without bounds tests.
__host__ __device__ inline int linv_rows(int M) { return (M + 255) & ~255; }
void launch_split_linv(const double* Linv, __bf16* pieces, int M, hipStream_t s);

// a5 variance: var[i] = sigma^2 || L^-1 phi_*(x_i) ||^2
int64_t predict_part_elems(int64_t Ns, int M, int* groups_out);
void launch_predict_var_f64(const double* xs, int64_t Ns, int p, int n, int M, const double* tab,
                            const double* Linv, double sigma2, double* part, double* var,
                            hipStream_t s, Prof* prof = nullptr);
// a5 mixed: mean by the FP64 Phi w kernel, variance by split-BF16 MFMA.
int64_t predict_mixed_part_elems(int64_t Ns, int M, int* groups_out);
void launch_predict_mixed(const double* xs, int64_t Ns, int p, int n, int M, const double* tab,
                          const uint16_t* midx, const uint32_t* pdesc, const __bf16* linv_pieces,
                          const double* w, double sigma2, double* part, double* mean, double* var,
                          hipStream_t s, Prof* prof = nullptr);
// Multi-index table: midx[c][j] = j*n + k_j(c), 8 uint16 per column.
void launch_midx(int p, int n, int M, uint16_t* midx, hipStream_t s);
// Per-column descriptors of the mixed prediction (pdesc_elems(M) uint32).
int64_t pdesc_elems(int M);
void launch_pdesc(int p, int n, int M, uint32_t* pdesc, hipStream_t s);

// C = alpha A B^T (row-major; B lower triangular if b_lower) on FP64 MFMA.
void launch_gemm_nt_f64(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc, int m,
                        int n, int k, double alpha, bool b_lower, hipStream_t s);
// Phi_* materialised, row-major [Ns][M] in FP64 (covariance blocks only).
void launch_phi_dense(const double* xs, int64_t Ns, int p, int n, int M, const double* tab, const uint16_t* midx,
                      double* out, hipStream_t s);
// Fit statistics for the log marginal likelihood (see posterior.hip):
// stats[0] = y^T y, [1] = sum log L_ii, [2] = sum log Lambda_m, [3] = b^T w,
// [4] = log p(y), [5] = N.  part holds kLmlParts doubles.
constexpr int kLmlParts = 256;
void launch_fit_stats(const double* y, int64_t N, const double* b, const double* w, const double* L,
                      const double* lam, int M, double sigma, double* part, double* stats, hipStream_t s);

// Zero fills as kernels (safe inside captured graphs).
void launch_fill_zero_int(int* p, int count, hipStream_t s);
void launch_fill_zero_f64(double* p, int64_t count, hipStream_t s);

// Device check that every element of v[count] is finite; sets *flag = 1 if not.
// flag = 1 if any of a[0..na) or b[0..nb) is not finite (one launch)
void launch_check_finite(const double* a, int64_t na, const double* b, int64_t nb, int* flag, hipStream_t s);

// Raise the dynamic-LDS limit of the kernels that need more than 64 KB.
hipError_t configure_kernels();

}  // namespace mgp
