// C ABI beyond the hot path: the log marginal likelihood of a fitted model,
// the full predictive covariance of a block of test points, and
// hyperparameter learning by maximising the log marginal likelihood.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "kernels.h"
#include "runtime.h"

using namespace mgp;

extern "C" {

gp_status gp_model_lml(const gp_model* model, double* lml) {
  if (!model || !lml) return fail(GP_EINVAL, "model/lml is NULL");
  if (hipSetDevice(model->ctx->device) != hipSuccess) return fail(GP_EDEVICE, "hipSetDevice");
  double st[8];
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(st, model->stats, sizeof(st), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(GP_EDEVICE, "gp_model_lml: %s", hipGetErrorString(e));
  *lml = st[4];
  return GP_OK;
}

gp_status gp_predict_cov(gp_ctx* ctx, const gp_model* model, const double* xs, int64_t Ns, double* cov, int64_t ld,
                         void* stream) {
  if (!ctx || !model) return fail(GP_EINVAL, "ctx/model is NULL");
  if (Ns < 0) return fail(GP_EINVAL, "Ns=%lld must be >= 0", (long long)Ns);
  if (Ns == 0) return GP_OK;
  if (!xs || !cov) return fail(GP_EINVAL, "xs/cov is NULL");
  if (ld < Ns) return fail(GP_EINVAL, "ld=%lld < Ns=%lld", (long long)ld, (long long)Ns);
  if (Ns > (int64_t)1 << 20) return fail(GP_EINVAL, "Ns=%lld: covariance blocks are limited to 2^20 points", (long long)Ns);
  if (!model->Linv)
    return fail(GP_EINVAL, "the model keeps no FP64 L^-1 (served models are lean); fit it with gp_fit");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(GP_EDEVICE, "hipSetDevice");
  hipStream_t s = (hipStream_t)stream;
  const int p = model->p, n = model->n, M = (int)model->M;
  const size_t zb = (size_t)Ns * M * sizeof(double);
  char* ws = nullptr;
  hipError_t e = hipMallocAsync((void**)&ws, 2 * zb, s);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EDEVICE, "covariance workspace of %zu bytes", 2 * zb);
  double* phi = (double*)ws;
  double* Z = (double*)(ws + zb);
  // Phi_* (Ns x M), Z = Phi_* L^-T (L^-1 lower: Z[i][r] sums c <= r), then
  // Sigma_* = sigma^2 Z Z^T  (eq. 12 in weight-space form)
  launch_phi_dense(xs, Ns, p, n, M, model->tab, model->midx, phi, s);
  launch_gemm_nt_f64(phi, M, model->Linv, M, Z, M, (int)Ns, M, M, 1.0, true, s);
  launch_gemm_nt_f64(Z, M, Z, M, cov, ld, (int)Ns, (int)Ns, M, model->sigma * model->sigma, false, s);
  hipFreeAsync(ws, s);
  e = hipGetLastError();
  if (e != hipSuccess) return fail(GP_EDEVICE, "gp_predict_cov: %s", hipGetErrorString(e));
  return GP_OK;
}

gp_status gp_learn(gp_ctx* ctx, const gp_params* start, const double* x, const double* y, int64_t N,
                   const gp_learn_opts* opts, void* stream, double* eps_out, double* alpha_out, double* sigma_out,
                   double* lml_out, int32_t* evals_out) {
  if (!ctx || !start || !x || !y) return fail(GP_EINVAL, "ctx/start/x/y is NULL");
  int64_t M = 0;
  gp_status st = validate_params(start, &M);
  if (st != GP_OK) return st;
  if (N < 1) return fail(GP_EINVAL, "N=%lld must be >= 1", (long long)N);
  gp_learn_opts o{};
  if (opts) o = *opts;
  const int max_evals = o.max_evals > 0 ? o.max_evals : 150;
  const double tol = o.tol > 0.0 ? o.tol : 1e-6;
  const int p = start->p;
  const int ne = o.per_dim ? p : 1;                 // eps parameters
  const int na = o.learn_alpha ? (o.per_dim ? p : 1) : 0;
  const int dim = ne + na + (o.learn_sigma ? 1 : 0);
  // theta: log eps (ne), log alpha (na), log sigma; a dimension without its
  // own parameter takes the first one
  std::vector<double> th0(dim);
  for (int j = 0; j < ne; ++j) th0[j] = log(start->eps[j]);
  for (int j = 0; j < na; ++j) th0[ne + j] = log(start->alpha[j]);
  if (o.learn_sigma) th0[ne + na] = log(start->sigma);
  int evals = 0;
  gp_status last_err = GP_OK;
  auto unpack = [&](const std::vector<double>& th, double* eps, double* alpha, double* sigma) {
    for (int j = 0; j < p; ++j) {
      eps[j] = exp(th[o.per_dim ? j : 0]);
      alpha[j] = na ? exp(th[ne + (o.per_dim ? j : 0)]) : start->alpha[j];
    }
    *sigma = o.learn_sigma ? exp(th[ne + na]) : start->sigma;
  };
  // objective: minus the log marginal likelihood of a fit at theta (+inf if
  // the fit fails, e.g. A not numerically SPD)
  auto f = [&](const std::vector<double>& th) {
    double eps[GP_MAX_P], alpha[GP_MAX_P], sigma;
    unpack(th, eps, alpha, &sigma);
    gp_params prm = *start;
    prm.eps = eps;
    prm.alpha = alpha;
    prm.sigma = sigma;
    ++evals;
    gp_model* m = nullptr;
    const gp_status s1 = gp_fit(ctx, &prm, x, y, N, stream, &m);
    if (s1 != GP_OK) {
      if (s1 != GP_ENOTSPD && s1 != GP_EINVAL) last_err = s1;
      return HUGE_VAL;
    }
    double v = 0.0;
    const gp_status s2 = gp_model_lml(m, &v);
    gp_model_free(m);
    if (s2 != GP_OK || !isfinite(v)) {
      if (s2 != GP_OK) last_err = s2;
      return HUGE_VAL;
    }
    return -v;
  };
  // Nelder-Mead (reflection 1, expansion 2, contraction 1/2, shrink 1/2) on
  // theta, initial simplex steps of 0.3 in each log-parameter
  std::vector<std::vector<double>> X(dim + 1, th0);
  std::vector<double> F(dim + 1, HUGE_VAL);
  for (int k = 0; k < dim; ++k) X[k + 1][k] += 0.3;
  for (int k = 0; k <= dim && evals < max_evals; ++k) F[k] = f(X[k]);
  if (last_err != GP_OK) return fail(last_err, "gp_learn: %s", gp_last_error(ctx));
  std::vector<int> ord(dim + 1);
  while (evals < max_evals) {
    for (int k = 0; k <= dim; ++k) ord[k] = k;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return F[a] < F[b]; });
    const int best = ord[0], worst = ord[dim], second = ord[dim - 1];
    if (isfinite(F[worst]) && F[worst] - F[best] <= tol) break;
    std::vector<double> c(dim, 0.0);
    for (int k = 0; k < dim; ++k)
      for (int q = 0; q < dim; ++q) c[q] += X[ord[k]][q] / dim;
    auto along = [&](double t) {
      std::vector<double> r(dim);
      for (int q = 0; q < dim; ++q) r[q] = c[q] + t * (X[worst][q] - c[q]);
      return r;
    };
    std::vector<double> xr = along(-1.0);
    const double fr = f(xr);
    if (fr < F[best]) {
      std::vector<double> xe = along(-2.0);
      const double fe = evals < max_evals ? f(xe) : HUGE_VAL;
      if (fe < fr) X[worst] = xe, F[worst] = fe;
      else X[worst] = xr, F[worst] = fr;
    } else if (fr < F[second]) {
      X[worst] = xr, F[worst] = fr;
    } else {
      const bool outside = fr < F[worst];
      std::vector<double> xc = along(outside ? -0.5 : 0.5);
      const double fc = evals < max_evals ? f(xc) : HUGE_VAL;
      if (fc < (outside ? fr : F[worst])) {
        X[worst] = xc, F[worst] = fc;
      } else {
        for (int k = 1; k <= dim && evals < max_evals; ++k) {
          const int i = ord[k];
          for (int q = 0; q < dim; ++q) X[i][q] = X[best][q] + 0.5 * (X[i][q] - X[best][q]);
          F[i] = f(X[i]);
        }
      }
    }
    if (last_err != GP_OK) return fail(last_err, "gp_learn: %s", gp_last_error(ctx));
  }
  int best = 0;
  for (int k = 1; k <= dim; ++k)
    if (F[k] < F[best]) best = k;
  if (!isfinite(F[best])) return fail(GP_ENOTSPD, "gp_learn: no evaluated point gave a finite log likelihood");
  double eps[GP_MAX_P], alpha[GP_MAX_P], sigma;
  unpack(X[best], eps, alpha, &sigma);
  if (eps_out) memcpy(eps_out, eps, p * sizeof(double));
  if (alpha_out) memcpy(alpha_out, alpha, p * sizeof(double));
  if (sigma_out) *sigma_out = sigma;
  if (lml_out) *lml_out = -F[best];
  if (evals_out) *evals_out = evals;
  return GP_OK;
}

}  // extern "C"
