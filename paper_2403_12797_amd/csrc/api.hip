// C ABI of libmercergp: validation, model lifetime, fit / predict drivers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>

#include "kernels.h"
#include "runtime.h"

namespace mgp {

thread_local std::string g_last_error;

gp_status fail(gp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(_e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(_e), __FILE__, __LINE__);                   \
  } while (0)

gp_status validate_params(const gp_params* prm, int64_t* M_out) {
  if (!prm) return fail(GP_EINVAL, "params is NULL");
  if (prm->p < 1 || prm->p > GP_MAX_P) return fail(GP_EINVAL, "p=%d outside 1..%d", prm->p, GP_MAX_P);
  if (prm->n < 1 || prm->n > GP_MAX_N) return fail(GP_EINVAL, "n=%d outside 1..%d", prm->n, GP_MAX_N);
  int64_t M = 1;
  for (int j = 0; j < prm->p; ++j) {
    M *= prm->n;
    if (M > GP_MAX_M) return fail(GP_EINVAL, "M=n^p exceeds %d (n=%d, p=%d)", GP_MAX_M, prm->n, prm->p);
  }
  if (!(prm->sigma > 0.0) || !isfinite(prm->sigma)) return fail(GP_EINVAL, "sigma must be finite and > 0");
  if (!prm->eps || !prm->alpha) return fail(GP_EINVAL, "eps/alpha must be host arrays of length p");
  for (int j = 0; j < prm->p; ++j) {
    if (!(prm->eps[j] > 0.0) || !isfinite(prm->eps[j])) return fail(GP_EINVAL, "eps[%d] must be finite and > 0", j);
    if (!(prm->alpha[j] > 0.0) || !isfinite(prm->alpha[j]))
      return fail(GP_EINVAL, "alpha[%d] must be finite and > 0", j);
  }
  if (prm->precision != GP_PREC_FP64 && !prec_mixed(prm->precision))
    return fail(GP_EINVAL, "unknown precision %d", prm->precision);
  if (prm->kernel != GP_KERNEL_SE && prm->kernel != GP_KERNEL_PERIODIC)
    return fail(GP_EINVAL, "unknown kernel %d", prm->kernel);
  if (prm->kernel == GP_KERNEL_PERIODIC)
    for (int j = 0; j < prm->p; ++j)
      if (prm->eps[j] > GP_MAX_PERIODIC_EPS)
        return fail(GP_EINVAL, "periodic kernel: eps[%d]=%g above %g", j, prm->eps[j], GP_MAX_PERIODIC_EPS);
  *M_out = M;
  return GP_OK;
}

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Sizes of a model's device regions, in the order model_alloc lays them out.
// A lean model (the served path) keeps only what prediction needs: the
// factor regions A, L, Dinv and (mixed precision) the FP64 L^-1 are sized
// zero here and live in the fit workspace instead (FitLayout).
static constexpr int kModelRegions = 14;
static void model_sizes(int64_t M, int precision, bool lean, size_t* sz) {
  const size_t MM = (size_t)M * M;
  const bool mixed = prec_mixed(precision);
  const size_t v[kModelRegions] = {kTabSize * 8, (size_t)M * 8, (size_t)M * 8, lean ? 0 : MM * 8, lean ? 0 : MM * 8,
                                   (lean && mixed) ? 0 : MM * 8,
                                   lean ? 0 : (size_t)ceil_div(M, kCholNb) * kCholNb * kCholNb * 8, (size_t)M * 8,
                                   (size_t)M * 8, 64,
                                   mixed ? 2 * (size_t)linv_rows((int)M) * linv_pitch((int)M) * 2 : 0,
                                   (size_t)M * 16, (size_t)pdesc_elems((int)M) * 4, 8 * sizeof(double)};
  for (int r = 0; r < kModelRegions; ++r) sz[r] = v[r];
}

// Device bytes a fitted model holds (used by admission control too).
size_t model_bytes(int64_t M, int precision, bool lean) {
  size_t sz[kModelRegions], b = 0;
  model_sizes(M, precision, lean, sz);
  for (size_t v : sz) b += v ? align_up(v) : 0;
  return b;
}

FitLayout fit_layout(int64_t N, int p, int n, int64_t M, int precision, int chunk, bool all_splits, bool lean) {
  FitLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align_up(bytes);
    return r;
  };
  L.lean = lean;
  if (prec_mixed(precision)) {
    L.g = gram_mixed_plan(N, p, n, (int)M, precision == GP_PREC_MIXED_F16, chunk);
    if (all_splits) L.g.splits_per_pass = L.g.splits_total, L.g.passes = 1;
    L.gpart = take((size_t)gram_mixed_part_elems(L.g) * 4);
    L.tab32 = take((size_t)gram_mixed_table_elems(N, p, n) * 4);
    L.hbuf = take((size_t)gram_mixed_hbuf_elems(L.g) * 8);
  } else {
    L.gpart = take((size_t)gram_f64_part_elems(N, (int)M, nullptr) * 8);
    L.tab32 = take(0);
    L.hbuf = take(0);
  }
  L.vpart = take((size_t)phiT_part_elems(N, (int)M) * 8);
  L.resid = take((size_t)N * 8);
  L.z = take((size_t)M * 8);
  L.r = take((size_t)M * 8);
  L.ltpart = take((size_t)ceil_div(M, 256) * M * 8);
  L.trws = take(trtri_workspace_elems((int)M) * 8);
  L.lmlpart = take(kLmlParts * 8);
  if (lean) {
    // A is factored in place (L = A); L^-1 here only for mixed precision
    L.A = take((size_t)M * M * 8);
    L.Dinv = take((size_t)ceil_div(M, kCholNb) * kCholNb * kCholNb * 8);
    L.Linv = prec_mixed(precision) ? take((size_t)M * M * 8) : 0;
  }
  L.total = o + 256;
  return L;
}

size_t fit_workspace_bytes(gp_ctx* ctx, int64_t N, int p, int n, int64_t M, int precision) {
  return fit_layout(N, p, n, M, precision, tuned_chunk(ctx, p, n, N), false, false).total;
}

size_t predict_workspace_bytes(int64_t Ns, int64_t M, int precision) {
  if (Ns <= 0) return 0;
  return (prec_mixed(precision) ? (size_t)predict_mixed_part_elems(Ns, (int)M, nullptr)
                                     : (size_t)predict_part_elems(Ns, (int)M, nullptr)) *
             8 +
         256;
}

void prof_mark(Prof* p, int phase, bool begin, hipStream_t s) {
  if (!p || !p->on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  hipEventRecord(e, s);
  std::lock_guard<std::mutex> lk(p->mu);
  if (begin) {
    if (p->open[phase]) hipEventDestroy(p->open[phase]);
    p->open[phase] = e;
  } else if (p->open[phase]) {
    p->pending[phase].emplace_back(p->open[phase], e);
    p->open[phase] = nullptr;
  } else {
    hipEventDestroy(e);
  }
}

void model_release(gp_model* m, hipStream_t s, bool sync_device) {
  if (!m) return;
  if (m->charged) {
    // a served model held by the caller: its bytes leave the admission budget
    m->ctx->resident_bytes.fetch_sub(m->bytes);
    m->charged = false;
    m->ctx->cv_work.notify_all();
  }
  if (m->base) {
    hipSetDevice(m->ctx->device);
    if (sync_device) hipDeviceSynchronize();
    hipFreeAsync(m->base, s);
    if (sync_device) hipStreamSynchronize(s);
  }
  delete m;
}

gp_status model_alloc(gp_ctx* ctx, const gp_params* prm, int64_t M, bool lean, hipStream_t s, gp_model** out) {
  gp_model* m = new gp_model();
  m->lean = lean;
  m->ctx = ctx;
  m->p = prm->p;
  m->n = prm->n;
  m->M = M;
  m->precision = prm->precision;
  m->kernel = prm->kernel;
  m->sigma = prm->sigma;
  for (int j = 0; j < prm->p; ++j) {
    m->eps[j] = prm->eps[j];
    m->alpha[j] = prm->alpha[j];
  }
  size_t sizes[kModelRegions];
  model_sizes(M, prm->precision, lean, sizes);
  size_t total = 0;
  for (size_t s : sizes) total += s ? align_up(s) : 0;
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = hipMallocAsync(&m->base, total, s);
  if (e != hipSuccess) {
    delete m;
    return fail(e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EDEVICE, "model allocation of %zu bytes: %s", total,
                hipGetErrorString(e));
  }
  m->bytes = total;
  char* b = (char*)m->base;
  size_t o = 0;
  auto take = [&](size_t s) -> void* {
    if (!s) return nullptr;
    void* r = b + o;
    o += align_up(s);
    return r;
  };
  m->tab = (double*)take(sizes[0]);
  m->lam = (double*)take(sizes[1]);
  m->reg = (double*)take(sizes[2]);
  m->A = (double*)take(sizes[3]);
  m->L = (double*)take(sizes[4]);
  m->Linv = (double*)take(sizes[5]);
  m->Dinv = (double*)take(sizes[6]);
  m->w = (double*)take(sizes[7]);
  m->b = (double*)take(sizes[8]);
  m->flags = (int*)take(sizes[9]);
  m->linv_pieces = prec_mixed(prm->precision) ? (__bf16*)take(sizes[10]) : nullptr;
  m->midx = (uint16_t*)take(sizes[11]);
  m->pdesc = (uint32_t*)take(sizes[12]);
  m->stats = (double*)take(sizes[13]);
  *out = m;
  return GP_OK;
}

// The fit in three parts so that many problems can share the Gram launch.
// head: flags, input checks, eigen tables (and the FP32 1-D tables, mixed).
void enqueue_fit_head(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                      hipStream_t s) {
  const int p = m->p, n = m->n, M = (int)m->M;
  EigArgs a;
  memset(&a, 0, sizeof(a));
  a.p = p;
  a.n = n;
  a.kind = m->kernel;
  a.sigma = m->sigma;
  for (int j = 0; j < p; ++j) {
    a.eps[j] = m->eps[j];
    a.alpha[j] = m->alpha[j];
  }
  char* wb = (char*)ws;
  launch_fill_zero_int(m->flags, 16, s);
  launch_check_finite(x, N * p, y, N, m->flags + 1, s);
  launch_eig_tables(a, m->tab, m->lam, m->reg, M, s);
  launch_midx(p, n, M, m->midx, s);
  if (prec_mixed(m->precision)) launch_pdesc(p, n, M, m->pdesc, s);
  if (prec_mixed(m->precision)) launch_gram_mixed_table(x, N, p, n, m->tab, (float*)(wb + L.tab32), s);
}

// tail: b = Phi^T y, Cholesky, L^-1, w with one FP64 refinement step, BF16 split.
void enqueue_fit_tail(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                      hipStream_t s) {
  const int p = m->p, n = m->n, M = (int)m->M;
  char* wb = (char*)ws;
  double* vpart = (double*)(wb + L.vpart);
  double* resid = (double*)(wb + L.resid);
  double* z = (double*)(wb + L.z);
  double* r = (double*)(wb + L.r);
  double* ltpart = (double*)(wb + L.ltpart);
  double* trws = (double*)(wb + L.trws);
  Prof* pr = &m->ctx->prof;
  prof_mark(pr, GP_PH_PHIT, true, s);
  launch_phiT_vec(x, y, N, p, n, M, m->tab, vpart, nullptr, nullptr, m->b, s);
  prof_mark(pr, GP_PH_PHIT, false, s);
  prof_mark(pr, GP_PH_CHOL, true, s);
  if (m->L != m->A) hipMemcpyAsync(m->L, m->A, (size_t)M * M * 8, hipMemcpyDeviceToDevice, s);
  launch_cholesky(m->L, M, m->Dinv, m->flags, s);
  prof_mark(pr, GP_PH_CHOL, false, s);
  prof_mark(pr, GP_PH_TRTRI, true, s);
  launch_trtri(m->L, m->Dinv, m->Linv, trws, M, m->flags, s);
  prof_mark(pr, GP_PH_TRTRI, false, s);
  prof_mark(pr, GP_PH_SOLVE, true, s);
  launch_lower_matvec(m->Linv, m->b, z, M, s);
  launch_lower_t_matvec(m->Linv, z, m->w, ltpart, M, s);
  launch_phi_matvec(x, N, p, n, M, m->tab, m->midx, m->w, y, resid, s);                 // y - Phi w
  launch_phiT_vec(x, resid, N, p, n, M, m->tab, vpart, m->reg, m->w, r, s);    // Phi^T(y - Phi w) - reg*w
  launch_lower_matvec(m->Linv, r, z, M, s);
  launch_lower_t_matvec(m->Linv, z, m->w, ltpart, M, s, m->w);   // w += L^-T z
  // y^T y, log det L, sum log Lambda, b^T w and the log marginal likelihood
  launch_fit_stats(y, N, m->b, m->w, m->L, m->lam, M, m->sigma, (double*)(wb + L.lmlpart), m->stats, s);
  prof_mark(pr, GP_PH_SOLVE, false, s);
  if (prec_mixed(m->precision)) {
    prof_mark(pr, GP_PH_SPLIT, true, s);
    launch_split_linv(m->Linv, m->linv_pieces, M, s);
    prof_mark(pr, GP_PH_SPLIT, false, s);
  }
}

// Enqueue the whole fit of one problem on stream s.  ws holds L.total bytes
// of a layout made for this problem (fit_layout); for a lean model the
// factor regions live in ws and the model keeps no pointer to them after
// this call (the device work still reads them, ordered on s before ws is
// freed).
void enqueue_fit(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                 hipStream_t s) {
  const int p = m->p, n = m->n, M = (int)m->M;
  char* wb = (char*)ws;
  Prof* pr = &m->ctx->prof;
  if (m->lean) {
    m->A = m->L = (double*)(wb + L.A);
    m->Dinv = (double*)(wb + L.Dinv);
    if (prec_mixed(m->precision)) m->Linv = (double*)(wb + L.Linv);
  }
  enqueue_fit_head(m, x, y, N, L, ws, s);
  // a3: A = Phi^T Phi + sigma^2 Lambda^-1
  if (prec_mixed(m->precision)) {
    launch_gram_mixed(x, N, p, n, M, L.g, m->precision == GP_PREC_MIXED_F16, m->tab, m->reg, (float*)(wb + L.gpart),
                      (float*)(wb + L.tab32), (double*)(wb + L.hbuf), m->A, s, pr);
  } else {
    launch_gram_f64(x, N, p, n, M, m->tab, m->reg, (double*)(wb + L.gpart), m->A, s, pr);
  }
  enqueue_fit_tail(m, x, y, N, L, ws, s);
  if (m->lean) {
    m->A = m->L = m->Dinv = nullptr;
    if (prec_mixed(m->precision)) m->Linv = nullptr;
  }
}

void enqueue_predict(const gp_model* m, const double* xs, int64_t Ns, double* mean, double* var, void* ws,
                     hipStream_t s, bool profile) {
  if (Ns <= 0) return;
  const int p = m->p, n = m->n, M = (int)m->M;
  const double s2 = m->sigma * m->sigma;
  Prof* pr = profile ? &m->ctx->prof : nullptr;
  if (prec_mixed(m->precision)) {
    launch_predict_mixed(xs, Ns, p, n, M, m->tab, m->midx, m->pdesc, m->linv_pieces, m->w, s2, (double*)ws, mean,
                         var, s, pr);
  } else {
    if (mean) {
      prof_mark(pr, GP_PH_PREDICT_MEAN, true, s);
      launch_phi_matvec(xs, Ns, p, n, M, m->tab, m->midx, m->w, nullptr, mean, s);
      prof_mark(pr, GP_PH_PREDICT_MEAN, false, s);
    }
    if (var) launch_predict_var_f64(xs, Ns, p, n, M, m->tab, m->Linv, s2, (double*)ws, var, s, pr);
  }
}

// ---------------------------------------------------------------- scratch
// Device memory of gp_predict_noalloc: the variance partial sums (the only
// workspace a prediction uses) live in this file-scope array, which every
// GPU the library runs on holds until the process ends.  In host code the
// name `scratch` is a host-side stand-in, not a device address: the device
// address is looked up once per device (scratch_init, from gp_ctx_create with
// that device current) and only that address is passed to kernels.
static __device__ __align__(256) unsigned char scratch[GP_NOALLOC_SCRATCH_BYTES];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices] = {};

static gp_status scratch_init(int device) {
  if (device < 0 || device >= kScratchDevices) return fail(GP_EDEVICE, "device %d has no scratch slot", device);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return GP_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    return fail(GP_EDEVICE, "device address of the scratch array: %s", hipGetErrorString(e));
  g_scratch_ptr[device] = ptr;
  return GP_OK;
}

}  // namespace mgp

using namespace mgp;

extern "C" {

const char* gp_last_error(const gp_ctx* ctx) {
  (void)ctx;  // messages are kept per calling thread
  return g_last_error.c_str();
}

gp_status gp_ctx_create(int device, size_t hbm_budget_bytes, gp_ctx** out) {
  if (!out) return fail(GP_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) return fail(GP_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (device < 0 || device >= count) return fail(GP_EINVAL, "device %d not in 0..%d", device, count - 1);
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(configure_kernels());
  {
    const gp_status sst = scratch_init(device);
    if (sst != GP_OK) return sst;
  }
  size_t freeb = 0, totalb = 0;
  HIP_TRY(hipMemGetInfo(&freeb, &totalb));
  gp_ctx* c = new gp_ctx();
  c->device = device;
  c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)freeb);
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  tune_load(c);
  gp_status st = scheduler_start(c);
  if (st != GP_OK) {
    delete c;
    return st;
  }
  *out = c;
  return GP_OK;
}

gp_status gp_ctx_destroy(gp_ctx* ctx) {
  if (!ctx) return GP_OK;
  scheduler_stop(ctx);
  delete ctx;
  return GP_OK;
}

gp_status gp_fit(gp_ctx* ctx, const gp_params* params, const double* x, const double* y, int64_t N, void* stream,
                 gp_model** out_model) {
  if (!ctx || !out_model) return fail(GP_EINVAL, "ctx/out_model is NULL");
  *out_model = nullptr;
  int64_t M = 0;
  gp_status st = validate_params(params, &M);
  if (st != GP_OK) return st;
  if (N < 1) return fail(GP_EINVAL, "N=%lld must be >= 1", (long long)N);
  if (!x || !y) return fail(GP_EINVAL, "x/y is NULL");
  if (fault_take(ctx, "oom")) return fail(GP_ENOMEM, "injected allocation failure");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  gp_model* m = nullptr;
  st = model_alloc(ctx, params, M, false, s, &m);
  if (st != GP_OK) return st;
  void* ws = nullptr;
  // the layout (and the Gram chunk in it) is fixed here, once
  const FitLayout L = fit_layout(N, params->p, params->n, M, params->precision,
                                 tuned_chunk(ctx, params->p, params->n, N), false, false);
  const size_t wsb = L.total;
  hipError_t e = hipMallocAsync(&ws, wsb, s);
  if (e != hipSuccess) {
    gp_model_free(m);
    return fail(e == hipErrorOutOfMemory ? GP_ENOMEM : GP_EDEVICE, "fit workspace of %zu bytes: %s", wsb,
                hipGetErrorString(e));
  }
  enqueue_fit(m, x, y, N, L, ws, s);
  hipFreeAsync(ws, s);
  int flags[2] = {0, 0};
  e = hipMemcpyAsync(flags, m->flags, sizeof(flags), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    gp_model_free(m);
    return fail(GP_EDEVICE, "fit: %s", hipGetErrorString(e));
  }
  if (flags[1]) {
    gp_model_free(m);
    return fail(GP_EINVAL, "x or y holds a non-finite value");
  }
  if (fault_take(ctx, "chol")) flags[0] = 1;
  if (flags[0]) {
    gp_model_free(m);
    return fail(GP_ENOTSPD, "Cholesky: non-positive pivot at column %d", flags[0] - 1);
  }
  *out_model = m;
  return GP_OK;
}

gp_status gp_predict(gp_ctx* ctx, const gp_model* model, const double* xs, int64_t Ns, double* mean, double* var,
                     void* stream) {
  if (!ctx || !model) return fail(GP_EINVAL, "ctx/model is NULL");
  if (Ns < 0) return fail(GP_EINVAL, "Ns=%lld must be >= 0", (long long)Ns);
  if (Ns == 0 || (!mean && !var)) return GP_OK;
  if (!xs) return fail(GP_EINVAL, "xs is NULL");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  const size_t wsb = predict_workspace_bytes(Ns, model->M, model->precision);
  HIP_TRY(hipMallocAsync(&ws, wsb, s));
  enqueue_predict(model, xs, Ns, mean, var, ws, s);
  HIP_TRY(hipFreeAsync(ws, s));
  HIP_TRY(hipGetLastError());
  return GP_OK;
}

gp_status gp_predict_noalloc(gp_ctx* ctx, const gp_model* model, const double* xs, int64_t Ns, double* mean,
                             double* var, void* stream) {
  if (!ctx || !model) return fail(GP_EINVAL, "ctx/model is NULL");
  if (Ns < 0) return fail(GP_EINVAL, "Ns=%lld must be >= 0", (long long)Ns);
  if (Ns == 0 || (!mean && !var)) return GP_OK;
  if (!xs) return fail(GP_EINVAL, "xs is NULL");
  const size_t wsb = predict_workspace_bytes(Ns, model->M, model->precision);
  if (wsb > (size_t)GP_NOALLOC_SCRATCH_BYTES)
    return fail(GP_EINVAL, "Ns=%lld at M=%lld needs %zu bytes of scratch; gp_predict_noalloc holds %zu",
                (long long)Ns, (long long)model->M, wsb, (size_t)GP_NOALLOC_SCRATCH_BYTES);
  void* ws = (ctx->device >= 0 && ctx->device < kScratchDevices) ? g_scratch_ptr[ctx->device] : nullptr;
  if (!ws) return fail(GP_EDEVICE, "no scratch address for device %d", ctx->device);
  HIP_TRY(hipSetDevice(ctx->device));
  enqueue_predict(model, xs, Ns, mean, var, ws, (hipStream_t)stream, false);
  HIP_TRY(hipGetLastError());
  return GP_OK;
}

gp_status gp_profile_enable(gp_ctx* ctx, int32_t on) {
  if (!ctx) return fail(GP_EINVAL, "ctx is NULL");
  Prof& p = ctx->prof;
  std::lock_guard<std::mutex> lk(p.mu);
  for (int k = 0; k < GP_PH_COUNT; ++k) {
    for (auto& pr : p.pending[k]) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    p.pending[k].clear();
    if (p.open[k]) hipEventDestroy(p.open[k]);
    p.open[k] = nullptr;
    p.ms[k] = 0.0;
    p.count[k] = 0;
  }
  p.on = on != 0;
  return GP_OK;
}

gp_status gp_profile_read(gp_ctx* ctx, int32_t phase, double* total_ms, int64_t* count) {
  if (!ctx) return fail(GP_EINVAL, "ctx is NULL");
  if (phase < 0 || phase >= GP_PH_COUNT) return fail(GP_EINVAL, "unknown phase %d", phase);
  Prof& p = ctx->prof;
  std::lock_guard<std::mutex> lk(p.mu);
  for (auto& pr : p.pending[phase]) {
    float ms = 0.0f;
    HIP_TRY(hipEventSynchronize(pr.second));
    HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
    p.ms[phase] += ms;
    p.count[phase] += 1;
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  p.pending[phase].clear();
  if (total_ms) *total_ms = p.ms[phase];
  if (count) *count = p.count[phase];
  return GP_OK;
}

gp_status gp_model_free(gp_model* model) {
  if (!model) return GP_OK;
  model_release(model, nullptr, true);
  return GP_OK;
}

gp_status gp_model_info(const gp_model* model, int32_t* p, int32_t* n, int64_t* M, int32_t* precision,
                        double* sigma) {
  if (!model) return fail(GP_EINVAL, "model is NULL");
  if (p) *p = model->p;
  if (n) *n = model->n;
  if (M) *M = model->M;
  if (precision) *precision = model->precision;
  if (sigma) *sigma = model->sigma;
  return GP_OK;
}

gp_status gp_model_weights(const gp_model* model, double* w_host) {
  if (!model || !w_host) return fail(GP_EINVAL, "model/w_host is NULL");
  return gp_model_get(model, GP_MODEL_W, w_host, model->M);
}

gp_status gp_model_get(const gp_model* model, int32_t what, double* host_out, int64_t count) {
  if (!model || !host_out) return fail(GP_EINVAL, "model/host_out is NULL");
  const int64_t M = model->M;
  const double* src = nullptr;
  int64_t len = 0;
  bool lower = false;
  switch (what) {
    case GP_MODEL_W: src = model->w; len = M; break;
    case GP_MODEL_LAMBDA: src = model->lam; len = M; break;
    case GP_MODEL_A: src = model->A; len = M * M; break;
    case GP_MODEL_B: src = model->b; len = M; break;
    case GP_MODEL_L: src = model->L; len = M * M; lower = true; break;
    case GP_MODEL_LINV: src = model->Linv; len = M * M; lower = true; break;
    default: return fail(GP_EINVAL, "unknown model array %d", what);
  }
  if (!src)
    return fail(GP_EINVAL, "array %d is not kept by this model (served models keep only what prediction needs)",
                what);
  if (count < len) return fail(GP_EINVAL, "count %lld < %lld", (long long)count, (long long)len);
  HIP_TRY(hipSetDevice(model->ctx->device));
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(host_out, src, (size_t)len * 8, hipMemcpyDeviceToHost));
  if (lower)
    for (int64_t r = 0; r < M; ++r)
      for (int64_t c = r + 1; c < M; ++c) host_out[r * M + c] = 0.0;
  return GP_OK;
}

}  // extern "C"
