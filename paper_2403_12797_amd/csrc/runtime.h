// Host-side runtime objects of libmercergp: context, model, served-request
// scheduler.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "kernels.h"

// Both mixed modes share everything but the Gram scheme.
inline bool prec_mixed(int precision) { return precision == GP_PREC_MIXED || precision == GP_PREC_MIXED_F16; }

struct gp_model {
  gp_ctx* ctx = nullptr;
  int p = 0, n = 0;
  int64_t M = 0;
  int precision = 0;
  int kernel = 0;   // gp_kernel
  double sigma = 0.0;
  double eps[GP_MAX_P] = {};
  double alpha[GP_MAX_P] = {};
  void* base = nullptr;  // one device allocation holding every array below
  size_t bytes = 0;
  double *tab = nullptr, *lam = nullptr, *reg = nullptr, *A = nullptr, *L = nullptr, *Linv = nullptr,
         *Dinv = nullptr, *w = nullptr, *b = nullptr;
  int* flags = nullptr;  // [0] Cholesky info, [1] non-finite input
  uint16_t* midx = nullptr;  // [M][8] multi-index table (1-D table rows per column)
  uint32_t* pdesc = nullptr; // [ceil16(M)] prediction column descriptors
  double* stats = nullptr;   // [8] fit statistics and log marginal likelihood (launch_fit_stats)
  __bf16* linv_pieces = nullptr;
  bool lean = false;     // keeps only what prediction needs (served models)
  bool charged = false;  // bytes counted in ctx->resident_bytes until freed
};

namespace mgp {

// Transient device memory of a fit: one block carved into these arrays
// (byte offsets).  all_splits keeps every Gram partial (no passes).
struct FitLayout {
  GramPlan g;
  size_t gpart, tab32, hbuf, vpart, resid, z, r, ltpart, trws, lmlpart, total;
  bool lean;
  size_t A, Dinv, Linv;  // lean models only: A (factored in place), Dinv, L^-1 (mixed)
};

// One served request (see gp_submit).
struct Request {
  int64_t id = 0;
  gp_request desc{};
  double eps[GP_MAX_P] = {}, alpha[GP_MAX_P] = {};
  size_t footprint = 0;   // device bytes held while in flight (workspace + model)
  size_t ws_bytes = 0;
  size_t fit_ws_bytes = 0;  // fit part of ws (the predict workspace follows it)
  size_t model_bytes = 0;   // lean model of a FIT kind (part of footprint)
  FitLayout layout{};       // fixed at submit: the Gram chunk is not looked up again
  int bypassed = 0;         // times a later request was admitted ahead of this one
  gp_status status = GP_PENDING;
  gp_model* model = nullptr;  // fitted model (FIT kinds)
  void* ws = nullptr;
  int slot = -1;
  bool inject_chol = false;
  double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int* flags_host = nullptr;   // pinned copy of the model flags
  Request* req = nullptr;
};

}  // namespace mgp

namespace mgp {
// Per-phase HIP-event timing (see gp_profile_enable).
struct Prof {
  std::mutex mu;
  bool on = false;
  hipEvent_t open[GP_PH_COUNT] = {};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[GP_PH_COUNT];
  double ms[GP_PH_COUNT] = {};
  int64_t count[GP_PH_COUNT] = {};
};
}  // namespace mgp

struct gp_ctx {
  int device = 0;
  size_t budget = 0;
  mgp::Prof prof;
  // served path
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler wake-up
  std::condition_variable cv_done;   // poll wake-up
  std::deque<mgp::Request*> queue;
  std::map<int64_t, mgp::Request*> requests;
  std::vector<mgp::Slot> slots;
  size_t in_flight_bytes = 0;
  // bytes of served models handed to the caller and not yet freed; they
  // count against the budget (atomic: model frees take no ctx lock)
  std::atomic<size_t> resident_bytes{0};
  int64_t next_id = 1;
  bool stop = false;
  std::thread thread;
  // fault injection: names of failures to report for the next request(s)
  std::string faults;
  // autotuned Gram chunk lengths: key (p, n, floor(log2 N)) -> chunk
  std::mutex tune_mu;
  std::map<int64_t, int> tune;
  std::string tune_path;
};

namespace mgp {
gp_status fail(gp_status st, const char* fmt, ...);
FitLayout fit_layout(int64_t N, int p, int n, int64_t M, int precision, int chunk, bool all_splits, bool lean);
void enqueue_fit_head(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                      hipStream_t s);
void enqueue_fit_tail(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                      hipStream_t s);
void tune_load(gp_ctx* ctx);
gp_status validate_params(const gp_params* prm, int64_t* M_out);
size_t model_bytes(int64_t M, int precision, bool lean);
size_t fit_workspace_bytes(gp_ctx* ctx, int64_t N, int p, int n, int64_t M, int precision);
// Gram chunk length chosen by the autotuner for (p, n, N) on this context,
// 0 if none (the planner's default applies).
int tuned_chunk(gp_ctx* ctx, int p, int n, int64_t N);
size_t predict_workspace_bytes(int64_t Ns, int64_t M, int precision);
gp_status model_alloc(gp_ctx* ctx, const gp_params* prm, int64_t M, bool lean, hipStream_t s, gp_model** out);
// Free a model's device memory stream-ordered on s (after a device-wide sync
// if sync_device) and delete it.
void model_release(gp_model* m, hipStream_t s, bool sync_device);
void enqueue_fit(gp_model* m, const double* x, const double* y, int64_t N, const FitLayout& L, void* ws,
                 hipStream_t s);
// (profile = false: no phase events, as for the no-allocation entry point)
void enqueue_predict(const gp_model* m, const double* xs, int64_t Ns, double* mean, double* var, void* ws,
                     hipStream_t s, bool profile = true);
gp_status scheduler_start(gp_ctx* ctx);
void scheduler_stop(gp_ctx* ctx);
// Consume one pending injected fault of this name (from MGP_FAULT or
// gp_ctx_inject_fault); returns true if one was pending.
bool fault_take(gp_ctx* ctx, const char* name);
}  // namespace mgp
