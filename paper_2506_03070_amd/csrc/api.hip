// C ABI entry points (declared in include/sap.h): argument validation,
// workspace management and the orchestration of Alg. 1 on one stream.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "common.h"

namespace sap {

// The last error message is kept per calling thread (errno-like), so
// concurrent sap_submit / sap_poll callers cannot race on it.
namespace {
thread_local std::string tl_err;
thread_local const sap_ctx *tl_err_ctx = nullptr;
}  // namespace

sap_status fail(sap_ctx *ctx, sap_status s, const std::string &msg) {
  if (ctx) {
    tl_err = msg;
    tl_err_ctx = ctx;
  }
  return s;
}

sap_status hip_fail(sap_ctx *ctx, hipError_t e, const char *what) {
  std::string msg = std::string("HIP error ") + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ") in " + what;
  return fail(ctx, SAP_EDEVICE, msg);
}

sap_status ensure_workspace(sap_ctx *ctx, size_t bytes, hipStream_t stream) {
  bytes = (bytes + 4095) & ~size_t(4095);
  if (bytes <= ctx->ws_size) return SAP_OK;
  if (bytes > ctx->budget)
    return fail(ctx, SAP_ENOMEM, "workspace of " + std::to_string(bytes) + " bytes exceeds the HBM budget of " +
                                     std::to_string(ctx->budget) + " bytes");
  if (ctx->ws) {
    SAP_HIP_TRY(hipStreamSynchronize(stream));
    SAP_HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_size = 0;
  }
  if (hipMalloc(&ctx->ws, bytes) != hipSuccess) {
    (void)hipGetLastError();
    ctx->ws = nullptr;
    return fail(ctx, SAP_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  ctx->ws_size = bytes;
  return SAP_OK;
}

static hipEvent_t take_event(sap_ctx *ctx) {
  if (!ctx->free_events.empty()) {
    hipEvent_t e = ctx->free_events.back();
    ctx->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

hipEvent_t prof_begin(sap_ctx *ctx, hipStream_t st) {
  if (!ctx->profiling) return nullptr;
  hipEvent_t e = take_event(ctx);
  if (e) (void)hipEventRecord(e, st);
  return e;
}

void prof_end(sap_ctx *ctx, int kernel, hipEvent_t begin, hipStream_t st) {
  if (!ctx->profiling || !begin) return;
  hipEvent_t e = take_event(ctx);
  if (!e) return;
  (void)hipEventRecord(e, st);
  ctx->pending[kernel].emplace_back(begin, e);
}

void prof_resolve(sap_ctx *ctx) {
  for (int k = 0; k < 2; ++k) {
    for (auto &pr : ctx->pending[k]) {
      float ms = 0.f;
      if (hipEventSynchronize(pr.second) == hipSuccess && hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
        ctx->prof_launches[k] += 1;
        ctx->prof_ms[k] += ms;
      }
      ctx->free_events.push_back(pr.first);
      ctx->free_events.push_back(pr.second);
    }
    ctx->pending[k].clear();
  }
}

namespace {

// Flags written by device checks and read back once per solve.
struct SolveFlags {
  int gen_error;
  int rank_deficient;
  int nonfinite_b;
  int bad_csr;
};

__global__ void zero_flags_kernel(SolveFlags *f) {
  if (threadIdx.x == 0) {
    f->gen_error = 0;
    f->rank_deficient = 0;
    f->nonfinite_b = 0;
    f->bad_csr = 0;
  }
}

__global__ __launch_bounds__(256) void finite_check_kernel(const double *__restrict__ b, int64_t m,
                                                           int *__restrict__ flag) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  int bad = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < m; i += stride)
    bad |= !isfinite(b[i]);
  if (bad) atomicOr(flag, 1);
}

// BF16 copy of an FP32 row-major matrix (round to nearest even), rows of
// ldo elements (ldo a multiple of 8: 16-byte rows).  The BF16-input sketch
// mode applies S to this copy.
__global__ __launch_bounds__(256) void to_bf16_kernel(const float *__restrict__ A, int64_t lda, int64_t m, int n,
                                                      __hip_bfloat16 *__restrict__ out, int64_t ldo) {
  const int64_t total = m * ldo;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / ldo;
    const int j = static_cast<int>(e - i * ldo);
    out[e] = __float2bfloat16(j < n ? A[i * lda + j] : 0.0f);
  }
}

sap_status check_sketch(sap_ctx *ctx, const sps_sketch *S) {
  if (!S) return fail(ctx, SAP_EINVAL, "sketch descriptor is NULL");
  if (S->m < 1) return fail(ctx, SAP_EINVAL, "sketch: m must be >= 1");
  if (S->d < 1) return fail(ctx, SAP_EINVAL, "sketch: d must be >= 1");
  if (S->zeta < 1 || S->zeta > 64) return fail(ctx, SAP_EINVAL, "sketch: zeta must be in [1, 64]");
  if (S->zeta > S->d) return fail(ctx, SAP_EINVAL, "sketch: zeta must not exceed d");
  if (!S->idx || !S->sign) return fail(ctx, SAP_EINVAL, "sketch: idx/sign must be device pointers");
  return SAP_OK;
}

}  // namespace
}  // namespace sap

using namespace sap;

extern "C" {

const char *sap_status_string(sap_status s) {
  switch (s) {
    case SAP_OK: return "SAP_OK";
    case SAP_EINVAL: return "SAP_EINVAL";
    case SAP_ENOMEM: return "SAP_ENOMEM";
    case SAP_RANK_DEFICIENT: return "SAP_RANK_DEFICIENT";
    case SAP_NOT_CONVERGED: return "SAP_NOT_CONVERGED";
    case SAP_PENDING: return "SAP_PENDING";
    case SAP_EDEVICE: return "SAP_EDEVICE";
    case SAP_ECANCELED: return "SAP_ECANCELED";
  }
  return "SAP_UNKNOWN";
}

sap_status sap_create(sap_ctx **out, int device, size_t hbm_budget) {
  if (!out) return SAP_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SAP_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return SAP_EDEVICE;
  sap_ctx *ctx = new sap_ctx();
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete ctx;
    return SAP_EDEVICE;
  }
  ctx->num_cus = prop.multiProcessorCount;
  size_t free_b = 0, total_b = 0;
  if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    delete ctx;
    return SAP_EDEVICE;
  }
  ctx->budget = hbm_budget ? hbm_budget : static_cast<size_t>(0.9 * static_cast<double>(free_b));
  if (apply_scratch_init(ctx) != SAP_OK) {
    delete ctx;
    return SAP_EDEVICE;
  }
  if (hipHostMalloc(&ctx->pinned, kPinnedBytes, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->batch_ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->batch_ev[1], hipEventDisableTiming) != hipSuccess) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (hipEvent_t e : ctx->batch_ev)
      if (e) (void)hipEventDestroy(e);
    delete ctx;
    return SAP_EDEVICE;
  }
  *out = ctx;
  return SAP_OK;
}

void sap_destroy(sap_ctx *ctx) {
  if (!ctx) return;
  serve_destroy(ctx);
  select_cache_free(ctx);
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  prof_resolve(ctx);
  for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
  batch_graphs_free(ctx);
  for (hipEvent_t e : ctx->batch_ev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ws) (void)hipFree(ctx->ws);
  delete ctx;
}

sap_status sap_profile_enable(sap_ctx *ctx, int enable) {
  if (!ctx) return SAP_EINVAL;
  ctx->profiling = enable != 0;
  return SAP_OK;
}

sap_status sap_profile_read(sap_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms, int reset) {
  if (!ctx || kernel < 0 || kernel > 1) return SAP_EINVAL;
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  prof_resolve(ctx);
  if (launches) *launches = ctx->prof_launches[kernel];
  if (total_ms) *total_ms = ctx->prof_ms[kernel];
  if (reset) {
    ctx->prof_launches[kernel] = 0;
    ctx->prof_ms[kernel] = 0.0;
  }
  return SAP_OK;
}

const char *sap_last_error(const sap_ctx *ctx) {
  if (!ctx) return "NULL context";
  return tl_err_ctx == ctx ? tl_err.c_str() : "";
}

sap_status sps_generate(sap_ctx *ctx, const sps_sketch *S, void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_sketch(ctx, S);
  if (s != SAP_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  s = ensure_workspace(ctx, 256, st);
  if (s != SAP_OK) return s;
  return launch_generate(ctx, S, static_cast<int *>(ctx->ws), st);
}

sap_status sps_apply(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda, sap_dtype a_type,
                     const double *b, int32_t n, void *Y, int64_t ldy, sap_dtype y_type, void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_sketch(ctx, S);
  if (s != SAP_OK) return s;
  if (!A || !Y) return fail(ctx, SAP_EINVAL, "sps_apply: A and Y must be device pointers");
  if (n < 1) return fail(ctx, SAP_EINVAL, "sps_apply: n must be >= 1");
  if (lda < n) return fail(ctx, SAP_EINVAL, "sps_apply: lda must be >= n");
  if (ldy < S->d) return fail(ctx, SAP_EINVAL, "sps_apply: ldy must be >= d");
  if (a_type != SAP_F64 && a_type != SAP_F32 && a_type != SAP_BF16)
    return fail(ctx, SAP_EINVAL, "sps_apply: a_type must be F64, F32 or BF16");
  if (y_type != SAP_F64 && y_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sps_apply: y_type must be F64 or F32");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  const int ncols = n + (b ? 1 : 0);
  s = ensure_workspace(ctx, apply_workspace_bytes(ctx, S->m, S->zeta, S->d, ncols, y_type) + 256, st);
  if (s != SAP_OK) return s;
  hipEvent_t pb = prof_begin(ctx, st);
  s = launch_apply(ctx, S, A, lda, a_type, b, n, Y, ldy, y_type, ctx->ws, st);
  prof_end(ctx, kProfApply, pb, st);
  return s;
}

sap_status sps_apply_noalloc(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda, sap_dtype a_type,
                             const double *b, int32_t n, void *Y, int64_t ldy, sap_dtype y_type, void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_sketch(ctx, S);
  if (s != SAP_OK) return s;
  if (!A || !Y) return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: A and Y must be device pointers");
  if (n < 1) return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: n must be >= 1");
  if (lda < n) return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: lda must be >= n");
  if (ldy < S->d) return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: ldy must be >= d");
  if (a_type != SAP_F64 && a_type != SAP_F32 && a_type != SAP_BF16)
    return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: a_type must be F64, F32 or BF16");
  if (y_type != SAP_F64 && y_type != SAP_F32)
    return fail(ctx, SAP_EINVAL, "sps_apply_noalloc: y_type must be F64 or F32");
  const int ncols = n + (b ? 1 : 0);
  const size_t need = apply_workspace_bytes(ctx, S->m, S->zeta, S->d, ncols, y_type);
  if (ctx->apply_scratch == nullptr || need > ctx->apply_scratch_bytes)
    return fail(ctx, SAP_ENOMEM, "sps_apply_noalloc: this apply needs " + std::to_string(need) +
                                     " bytes of scratch, more than the static buffer's " +
                                     std::to_string(ctx->apply_scratch_bytes));
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  return launch_apply(ctx, S, A, lda, a_type, b, n, Y, ldy, y_type, ctx->apply_scratch,
                      static_cast<hipStream_t>(stream));
}

sap_status sap_qr(sap_ctx *ctx, double *Y, int64_t ldy, int32_t rows, int32_t cols, double *tau, void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (!Y || !tau) return fail(ctx, SAP_EINVAL, "sap_qr: Y and tau must be device pointers");
  if (rows < 1 || cols < 1 || rows < cols) return fail(ctx, SAP_EINVAL, "sap_qr: need rows >= cols >= 1");
  if (ldy < rows) return fail(ctx, SAP_EINVAL, "sap_qr: ldy must be >= rows");
  if (rows > 16384) return fail(ctx, SAP_EINVAL, "sap_qr: more than 16384 rows is not supported");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  sap_status s = ensure_workspace(ctx, qr_workspace_bytes(rows, cols), st);
  if (s != SAP_OK) return s;
  return launch_qr(ctx, Y, ldy, rows, cols, tau, ctx->ws, st);
}

sap_status sap_trsv(sap_ctx *ctx, const double *R, int64_t ldr, int32_t n, int32_t trans, const double *rhs,
                    double *x, void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (!R || !rhs || !x) return fail(ctx, SAP_EINVAL, "sap_trsv: NULL pointer");
  if (n < 1 || ldr < n) return fail(ctx, SAP_EINVAL, "sap_trsv: need n >= 1 and ldr >= n");
  if (trans != 0 && trans != 1) return fail(ctx, SAP_EINVAL, "sap_trsv: trans must be 0 or 1");
  if (n > 8192) return fail(ctx, SAP_EINVAL, "sap_trsv: n > 8192 is not supported");
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t st = static_cast<hipStream_t>(stream);
  sap_status s = ensure_workspace(ctx, trsv_workspace_bytes(n), st);
  if (s != SAP_OK) return s;
  return launch_trsv(ctx, R, ldr, n, trans, rhs, x, ctx->ws, st);
}

static sap_status check_problem(sap_ctx *ctx, const sap_problem *p) {
  if (!p) return fail(ctx, SAP_EINVAL, "problem descriptor is NULL");
  if (p->n < 1) return fail(ctx, SAP_EINVAL, "problem: n must be >= 1");
  if (p->m < static_cast<int64_t>(p->n) + 1) return fail(ctx, SAP_EINVAL, "problem: need m >= n + 1");
  if (p->lda < p->n) return fail(ctx, SAP_EINVAL, "problem: lda must be >= n");
  if (!p->A || !p->b) return fail(ctx, SAP_EINVAL, "problem: A and b must be device pointers");
  if (p->n > 8192) return fail(ctx, SAP_EINVAL, "problem: n > 8192 is not supported");
  return SAP_OK;
}

sap_status sap_lsqr(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *x0,
                    double tol, int32_t maxiter, double *x, sap_info *info, void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_problem(ctx, prob);
  if (s != SAP_OK) return s;
  if (prob->a_type != SAP_F64 && prob->a_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sap_lsqr: A must be F64 or F32");
  if (!R || !x0 || !x) return fail(ctx, SAP_EINVAL, "sap_lsqr: NULL pointer");
  if (ldr < prob->n) return fail(ctx, SAP_EINVAL, "sap_lsqr: ldr must be >= n");
  if (maxiter < 0 || !(tol >= 0.0)) return fail(ctx, SAP_EINVAL, "sap_lsqr: need maxiter >= 0 and tol >= 0");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  s = ensure_workspace(ctx, lsqr_workspace_bytes(ctx, prob->m, prob->n), st);
  if (s != SAP_OK) return s;
  if (info) std::memset(info, 0, sizeof(*info));
  hipEvent_t e0, e1;
  SAP_HIP_TRY(hipEventCreate(&e0));
  SAP_HIP_TRY(hipEventCreate(&e1));
  SAP_HIP_TRY(hipEventRecord(e0, st));
  s = run_lsqr(ctx, prob, R, ldr, x0, nullptr, tol, maxiter, prob->a_type == SAP_F32 ? 1 : 0, 0, x, info, ctx->ws,
               st);
  (void)hipEventRecord(e1, st);
  (void)hipEventSynchronize(e1);
  prof_resolve(ctx);
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (info) {
    info->status = s;
    info->t_iterate_ms = ms;
  }
  return s;
}

sap_status sap_solve_batch(sap_ctx *ctx, int32_t count, const sap_problem *probs, const sap_params *params,
                           double *const *x, sap_info *info, void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (count < 1 || !probs || !params || !x) return fail(ctx, SAP_EINVAL, "sap_solve_batch: bad arguments");
  if (count > kMaxBatchCount) return fail(ctx, SAP_EINVAL, "sap_solve_batch: count must be at most 65535");
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  return run_batch(ctx, count, probs, params, x, info, static_cast<hipStream_t>(stream));
}

// Alg. 1 with LSQR (hb and ss null), heavy-ball momentum (App. D.3, hb) or
// the s-step form (App. D.4.2, ss) as the iterative method.
static sap_status solve_dense(sap_ctx *ctx, const sap_problem *prob, const sap_params *par_in,
                              const sap_hbm_params *hb, const sap_sstep_params *ss, double *x, sap_info *info,
                              void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_problem(ctx, prob);
  if (s != SAP_OK) return s;
  if (!par_in || !x) return fail(ctx, SAP_EINVAL, "sap_solve: NULL params or x");
  sap_params pv = *par_in;
  const sap_params *par = &pv;
  const int64_t m = prob->m;
  const int n = prob->n, nc = n + 1;
  if (pv.d == 0) {  // choose d for this problem (Sec. 4.3)
    if (!(pv.tol > 0.0 && pv.tol < 1.0)) return fail(ctx, SAP_EINVAL, "sap_solve: d = 0 needs tol in (0, 1)");
    if (pv.zeta < 1 || pv.zeta > 64) return fail(ctx, SAP_EINVAL, "sap_solve: zeta must be in [1, 64]");
    if (prob->a_type != SAP_F64 && prob->a_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sap_solve: bad A dtype");
    SAP_HIP_TRY(hipSetDevice(ctx->device));
    s = choose_d(ctx, prob, pv.zeta, pv.tol, &pv.d, static_cast<hipStream_t>(stream));
    if (s != SAP_OK) return s;
  }
  const int d = pv.d;
  if (d < nc) return fail(ctx, SAP_EINVAL, "sap_solve: need d >= n + 1");
  if (d > 16384) return fail(ctx, SAP_EINVAL, "sap_solve: d > 16384 is not supported");
  if (par->zeta < 1 || par->zeta > 64 || par->zeta > d) return fail(ctx, SAP_EINVAL, "sap_solve: zeta must be in [1, min(d, 64)]");
  if (par->maxiter < 0 || !(par->tol >= 0.0)) return fail(ctx, SAP_EINVAL, "sap_solve: need maxiter >= 0, tol >= 0");
  const int mode = par->mode;
  if (mode == SAP_MODE_FP64) {
    if (prob->a_type != SAP_F64) return fail(ctx, SAP_EINVAL, "sap_solve: FP64 mode needs an F64 A");
  } else if (mode == SAP_MODE_MIXED_FP32 || mode == SAP_MODE_MIXED_FP32_REFINE || mode == SAP_MODE_MIXED_BF16SA) {
    if (prob->a_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sap_solve: mixed modes need an F32 A");
    if (par->max_refine < 0) return fail(ctx, SAP_EINVAL, "sap_solve: max_refine must be >= 0");
  } else {
    return fail(ctx, SAP_EINVAL, "sap_solve: unsupported mode");
  }
  // fixed-count mode (Sec. 4.2): a set number of iterations, no stopping test
  int fixed = 0;
  if (par->fixed_iters != 0) {
    if (mode != SAP_MODE_FP64 && mode != SAP_MODE_MIXED_FP32)
      return fail(ctx, SAP_EINVAL, "sap_solve: fixed_iters needs the FP64 or MIXED_FP32 mode");
    if (par->fixed_iters > 0) {
      fixed = par->fixed_iters;
    } else {
      int32_t t = 0;
      if (sap_iteration_estimate(n, d, par->tol, &t) != SAP_OK)
        return fail(ctx, SAP_EINVAL, "sap_solve: fixed_iters < 0 needs tol in (0, 1)");
      fixed = t;
    }
  }
  // step size and momentum of the momentum method
  double hb_alpha = 0.0, hb_beta = 0.0;
  if (hb) {
    if (mode != SAP_MODE_FP64 && mode != SAP_MODE_MIXED_FP32)
      return fail(ctx, SAP_EINVAL, "sap_solve_hbm: mode must be FP64 or MIXED_FP32");
    if (hb->alpha > 0.0) {
      if (!(hb->beta >= 0.0 && hb->beta < 1.0)) return fail(ctx, SAP_EINVAL, "sap_solve_hbm: need 0 <= beta < 1");
      hb_alpha = hb->alpha;
      hb_beta = hb->beta;
    } else {
      const double c = hb->eta_scale > 0.0 ? hb->eta_scale : 1.0;
      const double eta = c * std::sqrt(static_cast<double>(n) / static_cast<double>(d));
      if (!(eta < 1.0)) return fail(ctx, SAP_EINVAL, "sap_solve_hbm: eta_scale sqrt(n/d) must be below 1");
      const double e2 = eta * eta;
      hb_alpha = hb->gradient_descent ? (1.0 - e2) * (1.0 - e2) / (1.0 + e2) : (1.0 - e2) * (1.0 - e2);
      hb_beta = hb->gradient_descent ? 0.0 : e2;
    }
  }
  // block size and Chebyshev interval of the s-step form: the embedding
  // bound puts Z's spectrum in [(1 - eta)^2, (1 + eta)^2], eta = c sqrt(n/d)
  double ss_lo = 0.0, ss_hi = 0.0;
  if (ss) {
    if (mode != SAP_MODE_FP64 && mode != SAP_MODE_MIXED_FP32)
      return fail(ctx, SAP_EINVAL, "sap_solve_sstep: mode must be FP64 or MIXED_FP32");
    if (ss->s < 1 || ss->s > 16) return fail(ctx, SAP_EINVAL, "sap_solve_sstep: need 1 <= s <= 16");
    const double c = ss->eta_scale > 0.0 ? ss->eta_scale : 1.0;
    const double eta = c * std::sqrt(static_cast<double>(n) / static_cast<double>(d));
    if (!(eta < 1.0)) return fail(ctx, SAP_EINVAL, "sap_solve_sstep: eta_scale sqrt(n/d) must be below 1");
    ss_lo = (1.0 - eta) * (1.0 - eta);
    ss_hi = (1.0 + eta) * (1.0 + eta);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));

  // The sketch is accumulated in FP64 in both forms: with an FP32 sketch the
  // preconditioner of an ill-conditioned A is perturbed enough to cost ~15%
  // more iterations, and the FP64 accumulator is the faster LDS path.
  const sap_dtype y_type = SAP_F64;
  const size_t bytes_flags = 256;
  const size_t bytes_idx = static_cast<size_t>(m) * par->zeta * sizeof(int32_t);
  const size_t bytes_sign = static_cast<size_t>(m) * sizeof(uint64_t);
  const size_t bytes_Y = static_cast<size_t>(d) * nc * sizeof(double);
  const size_t bytes_tau = static_cast<size_t>(nc) * sizeof(double);
  const size_t bytes_apply = apply_workspace_bytes(ctx, m, par->zeta, d, nc, y_type);
  const size_t bytes_qr = qr_workspace_bytes(d, nc);
  const size_t bytes_lsqr = lsqr_workspace_bytes(ctx, m, n);
  size_t scratch = bytes_apply > bytes_qr ? bytes_apply : bytes_qr;
  scratch = scratch > bytes_lsqr ? scratch : bytes_lsqr;
  const bool bf16sa = mode == SAP_MODE_MIXED_BF16SA;
  const int64_t ld_bf = (static_cast<int64_t>(n) + 7) / 8 * 8;
  const size_t bytes_bf = bf16sa ? static_cast<size_t>(m) * ld_bf * sizeof(__hip_bfloat16) : 0;
  const size_t bytes_ss = ss ? sstep_workspace_bytes(n, ss->s) : 0;
  const size_t total =
      10 * 256 + bytes_flags + bytes_idx + bytes_sign + bytes_Y + bytes_tau + bytes_bf + bytes_ss + scratch;
  s = ensure_workspace(ctx, total, st);
  if (s != SAP_OK) return s;
  Carve cv(ctx->ws);
  SolveFlags *flags = cv.take<SolveFlags>(1);
  int32_t *idx = cv.take<int32_t>(static_cast<size_t>(m) * par->zeta);
  uint64_t *sign = cv.take<uint64_t>(static_cast<size_t>(m));
  double *Y = cv.take<double>(static_cast<size_t>(d) * nc);
  double *tau = cv.take<double>(nc);
  __hip_bfloat16 *Abf = bf16sa ? cv.take<__hip_bfloat16>(static_cast<size_t>(m) * ld_bf) : nullptr;
  void *work = cv.take<char>(scratch);
  void *swork = ss ? cv.take<char>(bytes_ss) : nullptr;

  if (info) std::memset(info, 0, sizeof(*info));
  hipEvent_t ev[5];
  for (auto &e : ev) SAP_HIP_TRY(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int k = 0; k < 5; ++k) (void)hipEventDestroy(e[k]);
    }
  } guard{ev};

  zero_flags_kernel<<<1, 64, 0, st>>>(flags);
  finite_check_kernel<<<256, 256, 0, st>>>(prob->b, m, &flags->nonfinite_b);
  SAP_HIP_TRY(hipGetLastError());
  SAP_HIP_TRY(hipEventRecord(ev[0], st));
  sps_sketch S{m, d, par->zeta, par->seed, 0, idx, sign};
  s = launch_generate(ctx, &S, &flags->gen_error, st);
  if (s != SAP_OK) return s;
  SAP_HIP_TRY(hipEventRecord(ev[1], st));
  if (bf16sa) {  // the BF16 copy is part of the apply phase's cost
    const int64_t tot = m * ld_bf;
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((tot + 255) / 256, int64_t(ctx->num_cus) * 16));
    to_bf16_kernel<<<g, 256, 0, st>>>(static_cast<const float *>(prob->A), prob->lda, m, n, Abf, ld_bf);
    SAP_HIP_TRY(hipGetLastError());
  }
  hipEvent_t pb_apply = prof_begin(ctx, st);
  s = bf16sa ? launch_apply(ctx, &S, Abf, ld_bf, SAP_BF16, prob->b, n, Y, d, y_type, work, st)
             : launch_apply(ctx, &S, prob->A, prob->lda, prob->a_type, prob->b, n, Y, d, y_type, work, st);
  if (s != SAP_OK) return s;
  prof_end(ctx, kProfApply, pb_apply, st);
  SAP_HIP_TRY(hipEventRecord(ev[2], st));
  s = launch_qr(ctx, Y, d, d, nc, tau, work, st);
  if (s != SAP_OK) return s;
  s = launch_rank_check(ctx, Y, d, n, d, &flags->rank_deficient, st);
  if (s != SAP_OK) return s;
  SAP_HIP_TRY(hipEventRecord(ev[3], st));
  SolveFlags hf{};
  SAP_HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  if (hf.nonfinite_b) return fail(ctx, SAP_EINVAL, "sap_solve: b has non-finite entries");
  if (hf.gen_error) return fail(ctx, SAP_EDEVICE, "sap_solve: sketch generation hit its round cap");
  if (hf.rank_deficient == 2) return fail(ctx, SAP_EINVAL, "sap_solve: the sketch's R is not finite (non-finite A)");
  if (hf.rank_deficient) {
    if (info) info->status = SAP_RANK_DEFICIENT;
    return fail(ctx, SAP_RANK_DEFICIENT, "sap_solve: R is numerically singular (A rank deficient)");
  }
  // x0 = R^-1 (Q^T S b)[0:n]: column n of the factored sketch.
  // MIXED_BF16SA iterates as MIXED_FP32_REFINE (FP32 passes, FP64 refinement)
  const int lsqr_mode = (mode == SAP_MODE_FP64) ? 0 : (mode == SAP_MODE_MIXED_FP32 ? 1 : 2);
  sap_info li{};
  if (ss)
    s = run_sstep(ctx, prob, Y, d, Y + static_cast<int64_t>(n) * d, fixed ? 0.0 : par->tol,
                  fixed ? fixed : par->maxiter, lsqr_mode, ss->s, ss_lo, ss_hi, x, &li, work, swork, st);
  else if (hb)
    s = run_hbm(ctx, prob, Y, d, Y + static_cast<int64_t>(n) * d, fixed ? 0.0 : par->tol,
                fixed ? fixed : par->maxiter, lsqr_mode, hb_alpha, hb_beta, x, &li, work, st);
  else
    s = run_lsqr(ctx, prob, Y, d, nullptr, Y + static_cast<int64_t>(n) * d, fixed ? 0.0 : par->tol,
                 fixed ? fixed : par->maxiter, lsqr_mode, par->max_refine, x, &li, work, st);
  if (s != SAP_OK && s != SAP_NOT_CONVERGED) return s;
  if (fixed && s == SAP_NOT_CONVERGED) s = SAP_OK;  // the set count was run
  SAP_HIP_TRY(hipEventRecord(ev[4], st));
  SAP_HIP_TRY(hipEventSynchronize(ev[4]));
  prof_resolve(ctx);
  if (info) {
    *info = li;
    info->status = s;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    info->t_generate_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
    info->t_apply_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[2], ev[3]);
    info->t_qr_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[3], ev[4]);
    info->t_iterate_ms = ms;
    info->d_used = d;
  }
  if (s == SAP_NOT_CONVERGED) (void)fail(ctx, s, "sap_solve: maxiter reached before the stopping test");
  return s;
}

sap_status sap_solve(sap_ctx *ctx, const sap_problem *prob, const sap_params *params, double *x, sap_info *info,
                     void *stream) {
  return solve_dense(ctx, prob, params, nullptr, nullptr, x, info, stream);
}

sap_status sap_solve_hbm(sap_ctx *ctx, const sap_problem *prob, const sap_params *params,
                         const sap_hbm_params *hbm, double *x, sap_info *info, void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (!hbm) return fail(ctx, SAP_EINVAL, "sap_solve_hbm: NULL momentum parameters");
  return solve_dense(ctx, prob, params, hbm, nullptr, x, info, stream);
}

sap_status sap_solve_sstep(sap_ctx *ctx, const sap_problem *prob, const sap_params *params,
                           const sap_sstep_params *ss, double *x, sap_info *info, void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (!ss) return fail(ctx, SAP_EINVAL, "sap_solve_sstep: NULL s-step parameters");
  return solve_dense(ctx, prob, params, nullptr, ss, x, info, stream);
}

static sap_status check_csr(sap_ctx *ctx, const sap_csr *A) {
  if (!A) return fail(ctx, SAP_EINVAL, "sparse A descriptor is NULL");
  if (A->n < 1 || A->n > 8192) return fail(ctx, SAP_EINVAL, "sparse A: need 1 <= n <= 8192");
  if (A->m < static_cast<int64_t>(A->n) + 1) return fail(ctx, SAP_EINVAL, "sparse A: need m >= n + 1");
  if (A->m >= (int64_t(1) << 31)) return fail(ctx, SAP_EINVAL, "sparse A: need m < 2^31");
  if (A->nnz < 0 || !A->indptr || (A->nnz > 0 && (!A->indices || !A->values)))
    return fail(ctx, SAP_EINVAL, "sparse A: bad pointers or nnz");
  if (A->v_type != SAP_F64 && A->v_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sparse A: values must be F64 or F32");
  return SAP_OK;
}

static SparseA to_sparse(const sap_csr *A) {
  SparseA s;
  s.m = A->m;
  s.n = A->n;
  s.nnz = A->nnz;
  s.indptr = A->indptr;
  s.indices = A->indices;
  s.values = A->values;
  s.v_type = A->v_type;
  return s;
}

sap_status sps_apply_csr(sap_ctx *ctx, const sps_sketch *S, const sap_csr *A, const double *b, double *Y, int64_t ldy,
                         void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_sketch(ctx, S);
  if (s != SAP_OK) return s;
  s = check_csr(ctx, A);
  if (s != SAP_OK) return s;
  if (S->m != A->m) return fail(ctx, SAP_EINVAL, "sps_apply_csr: the sketch must have m columns");
  if (!Y || ldy < S->d) return fail(ctx, SAP_EINVAL, "sps_apply_csr: need Y and ldy >= d");
  if (S->d >= 20000) return fail(ctx, SAP_EINVAL, "sps_apply_csr: d >= 20000 is not supported");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  const SparseA sa = to_sparse(A);
  s = ensure_workspace(ctx, csr_apply_workspace_bytes(sa, S->d) + 512, st);
  if (s != SAP_OK) return s;
  Carve cv(ctx->ws);
  int *bad = cv.take<int>(1);
  void *work = cv.take<char>(csr_apply_workspace_bytes(sa, S->d));
  hipEvent_t pb = prof_begin(ctx, st);
  s = launch_csr_apply(ctx, S, sa, b, Y, ldy, bad, work, st);
  prof_end(ctx, kProfApply, pb, st);
  if (s != SAP_OK) return s;
  int hbad = 0;
  SAP_HIP_TRY(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  if (hbad)
    return fail(ctx, SAP_EINVAL,
                "sps_apply_csr: indptr must start at 0, end at nnz and not decrease; column indices must lie in [0, n)");
  return SAP_OK;
}

sap_status sap_solve_csr(sap_ctx *ctx, const sap_csr *A, const double *b, const sap_params *par_in, double *x,
                         sap_info *info, void *stream) {
  if (!ctx) return SAP_EINVAL;
  sap_status s = check_csr(ctx, A);
  if (s != SAP_OK) return s;
  if (!par_in || !x || !b) return fail(ctx, SAP_EINVAL, "sap_solve_csr: NULL params, b or x");
  sap_params pv = *par_in;
  const int64_t m = A->m;
  const int n = A->n, nc = n + 1;
  if (pv.d == 0) {  // eq. (4.2) with cost ratio 1
    int32_t d42 = 0;
    if (!(pv.tol > 0.0 && pv.tol < 1.0) || sap_embedding_dim(m, n, pv.tol, 1.0, &d42) != SAP_OK)
      return fail(ctx, SAP_EINVAL, "sap_solve_csr: d = 0 needs tol in (0, 1)");
    pv.d = static_cast<int32_t>(std::min<int64_t>(std::min<int64_t>(d42, 16384), m));
  }
  const int d = pv.d;
  if (d < nc || d > 16384) return fail(ctx, SAP_EINVAL, "sap_solve_csr: need n + 1 <= d <= 16384");
  if (pv.zeta < 1 || pv.zeta > 64 || pv.zeta > d) return fail(ctx, SAP_EINVAL, "sap_solve_csr: bad zeta");
  if (pv.maxiter < 0 || !(pv.tol >= 0.0)) return fail(ctx, SAP_EINVAL, "sap_solve_csr: need maxiter >= 0, tol >= 0");
  if (pv.mode == SAP_MODE_FP64) {
    if (A->v_type != SAP_F64) return fail(ctx, SAP_EINVAL, "sap_solve_csr: FP64 mode needs F64 values");
  } else if (pv.mode == SAP_MODE_MIXED_FP32) {
    if (A->v_type != SAP_F32) return fail(ctx, SAP_EINVAL, "sap_solve_csr: MIXED_FP32 needs F32 values");
  } else {
    return fail(ctx, SAP_EINVAL, "sap_solve_csr: mode must be FP64 or MIXED_FP32");
  }
  int fixed = 0;
  if (pv.fixed_iters > 0) fixed = pv.fixed_iters;
  else if (pv.fixed_iters < 0 && sap_iteration_estimate(n, d, pv.tol, &fixed) != SAP_OK)
    return fail(ctx, SAP_EINVAL, "sap_solve_csr: fixed_iters < 0 needs tol in (0, 1)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  const SparseA sa = to_sparse(A);
  size_t scratch = csr_apply_workspace_bytes(sa, d);
  scratch = std::max(scratch, qr_workspace_bytes(d, nc));
  scratch = std::max(scratch, lsqr_workspace_bytes(ctx, m, n));
  const size_t total = 8 * 256 + 256 + static_cast<size_t>(m) * pv.zeta * sizeof(int32_t) +
                       static_cast<size_t>(m) * sizeof(uint64_t) + static_cast<size_t>(d) * nc * sizeof(double) +
                       static_cast<size_t>(nc) * sizeof(double) + scratch;
  s = ensure_workspace(ctx, total, st);
  if (s != SAP_OK) return s;
  Carve cv(ctx->ws);
  SolveFlags *flags = cv.take<SolveFlags>(1);
  int32_t *idx = cv.take<int32_t>(static_cast<size_t>(m) * pv.zeta);
  uint64_t *sign = cv.take<uint64_t>(static_cast<size_t>(m));
  double *Y = cv.take<double>(static_cast<size_t>(d) * nc);
  double *tau = cv.take<double>(nc);
  void *work = cv.take<char>(scratch);
  if (info) std::memset(info, 0, sizeof(*info));
  hipEvent_t ev[5];
  for (auto &e : ev) SAP_HIP_TRY(hipEventCreate(&e));
  struct EvGuard {
    hipEvent_t *e;
    ~EvGuard() {
      for (int k = 0; k < 5; ++k) (void)hipEventDestroy(e[k]);
    }
  } guard{ev};
  zero_flags_kernel<<<1, 64, 0, st>>>(flags);
  finite_check_kernel<<<256, 256, 0, st>>>(b, m, &flags->nonfinite_b);
  SAP_HIP_TRY(hipGetLastError());
  SAP_HIP_TRY(hipEventRecord(ev[0], st));
  sps_sketch S{m, d, pv.zeta, pv.seed, 0, idx, sign};
  s = launch_generate(ctx, &S, &flags->gen_error, st);
  if (s != SAP_OK) return s;
  SAP_HIP_TRY(hipEventRecord(ev[1], st));
  hipEvent_t pb_apply = prof_begin(ctx, st);
  s = launch_csr_apply(ctx, &S, sa, b, Y, d, &flags->bad_csr, work, st);
  if (s != SAP_OK) return s;
  prof_end(ctx, kProfApply, pb_apply, st);
  SAP_HIP_TRY(hipEventRecord(ev[2], st));
  s = launch_qr(ctx, Y, d, d, nc, tau, work, st);
  if (s != SAP_OK) return s;
  s = launch_rank_check(ctx, Y, d, n, d, &flags->rank_deficient, st);
  if (s != SAP_OK) return s;
  SAP_HIP_TRY(hipEventRecord(ev[3], st));
  SolveFlags hf{};
  SAP_HIP_TRY(hipMemcpyAsync(&hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  if (hf.bad_csr)
    return fail(ctx, SAP_EINVAL,
                "sap_solve_csr: indptr must start at 0, end at nnz and not decrease; column indices must lie in [0, n)");
  if (hf.nonfinite_b) return fail(ctx, SAP_EINVAL, "sap_solve_csr: b has non-finite entries");
  if (hf.gen_error) return fail(ctx, SAP_EDEVICE, "sap_solve_csr: sketch generation hit its round cap");
  if (hf.rank_deficient == 2)
    return fail(ctx, SAP_EINVAL, "sap_solve_csr: the sketch's R is not finite (non-finite A)");
  if (hf.rank_deficient) {
    if (info) info->status = SAP_RANK_DEFICIENT;
    return fail(ctx, SAP_RANK_DEFICIENT, "sap_solve_csr: R is numerically singular (A rank deficient)");
  }
  sap_problem prob{m, n, nullptr, n, A->v_type, b};
  sap_info li{};
  s = run_lsqr(ctx, &prob, Y, d, nullptr, Y + static_cast<int64_t>(n) * d, fixed ? 0.0 : pv.tol,
               fixed ? fixed : pv.maxiter, pv.mode == SAP_MODE_FP64 ? 0 : 1, 0, x, &li, work, st, &sa);
  if (s != SAP_OK && s != SAP_NOT_CONVERGED) return s;
  if (fixed && s == SAP_NOT_CONVERGED) s = SAP_OK;
  SAP_HIP_TRY(hipEventRecord(ev[4], st));
  SAP_HIP_TRY(hipEventSynchronize(ev[4]));
  prof_resolve(ctx);
  if (info) {
    *info = li;
    info->status = s;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, ev[0], ev[1]);
    info->t_generate_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[1], ev[2]);
    info->t_apply_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[2], ev[3]);
    info->t_qr_ms = ms;
    (void)hipEventElapsedTime(&ms, ev[3], ev[4]);
    info->t_iterate_ms = ms;
    info->d_used = d;
  }
  if (s == SAP_NOT_CONVERGED) (void)fail(ctx, s, "sap_solve_csr: maxiter reached before the stopping test");
  return s;
}

sap_status sap_serve_start(sap_ctx *ctx, size_t arena_bytes, int32_t max_active) {
  if (!ctx) return SAP_EINVAL;
  return serve_start(ctx, arena_bytes, max_active);
}

sap_status sap_submit(sap_ctx *ctx, const sap_problem *prob, const sap_params *params, double *x, uint64_t *ticket,
                      void *stream) {
  if (!ctx) return SAP_EINVAL;
  return serve_submit(ctx, prob, params, x, ticket, static_cast<hipStream_t>(stream));
}

sap_status sap_poll(sap_ctx *ctx, uint64_t ticket, sap_info *info, int32_t wait) {
  if (!ctx) return SAP_EINVAL;
  return serve_poll(ctx, ticket, info, wait);
}

sap_status sap_cancel(sap_ctx *ctx, uint64_t ticket) {
  if (!ctx) return SAP_EINVAL;
  return serve_cancel(ctx, ticket);
}

sap_status sap_serve_stats(sap_ctx *ctx, int64_t *stats) {
  if (!ctx || !stats) return SAP_EINVAL;
  return serve_stats(ctx, stats);
}

}  // extern "C"
