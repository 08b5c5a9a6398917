// Machine-aware choice of the embedding dimension (Sec. 4.3).
//
// Eq. (4.2) balances the QR work d n^2 against the iteration work t(d) m n
// with the two unit costs taken equal, and assumes the sketch costs the same
// at every d.  On this GPU neither holds exactly: the apply's cost steps with
// the LDS strip width that d allows, and the QR's with its panel path.  So
// the candidates are priced with the library's own kernels, timed on a slab
// of the caller's problem, once per context and (n, dtype, zeta, d):
//   apply(d): the sketch apply of the first m_s = min(m, 65536) rows at d,
//             scaled by m / m_s;
//   qr(d):    the Householder QR of that d x (n+1) sketch (independent of m);
//   a m + f:  one LSQR iteration, from iterations timed on the slab and on
//             half of it (each as the difference of a 9- and a 3-iteration
//             run, which removes the per-solve set-up);
// and the candidate minimising apply(d) + qr(d) + (t(d) + 1)(a m + f) wins,
// t(d) the eq. (4.1) estimate ceil(2 log eps / log(n/d)).
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>
#include <vector>

#include "common.h"

namespace sap {

struct SelectCache {
  struct Entry {
    double apply_ms_per_row = 0.0;  // apply time per row of A at this d
    double qr_ms = 0.0;
  };
  // (n, dtype, zeta, d) -> timings; (n, dtype) -> iteration fit (a per row, f)
  std::map<std::tuple<int, int, int, int>, Entry> phase;
  std::map<std::tuple<int, int>, std::pair<double, double>> iter_fit;
};

void select_cache_free(sap_ctx *ctx) {
  delete static_cast<SelectCache *>(ctx->select_cache);
  ctx->select_cache = nullptr;
}

namespace {

constexpr int64_t kSlabRows = 65536;
constexpr int64_t kMinCalibrateRows = 4096;
constexpr int kMaxD = 16384;  // sap_solve's limit (the QR panel holds a column in registers)

__global__ void zero_f64_kernel(double *x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

std::vector<int> candidates(int64_t m, int n, double eps) {
  static const double ks[] = {1.25, 1.5, 2.0, 2.5, 3.0, 4.0, 5.0, 6.0, 8.0, 10.0, 12.0};
  const int hi = static_cast<int>(std::min<int64_t>(m, kMaxD));
  std::vector<int> c;
  for (double k : ks) c.push_back(static_cast<int>(std::ceil(k * n)));
  int32_t d42 = 0;
  if (sap_embedding_dim(m, n, eps, 1.0, &d42) == SAP_OK) c.push_back(d42);
  for (int &v : c) v = std::max(n + 1, std::min(v, hi));
  std::sort(c.begin(), c.end());
  c.erase(std::unique(c.begin(), c.end()), c.end());
  return c;
}

// Time (ms) of a blocking host call bracketed by events on `st`.
template <typename F>
sap_status timed(sap_ctx *ctx, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double *ms, F &&f) {
  SAP_HIP_TRY(hipEventRecord(e0, st));
  const sap_status s = f();
  if (s != SAP_OK && s != SAP_NOT_CONVERGED) return s;
  SAP_HIP_TRY(hipEventRecord(e1, st));
  SAP_HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  SAP_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  *ms = t;
  return SAP_OK;
}

sap_status calibrate(sap_ctx *ctx, SelectCache &cache, const sap_problem *prob, int zeta,
                     const std::vector<int> &need_d, bool need_fit, hipStream_t st) {
  const int n = prob->n, nc = n + 1;
  const int64_t ms = std::min<int64_t>(prob->m, kSlabRows);
  const int dmax = *std::max_element(need_d.begin(), need_d.end());
  const sap_dtype at = prob->a_type;
  // the apply's and the QR's workspace depend on d, and not monotonically
  // (a small d gives wide LDS strips and so row slices with partial sums):
  // size the scratch for every d timed here
  size_t scratch = lsqr_workspace_bytes(ctx, ms, n);
  for (int d : need_d) {
    scratch = std::max(scratch, apply_workspace_bytes(ctx, ms, zeta, d, nc, SAP_F64));
    scratch = std::max(scratch, qr_workspace_bytes(d, nc));
  }
  scratch = std::max(scratch, apply_workspace_bytes(ctx, ms, zeta, dmax, nc, SAP_F64));
  scratch = std::max(scratch, qr_workspace_bytes(dmax, nc));
  const size_t total = 8 * 256 + static_cast<size_t>(ms) * zeta * sizeof(int32_t) + ms * sizeof(uint64_t) +
                       static_cast<size_t>(dmax) * nc * sizeof(double) + 3 * static_cast<size_t>(nc) * sizeof(double) +
                       sizeof(int) * 4 + scratch;
  sap_status s = ensure_workspace(ctx, total, st);
  if (s != SAP_OK) return s;
  Carve cv(ctx->ws);
  int32_t *idx = cv.take<int32_t>(static_cast<size_t>(ms) * zeta);
  uint64_t *sign = cv.take<uint64_t>(ms);
  double *Y = cv.take<double>(static_cast<size_t>(dmax) * nc);
  double *tau = cv.take<double>(nc);
  double *x0 = cv.take<double>(nc);
  double *xs = cv.take<double>(nc);
  int *gen_err = cv.take<int>(4);
  void *work = cv.take<char>(scratch);
  hipEvent_t e0, e1;
  SAP_HIP_TRY(hipEventCreate(&e0));
  SAP_HIP_TRY(hipEventCreate(&e1));
  struct Guard {
    hipEvent_t a, b;
    ~Guard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } guard{e0, e1};
  SAP_HIP_TRY(hipMemsetAsync(gen_err, 0, sizeof(int), st));
  // the apply and QR at each candidate d; the last leaves the slab's R at dmax in Y
  std::vector<int> ds = need_d;
  if (need_fit && ds.back() != dmax) ds.push_back(dmax);
  for (int d : ds) {
    sps_sketch S{ms, d, zeta, 0x5e1ec7ULL, 0, idx, sign};
    s = launch_generate(ctx, &S, gen_err, st);
    if (s != SAP_OK) return s;
    // warm the kernels at this shape once, then time
    s = launch_apply(ctx, &S, prob->A, prob->lda, at, prob->b, n, Y, d, SAP_F64, work, st);
    if (s != SAP_OK) return s;
    double t_apply = 0.0, t_qr = 0.0;
    s = timed(ctx, st, e0, e1, &t_apply, [&] {
      return launch_apply(ctx, &S, prob->A, prob->lda, at, prob->b, n, Y, d, SAP_F64, work, st);
    });
    if (s != SAP_OK) return s;
    s = timed(ctx, st, e0, e1, &t_qr, [&] { return launch_qr(ctx, Y, d, d, nc, tau, work, st); });
    if (s != SAP_OK) return s;
    SelectCache::Entry &en = cache.phase[std::make_tuple(n, static_cast<int>(at), zeta, d)];
    en.apply_ms_per_row = t_apply / static_cast<double>(ms);
    en.qr_ms = t_qr;
  }
  if (need_fit) {
    // one iteration on the slab and on half of it, each as the difference of
    // a 9- and a 3-iteration run from x0 = 0 (tol 0: the runs go to maxiter)
    zero_f64_kernel<<<(n + 255) / 256, 256, 0, st>>>(x0, n);
    SAP_HIP_TRY(hipGetLastError());
    const int mode = (at == SAP_F32) ? 1 : 0;
    double per[2] = {0.0, 0.0};
    const int64_t rows[2] = {ms, std::max<int64_t>(n + 1, ms / 2)};
    for (int k = 0; k < 2; ++k) {
      sap_problem slab = *prob;
      slab.m = rows[k];
      double t3 = 0.0, t9 = 0.0;
      for (int rep = 0; rep < 2; ++rep) {  // the first round warms the kernels
        sap_info inf{};
        s = timed(ctx, st, e0, e1, &t3,
                  [&] { return run_lsqr(ctx, &slab, Y, dmax, x0, nullptr, 0.0, 3, mode, 0, xs, &inf, work, st); });
        if (s != SAP_OK) return s;
        s = timed(ctx, st, e0, e1, &t9,
                  [&] { return run_lsqr(ctx, &slab, Y, dmax, x0, nullptr, 0.0, 9, mode, 0, xs, &inf, work, st); });
        if (s != SAP_OK) return s;
      }
      per[k] = std::max(0.0, (t9 - t3) / 6.0);
    }
    const double a = std::max(0.0, (per[0] - per[1]) / static_cast<double>(rows[0] - rows[1]));
    const double f = std::max(0.0, per[0] - a * static_cast<double>(rows[0]));
    cache.iter_fit[std::make_tuple(n, static_cast<int>(at))] = {a, f};
  }
  int herr = 0;
  SAP_HIP_TRY(hipMemcpyAsync(&herr, gen_err, sizeof(int), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  if (herr) return fail(ctx, SAP_EDEVICE, "sap_choose_d: sketch generation hit its round cap");
  return SAP_OK;
}

}  // namespace

sap_status choose_d(sap_ctx *ctx, const sap_problem *prob, int zeta, double eps, int32_t *d, hipStream_t st) {
  const int n = prob->n;
  const int64_t m = prob->m;
  int32_t d42 = 0;
  if (sap_embedding_dim(m, n, eps, 1.0, &d42) != SAP_OK) return fail(ctx, SAP_EINVAL, "sap_choose_d: bad shape");
  if (m < kMinCalibrateRows || n + 1 > kMaxD) {
    *d = std::max(n + 1, std::min<int32_t>(d42, static_cast<int32_t>(std::min<int64_t>(m, kMaxD))));
    return SAP_OK;
  }
  if (!ctx->select_cache) ctx->select_cache = new SelectCache();
  SelectCache &cache = *static_cast<SelectCache *>(ctx->select_cache);
  const std::vector<int> cand = candidates(m, n, eps);
  std::vector<int> need;
  for (int dc : cand)
    if (!cache.phase.count(std::make_tuple(n, static_cast<int>(prob->a_type), zeta, dc))) need.push_back(dc);
  const bool need_fit = !cache.iter_fit.count(std::make_tuple(n, static_cast<int>(prob->a_type)));
  if (!need.empty() || need_fit) {
    std::vector<int> nd = need.empty() ? std::vector<int>{cand.back()} : need;
    sap_status s = calibrate(ctx, cache, prob, zeta, nd, need_fit, st);
    if (s != SAP_OK) return s;
  }
  const auto fit = cache.iter_fit[std::make_tuple(n, static_cast<int>(prob->a_type))];
  const double per_iter = fit.first * static_cast<double>(m) + fit.second;
  double best = INFINITY;
  int best_d = cand.front();
  for (int dc : cand) {
    const SelectCache::Entry &en = cache.phase[std::make_tuple(n, static_cast<int>(prob->a_type), zeta, dc)];
    int32_t t = 0;
    if (sap_iteration_estimate(n, dc, eps, &t) != SAP_OK) continue;
    const double cost = en.apply_ms_per_row * static_cast<double>(m) + en.qr_ms + (t + 1.0) * per_iter;
    if (cost < best) {
      best = cost;
      best_d = dc;
    }
  }
  *d = best_d;
  return SAP_OK;
}

}  // namespace sap

using namespace sap;

extern "C" sap_status sap_choose_d(sap_ctx *ctx, const sap_problem *prob, int32_t zeta, double eps, int32_t *d,
                                   void *stream) {
  if (!ctx) return SAP_EINVAL;
  if (!prob || !d) return fail(ctx, SAP_EINVAL, "sap_choose_d: NULL argument");
  if (prob->n < 1 || prob->m < static_cast<int64_t>(prob->n) + 1 || prob->lda < prob->n || !prob->A || !prob->b)
    return fail(ctx, SAP_EINVAL, "sap_choose_d: bad problem");
  if (prob->a_type != SAP_F64 && prob->a_type != SAP_F32)
    return fail(ctx, SAP_EINVAL, "sap_choose_d: A must be F64 or F32");
  if (zeta < 1 || zeta > 64) return fail(ctx, SAP_EINVAL, "sap_choose_d: zeta must be in [1, 64]");
  if (!(eps > 0.0 && eps < 1.0)) return fail(ctx, SAP_EINVAL, "sap_choose_d: eps must be in (0, 1)");
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  return choose_d(ctx, prob, zeta, eps, d, static_cast<hipStream_t>(stream));
}
