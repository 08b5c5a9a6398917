// Internal helpers shared by the gfx950 kernels and the host-side API.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "../../include/sap.h"

namespace sap {

constexpr int kWave = 64;  // CDNA wavefront width

// ---------------------------------------------------------------- device ---
// [wave-helpers-begin] (wavefront reductions used by the fused LSQR pass; the
// benchmark hashes this region and the pass kernel's to tell whether HBM
// counters taken on the pass still describe it)
// Butterfly sum over the 64 lanes of a wavefront; every lane receives the
// total.  The order of additions is fixed, so the result is deterministic.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T o = __shfl_xor(v, off, kWave);
    v = v > o ? v : o;
  }
  return v;
}

// DPP lane permutation of a double (both 32-bit halves moved alike).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ double readlane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float readlane(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// DPP move restricted to the rows in ROWMASK; lanes of the other rows read 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_mov_rows(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_mov_rows(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xF, false));
}

// Sum over the 64 lanes of a wavefront returned as a wave-uniform value.
// Within each row of 16 lanes: quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror leave the row sum in every lane; row_bcast:15
// into rows 1 and 3 then row_bcast:31 into rows 2 and 3 accumulate the four
// row sums into row 3, and lane 63 is read.  Fixed order, so the result is
// deterministic.  Every lane of the wave must be active.
template <typename T>
__device__ __forceinline__ T wave_sum_u(T v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  v += dpp_mov<0x140>(v);
  v += dpp_mov_rows<0x142, 0xA>(v);
  v += dpp_mov_rows<0x143, 0xC>(v);
  return readlane(v, 63);
}

// [wave-helpers-end]

// Broadcast a double held by lane `src` (wave-uniform) to all lanes.
__device__ __forceinline__ double wave_bcast(double v, int src) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Sum over a workgroup of `nwaves` waves.  `scratch` is LDS of >= nwaves
// doubles.  All threads receive the total.  Contains two barriers.
__device__ __forceinline__ double block_sum(double v, double *scratch, int nwaves) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nwaves; ++w) s += scratch[w];
  return s;
}

// ------------------------------------------------------------------ host ---
#define SAP_HIP_TRY(expr)                                          \
  do {                                                             \
    hipError_t _e = (expr);                                        \
    if (_e != hipSuccess) return ::sap::hip_fail(ctx, _e, #expr);  \
  } while (0)

// Streaming load of V consecutive elements (16 bytes or fewer) with the
// nontemporal hint: data read once per pass should not displace what the
// caches hold for reuse.  On gfx950 a read-only stream reaches ~90% of the
// HBM peak this way, ~80% with ordinary loads.
template <typename T, int V>
__device__ __forceinline__ void load_stream(const T *p, T (&out)[V]) {
  if constexpr (V == 1) {
    out[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T vec_t __attribute__((ext_vector_type(V)));
    const vec_t v = __builtin_nontemporal_load(reinterpret_cast<const vec_t *>(p));
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = v[e];
  }
}

// Global-memory views.  A pointer that a kernel reads from device memory (a
// field of a work-item descriptor) is generic to the compiler, which then
// emits flat loads and stores; a flat access also counts against the LDS
// wait counter, so every LDS or cross-lane wait in a loop drains the loads
// in flight.  Through these views the accesses are global ones.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ const gmem<T> *gview(const T *p) {
  return (const gmem<T> *)p;
}
template <typename T>
__device__ __forceinline__ gmem<T> *gview(T *p) {
  return (gmem<T> *)p;
}
template <typename T, int V>
__device__ __forceinline__ void load_stream(const gmem<T> *p, T (&out)[V]) {
  if constexpr (V == 1) {
    out[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T vec_t __attribute__((ext_vector_type(V)));
    const vec_t v = __builtin_nontemporal_load(reinterpret_cast<const gmem<vec_t> *>(p));
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = v[e];
  }
}

// Device-resident LSQR state.  All recurrence scalars stay on the device so
// that an iteration needs no host round trip.

struct LsqrState {
  double alpha, beta, rhobar, phibar;
  double c_ap, c_u;           // next pass computes u <- c_ap * (A p) + c_u * u
  double alpha_new, beta_new; // alpha_{t+1}, beta_{t+1} from the lower solve
  double normb, tol;
  double resid_est, normar_est;
  int32_t iter, maxiter;
  int32_t done, converged;
  int32_t init;          // 1: the next step is the initialisation step
  int32_t total_iters;   // iterations done
  int32_t proceed;       // alpha_{t+1} > 0 and beta_{t+1} > 0
  int32_t steps;         // completed lower/upper solve pairs (flag epoch)
  int32_t rel;           // 1: phibar is tested against beta_1 of this run (inner solves)
  int32_t pad;
  double normref;        // scale of the phibar test: ||b||, or beta_1 when rel
  double normar0;        // ||(A M)^T r|| at the initialisation step (rel runs)
  // Residual refinement kept on the device (batched and served forms): the
  // outer loop around the FP32 inner solves.
  int32_t refine;        // 1: FP32 inner solves, FP64 residual refinement
  int32_t refinements;   // inner solves finished so far
  int32_t max_refine;    // cap on the inner solves
  int32_t final_done;    // the outer loop has stopped (converged or gave up)
  double target;         // stop when ||x - x_prev|| <= target ||x||
  double prev_delta;     // the previous correction ||x - x_prev||
};

}  // namespace sap

namespace sap {
struct Server;
}

struct sap_ctx {
  sap::Server *server = nullptr;  // served form (continuous batching), created on demand
  int device = 0;
  int num_cus = 256;
  size_t budget = 0;

  void *ws = nullptr;
  size_t ws_size = 0;
  // device address of this GPU's copy of the static scratch array used by
  // sps_apply_noalloc (set once at sap_create; never allocated or freed)
  void *apply_scratch = nullptr;
  size_t apply_scratch_bytes = 0;
  // per-context timings of sap_choose_d (select.hip)
  void *select_cache = nullptr;
  // captured LSQR / momentum iteration batches, replayed as hipGraphs
  // (lsqr.hip), and the pinned host slots and events through which the
  // state of one batch is read while the next one runs
  void *batch_graphs = nullptr;
  void *pinned = nullptr;
  hipEvent_t batch_ev[2] = {nullptr, nullptr};
  // kernel timing (sap_profile_enable): pending event pairs per kernel,
  // resolved into launch counts and milliseconds; free events are reused
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[2];
  std::vector<hipEvent_t> free_events;
  int64_t prof_launches[2] = {0, 0};
  double prof_ms[2] = {0.0, 0.0};
};

namespace sap {

sap_status fail(sap_ctx *ctx, sap_status s, const std::string &msg);
sap_status hip_fail(sap_ctx *ctx, hipError_t e, const char *what);
// Grow the context workspace to at least `bytes` (synchronises `stream` when
// it has to reallocate).  Returns SAP_ENOMEM beyond the budget.
sap_status ensure_workspace(sap_ctx *ctx, size_t bytes, hipStream_t stream);

// Bump allocator over a workspace region (256-byte aligned pieces).
struct Carve {
  char *base;
  size_t off = 0;
  explicit Carve(void *b) : base(static_cast<char *>(b)) {}
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = reinterpret_cast<T *>(base + off);
    off += count * sizeof(T);
    return p;
  }
  size_t used() const { return (off + 255) & ~size_t(255); }
};

// Kernel timing helpers: begin records an event before a launch, end after
// it; resolve waits for pending events and accumulates their durations.
enum ProfKernel { kProfPass = 0, kProfApply = 1 };
hipEvent_t prof_begin(sap_ctx *ctx, hipStream_t st);
void prof_end(sap_ctx *ctx, int kernel, hipEvent_t begin, hipStream_t st);
void prof_resolve(sap_ctx *ctx);

// ------------------------------------------------------- internal launchers
// Sketch generation (sketch.hip).
sap_status launch_generate(sap_ctx *ctx, const sps_sketch *S, int *err_word, hipStream_t st);

// Sketch apply (apply.hip).  Workspace bytes for partial sums first.
size_t apply_workspace_bytes(sap_ctx *ctx, int64_t m, int zeta, int d, int ncols, sap_dtype y_type);
sap_status launch_apply(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda,
                        sap_dtype a_type, const double *b, int n, void *Y, int64_t ldy,
                        sap_dtype y_type, void *work, hipStream_t st);

// Static scratch of the allocation-free apply (apply.hip): its size, and the
// lookup of this device's copy (once per context, with the device current).
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
sap_status apply_scratch_init(sap_ctx *ctx);

// Embedding-dimension choice (select.hip): d for a problem, timings cached
// per context; the cache is freed by sap_destroy.
sap_status choose_d(sap_ctx *ctx, const sap_problem *prob, int zeta, double eps, int32_t *d, hipStream_t st);
void select_cache_free(sap_ctx *ctx);

// Householder QR (qr.hip).
size_t qr_workspace_bytes(int rows, int cols);
sap_status launch_qr(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau,
                     void *work, hipStream_t st);
// Rank test of R's diagonal; writes 1 to *flag when deficient.
sap_status launch_rank_check(sap_ctx *ctx, const double *R, int64_t ldr, int n, int d, int *flag,
                             hipStream_t st);

// Triangular solves (lsqr.hip, trsv.hip).  Blocking (reads an error word).
size_t trsv_workspace_bytes(int n);
sap_status launch_trsv(sap_ctx *ctx, const double *R, int64_t ldr, int n, int trans,
                       const double *rhs, double *x, void *work, hipStream_t st);

// Sparse A in CSR form (sparse.hip): row i holds entries indptr[i] ..
// indptr[i+1]-1 (columns `indices`, values of type v_type, F64 or F32).
struct SparseA {
  int64_t m = 0;
  int n = 0;
  int64_t nnz = 0;
  const int64_t *indptr = nullptr;
  const int32_t *indices = nullptr;
  const void *values = nullptr;
  sap_dtype v_type = SAP_F64;
};
size_t csr_apply_workspace_bytes(const SparseA &A, int d);
// Y (F64, ldy) = S [A b], asynchronous.  *bad (device) is cleared, then set
// when the CSR arrays fail the check (Y is then garbage); the caller reads it.
sap_status launch_csr_apply(sap_ctx *ctx, const sps_sketch *S, const SparseA &A, const double *b, double *Y,
                            int64_t ldy, int *bad, void *work, hipStream_t st);
int csr_pass_grid(sap_ctx *ctx, const SparseA &A);
void launch_csr_pass(sap_ctx *ctx, const SparseA &A, int grid, const double *p, const double *u_in, double *u_out,
                     const LsqrState *st, double *qpart, double *nrmpart, hipStream_t s);

// LSQR driver (lsqr.hip).  When z is non-null, x0 is ignored and the initial
// guess is R^-1 z (the sketch-and-solve solution of Alg. 1).
// mode 0: A in FP64; mode 1: A stored in FP32 (FP64 arithmetic); mode 2: A
// stored in FP32, FP64 residual refinement around FP32 inner solves.
size_t lsqr_workspace_bytes(sap_ctx *ctx, int64_t m, int n);
// With sp non-null the passes run on that CSR matrix (modes 0 and 1; prob
// then gives only m, n and b).
sap_status run_lsqr(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr,
                    const double *x0, const double *z, double tol, int maxiter, int mode, int max_refine,
                    double *x, sap_info *info, void *work, hipStream_t st, const SparseA *sp = nullptr);
// The iteration-batch graph cache (lsqr.hip), freed with the context.
void batch_graphs_free(sap_ctx *ctx);
constexpr size_t kPinnedBytes = 4096;
// Problems of one sap_solve_batch call: the batched launches index them in a
// grid dimension limited to 65535 blocks.
constexpr int kMaxBatchCount = 65535;

// Heavy-ball momentum (App. D.3) in place of LSQR (lsqr.hip): x0 = R^-1 z,
// step alpha, momentum beta; the LSQR workspace; mode 0 (FP64) or 1 (FP32 A).
// The s-step form of App. D.4.2 (s_steps Krylov steps per block, the
// Chebyshev basis on [lo, hi]); swork: sstep_workspace_bytes(n, s_steps).
size_t sstep_workspace_bytes(int n, int s);
sap_status run_sstep(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *z,
                     double tol, int maxiter, int mode, int s_steps, double lo, double hi, double *x, sap_info *info,
                     void *work, void *swork, hipStream_t s);
sap_status run_hbm(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *z,
                   double tol, int maxiter, int mode, double alpha, double beta, double *x, sap_info *info,
                   void *work, hipStream_t st);

// Served form (batch.hip).
sap_status serve_start(sap_ctx *ctx, size_t arena_bytes, int max_slots);
sap_status serve_submit(sap_ctx *ctx, const sap_problem *p, const sap_params *q, double *x, uint64_t *ticket,
                        hipStream_t stream);
sap_status serve_poll(sap_ctx *ctx, uint64_t ticket, sap_info *info, int wait);
sap_status serve_cancel(sap_ctx *ctx, uint64_t ticket);
sap_status serve_stats(sap_ctx *ctx, int64_t *out);
void serve_destroy(sap_ctx *ctx);

// Batched form (batch.hip).
sap_status run_batch(sap_ctx *ctx, int count, const sap_problem *probs, const sap_params *par, double *const *x,
                     sap_info *infos, hipStream_t user_stream);

}  // namespace sap
