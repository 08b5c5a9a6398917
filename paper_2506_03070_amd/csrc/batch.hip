// Batched sketch-and-precondition: many independent, unevenly sized
// least-squares problems solved together, each phase of Alg. 1 one launch
// over all problems.
//
//   generate : one lane per sketch column of every problem (binary search of
//              the column prefix), stream word = problem index;
//   apply    : one workgroup per (problem, 16-column tile), the tile's d rows
//              in LDS (d <= 2048 for FP32 accumulation, <= 1250 for FP64);
//   QR       : one launch per panel step for all problems (2-D grid:
//              trailing block x problem), shapes from the largest d;
//   LSQR     : per iteration one packed pass over all problems (work items =
//              (problem, row chunk); several short rows per wavefront), then
//              the two chain triangular solves on a (block, problem) grid;
//              the iterations are replayed from a captured hipGraph until a
//              device counter says every problem has stopped.
// The pass reads A in its storage precision (FP32 or FP64) and accumulates
// in FP64 (on gfx950 the FP64 vector rate keeps this pass HBM-bound), except
// for problems in the refinement form (SAP_MODE_MIXED_FP32_REFINE): their
// inner LSQR solves run the pass in FP32 (products, accumulation and u), each
// restart forms the residual r = b - A x with FP64 accumulation, and a
// per-problem device kernel keeps the outer loop (x += delta until
// ||delta|| <= tol ||x||), so one batch can mix both forms.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <tuple>
#include <type_traits>
#include <vector>

#include "common.h"
#include "lsqr_dev.h"
#include "qr_dev.h"
#include "sketch_dev.h"
#include "trsv.h"

namespace sap {

// Per-problem descriptor (device resident).
struct BatchItem {
  const void *A;
  int64_t lda;
  const double *b;
  double *x;
  int64_t m;
  int32_t n, d, zeta, maxiter;
  double tol, h;
  uint64_t seed, stream;
  int64_t col_base;  // prefix of m over the problems (sketch columns)
  int32_t *idx;
  uint64_t *sign;
  double *Y;         // FP64 sketch, d x (n+1), factored in place
  double *tau, *T0, *T1;
  double *Rt, *Dup, *Dlo;
  int *flags;        // 3 * nblk: lower, upper, x0
  LsqrState *st;
  double *u, *y, *v, *w, *p;
  double *qpart, *nrmpart;
  int32_t G, nblk;
  int64_t rows_per_chunk;
  int32_t rank_deficient, pad;
  int32_t refine, max_refine;  // refinement form (FP32 inner solves), its cap (0 = 10)
  double *xprev;               // x before the current inner solve (refinement form)
  // sketch apply in row slices: aslices work items per strip, each over arows
  // rows of [A b]; with more than one, unscaled partial sketches land in
  // Ypart (slice-major, each d x (n+1) column-major) and are summed into Y
  double *Ypart;
  int64_t arows;
  int32_t aslices;
  // A is this form's repacked copy: rows of whole 16-byte vectors whose
  // entries past n are zero, m * lda elements in all
  int32_t zero_pad;
};

// Row slices of a problem's sketch apply: about kApplySliceRows rows each, at
// most kMaxApplySlices, and their partial sketches no larger than half of
// the problem's FP32 A.  Short slices let the one or two requests a served
// round admits spread over many CUs (a request of 1e5 rows and 129 columns
// in strips of 32 makes 5 x 13 work items).
constexpr int64_t kApplySliceRows = 8192;
constexpr int kMaxApplySlices = 32;
inline int apply_slices(int64_t m, int n, int d) {
  int sl = static_cast<int>(std::min<int64_t>(kMaxApplySlices, (m + kApplySliceRows - 1) / kApplySliceRows));
  while (sl > 1 && static_cast<double>(sl) * (n + 1) * d * 8.0 > 2.0 * static_cast<double>(m) * n) --sl;
  return std::max(1, sl);
}

namespace {

using namespace qr_dev;

constexpr double kInnerTolF32 = 0x1p-23;  // FP32 resolution of the inner solves' test

constexpr int kBThreads = 1024;
constexpr int kBWaves = kBThreads / kWave;
constexpr size_t kBatchLds = 160000;  // LDS bytes for the sketch strip of one workgroup
constexpr int kXcdsB = 8;

// ---- generate --------------------------------------------------------------
template <int ZMAX>
__global__ __launch_bounds__(256) void batch_generate_kernel(const BatchItem *__restrict__ items, int count,
                                                             int64_t total, int *__restrict__ err) {
  const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= total) return;
  int lo = 0, hi = count - 1;  // last item with col_base <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].col_base <= g) lo = mid;
    else hi = mid - 1;
  }
  const BatchItem &it = items[lo];
  sketch_dev::generate_column<ZMAX>(g - it.col_base, it.d, it.zeta, it.seed, it.stream, it.idx, it.sign, err);
}

// ---- apply -----------------------------------------------------------------
// Work item = (problem, strip of W columns, row slice): the strip of Y (d + 1
// spare rows by W columns) is accumulated in FP64 in LDS over the slice's
// rows; a problem of one slice writes h times it into Y, otherwise into its
// slice of Ypart (summed by batch_apply_reduce_kernel).  work.y packs the
// strip (low 20 bits) and the slice.
template <typename TA, int W>
__global__ __launch_bounds__(kBThreads) void batch_apply_kernel(const BatchItem *__restrict__ items,
                                                                const int2 *__restrict__ work, int nwork) {
  using TY = double;
  constexpr int kTileColsB = W;
  extern __shared__ unsigned char lds_raw[];
  TY *acc = reinterpret_cast<TY *>(lds_raw);
  const int per_xcd = (nwork + kXcdsB - 1) / kXcdsB;
  const int wi = (blockIdx.x % kXcdsB) * per_xcd + blockIdx.x / kXcdsB;
  if (wi >= nwork) return;
  const int2 wk = work[wi];
  const BatchItem &it = items[wk.x];
  const int strip = wk.y & 0xFFFFF, slice = wk.y >> 20;
  const int c0 = strip * kTileColsB;
  const int d = it.d, n = it.n, ncols = it.n + 1, zeta = it.zeta;
  const gmem<TA> *__restrict__ A = gview(static_cast<const TA *>(it.A));
  const gmem<double> *__restrict__ bvec = gview(it.b);
  const gmem<uint64_t> *__restrict__ sgn = gview(it.sign);
  const gmem<int32_t> *__restrict__ idx = gview(it.idx);
  for (int e = threadIdx.x; e < (d + 1) * kTileColsB; e += kBThreads) acc[e] = TY(0);
  __syncthreads();
  // One row of [A b] per group of 16 lanes: its 16-column piece is loaded
  // once and added into the zeta target rows; all loads of a batch of rows
  // are issued before the adds.
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  constexpr int RPW = kWave / kTileColsB;  // rows per wave instruction
  const int g = lane / kTileColsB, c = lane % kTileColsB;
  const int col = c0 + c;
  const bool col_a = col < n, col_b = col == n;
  const int64_t r_lo = static_cast<int64_t>(slice) * it.arows;
  const int64_t m = min(it.m, r_lo + it.arows);  // end of this slice's rows
  constexpr int U = 8;
  constexpr int64_t kStride = static_cast<int64_t>(kBWaves) * RPW * U;
  const bool fast = zeta == 8 && (reinterpret_cast<uintptr_t>(it.idx) % 16 == 0);
  for (int64_t base = r_lo + static_cast<int64_t>(wave) * RPW * U + g; base < m; base += kStride) {
    if (fast) {
      TY val[U];
      uint32_t sg[U];
      typedef int iv4 __attribute__((ext_vector_type(4)));
      iv4 ix[U][2];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t i0 = base + u * RPW;
        const bool ok = i0 < m;
        const int64_t i = ok ? i0 : m - 1;
        TY a = TY(0);
        if (col_a) a = static_cast<TY>(A[i * it.lda + col]);
        else if (col_b) a = static_cast<TY>(bvec[i]);
        val[u] = ok ? a : TY(0);
        sg[u] = static_cast<uint32_t>(sgn[i]);
        const gmem<iv4> *ip = reinterpret_cast<const gmem<iv4> *>(idx + i * 8);
        ix[u][0] = ip[0];
        ix[u][1] = ip[1];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int rr[8] = {ix[u][0].x, ix[u][0].y, ix[u][0].z, ix[u][0].w,
                           ix[u][1].x, ix[u][1].y, ix[u][1].z, ix[u][1].w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int r = static_cast<unsigned>(rr[k]) < static_cast<unsigned>(d) ? rr[k] : d;  // spare row
          atomicAdd(acc + r * kTileColsB + c, ((sg[u] >> k) & 1u) ? val[u] : -val[u]);
        }
      }
    } else {
      for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * RPW;
        if (i >= m) break;
        TY a = TY(0);
        if (col_a) a = static_cast<TY>(A[i * it.lda + col]);
        else if (col_b) a = static_cast<TY>(bvec[i]);
        const uint64_t sg = sgn[i];
        const gmem<int32_t> *ri = idx + i * zeta;
        for (int k0 = 0; k0 < zeta; k0 += 4) {
          int rr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) rr[q] = (k0 + q < zeta) ? ri[k0 + q] : -1;
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (static_cast<unsigned>(rr[q]) < static_cast<unsigned>(d))
              atomicAdd(acc + rr[q] * kTileColsB + c, ((sg >> (k0 + q)) & 1ull) ? a : -a);
        }
      }
    }
  }
  __syncthreads();
  const bool direct = it.aslices <= 1;
  double *Y = direct ? it.Y : it.Ypart + static_cast<int64_t>(slice) * d * ncols;
  const TY hs = direct ? static_cast<TY>(it.h) : TY(1);
  for (int e = threadIdx.x; e < d * kTileColsB; e += kBThreads) {
    const int q = e / d, r = e % d;
    const int cc = c0 + q;
    if (cc < ncols) Y[r + static_cast<int64_t>(cc) * d] = acc[r * kTileColsB + q] * hs;
  }
}

// Y = h * (sum of the slice partials, slice order) for the problems whose
// apply ran in several row slices.  Grid: (element blocks of 256, problems).
__global__ __launch_bounds__(256) void batch_apply_reduce_kernel(const BatchItem *__restrict__ items) {
  const BatchItem &it = items[blockIdx.y];
  if (it.aslices <= 1) return;
  const int64_t tot = static_cast<int64_t>(it.d) * (it.n + 1);
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= tot) return;
  double s = 0.0;
  for (int k = 0; k < it.aslices; ++k) s += it.Ypart[k * tot + e];
  it.Y[e] = s * it.h;
}

// ---- QR ----------------------------------------------------------------------
template <int S, int NB>
__global__ __launch_bounds__(kPanelThreads) void batch_qr_first_kernel(const BatchItem *__restrict__ items) {
  __shared__ PanelShared<NB> sh;
  const BatchItem &it = items[blockIdx.x];
  const int rows = it.d, cols = it.n + 1;
  const int nb = cols < NB ? cols : NB;
  double P[S][NB];
  load_block<S, NB>(it.Y, rows, 0, rows, 0, nb, P);
  factor_panel<S, NB>(P, sh, nb, rows, 0, 0, it.tau, it.T0);
  store_block<S, NB>(it.Y, rows, 0, rows, 0, nb, P);
}

template <int S, int NB>
__global__ __launch_bounds__(kPanelThreads) void batch_qr_step_kernel(const BatchItem *__restrict__ items, int step) {
  __shared__ PanelShared<NB> sh;
  const BatchItem &it = items[blockIdx.y];
  const int rows = it.d, cols = it.n + 1;
  const int k0 = step * NB;
  const int nb = min(NB, cols - k0);
  if (nb <= 0 || k0 + nb >= cols) return;  // no trailing columns at this step
  const int trailing = cols - (k0 + nb);
  if (static_cast<int>(blockIdx.x) * NB >= trailing) return;
  const int c0 = k0 + nb + static_cast<int>(blockIdx.x) * NB;
  const int ncb = min(NB, cols - c0);
  const int dr = rows - k0;
  const double *Tcur = (step & 1) ? it.T1 : it.T0;
  double *Tnext = (step & 1) ? it.T0 : it.T1;
  double C[S][NB];
  load_block<S, NB>(it.Y, rows, k0, dr, c0, ncb, C);
  apply_panel_qt<S, NB>(it.Y, rows, dr, k0, nb, Tcur, C, ncb, sh);
  if (blockIdx.x == 0) factor_panel<S, NB>(C, sh, ncb, rows - c0, c0 - k0, c0, it.tau, Tnext);
  store_block<S, NB>(it.Y, rows, k0, dr, c0, ncb, C);
}

__global__ __launch_bounds__(256) void batch_rank_kernel(BatchItem *__restrict__ items) {
  __shared__ double smax[4], smin[4];
  BatchItem &it = items[blockIdx.x];
  double mx = 0.0, mn = INFINITY;
  for (int k = threadIdx.x; k < it.n; k += 256) {
    const double a = fabs(it.Y[k + static_cast<int64_t>(k) * it.d]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
  mx = wave_max(mx);
  mn = -wave_max(-mn);
  if ((threadIdx.x & 63) == 0) {
    smax[threadIdx.x / 64] = mx;
    smin[threadIdx.x / 64] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < 4; ++w) {
      mx = fmax(mx, smax[w]);
      mn = fmin(mn, smin[w]);
    }
    it.rank_deficient = !(mn > static_cast<double>(it.d) * 0x1p-53 * mx);
  }
}

// ---- triangular-solve preparation and x0 ------------------------------------
__global__ __launch_bounds__(256) void batch_trsv_prepare_kernel(const BatchItem *__restrict__ items) {
  __shared__ TrsvPrepShared sh;
  const BatchItem &it = items[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= it.nblk) return;
  trsv_invert_diag_block(it.Y, it.d, it.n, static_cast<int>(blockIdx.x), it.Dup, it.Dlo, sh);
}

__global__ __launch_bounds__(256) void batch_transpose_kernel(const BatchItem *__restrict__ items) {
  __shared__ double tile[32][33];
  const BatchItem &it = items[blockIdx.z];
  const int nt = (it.n + 31) / 32;
  if (static_cast<int>(blockIdx.x) >= nt || static_cast<int>(blockIdx.y) >= nt) return;
  trsv_transpose_tile(it.Y, it.d, it.n, static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y), it.Rt, tile);
}

// Fresh LSQR state, cleared flags, ||b||.
__global__ __launch_bounds__(1024) void batch_init_kernel(const BatchItem *__restrict__ items) {
  __shared__ double scr[16];
  const BatchItem &it = items[blockIdx.x];
  for (int i = threadIdx.x; i < 3 * it.nblk; i += 1024) it.flags[i] = 0;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < it.m; i += 1024) s += it.b[i] * it.b[i];
  s = wg_sum(s, scr);
  if (threadIdx.x == 0) {
    LsqrState *st = it.st;
    st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
    st->alpha_new = st->beta_new = 0.0;
    st->c_ap = -1.0;
    st->c_u = 1.0;
    st->normb = sqrt(s);
    st->tol = it.tol;
    st->resid_est = st->normar_est = 0.0;
    st->iter = 0;
    st->maxiter = it.maxiter;
    st->done = it.rank_deficient ? 1 : 0;
    st->converged = 0;
    st->init = 1;
    st->proceed = 0;
    st->total_iters = 0;
    st->steps = 0;
    st->rel = it.refine ? 1 : 0;
    if (it.refine) st->tol = kInnerTolF32;
    st->refine = it.refine;
    st->refinements = 0;
    st->max_refine = it.max_refine > 0 ? it.max_refine : 10;
    st->final_done = it.rank_deficient ? 1 : 0;
    st->target = it.tol;
    st->prev_delta = INFINITY;
  }
}

// x0 = R^-1 z (z = column n of the factored sketch), chain over the blocks.
__global__ __launch_bounds__(kTrsvThreads) void batch_x0_kernel(const BatchItem *__restrict__ items, int *err) {
  __shared__ LowerShared sh;
  const BatchItem &it = items[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= it.nblk) return;
  if (it.rank_deficient) return;
  const int n = it.n;
  const int b = it.nblk - 1 - static_cast<int>(blockIdx.x);
  const double *z = it.Y + static_cast<int64_t>(n) * it.d;
  if (threadIdx.x < kTrsvB) {
    const int row = b * kTrsvB + threadIdx.x;
    sh.rb[threadIdx.x] = row < n ? z[row] : 0.0;
  }
  __syncthreads();
  chain_block<true>(it.Y, it.d, n, it.Dup, it.x, it.flags + 2 * it.nblk, 1, b, sh.rb, sh.red, err);
}

// ---- repacking of unaligned rows -------------------------------------------
// A problem whose rows do not start on 16-byte boundaries (lda not a multiple
// of 16 / element size, or A itself unaligned) can only be read element by
// element.  Before the solve its rows are copied once into a buffer with
// lda_pad = n rounded up to 16 bytes, so that every pass reads it with
// 16-byte loads; the columns past n are never read.
struct RepackJob {
  const void *src;
  int64_t lda_src;
  void *dst;
  int64_t lda_dst;
  int64_t m;
  int32_t n, pad;
};
constexpr int kRepackRows = 256;  // rows per work item

template <typename TA>
__global__ __launch_bounds__(256) void batch_repack_kernel(const RepackJob *__restrict__ jobs,
                                                           const int2 *__restrict__ work) {
  constexpr int V = 16 / static_cast<int>(sizeof(TA));
  typedef TA vec_t __attribute__((ext_vector_type(V)));
  const int2 wk = work[blockIdx.x];
  const RepackJob &jb = jobs[wk.x];
  const TA *__restrict__ src = static_cast<const TA *>(jb.src);
  TA *__restrict__ dst = static_cast<TA *>(jb.dst);
  const int n = jb.n;
  const int nv = (n + V - 1) / V;  // vectors per row
  const int64_t r0 = static_cast<int64_t>(wk.y) * kRepackRows;
  const int64_t r1 = min(jb.m, r0 + kRepackRows);
  const int64_t total = (r1 - r0) * nv;
  for (int64_t e = threadIdx.x; e < total; e += 256) {
    const int64_t row = r0 + e / nv;
    const int c = static_cast<int>(e % nv) * V;
    vec_t v;
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] = c + q < n ? src[row * jb.lda_src + c + q] : TA(0);
    *reinterpret_cast<vec_t *>(dst + row * jb.lda_dst + c) = v;
  }
}

// ---- LSQR iteration -----------------------------------------------------------
// Packed pass: L lanes serve one row (L = the power of two covering n/VEC,
// at most 64, chosen per problem), so a wavefront handles 64/L rows at once.
// u <- c_ap (A p) + c_u u_in with FP64 accumulation; q += u_i A[i, :].
// At the initialisation step (st->init) the pass reads u_in = b and p = x.
// p sits in LDS (read per element), q in registers; the waves' q partials
// are combined through one LDS vector in wave order.
// PF: 512-thread workgroups with two row groups in flight per wave (the next
// group's loads issued before the current one is reduced); otherwise 1024
// threads and one group at a time.  The served form, whose rounds hold a few
// large requests, uses PF; the batched form, many small problems, the other
// (more waves to cover the per-row shuffles).
// The body of the pass for compute type TC (FP64, or FP32 in the inner
// solves of the refinement form) and u storage type TU (FP32 in the
// refinement form, whose residual pass computes in FP64 and rounds u).
// v plus the value of another lane of its row of 16, chosen by a DPP
// control: 0xB1 (quad_perm 1,0,3,2: lane ^ 1), 0x4E (quad_perm 2,3,0,1:
// lane ^ 2), 0x141 (row_half_mirror: lane 7 - i within 8, the other quad),
// 0x140 (row_mirror: lane 15 - i within 16, the other half).  A VALU move,
// no LDS round trip.
template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int mlo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xF, 0xF, false);
  const int mhi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(mhi, mlo);
}

template <typename TA, typename TC, typename TU, int VEC, int KJ, int U, bool PF, int TH>
__device__ __forceinline__ void batch_pass_body(const BatchItem &it, int chunk, int tune, TC *psh, TC *qacc,
                                                double *nsh) {
  constexpr int NW = TH / kWave;
  const LsqrState *st = it.st;
  const int n = it.n;
  const bool init = st->init != 0;
  const double *__restrict__ pv = init ? it.x : it.p;
  const gmem<TU> *__restrict__ uin = init ? nullptr : gview(reinterpret_cast<const TU *>(it.u));
  const gmem<double> *__restrict__ bin = gview(it.b);
  gmem<TU> *uout = gview(reinterpret_cast<TU *>(it.u));
  const TC c_ap = static_cast<TC>(st->c_ap), c_u = static_cast<TC>(st->c_u);
  // kje (<= KJ) vectors of a row per lane, on L lanes: fewer vectors per
  // lane while a row would otherwise sit on fewer than 8 lanes, so that each
  // load instruction reads whole 128-byte lines of a short row.
  int kje = KJ, L = 1;
  for (;;) {
    L = 1;
    while (L * VEC * kje < n && L < 64) L <<= 1;
    if (L >= 8 || kje == 1) break;
    kje >>= 1;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int slot = lane / L, sub = lane % L;
  const int RS = kWave / L;  // rows per wavefront step
  const gmem<TA> *__restrict__ A = gview(static_cast<const TA *>(it.A));
  const int64_t lda = it.lda;

  for (int c = threadIdx.x; c < 64 * VEC * KJ; c += TH) {
    psh[c] = c < n ? static_cast<TC>(pv[c]) : TC(0);
    qacc[c] = TC(0);
  }
  __syncthreads();
  TC q[KJ][VEC];
#pragma unroll
  for (int j = 0; j < KJ; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) q[j][e] = TC(0);
  const int64_t r0 = static_cast<int64_t>(chunk) * it.rows_per_chunk;
  const int64_t r1 = min(it.m, r0 + it.rows_per_chunk);
  double nrm = 0.0;
  const int64_t gstride = static_cast<int64_t>(NW) * RS * U;
  // Loads without per-lane branches: a row past the chunk reads the chunk's
  // last row (its results are dropped), a lane past the row's whole vectors
  // reads the last whole vector (its p entries are zero and its q sums are
  // never stored).  Only the vector that straddles n (n % VEC != 0) is read
  // element by element, unless the rows are zero-padded to whole vectors.
  const bool straddle = (n % VEC) != 0 && !it.zero_pad;
  const int cf = (it.zero_pad ? n + VEC - 1 : n) / VEC * VEC;  // columns read as whole vectors
  const int clast = cf - VEC;  // start of the last whole vector (< 0: none)
  auto load_group = [&](int64_t base, TA (&a)[U][KJ][VEC], TC (&ui)[U]) {
#pragma unroll
    for (int uu = 0; uu < U; ++uu) {
      const int64_t row = base + uu * RS + slot;
      const int64_t rowc = row < r1 ? row : r1 - 1;
      const gmem<TA> *arow = A + rowc * lda;
#pragma unroll
      for (int j = 0; j < KJ; ++j) {
        if (j > 0 && j >= kje) break;
        const int c = (sub + L * j) * VEC;
        if (clast >= 0) {
          load_stream<TA, VEC>(arow + min(c, clast), a[uu][j]);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[uu][j][e] = TA(0);
        }
        if (straddle && c == cf) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[uu][j][e] = (c + e < n) ? __builtin_nontemporal_load(arow + c + e) : TA(0);
        }
      }
      ui[uu] = init ? static_cast<TC>(bin[rowc]) : static_cast<TC>(uin[rowc]);
    }
  };
  // u_i <- c_ap (A_i p) + c_u u_i and q += u_i A_i for row i.
  auto update_row = [&](int64_t row, TC s, TA (&ar)[KJ][VEC], TC ui) {
    if (row >= r1) return;
    const TC uh = c_ap * s + c_u * ui;
    const TU us = static_cast<TU>(uh);
#pragma unroll
    for (int j = 0; j < KJ; ++j) {
      if (j > 0 && j >= kje) break;
#pragma unroll
      for (int e = 0; e < VEC; ++e) q[j][e] += static_cast<TC>(us) * static_cast<TC>(ar[j][e]);
    }
    if (sub == 0) {
      if (!tune) uout[row] = us;
      nrm += static_cast<double>(us) * static_cast<double>(us);
    }
  };
  auto dot_row = [&](TA (&ar)[KJ][VEC]) {
    TC s = TC(0);
#pragma unroll
    for (int j = 0; j < KJ; ++j) {
      if (j > 0 && j >= kje) break;
#pragma unroll
      for (int e = 0; e < VEC; ++e) s += static_cast<TC>(ar[j][e]) * psh[(sub + L * j) * VEC + e];
    }
    return s;
  };
  // Each row's dot product is reduced over its L lanes.  With 512 threads
  // (registers to spare) the U rows of a group are reduced together, one
  // cross-lane round trip per step for all of them; with 1024 threads (128
  // registers) one row at a time, which keeps fewer values live.
  auto compute_group = [&](int64_t base, TA (&a)[U][KJ][VEC], TC (&ui)[U]) {
    if constexpr (TH <= 512) {
      TC s[U];
#pragma unroll
      for (int uu = 0; uu < U; ++uu) s[uu] = dot_row(a[uu]);
      // within a row of 16 lanes by DPP moves (the L lanes of a row are
      // aligned), beyond it by cross-lane shuffles
      if (L >= 2) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) s[uu] = dpp_add<0xB1>(s[uu]);
      }
      if (L >= 4) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) s[uu] = dpp_add<0x4E>(s[uu]);
      }
      if (L >= 8) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) s[uu] = dpp_add<0x141>(s[uu]);
      }
      if (L >= 16) {
#pragma unroll
        for (int uu = 0; uu < U; ++uu) s[uu] = dpp_add<0x140>(s[uu]);
      }
      for (int off = 16; off < L; off <<= 1) {
        TC t[U];
#pragma unroll
        for (int uu = 0; uu < U; ++uu) t[uu] = __shfl_xor(s[uu], off, kWave);
#pragma unroll
        for (int uu = 0; uu < U; ++uu) s[uu] += t[uu];
      }
#pragma unroll
      for (int uu = 0; uu < U; ++uu) update_row(base + uu * RS + slot, s[uu], a[uu], ui[uu]);
    } else {
#pragma unroll
      for (int uu = 0; uu < U; ++uu) {
        TC s = dot_row(a[uu]);
        for (int off = L >> 1; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
        update_row(base + uu * RS + slot, s, a[uu], ui[uu]);
      }
    }
  };
  int64_t base = r0 + static_cast<int64_t>(wave) * RS * U;
  if constexpr (PF) {
    TA a0[U][KJ][VEC], a1[U][KJ][VEC];
    TC u0[U], u1[U];
    if (base < r1) load_group(base, a0, u0);
    for (; base < r1; base += 2 * gstride) {
      if (base + gstride < r1) load_group(base + gstride, a1, u1);
      compute_group(base, a0, u0);
      if (base + gstride < r1) {
        if (base + 2 * gstride < r1) load_group(base + 2 * gstride, a0, u0);
        compute_group(base + gstride, a1, u1);
      }
    }
  } else {
    for (; base < r1; base += gstride) {
      TA a[U][KJ][VEC];
      TC ui[U];
      load_group(base, a, ui);
      compute_group(base, a, ui);
    }
  }
  // combine the row slots of the wavefront (lanes with equal `sub`), then
  // waves; as above, all values per step where registers allow
  if constexpr (TH <= 512) {
    for (int off = L; off < kWave; off <<= 1) {
      TC t[KJ][VEC];
#pragma unroll
      for (int j = 0; j < KJ; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) t[j][e] = __shfl_xor(q[j][e], off, kWave);
#pragma unroll
      for (int j = 0; j < KJ; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) q[j][e] += t[j][e];
    }
  } else {
#pragma unroll
    for (int j = 0; j < KJ; ++j)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        TC v = q[j][e];
        for (int off = L; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
        q[j][e] = v;
      }
  }
  nrm = wave_sum(nrm);
  if (lane == 0) nsh[wave] = nrm;
  for (int w = 0; w < NW; ++w) {
    if (wave == w && slot == 0) {
#pragma unroll
      for (int j = 0; j < KJ; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) qacc[(sub + L * j) * VEC + e] += q[j][e];
    }
    __syncthreads();
  }
  gmem<double> *qdst = gview(it.qpart) + static_cast<int64_t>(chunk) * n;
  for (int c = threadIdx.x; c < n; c += TH) qdst[c] = static_cast<double>(qacc[c]);
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < NW; ++w) sum += nsh[w];
    gview(it.nrmpart)[chunk] = sum;
  }
}

// Packed pass: L lanes serve one row (L = the power of two covering n/VEC,
// at most 64, chosen per problem), so a wavefront handles 64/L rows at once.
// u <- c_ap (A p) + c_u u_in; q += u_i A[i, :].  At the initialisation step
// (st->init) the pass reads u_in = b and p = x.  p sits in LDS (read per
// element), q in registers; the waves' q partials are combined through one
// LDS vector in wave order.  FP64 arithmetic, except the inner solves of the
// refinement form (FP32 arithmetic and u; their residual pass is FP64 with u
// rounded to FP32).
// PF: 512-thread workgroups with two row groups in flight per wave (the next
// group's loads issued before the current one is reduced); otherwise 1024
// threads and one group at a time.  The served form, whose rounds hold a few
// large requests, uses PF; the batched form, many small problems, the other
// (more waves to cover the per-row shuffles).
// skip_inner: the FP32 inner passes of the refinement form are left to
// batch_pass_inner_kernel (launched after this one), whose single FP32 code
// path needs far fewer registers than this kernel's FP64 ones.
template <typename TA, int VEC, int KJ, int U, bool PF>
__global__ __launch_bounds__(PF ? 512 : kBThreads) void batch_pass_kernel(const BatchItem *__restrict__ items,
                                                                          const int2 *__restrict__ work, int nwork,
                                                                          int tune, int skip_inner) {
  constexpr int TH = PF ? 512 : kBThreads;
  constexpr int NW = TH / kWave;
  __shared__ double psh[64 * VEC * KJ];
  __shared__ double qacc[64 * VEC * KJ];
  __shared__ double nsh[NW];
  const int2 wk = work[blockIdx.x];
  const BatchItem &it = items[wk.x];
  const LsqrState *st = it.st;
  if (st->done && !tune) return;
  if (!it.refine)
    batch_pass_body<TA, double, double, VEC, KJ, U, PF, TH>(it, wk.y, tune, psh, qacc, nsh);
  else if (st->init)
    batch_pass_body<TA, double, float, VEC, KJ, U, PF, TH>(it, wk.y, tune, psh, qacc, nsh);
  else if (!skip_inner)
    batch_pass_body<TA, float, float, VEC, KJ, U, PF, TH>(it, wk.y, tune, reinterpret_cast<float *>(psh),
                                                          reinterpret_cast<float *>(qacc), nsh);
}

// The FP32 inner passes of the refinement form alone (FP32 A, arithmetic and
// u): 512-thread workgroups, two row groups in flight per wave.  Items of
// other kinds return at once (batch_pass_kernel takes them).
template <int VEC, int KJ, int U>
__global__ __launch_bounds__(512) void batch_pass_inner_kernel(const BatchItem *__restrict__ items,
                                                               const int2 *__restrict__ work, int nwork) {
  constexpr int NW = 512 / kWave;
  __shared__ double psh[64 * VEC * KJ];
  __shared__ double qacc[64 * VEC * KJ];
  __shared__ double nsh[NW];
  const int2 wk = work[blockIdx.x];
  const BatchItem &it = items[wk.x];
  const LsqrState *st = it.st;
  if (st->done || !it.refine || st->init) return;
  batch_pass_body<float, float, float, VEC, KJ, U, true, 512>(it, wk.y, 0, reinterpret_cast<float *>(psh),
                                                              reinterpret_cast<float *>(qacc), nsh);
}

__global__ __launch_bounds__(kTrsvThreads) void batch_lower_kernel(const BatchItem *__restrict__ items, int *err) {
  __shared__ LowerShared sh;
  const BatchItem &it = items[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= it.nblk) return;
  LsqrState *st = it.st;
  if (st->done) return;
  const int n = it.n, b = blockIdx.x;
  const int epoch = st->steps + 1;
  reduce_q_block(it.qpart, it.G, n, b, sh);
  chain_block<false>(it.Rt, n, n, it.Dlo, it.y, it.flags, epoch, b, sh.rb, sh.red, err);
  if (b != it.nblk - 1) return;
  lower_epilogue(n, it.G, it.nrmpart, it.y, it.v, st, sh);
}

__global__ __launch_bounds__(kTrsvThreads) void batch_upper_kernel(const BatchItem *__restrict__ items, int *err,
                                                                   int *done_count) {
  __shared__ LowerShared sh;
  const BatchItem &it = items[blockIdx.y];
  if (static_cast<int>(blockIdx.x) >= it.nblk) return;
  LsqrState *st = it.st;
  if (st->done) return;
  const int n = it.n;
  const int b = it.nblk - 1 - static_cast<int>(blockIdx.x);
  const int epoch = st->steps + 1;
  if (threadIdx.x < kTrsvB) {
    const int row = b * kTrsvB + threadIdx.x;
    sh.rb[threadIdx.x] = row < n ? it.v[row] : 0.0;
  }
  __syncthreads();
  chain_block<true>(it.Y, it.d, n, it.Dup, it.p, it.flags + it.nblk, epoch, b, sh.rb, sh.red, err);
  if (b != 0) return;
  upper_epilogue(n, it.p, it.w, it.x, st, it.refine ? nullptr : done_count);
}

// The outer loop of the refinement form, after each iteration: for every
// problem whose inner solve has just stopped, compare the correction it made
// with x.  Converged (||x - x_prev|| <= tol ||x||, which includes a restart
// that found r or (A M)^T r exactly zero), stagnated (a correction no smaller
// than the previous one: the FP32 inner solves cannot resolve the remaining
// error), out of iterations or out of refinements: the problem is finished
// and counted in *done_count.  Otherwise x_prev = x and the LSQR state
// restarts with an initialisation step, whose pass forms the FP64 residual
// of the current x.  The flag epochs (steps) keep counting.
__global__ __launch_bounds__(1024) void batch_refine_kernel(const BatchItem *__restrict__ items, int *done_count) {
  __shared__ double scr[16];
  __shared__ int restart;
  const BatchItem &it = items[blockIdx.x];
  if (!it.refine) return;
  LsqrState *st = it.st;
  if (!st->done || st->final_done) return;
  const int n = it.n;
  double a = 0.0, bb = 0.0;
  for (int c = threadIdx.x; c < n; c += 1024) {
    const double xc = it.x[c];
    const double dx = xc - it.xprev[c];
    a += dx * dx;
    bb += xc * xc;
  }
  a = sqrt(wg_sum(a, scr));
  bb = sqrt(wg_sum(bb, scr));
  if (threadIdx.x == 0) {
    const int nref = st->refinements + 1;
    st->refinements = nref;
    const bool conv = a <= st->target * bb;
    const bool give_up = a >= st->prev_delta || st->total_iters >= st->maxiter || nref >= st->max_refine;
    if (conv || give_up) {
      st->converged = conv ? 1 : 0;
      st->final_done = 1;
      atomicAdd(done_count, 1);
      restart = 0;
    } else {
      st->prev_delta = a;
      st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
      st->alpha_new = st->beta_new = 0.0;
      st->c_ap = -1.0;
      st->c_u = 1.0;
      st->resid_est = st->normar_est = 0.0;
      st->iter = 0;
      st->converged = 0;
      st->proceed = 0;
      st->init = 1;
      st->done = 0;
      restart = 1;
    }
  }
  __syncthreads();
  if (restart)
    for (int c = threadIdx.x; c < n; c += 1024) it.xprev[c] = it.x[c];
}

// x_prev = x0 for the problems in the refinement form (after the x0 solve).
__global__ __launch_bounds__(256) void batch_save_x_kernel(const BatchItem *__restrict__ items) {
  const BatchItem &it = items[blockIdx.x];
  if (!it.refine || it.rank_deficient) return;
  for (int c = threadIdx.x; c < it.n; c += 256) it.xprev[c] = it.x[c];
}

__global__ void batch_count_rank_kernel(const BatchItem *__restrict__ items, int count, int *done_count) {
  if (threadIdx.x != 0) return;
  int c = 0;
  for (int k = 0; k < count; ++k) c += items[k].rank_deficient ? 1 : 0;
  *done_count = c;
}

// done[k] = problem k has stopped (served form).
__global__ void serve_done_kernel(const BatchItem *__restrict__ items, int count, int *__restrict__ done) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) done[k] = items[k].refine ? items[k].st->final_done : items[k].st->done;
}

template <int S, int NB>
void launch_batch_qr(const BatchItem *items, int count, int max_cols, hipStream_t st) {
  batch_qr_first_kernel<S, NB><<<count, kPanelThreads, 0, st>>>(items);
  const int nsteps = (max_cols + NB - 1) / NB;
  for (int step = 0; step < nsteps; ++step) {
    const int trailing = max_cols - step * NB - NB;
    if (trailing <= 0) break;
    const int blocks = (trailing + NB - 1) / NB;
    batch_qr_step_kernel<S, NB><<<dim3(blocks, count), kPanelThreads, 0, st>>>(items, step);
  }
}

struct PassChoice {
  const void *fn;
  int vec, kj;
  int threads;
  const void *inner_fn = nullptr;  // FP32 inner passes of the refinement form (FP32 A only)
};

// E = KJ * VEC elements of a row per lane: 8 while the widest problem has
// at most 512 columns, else 16; a problem of n columns puts L = n/E lanes
// (rounded up to a power of two) on a row, so a wavefront works on 64/L rows
// at once.
// U = row groups in flight per lane, as many as the registers allow without
// spilling (the per-element loads of an unaligned row each need an address).
template <typename TA>
PassChoice pick_batch_pass(int n_max, bool aligned, bool pf) {
  constexpr int vmax = 16 / static_cast<int>(sizeof(TA));
  constexpr bool f32 = sizeof(TA) == 4;
  auto fn = [](auto kernel) { return reinterpret_cast<const void *>(kernel); };
  const int th = pf ? 512 : kBThreads;
  PassChoice c;
  if (n_max <= 512) {
    if (aligned) {
      c = {pf ? fn(&batch_pass_kernel<TA, vmax, 8 / vmax, f32 ? 4 : 2, true>)
              : fn(&batch_pass_kernel<TA, vmax, 8 / vmax, f32 ? 4 : 2, false>), vmax, 8 / vmax, th};
      c.inner_fn = fn(&batch_pass_inner_kernel<vmax, 8 / vmax, f32 ? 4 : 2>);
    } else {
      c = {pf ? fn(&batch_pass_kernel<TA, 1, 8, 2, true>) : fn(&batch_pass_kernel<TA, 1, 8, 2, false>), 1, 8, th};
      c.inner_fn = fn(&batch_pass_inner_kernel<1, 8, 2>);
    }
  } else if (aligned) {
    c = {pf ? fn(&batch_pass_kernel<TA, vmax, 16 / vmax, f32 ? 2 : 1, true>)
            : fn(&batch_pass_kernel<TA, vmax, 16 / vmax, f32 ? 2 : 1, false>), vmax, 16 / vmax, th};
    c.inner_fn = fn(&batch_pass_inner_kernel<vmax, 16 / vmax, f32 ? 2 : 1>);
  } else {
    c = {pf ? fn(&batch_pass_kernel<TA, 1, 16, 1, true>) : fn(&batch_pass_kernel<TA, 1, 16, 1, false>), 1, 16, th};
    c.inner_fn = fn(&batch_pass_inner_kernel<1, 16, 1>);
  }
  if (!f32) c.inner_fn = nullptr;  // the refinement form needs FP32 A
  return c;
}

// One pass over every work item.  split (when some problem is in the
// refinement form): its FP32 inner passes run in batch_pass_inner_kernel.
void launch_pass_fn(const PassChoice &pc, const BatchItem *items, const int2 *work, int nwork, int tune,
                    hipStream_t st, bool split = false) {
  const BatchItem *it_ = items;
  const int2 *w_ = work;
  int nw = nwork, tn = tune;
  const bool sp = split && pc.inner_fn && !tune;
  int skip = sp ? 1 : 0;
  void *args[] = {&it_, &w_, &nw, &tn, &skip};
  (void)hipLaunchKernel(pc.fn, dim3(nwork), dim3(pc.threads), args, 0, st);
  if (sp) {
    void *iargs[] = {&it_, &w_, &nw};
    (void)hipLaunchKernel(pc.inner_fn, dim3(nwork), dim3(512), iargs, 0, st);
  }
}

}  // namespace

// ----------------------------------------------------------------------------
// Shared pieces of the batched and served forms.

// Strip width of the batched sketch apply: the widest power of two (4..32)
// whose FP64 strip of d_max + 1 rows fits in the LDS budget.
int batch_apply_width(int d_max) {
  int w = 32;
  while (w > 4 && static_cast<size_t>(d_max + 1) * w * sizeof(double) > kBatchLds) w /= 2;
  return w;
}

// Bytes of one problem's workspace (rows_per_chunk >= kMinRowsPerChunk).
constexpr int64_t kMinRowsPerChunk = 1024;

size_t item_bytes(int64_t m, int n, int d, int zeta, sap_dtype at) {
  (void)at;
  const int nc = n + 1;
  const int nblk = (n + kTrsvB - 1) / kTrsvB;
  const int64_t gmax = (m + kMinRowsPerChunk - 1) / kMinRowsPerChunk;
  size_t b = 0;
  b += 256 + sizeof(int32_t) * m * zeta;
  b += 256 + sizeof(uint64_t) * m;
  b += 256 + sizeof(double) * d * nc;
  b += 256 + sizeof(double) * nc;             // tau, one per column
  b += 2 * (256 + sizeof(double) * 256);      // T of two panels (NB x NB <= 256)
  b += 256 + sizeof(double) * n * n;
  b += 2 * (256 + sizeof(double) * nblk * kTrsvB * kTrsvB);
  b += 256 + sizeof(int) * 3 * nblk;
  b += 256 + sizeof(LsqrState);
  b += 256 + sizeof(double) * m;
  b += 5 * (256 + sizeof(double) * n);
  b += 256 + sizeof(double) * gmax * n;
  b += 256 + sizeof(double) * gmax;
  const int sl = apply_slices(m, n, d);
  if (sl > 1) b += 256 + sizeof(double) * static_cast<size_t>(sl) * d * nc;
  return (b + 256 + 255) / 256 * 256;  // a multiple of 256: consecutive items stay aligned
}

// Fill the workspace pointers of `it` from memory at `base`.
void carve_item(BatchItem &it, void *base, sap_dtype at, int64_t rows_per_chunk) {
  Carve cv(base);
  const int64_t m = it.m;
  const int n = it.n, d = it.d, nc = n + 1;
  it.nblk = (n + kTrsvB - 1) / kTrsvB;
  it.idx = cv.take<int32_t>(static_cast<size_t>(m) * it.zeta);
  it.sign = cv.take<uint64_t>(m);
  (void)at;
  it.Y = cv.take<double>(static_cast<size_t>(d) * nc);
  it.tau = cv.take<double>(nc);
  it.T0 = cv.take<double>(256);
  it.T1 = cv.take<double>(256);
  it.Rt = cv.take<double>(static_cast<size_t>(n) * n);
  it.Dup = cv.take<double>(static_cast<size_t>(it.nblk) * kTrsvB * kTrsvB);
  it.Dlo = cv.take<double>(static_cast<size_t>(it.nblk) * kTrsvB * kTrsvB);
  it.flags = cv.take<int>(3 * it.nblk);
  it.st = cv.take<LsqrState>(1);
  it.u = cv.take<double>(m);
  it.y = cv.take<double>(n);
  it.v = cv.take<double>(n);
  it.w = cv.take<double>(n);
  it.p = cv.take<double>(n);
  it.xprev = cv.take<double>(n);
  const int64_t gmax = (m + kMinRowsPerChunk - 1) / kMinRowsPerChunk;
  it.qpart = cv.take<double>(static_cast<size_t>(gmax) * n);
  it.nrmpart = cv.take<double>(gmax);
  it.rows_per_chunk = rows_per_chunk;
  it.G = static_cast<int>((m + rows_per_chunk - 1) / rows_per_chunk);
  it.aslices = apply_slices(m, n, d);
  it.arows = (m + it.aslices - 1) / it.aslices;
  it.Ypart = it.aslices > 1 ? cv.take<double>(static_cast<size_t>(it.aslices) * d * nc) : nullptr;
}

// Phases S1-S7 setup for the `count` problems of a device items array:
// sketches, apply, QR, rank test, factor preparation, LSQR state and x0.
// dflags: [0] wait error, [1] done counter (incremented for rank-deficient
// problems here), [2] generation error.
sap_status setup_items(sap_ctx *ctx, BatchItem *ditems, const std::vector<BatchItem> &items, const int2 *dapply,
                       int napply, int *dflags, sap_dtype at, hipStream_t st) {
  const int count = static_cast<int>(items.size());
  int n_max = 0, d_max = 0, zeta_max = 0;
  int64_t total_cols = 0;
  for (const auto &it : items) {
    n_max = std::max(n_max, it.n);
    d_max = std::max(d_max, it.d);
    zeta_max = std::max(zeta_max, it.zeta);
    total_cols = std::max(total_cols, it.col_base + it.m);
  }
  const unsigned grid = static_cast<unsigned>((total_cols + 255) / 256);
  if (zeta_max <= 8) batch_generate_kernel<8><<<grid, 256, 0, st>>>(ditems, count, total_cols, dflags + 2);
  else if (zeta_max <= 16) batch_generate_kernel<16><<<grid, 256, 0, st>>>(ditems, count, total_cols, dflags + 2);
  else if (zeta_max <= 32) batch_generate_kernel<32><<<grid, 256, 0, st>>>(ditems, count, total_cols, dflags + 2);
  else batch_generate_kernel<64><<<grid, 256, 0, st>>>(ditems, count, total_cols, dflags + 2);
  const int per_xcd = (napply + kXcdsB - 1) / kXcdsB;
  const int w = batch_apply_width(d_max);
  const size_t lds = static_cast<size_t>(d_max + 1) * w * sizeof(double);  // plus a spare row
  const dim3 ag(static_cast<unsigned>(per_xcd * kXcdsB));
  if (at == SAP_F32) {
    switch (w) {
      case 32: batch_apply_kernel<float, 32><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      case 16: batch_apply_kernel<float, 16><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      case 8: batch_apply_kernel<float, 8><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      default: batch_apply_kernel<float, 4><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
    }
  } else {
    switch (w) {
      case 32: batch_apply_kernel<double, 32><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      case 16: batch_apply_kernel<double, 16><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      case 8: batch_apply_kernel<double, 8><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
      default: batch_apply_kernel<double, 4><<<ag, kBThreads, lds, st>>>(ditems, dapply, napply); break;
    }
  }
  {
    const int64_t tot_max = static_cast<int64_t>(d_max) * (n_max + 1);
    batch_apply_reduce_kernel<<<dim3(static_cast<unsigned>((tot_max + 255) / 256), count), 256, 0, st>>>(ditems);
  }
  SAP_HIP_TRY(hipGetLastError());
  const int sh = (d_max + kPanelThreads - 1) / kPanelThreads;
  const int cols = n_max + 1;
  // 4-column steps: twice the launches of 8-column ones, each with half the
  // panel's dependent column reductions on the critical path (served
  // stream p50 7.2 -> 6.5 ms, 512-problem batch 194 -> 189 ms)
  if (sh <= 1) launch_batch_qr<1, 4>(ditems, count, cols, st);
  else if (sh <= 2) launch_batch_qr<2, 4>(ditems, count, cols, st);
  else if (sh <= 4) launch_batch_qr<4, 4>(ditems, count, cols, st);
  else launch_batch_qr<8, 4>(ditems, count, cols, st);
  SAP_HIP_TRY(hipGetLastError());
  batch_rank_kernel<<<count, 256, 0, st>>>(ditems);
  const int nblk_max = (n_max + kTrsvB - 1) / kTrsvB;
  const int nt_max = (n_max + 31) / 32;
  batch_trsv_prepare_kernel<<<dim3(nblk_max, count), 256, 0, st>>>(ditems);
  batch_transpose_kernel<<<dim3(nt_max, nt_max, count), 256, 0, st>>>(ditems);
  batch_init_kernel<<<count, 1024, 0, st>>>(ditems);
  batch_x0_kernel<<<dim3(nblk_max, count), kTrsvThreads, 0, st>>>(ditems, dflags);
  batch_save_x_kernel<<<count, 256, 0, st>>>(ditems);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

// Shapes of the batch that select kernels, and the cached autotune choice.
struct BatchTuneKey {
  int a_type, n_bucket, count;
  bool operator<(const BatchTuneKey &o) const {
    return std::tie(a_type, n_bucket, count) < std::tie(o.a_type, o.n_bucket, o.count);
  }
};
struct BatchTune {
  int64_t chunk_elems;  // elements of A per pass work item
  bool pf;              // the pass variant: 512-thread workgroups with two row groups in flight
};

// Rows of a pass work item for a problem of n columns: about `elems`
// elements of A, at least kMinRowsPerChunk rows.
int64_t batch_chunk_rows(int n, int64_t elems) {
  return std::max<int64_t>(kMinRowsPerChunk, elems / std::max(1, n));
}
static std::map<BatchTuneKey, BatchTune> g_tune_rows;

// d = 0 (choose: eq. (4.2)'s d with cost ratio 1, within the batched form's
// limit) and the fixed-count mode (maxiter = the set count, tol = 0).
// Returns false when they cannot be resolved.
constexpr int kBatchMaxD = 4096;
bool resolve_params(const sap_problem &p, sap_params &q, int *fixed) {
  *fixed = 0;
  if (q.d == 0) {
    int32_t d42 = 0;
    if (!(q.tol > 0.0 && q.tol < 1.0) || sap_embedding_dim(p.m, p.n, q.tol, 1.0, &d42) != SAP_OK) return false;
    q.d = static_cast<int32_t>(std::min<int64_t>(std::min<int64_t>(d42, kBatchMaxD), p.m));
  }
  if (q.fixed_iters != 0) {
    if (q.mode != SAP_MODE_FP64 && q.mode != SAP_MODE_MIXED_FP32) return false;
    int32_t t = q.fixed_iters;
    if (t < 0 && (q.d <= p.n || sap_iteration_estimate(p.n, q.d, q.tol, &t) != SAP_OK)) return false;
    *fixed = t;
    q.maxiter = t;
    q.tol = 0.0;
  }
  return true;
}

sap_status run_batch(sap_ctx *ctx, int count, const sap_problem *probs, const sap_params *par_in, double *const *x,
                     sap_info *infos, hipStream_t user_stream) {
  if (count < 1) return fail(ctx, SAP_EINVAL, "sap_solve_batch: count must be >= 1");
  std::vector<sap_params> par_v(par_in, par_in + count);
  std::vector<int> fixed_v(count, 0);
  for (int k = 0; k < count; ++k)
    if (!resolve_params(probs[k], par_v[k], &fixed_v[k]))
      return fail(ctx, SAP_EINVAL, "sap_solve_batch: bad d = 0 or fixed_iters request");
  const sap_params *par = par_v.data();
  const sap_dtype at = probs[0].a_type;
  int n_max = 0, maxiter_max = 0;
  bool aligned = true;
  for (int k = 0; k < count; ++k) {
    const sap_problem &p = probs[k];
    const sap_params &q = par[k];
    if (p.a_type != at) return fail(ctx, SAP_EINVAL, "sap_solve_batch: all problems need the same A dtype");
    if (at != SAP_F32 && at != SAP_F64) return fail(ctx, SAP_EINVAL, "sap_solve_batch: A must be F32 or F64");
    if (!p.A || !p.b || !x[k]) return fail(ctx, SAP_EINVAL, "sap_solve_batch: NULL pointer");
    if (p.n < 1 || p.m < static_cast<int64_t>(p.n) + 1 || p.lda < p.n || p.m > (int64_t(1) << 31))
      return fail(ctx, SAP_EINVAL, "sap_solve_batch: bad problem shape");
    if (q.d < p.n + 1 || q.zeta < 1 || q.zeta > 64 || q.zeta > q.d || q.maxiter < 0 || !(q.tol >= 0.0) ||
        q.max_refine < 0)
      return fail(ctx, SAP_EINVAL, "sap_solve_batch: bad parameters");
    if (q.mode != SAP_MODE_FP64 && q.mode != SAP_MODE_MIXED_FP32 && q.mode != SAP_MODE_MIXED_FP32_REFINE)
      return fail(ctx, SAP_EINVAL, "sap_solve_batch: mode must be FP64, MIXED_FP32 or MIXED_FP32_REFINE");
    if (q.mode == SAP_MODE_MIXED_FP32_REFINE && at != SAP_F32)
      return fail(ctx, SAP_EINVAL, "sap_solve_batch: the refinement form needs FP32 A");
    const size_t es = (at == SAP_F32) ? 4 : 8;
    if (q.d > kBatchMaxD) return fail(ctx, SAP_EINVAL, "sap_solve_batch: d > 4096 is not supported by the batched form");
    n_max = std::max(n_max, p.n);
    maxiter_max = std::max(maxiter_max, q.maxiter);
    const int vm = 16 / static_cast<int>(es);
    if (reinterpret_cast<uintptr_t>(p.A) % 16 != 0 || p.lda % vm != 0) aligned = false;
  }
  if (n_max > 1024) return fail(ctx, SAP_EINVAL, "sap_solve_batch: n > 1024 is not supported");

  // ---- unaligned rows: repack into 16-byte-aligned rows when memory allows ----
  const size_t es_a = (at == SAP_F32) ? 4 : 8;
  const int vm_a = 16 / static_cast<int>(es_a);
  std::vector<int> repack_idx;   // problems to repack
  size_t repack_bytes = 0;
  int64_t repack_chunks = 0;
  if (!aligned) {
    for (int k = 0; k < count; ++k) {
      const sap_problem &p = probs[k];
      if (reinterpret_cast<uintptr_t>(p.A) % 16 == 0 && p.lda % vm_a == 0) continue;
      const int64_t ldp = (p.n + vm_a - 1) / vm_a * vm_a;
      repack_idx.push_back(k);
      repack_bytes += 256 + static_cast<size_t>(p.m) * ldp * es_a;
      repack_chunks += (p.m + kRepackRows - 1) / kRepackRows;
    }
  }

  // ---- workspace layout ---------------------------------------------------------
  const BatchTuneKey key{static_cast<int>(at), (n_max + 63) / 64, count};
  int64_t chunk_elems = int64_t(1) << 19;
  bool pass_pf = false;
  auto tit = g_tune_rows.find(key);
  const bool have_tune = tit != g_tune_rows.end();
  if (have_tune) {
    chunk_elems = tit->second.chunk_elems;
    pass_pf = tit->second.pf;
  }
  std::vector<size_t> need(count);
  size_t total = 8 * 256 + sizeof(BatchItem) * count + static_cast<size_t>(count) * 256;
  int64_t total_chunks_max = 0;
  for (int k = 0; k < count; ++k) {
    need[k] = item_bytes(probs[k].m, probs[k].n, par[k].d, par[k].zeta, at);
    total += need[k];
    total_chunks_max += (probs[k].m + kMinRowsPerChunk - 1) / kMinRowsPerChunk;
  }
  int d_max = 0;
  for (int k = 0; k < count; ++k) d_max = std::max(d_max, par[k].d);
  const int aw = batch_apply_width(d_max);
  const int tiles_max = (n_max + 1 + aw - 1) / aw;
  total += 256 + sizeof(int2) * (total_chunks_max + 16);
  total += 256 + sizeof(int2) * (static_cast<size_t>(count) * tiles_max * kMaxApplySlices + 16);
  const size_t repack_total = repack_idx.empty() ? 0
                                                 : repack_bytes + 2 * 256 + sizeof(RepackJob) * repack_idx.size() +
                                                       sizeof(int2) * static_cast<size_t>(repack_chunks);
  const bool repack = !repack_idx.empty() && total + repack_total <= ctx->budget;
  if (repack) total += repack_total;
  sap_status s = ensure_workspace(ctx, total, user_stream);
  if (s != SAP_OK) return s;
  Carve cv(ctx->ws);
  int *dflags = cv.take<int>(8);  // [0] wait error, [1] done count, [2] generation error
  BatchItem *ditems = cv.take<BatchItem>(count);
  std::vector<BatchItem> items(count);
  int64_t col_base = 0;
  bool any_refine = false;
  for (int k = 0; k < count; ++k) {
    BatchItem &it = items[k];
    const sap_problem &p = probs[k];
    const sap_params &q = par[k];
    it = BatchItem{};
    it.A = p.A;
    it.lda = p.lda;
    it.b = p.b;
    it.x = x[k];
    it.m = p.m;
    it.n = p.n;
    it.d = q.d;
    it.zeta = q.zeta;
    it.maxiter = q.maxiter;
    it.tol = q.tol;
    it.h = 1.0 / std::sqrt(static_cast<double>(q.zeta));
    it.seed = q.seed;
    it.stream = static_cast<uint64_t>(k);
    it.refine = q.mode == SAP_MODE_MIXED_FP32_REFINE ? 1 : 0;
    it.max_refine = q.max_refine;
    any_refine = any_refine || it.refine;
    it.col_base = col_base;
    col_base += p.m;
    carve_item(it, cv.take<char>(need[k]), at, batch_chunk_rows(p.n, chunk_elems));
  }
  int2 *dpass = cv.take<int2>(total_chunks_max + 16);
  int2 *dapply = cv.take<int2>(static_cast<size_t>(count) * tiles_max * kMaxApplySlices + 16);
  std::vector<RepackJob> jobs;
  std::vector<int2> repack_work;
  RepackJob *djobs = nullptr;
  int2 *drepack = nullptr;
  if (repack) {
    djobs = cv.take<RepackJob>(repack_idx.size());
    drepack = cv.take<int2>(static_cast<size_t>(repack_chunks));
    for (int k : repack_idx) {
      BatchItem &it = items[k];
      const int64_t ldp = (it.n + vm_a - 1) / vm_a * vm_a;
      RepackJob jb{};
      jb.src = it.A;
      jb.lda_src = it.lda;
      jb.dst = cv.take<char>(static_cast<size_t>(it.m) * ldp * es_a);
      jb.lda_dst = ldp;
      jb.m = it.m;
      jb.n = it.n;
      const int j = static_cast<int>(jobs.size());
      for (int64_t c = 0; c < (it.m + kRepackRows - 1) / kRepackRows; ++c)
        repack_work.push_back(make_int2(j, static_cast<int>(c)));
      jobs.push_back(jb);
      it.A = jb.dst;  // the solve reads the repacked rows
      it.zero_pad = 1;
      it.lda = ldp;
    }
    aligned = true;
  }

  // work tables
  std::vector<int2> apply_work;
  for (int k = 0; k < count; ++k) {
    const int tiles = (items[k].n + 1 + aw - 1) / aw;
    for (int t = 0; t < tiles; ++t)
      for (int sl = 0; sl < items[k].aslices; ++sl) apply_work.push_back(make_int2(k, t | (sl << 20)));
  }
  // Pass work items of about `elems` elements each, the largest first (each
  // problem's last, shorter item goes to the end of the launch).
  auto pass_table = [&](int64_t elems) {
    std::vector<std::pair<int64_t, int2>> v;
    for (int k = 0; k < count; ++k) {
      const int64_t rows = batch_chunk_rows(items[k].n, elems);
      const int G = static_cast<int>((items[k].m + rows - 1) / rows);
      for (int g = 0; g < G; ++g) {
        const int64_t r = std::min<int64_t>(items[k].m, (g + 1) * rows) - g * rows;
        v.push_back({r * items[k].n, make_int2(k, g)});
      }
    }
    std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<int2> wt(v.size());
    for (size_t i = 0; i < v.size(); ++i) wt[i] = v[i].second;
    return wt;
  };

  // internal stream (graph capture needs a non-default stream)
  hipStream_t st = nullptr;
  SAP_HIP_TRY(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } sguard{st};
  hipEvent_t ev_in;
  SAP_HIP_TRY(hipEventCreateWithFlags(&ev_in, hipEventDisableTiming));
  SAP_HIP_TRY(hipEventRecord(ev_in, user_stream));
  SAP_HIP_TRY(hipStreamWaitEvent(st, ev_in, 0));
  (void)hipEventDestroy(ev_in);

  SAP_HIP_TRY(hipMemsetAsync(dflags, 0, 8 * sizeof(int), st));
  if (repack) {
    SAP_HIP_TRY(hipMemcpyAsync(djobs, jobs.data(), sizeof(RepackJob) * jobs.size(), hipMemcpyHostToDevice, st));
    SAP_HIP_TRY(hipMemcpyAsync(drepack, repack_work.data(), sizeof(int2) * repack_work.size(), hipMemcpyHostToDevice, st));
    if (at == SAP_F32)
      batch_repack_kernel<float><<<static_cast<unsigned>(repack_work.size()), 256, 0, st>>>(djobs, drepack);
    else
      batch_repack_kernel<double><<<static_cast<unsigned>(repack_work.size()), 256, 0, st>>>(djobs, drepack);
    SAP_HIP_TRY(hipGetLastError());
  }
  SAP_HIP_TRY(hipMemcpyAsync(ditems, items.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, st));
  SAP_HIP_TRY(hipMemcpyAsync(dapply, apply_work.data(), sizeof(int2) * apply_work.size(), hipMemcpyHostToDevice, st));
  s = setup_items(ctx, ditems, items, dapply, static_cast<int>(apply_work.size()), dflags, at, st);
  if (s != SAP_OK) return s;
  batch_count_rank_kernel<<<1, 64, 0, st>>>(ditems, count, dflags + 1);
  const int nblk_max = (n_max + kTrsvB - 1) / kTrsvB;
  // The rank test wrote its flag into the device items: take them back so
  // that the re-uploads below keep it.
  SAP_HIP_TRY(hipMemcpyAsync(items.data(), ditems, sizeof(BatchItem) * count, hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));

  // ---- autotune the pass once per batch shape: elements per work item and
  // the variant (1024-thread workgroups, one row group in flight per wave,
  // or 512-thread workgroups with two), each timed on the device ----
  auto pick = [&](bool pf) {
    return (at == SAP_F32) ? pick_batch_pass<float>(n_max, aligned, pf) : pick_batch_pass<double>(n_max, aligned, pf);
  };
  if (!have_tune) {
    const int64_t cands[] = {int64_t(1) << 18, int64_t(1) << 19, int64_t(1) << 20, int64_t(1) << 21};
    float best_ms = 1e30f;
    int64_t best = chunk_elems;
    bool best_pf = false;
    hipEvent_t e0, e1;
    SAP_HIP_TRY(hipEventCreate(&e0));
    SAP_HIP_TRY(hipEventCreate(&e1));
    for (const bool pf : {false, true}) {
      const PassChoice pcv = pick(pf);
      for (int64_t c : cands) {
        std::vector<int2> wt = pass_table(c);
        std::vector<BatchItem> tmp = items;
        for (auto &it : tmp) {
          it.rows_per_chunk = batch_chunk_rows(it.n, c);
          it.G = static_cast<int>((it.m + it.rows_per_chunk - 1) / it.rows_per_chunk);
        }
        SAP_HIP_TRY(hipMemcpyAsync(ditems, tmp.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, st));
        SAP_HIP_TRY(hipMemcpyAsync(dpass, wt.data(), sizeof(int2) * wt.size(), hipMemcpyHostToDevice, st));
        float ms_best = 1e30f;
        for (int rep = 0; rep < 2; ++rep) {
          SAP_HIP_TRY(hipEventRecord(e0, st));
          launch_pass_fn(pcv, ditems, dpass, static_cast<int>(wt.size()), 1, st);
          SAP_HIP_TRY(hipEventRecord(e1, st));
          SAP_HIP_TRY(hipEventSynchronize(e1));
          float ms = 0.f;
          SAP_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
          ms_best = std::min(ms_best, ms);
        }
        if (ms_best < best_ms) {
          best_ms = ms_best;
          best = c;
          best_pf = pf;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    chunk_elems = best;
    pass_pf = best_pf;
    g_tune_rows[key] = BatchTune{best, best_pf};
    for (auto &it : items) {
      it.rows_per_chunk = batch_chunk_rows(it.n, best);
      it.G = static_cast<int>((it.m + it.rows_per_chunk - 1) / it.rows_per_chunk);
    }
    SAP_HIP_TRY(hipMemcpyAsync(ditems, items.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, st));
  }
  const PassChoice pc = pick(pass_pf);
  std::vector<int2> pass_work = pass_table(chunk_elems);
  SAP_HIP_TRY(hipMemcpyAsync(dpass, pass_work.data(), sizeof(int2) * pass_work.size(), hipMemcpyHostToDevice, st));
  const int npass = static_cast<int>(pass_work.size());

  // ---- S7-S8: iterations, replayed from a captured graph ----
  const int kIterPerGraph = 8;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  SAP_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < kIterPerGraph; ++k) {
    launch_pass_fn(pc, ditems, dpass, npass, 0, st, any_refine);
    batch_lower_kernel<<<dim3(nblk_max, count), kTrsvThreads, 0, st>>>(ditems, dflags);
    batch_upper_kernel<<<dim3(nblk_max, count), kTrsvThreads, 0, st>>>(ditems, dflags, dflags + 1);
    if (any_refine) batch_refine_kernel<<<count, 1024, 0, st>>>(ditems, dflags + 1);
  }
  hipError_t ce = hipStreamEndCapture(st, &graph);
  if (ce != hipSuccess) return hip_fail(ctx, ce, "hipStreamEndCapture");
  ce = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
  if (ce != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return hip_fail(ctx, ce, "hipGraphInstantiate");
  }
  struct GraphGuard {
    hipGraph_t g;
    hipGraphExec_t e;
    ~GraphGuard() {
      (void)hipGraphExecDestroy(e);
      (void)hipGraphDestroy(g);
    }
  } gguard{graph, gexec};
  int hflags[3] = {0, 0, 0};
  // every restart of the refinement form takes one step that is not an
  // iteration (the residual pass), at most max_refine of them per problem
  int refine_steps = 0;
  for (int k = 0; k < count; ++k)
    if (items[k].refine) refine_steps = std::max(refine_steps, items[k].max_refine > 0 ? items[k].max_refine : 10);
  const int max_launches = (maxiter_max + refine_steps + 1) / kIterPerGraph + 2;
  bool finished = false;
  for (int l = 0; l < max_launches; ++l) {
    SAP_HIP_TRY(hipGraphLaunch(gexec, st));
    SAP_HIP_TRY(hipMemcpyAsync(hflags, dflags, sizeof(hflags), hipMemcpyDeviceToHost, st));
    SAP_HIP_TRY(hipStreamSynchronize(st));
    if (hflags[0]) return fail(ctx, SAP_EDEVICE, "sap_solve_batch: a triangular-solve wait expired");
    if (hflags[1] >= count) {
      finished = true;
      break;
    }
  }
  if (hflags[2]) return fail(ctx, SAP_EDEVICE, "sap_solve_batch: sketch generation hit its round cap");
  if (!finished) return fail(ctx, SAP_EDEVICE, "sap_solve_batch: device never reported completion");

  // per-problem results
  std::vector<LsqrState> states(count);
  std::vector<BatchItem> back(count);
  SAP_HIP_TRY(hipMemcpyAsync(back.data(), ditems, sizeof(BatchItem) * count, hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  for (int k = 0; k < count; ++k)
    SAP_HIP_TRY(hipMemcpyAsync(&states[k], back[k].st, sizeof(LsqrState), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  // order the caller's stream after this work
  hipEvent_t ev_out;
  SAP_HIP_TRY(hipEventCreateWithFlags(&ev_out, hipEventDisableTiming));
  SAP_HIP_TRY(hipEventRecord(ev_out, st));
  SAP_HIP_TRY(hipStreamWaitEvent(user_stream, ev_out, 0));
  (void)hipEventDestroy(ev_out);
  bool all_ok = true;
  for (int k = 0; k < count; ++k) {
    const bool ran_fixed = fixed_v[k] > 0 && states[k].total_iters >= fixed_v[k];
    sap_status sk = back[k].rank_deficient ? SAP_RANK_DEFICIENT
                                           : ((states[k].converged || ran_fixed) ? SAP_OK : SAP_NOT_CONVERGED);
    if (sk != SAP_OK) all_ok = false;
    if (infos) {
      std::memset(&infos[k], 0, sizeof(sap_info));
      infos[k].status = sk;
      infos[k].iters = states[k].total_iters;
      infos[k].refinements = states[k].refinements;
      infos[k].d_used = par[k].d;
      infos[k].resid_est = states[k].resid_est;
      infos[k].normar_est = states[k].normar_est;
    }
  }
  if (!all_ok) (void)fail(ctx, SAP_NOT_CONVERGED, "sap_solve_batch: some problems did not converge or were rank deficient (see info)");
  return all_ok ? SAP_OK : SAP_NOT_CONVERGED;
}

// ----------------------------------------------------------------------------
// Served form: continuous batching.  A scheduler thread owns a device arena
// and admits queued requests (first in, first out) whenever their workspace
// footprint fits; a round runs the setup phases of the newly admitted
// requests as one batch and then a few LSQR iterations of every active
// request as one batch; finished requests retire at the end of a round and
// free their memory, so requests that arrive while others run join the next
// round.  Requests are independent: a result does not depend on what else is
// in flight (only the floating-point order of the LDS sketch adds varies).

struct ServeRequest {
  uint64_t ticket = 0;
  sap_problem prob{};
  sap_params par{};
  double *x = nullptr;
  int fixed = 0;  // fixed-count mode: the set number of iterations
  size_t bytes = 0, offset = 0;
  BatchItem item{};
  hipEvent_t ready = nullptr;  // inputs written: recorded on the submitter's stream
  int state = 0;  // 0 queued, 1 active, 2 finished
  bool cancel = false;
  sap_status status = SAP_PENDING;
  sap_info info{};
  std::chrono::steady_clock::time_point t_submit, t_admit, t_done;
};

struct Arena {  // first-fit sub-allocator over one device allocation
  char *base = nullptr;
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  void init(void *b, size_t n) {
    base = static_cast<char *>(b);
    size = n;
    free_.clear();
    free_[0] = n;
    used = 0;
  }
  bool alloc(size_t n, size_t *off) {
    n = (n + 4095) & ~size_t(4095);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t o = it->first;
        free_.erase(it);
        if (rest) free_[o + n] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 4095) & ~size_t(4095);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Server {
  sap_ctx *ctx = nullptr;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  std::deque<ServeRequest *> queued;
  std::vector<ServeRequest *> active;
  std::unordered_map<uint64_t, std::unique_ptr<ServeRequest>> reqs;
  std::thread th;
  bool stop = false;
  bool failed = false;
  std::string fail_msg;
  uint64_t next_ticket = 1;
  sap_dtype at = SAP_F32;
  bool at_set = false;
  Arena arena;
  void *arena_mem = nullptr;
  hipStream_t st = nullptr;        // iterations of the active requests
  hipStream_t st_setup = nullptr;  // setup of newly admitted requests, overlapping the iterations
  int max_slots = 0;
  int iters_per_round = 8;
  BatchItem *d_active = nullptr, *d_new = nullptr;
  int2 *d_pass = nullptr, *d_apply = nullptr;
  int *d_flags = nullptr, *d_flags_setup = nullptr, *d_done = nullptr;
  void *scratch = nullptr;
  int64_t n_submitted = 0, n_completed = 0, n_rejected = 0;
  // a round's iteration launches, captured once per launch shape and
  // replayed while the active set keeps that shape (the launches read the
  // requests' parameters from d_active, so only the shape is baked in)
  struct RoundGraph {
    int64_t key[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    hipGraphExec_t exec = nullptr;
  } round_graphs[4];
  int rg_next = 0;
};

namespace {

// Rows per pass work item of a served request: about 2 MB of A per item
// (power of two in [1024, 8192] rows), so that the few requests a round holds
// still spread over the whole GPU in even pieces.
int64_t serve_rows_per_chunk(int n, sap_dtype at) {
  const int64_t row_bytes = static_cast<int64_t>(n) * (at == SAP_F32 ? 4 : 8);
  int64_t r = 1024;
  while (r < 8192 && 2 * r * row_bytes <= (int64_t(2) << 20)) r *= 2;
  return r;
}
constexpr int kServeMaxChunks = 1 << 20;
constexpr int kServeMaxApply = 1 << 20;

// A device error ends serving: every request not finished yet fails.
void serve_fail_all(Server *S, const std::string &msg, std::vector<ServeRequest *> &fresh) {
  std::lock_guard<std::mutex> lk(S->mu);
  S->failed = true;
  S->fail_msg = msg;
  auto fail_one = [](ServeRequest *r) {
    if (r->ready) (void)hipEventDestroy(r->ready);
    r->ready = nullptr;
    r->state = 2;
    r->status = SAP_EDEVICE;
    r->info.status = SAP_EDEVICE;
  };
  for (ServeRequest *r : S->active) fail_one(r);
  for (ServeRequest *r : fresh) fail_one(r);
  for (ServeRequest *r : S->queued) fail_one(r);
  S->active.clear();
  S->queued.clear();
  fresh.clear();
  S->cv_done.notify_all();
}

// One round: the setup of the newly admitted requests (one batched launch
// sequence on the setup stream) overlaps 8 iterations of the active ones on
// the iteration stream; finished requests retire, and the new ones join the
// active set for the next round.
hipError_t serve_round(Server *S, std::vector<ServeRequest *> &fresh) {
  hipStream_t st = S->st, ss = S->st_setup;
  const sap_dtype at = S->at;
  hipError_t e;
  // ---- setup of the newly admitted requests (enqueued only) ----
  std::vector<BatchItem> new_items(fresh.size());
  int setup_flags[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (!fresh.empty()) {
    std::vector<int2> apply_work;
    int64_t col_base = 0;
    int d_max = 0;
    for (ServeRequest *r : fresh) d_max = std::max(d_max, r->item.d);
    const int aw = batch_apply_width(d_max);
    for (size_t k = 0; k < fresh.size(); ++k) {
      ServeRequest *r = fresh[k];
      BatchItem &it = r->item;
      it.col_base = col_base;
      col_base += it.m;
      new_items[k] = it;
      const int tiles = (it.n + 1 + aw - 1) / aw;
      for (int t = 0; t < tiles; ++t)
        for (int sl = 0; sl < it.aslices; ++sl) apply_work.push_back(make_int2(static_cast<int>(k), t | (sl << 20)));
    }
    if (static_cast<int>(apply_work.size()) > kServeMaxApply) return hipErrorInvalidValue;
    for (ServeRequest *r : fresh)
      if ((e = hipStreamWaitEvent(ss, r->ready, 0)) != hipSuccess) return e;
    if ((e = hipMemsetAsync(S->d_flags_setup, 0, 8 * sizeof(int), ss)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(S->d_new, new_items.data(), sizeof(BatchItem) * new_items.size(), hipMemcpyHostToDevice, ss)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(S->d_apply, apply_work.data(), sizeof(int2) * apply_work.size(), hipMemcpyHostToDevice, ss)) != hipSuccess) return e;
    if (setup_items(S->ctx, S->d_new, new_items, S->d_apply, static_cast<int>(apply_work.size()), S->d_flags_setup, at, ss) != SAP_OK)
      return hipErrorLaunchFailure;
    // the rank test wrote its flag into the device copy of each item
    if ((e = hipMemcpyAsync(new_items.data(), S->d_new, sizeof(BatchItem) * new_items.size(), hipMemcpyDeviceToHost, ss)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(setup_flags, S->d_flags_setup, sizeof(setup_flags), hipMemcpyDeviceToHost, ss)) != hipSuccess) return e;
  }
  // ---- iterations of the active requests ----
  std::vector<ServeRequest *> act;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    act = S->active;
  }
  const int count = static_cast<int>(act.size());
  std::vector<int> done(count), hflags(8, 0);
  if (count > 0) {
    std::vector<BatchItem> items(count);
    std::vector<int2> pass_work;
    int n_max = 0;
    bool aligned = true;
    bool any_refine = false;
    const int vm = (at == SAP_F32) ? 4 : 2;
    for (int k = 0; k < count; ++k) {
      items[k] = act[k]->item;
      n_max = std::max(n_max, items[k].n);
      any_refine = any_refine || items[k].refine;
      if (reinterpret_cast<uintptr_t>(items[k].A) % 16 != 0 || items[k].lda % vm != 0) aligned = false;
      for (int g = 0; g < items[k].G; ++g) pass_work.push_back(make_int2(k, g));
    }
    // the largest work items first: each request's shorter last item runs at the end
    auto item_elems = [&](int2 w) {
      const BatchItem &it = items[w.x];
      return (std::min<int64_t>(it.m, (w.y + int64_t(1)) * it.rows_per_chunk) - w.y * it.rows_per_chunk) * it.n;
    };
    std::stable_sort(pass_work.begin(), pass_work.end(),
                     [&](int2 a, int2 b) { return item_elems(a) > item_elems(b); });
    if (static_cast<int>(pass_work.size()) > kServeMaxChunks) return hipErrorInvalidValue;
    if ((e = hipMemcpyAsync(S->d_active, items.data(), sizeof(BatchItem) * count, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(S->d_pass, pass_work.data(), sizeof(int2) * pass_work.size(), hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    const PassChoice pc = (at == SAP_F32) ? pick_batch_pass<float>(n_max, aligned, true)
                                           : pick_batch_pass<double>(n_max, aligned, true);
    const int nblk_max = (n_max + kTrsvB - 1) / kTrsvB;
    const int nwork = static_cast<int>(pass_work.size());
    auto launch_iters = [&](hipStream_t ls) {
      for (int k = 0; k < S->iters_per_round; ++k) {
        launch_pass_fn(pc, S->d_active, S->d_pass, nwork, 0, ls, any_refine);
        batch_lower_kernel<<<dim3(nblk_max, count), kTrsvThreads, 0, ls>>>(S->d_active, S->d_flags);
        batch_upper_kernel<<<dim3(nblk_max, count), kTrsvThreads, 0, ls>>>(S->d_active, S->d_flags,
                                                                          S->d_flags + 1);
        if (any_refine) batch_refine_kernel<<<count, 1024, 0, ls>>>(S->d_active, S->d_flags + 1);
      }
    };
    const int64_t key[8] = {static_cast<int64_t>(reinterpret_cast<uintptr_t>(pc.fn)), pc.threads, nwork, count,
                            nblk_max, any_refine ? 1 : 0, S->iters_per_round, 1};
    hipGraphExec_t ex = nullptr;
    for (auto &g : S->round_graphs)
      if (g.exec && std::equal(key, key + 8, g.key)) ex = g.exec;
    if (!ex && !S->ctx->profiling && hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      launch_iters(st);
      hipGraph_t graph = nullptr;
      if (hipStreamEndCapture(st, &graph) == hipSuccess && graph) {
        if (hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0) != hipSuccess) ex = nullptr;
        (void)hipGraphDestroy(graph);
      }
      (void)hipGetLastError();
      if (ex) {
        auto &slot = S->round_graphs[S->rg_next];
        S->rg_next = (S->rg_next + 1) % 4;
        if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
        slot.exec = ex;
        std::copy(key, key + 8, slot.key);
      }
    }
    if (ex) {
      if ((e = hipGraphLaunch(ex, st)) != hipSuccess) return e;
    } else {
      launch_iters(st);
    }
    serve_done_kernel<<<(count + 255) / 256, 256, 0, st>>>(S->d_active, count, S->d_done);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(done.data(), S->d_done, sizeof(int) * count, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(hflags.data(), S->d_flags, sizeof(int) * 8, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (hflags[0] || hflags[2]) return hipErrorLaunchFailure;
  }
  // ---- retire finished (or cancelled) requests ----
  std::vector<ServeRequest *> finished;
  for (int k = 0; k < count; ++k) {
    ServeRequest *r = act[k];
    bool cancel;
    {
      std::lock_guard<std::mutex> lk(S->mu);
      cancel = r->cancel;
    }
    if (done[k] || cancel) finished.push_back(r);
  }
  if (!finished.empty()) {
    std::vector<LsqrState> states(finished.size());
    for (size_t k = 0; k < finished.size(); ++k) {
      if ((e = hipMemcpyAsync(&states[k], finished[k]->item.st, sizeof(LsqrState), hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    }
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    const auto now = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t k = 0; k < finished.size(); ++k) {
      ServeRequest *r = finished[k];
      sap_status stt;
      if (r->cancel) stt = SAP_ECANCELED;
      else if (r->item.rank_deficient) stt = SAP_RANK_DEFICIENT;
      else stt = (states[k].converged || (r->fixed > 0 && states[k].total_iters >= r->fixed)) ? SAP_OK
                                                                                               : SAP_NOT_CONVERGED;
      r->status = stt;
      r->t_done = now;
      std::memset(&r->info, 0, sizeof(r->info));
      r->info.status = stt;
      r->info.iters = states[k].total_iters;
      r->info.refinements = states[k].refinements;
      r->info.d_used = r->par.d;
      r->info.resid_est = states[k].resid_est;
      r->info.normar_est = states[k].normar_est;
      r->info.t_queue_ms = std::chrono::duration<double, std::milli>(r->t_admit - r->t_submit).count();
      r->info.t_total_ms = std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count();
      r->state = 2;
      S->arena.release(r->offset, r->bytes);
      S->active.erase(std::find(S->active.begin(), S->active.end(), r));
      S->n_completed += 1;
    }
    S->cv_done.notify_all();
    S->cv.notify_all();
  }
  // ---- the new requests join the active set ----
  if (!fresh.empty()) {
    if ((e = hipStreamSynchronize(ss)) != hipSuccess) return e;
    if (setup_flags[0] || setup_flags[2]) return hipErrorLaunchFailure;
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t k = 0; k < fresh.size(); ++k) {
      (void)hipEventDestroy(fresh[k]->ready);
      fresh[k]->ready = nullptr;
      fresh[k]->item = new_items[k];
      S->active.push_back(fresh[k]);
    }
    fresh.clear();
    S->cv.notify_all();
  }
  return hipSuccess;
}

void serve_loop(Server *S) {
  (void)hipSetDevice(S->ctx->device);
  for (;;) {
    std::vector<ServeRequest *> fresh;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] { return S->stop || !S->queued.empty() || !S->active.empty(); });
      if (S->stop) return;
      // drop cancelled requests still in the queue
      for (auto it = S->queued.begin(); it != S->queued.end();) {
        if ((*it)->cancel) {
          (void)hipEventDestroy((*it)->ready);
          (*it)->ready = nullptr;
          (*it)->state = 2;
          (*it)->status = SAP_ECANCELED;
          (*it)->info.status = SAP_ECANCELED;
          it = S->queued.erase(it);
          S->cv_done.notify_all();
        } else {
          ++it;
        }
      }
      // admit in arrival order while the head of the queue fits
      const auto now = std::chrono::steady_clock::now();
      while (!S->queued.empty() && static_cast<int>(S->active.size() + fresh.size()) < S->max_slots) {
        ServeRequest *r = S->queued.front();
        size_t off = 0;
        if (!S->arena.alloc(r->bytes, &off)) break;
        r->offset = off;
        r->state = 1;
        r->t_admit = now;
        carve_item(r->item, S->arena.base + off, S->at, serve_rows_per_chunk(r->item.n, S->at));
        S->queued.pop_front();
        fresh.push_back(r);
      }
    }
    const hipError_t e = serve_round(S, fresh);
    if (e != hipSuccess) {
      serve_fail_all(S, std::string("served round failed: ") + hipGetErrorString(e), fresh);
      return;
    }
  }
}

}  // namespace

void serve_destroy(sap_ctx *ctx) {
  Server *S = ctx->server;
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->th.joinable()) S->th.join();
  (void)hipSetDevice(ctx->device);
  for (auto &kv : S->reqs)
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
  if (S->st) (void)hipStreamSynchronize(S->st);
  if (S->st_setup) (void)hipStreamSynchronize(S->st_setup);
  for (auto &g : S->round_graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (S->st) (void)hipStreamDestroy(S->st);
  if (S->st_setup) (void)hipStreamDestroy(S->st_setup);
  if (S->arena_mem) (void)hipFree(S->arena_mem);
  if (S->scratch) (void)hipFree(S->scratch);
  delete S;
  ctx->server = nullptr;
}

sap_status serve_start(sap_ctx *ctx, size_t arena_bytes, int max_slots) {
  if (ctx->server) return fail(ctx, SAP_EINVAL, "sap_serve_start: already serving");
  if (max_slots < 1 || max_slots > 4096) return fail(ctx, SAP_EINVAL, "sap_serve_start: max_slots must be in [1, 4096]");
  if (arena_bytes == 0) arena_bytes = std::min<size_t>(ctx->budget / 2, size_t(64) << 30);
  if (arena_bytes > ctx->budget) return fail(ctx, SAP_ENOMEM, "sap_serve_start: arena exceeds the HBM budget");
  std::unique_ptr<Server> S(new Server());
  S->ctx = ctx;
  S->max_slots = max_slots;
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  if (hipMalloc(&S->arena_mem, arena_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, SAP_ENOMEM, "sap_serve_start: could not allocate the arena");
  }
  S->arena.init(S->arena_mem, arena_bytes);
  const size_t scratch = 8 * 256 + 2 * sizeof(BatchItem) * max_slots + sizeof(int2) * (kServeMaxChunks + kServeMaxApply) +
                         sizeof(int) * (16 + max_slots);
  if (hipMalloc(&S->scratch, scratch) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(S->arena_mem);
    return fail(ctx, SAP_ENOMEM, "sap_serve_start: could not allocate the scheduler scratch");
  }
  Carve cv(S->scratch);
  S->d_flags = cv.take<int>(8);
  S->d_flags_setup = cv.take<int>(8);
  S->d_done = cv.take<int>(max_slots);
  S->d_active = cv.take<BatchItem>(max_slots);
  S->d_new = cv.take<BatchItem>(max_slots);
  S->d_pass = cv.take<int2>(kServeMaxChunks);
  S->d_apply = cv.take<int2>(kServeMaxApply);
  SAP_HIP_TRY(hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking));
  SAP_HIP_TRY(hipStreamCreateWithFlags(&S->st_setup, hipStreamNonBlocking));
  ctx->server = S.release();
  ctx->server->th = std::thread(serve_loop, ctx->server);
  return SAP_OK;
}

sap_status serve_submit(sap_ctx *ctx, const sap_problem *p, const sap_params *q_in, double *x, uint64_t *ticket,
                        hipStream_t stream) {
  if (!p || !q_in || !x || !ticket) return fail(ctx, SAP_EINVAL, "sap_submit: NULL argument");
  sap_params qv = *q_in;
  int fixed = 0;
  if (!resolve_params(*p, qv, &fixed)) return fail(ctx, SAP_EINVAL, "sap_submit: bad d = 0 or fixed_iters request");
  const sap_params *q = &qv;
  {
    static std::mutex start_mu;
    std::lock_guard<std::mutex> lk(start_mu);
    if (!ctx->server) {
      sap_status s = serve_start(ctx, 0, 1024);
      if (s != SAP_OK) return s;
    }
  }
  Server *S = ctx->server;
  if (p->a_type != SAP_F32 && p->a_type != SAP_F64) return fail(ctx, SAP_EINVAL, "sap_submit: A must be F32 or F64");
  if (!p->A || !p->b) return fail(ctx, SAP_EINVAL, "sap_submit: NULL device pointer");
  if (p->n < 1 || p->n > 1024 || p->m < static_cast<int64_t>(p->n) + 1 || p->lda < p->n || p->m > (int64_t(1) << 31))
    return fail(ctx, SAP_EINVAL, "sap_submit: bad problem shape (n <= 1024, m >= n + 1)");
  if (q->d < p->n + 1 || q->d > 4096 || q->zeta < 1 || q->zeta > 64 ||
      q->zeta > q->d || q->maxiter < 0 || !(q->tol >= 0.0) || q->max_refine < 0)
    return fail(ctx, SAP_EINVAL, "sap_submit: bad parameters");
  if (q->mode != SAP_MODE_FP64 && q->mode != SAP_MODE_MIXED_FP32 && q->mode != SAP_MODE_MIXED_FP32_REFINE)
    return fail(ctx, SAP_EINVAL, "sap_submit: mode must be FP64, MIXED_FP32 or MIXED_FP32_REFINE");
  if (q->mode == SAP_MODE_MIXED_FP32_REFINE && p->a_type != SAP_F32)
    return fail(ctx, SAP_EINVAL, "sap_submit: the refinement form needs FP32 A");
  const size_t bytes = item_bytes(p->m, p->n, q->d, q->zeta, p->a_type);
  hipEvent_t ready = nullptr;
  SAP_HIP_TRY(hipSetDevice(ctx->device));
  SAP_HIP_TRY(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  if (hipEventRecord(ready, stream) != hipSuccess) {
    (void)hipEventDestroy(ready);
    return fail(ctx, SAP_EDEVICE, "sap_submit: could not record the input event");
  }
  struct EvOwner {
    hipEvent_t e;
    ~EvOwner() {
      if (e) (void)hipEventDestroy(e);
    }
  } owner{ready};
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->failed) return fail(ctx, SAP_EDEVICE, S->fail_msg);
  if (S->at_set && p->a_type != S->at) return fail(ctx, SAP_EINVAL, "sap_submit: all served problems share one A dtype");
  if (bytes > S->arena.size) {
    S->n_rejected += 1;
    return fail(ctx, SAP_ENOMEM, "sap_submit: the request can never fit in the serving arena");
  }
  S->at = p->a_type;
  S->at_set = true;
  std::unique_ptr<ServeRequest> r(new ServeRequest());
  r->ticket = S->next_ticket++;
  r->prob = *p;
  r->par = *q;
  r->fixed = fixed;
  r->x = x;
  r->bytes = bytes;
  r->ready = ready;
  owner.e = nullptr;
  r->t_submit = std::chrono::steady_clock::now();
  BatchItem &it = r->item;
  it.A = p->A;
  it.lda = p->lda;
  it.b = p->b;
  it.x = x;
  it.m = p->m;
  it.n = p->n;
  it.d = q->d;
  it.zeta = q->zeta;
  it.maxiter = q->maxiter;
  it.tol = q->tol;
  it.h = 1.0 / std::sqrt(static_cast<double>(q->zeta));
  it.seed = q->seed;
  it.stream = 0;  // the sketch sap_solve draws for the same seed
  it.refine = q->mode == SAP_MODE_MIXED_FP32_REFINE ? 1 : 0;
  it.max_refine = q->max_refine;
  *ticket = r->ticket;
  S->queued.push_back(r.get());
  S->reqs[r->ticket] = std::move(r);
  S->n_submitted += 1;
  S->cv.notify_all();
  return SAP_OK;
}

sap_status serve_poll(sap_ctx *ctx, uint64_t ticket, sap_info *info, int wait) {
  Server *S = ctx->server;
  if (!S) return fail(ctx, SAP_EINVAL, "sap_poll: nothing was submitted");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(ctx, SAP_EINVAL, "sap_poll: unknown ticket");
  ServeRequest *r = it->second.get();
  if (wait) S->cv_done.wait(lk, [&] { return r->state == 2; });
  if (r->state != 2) {
    if (info) {
      std::memset(info, 0, sizeof(*info));
      info->status = SAP_PENDING;
    }
    return SAP_PENDING;
  }
  const sap_status s = r->status;
  if (info) *info = r->info;
  S->reqs.erase(it);
  return s;
}

sap_status serve_cancel(sap_ctx *ctx, uint64_t ticket) {
  Server *S = ctx->server;
  if (!S) return fail(ctx, SAP_EINVAL, "sap_cancel: nothing was submitted");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return fail(ctx, SAP_EINVAL, "sap_cancel: unknown ticket");
  it->second->cancel = true;
  S->cv.notify_all();
  return SAP_OK;
}

sap_status serve_stats(sap_ctx *ctx, int64_t *out) {
  Server *S = ctx->server;
  if (!S) {
    for (int k = 0; k < 7; ++k) out[k] = 0;
    return SAP_OK;
  }
  std::lock_guard<std::mutex> lk(S->mu);
  out[0] = S->n_submitted;
  out[1] = S->n_completed;
  out[2] = static_cast<int64_t>(S->active.size());
  out[3] = static_cast<int64_t>(S->queued.size());
  out[4] = S->n_rejected;
  out[5] = static_cast<int64_t>(S->arena.used);
  out[6] = static_cast<int64_t>(S->arena.size);
  return SAP_OK;
}

}  // namespace sap
