// Preconditioned LSQR (Alg. 2) on A M, M = R^-1, for gfx950.
//
// One iteration is five kernels on one stream, with no host round trip:
//   1. pass   : one sweep over A computing, for every row i,
//                 u_i <- c_ap (A p)_i + c_u u_i        (p = M v_t)
//               and accumulating q = A^T u and ||u||^2 from the same
//               registers.  This is the one-synchronisation reorganisation
//               of App. D.4.1: A^T is applied to the unnormalised u_hat and
//               the scale 1/beta is folded into the next step, so A is read
//               once per iteration instead of twice.  Each workgroup writes
//               one partial q.
//   2. q_slices: the partials summed in fixed-order slices;
//   3. mtq    : v_hat = M^T q / beta - beta v and the partials of ||v_hat||^2
//               (M = R^-1 formed once per solve, Sec. 3.2);
//   4. mv     : alpha, v = v_hat / alpha, p = M v;
//   5. update : plane rotation, x += (phi/rho) w, w = p - (theta/rho) w, the
//               stopping test and the coefficients of the next pass.
// All scalars stay in device memory.  Kernels early-exit once the device
// `done` flag is set, so the host enqueues iterations in batches of eight
// (captured once into a hipGraph and replayed) and reads the flag once per
// batch, while the next batch runs.  The same file holds the refinement form
// (FP32 inner passes, FP64 residual restarts) and heavy-ball momentum
// (App. D.3), which reuses the pass with p = x and u_in = b.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>

#include "common.h"
#include "trsv.h"
#include "lsqr_dev.h"

namespace sap {
namespace {

constexpr int kPassThreads = 512;
constexpr int kPassWaves = kPassThreads / kWave;
constexpr int kMaxN = 8192;
constexpr int kMaxSstep = 16;  // steps per block of the s-step form

// [fused-pass-begin] (the benchmark hashes this region, with the wavefront
// helpers, to tell whether HBM counters taken on the pass still describe it)
// --------------------------------------------------------------------------
// Fused pass.  MODE 0: A in FP64.  MODE 1: A stored in FP32 (the mixed
// form): p, the accumulation and u are FP64, an FP32 element is widened
// exactly, so the pass reads half the bytes for the same arithmetic.
// The refinement form uses two more: MODE 2, the inner iterations, with p,
// the accumulation and u in FP32; MODE 3, the residual pass r = b - A x with
// FP64 accumulation, whose u output (the inner right-hand side) is FP32.
template <int MODE>
struct PassTypes;
template <>
struct PassTypes<0> {
  using TA = double; using TC = double; using TUI = double; using TUO = double;
};
template <>
struct PassTypes<1> {
  using TA = float; using TC = double; using TUI = double; using TUO = double;
};
template <>
struct PassTypes<2> {
  using TA = float; using TC = float; using TUI = float; using TUO = float;
};
template <>
struct PassTypes<3> {
  using TA = float; using TC = double; using TUI = double; using TUO = float;
};

// Rows of a row group per step: 16 / (J VEC) for short rows (at most 4), one
// row for rows of 16 or more elements per lane, except that FP32 storage with
// FP64 arithmetic (modes 1 and 3) then takes two rows: as many bytes in
// flight per wave as the FP64 pass at the same occupancy, which the FP64
// accumulators set (FP32 pass over 2^22 x 4096: 5.8 -> 6.8 TB/s).
__host__ __device__ constexpr int pass_rows(int mode, int jv) {
  if (jv >= 16) return (mode == 1 || mode == 3) ? 2 : 1;
  return 16 / jv > 4 ? 4 : 16 / jv;
}

// WC waves split the columns of a row (64*VEC*J columns each); WR = kPassWaves/WC
// row groups share the workgroup.
//
// Row distribution: workgroup g first takes rows [g S, (g+1) S) (S =
// rows_per_wg, a whole number of steps); the rows from dyn_begin = grid S to
// m are claimed in chunks of `chunk` rows from the counter dyn[0], so that
// workgroups on faster XCDs take more of the tail (the eight XCDs finish a
// static split up to ~7% apart).  The last workgroup to finish resets
// dyn[0..1] to zero for the next launch; they must be zero before the first.
// The rows a workgroup sums into its partials then depend on timing, so q
// and ||u||^2 are reproducible to rounding only.
template <int MODE, int VEC, int J, int WC>
__global__ __launch_bounds__(kPassThreads) void lsqr_pass_kernel(
    const typename PassTypes<MODE>::TA *__restrict__ A, int64_t lda, int64_t m, int n,
    const typename PassTypes<MODE>::TC *__restrict__ p, const typename PassTypes<MODE>::TUI *u_in,
    typename PassTypes<MODE>::TUO *u_out, const LsqrState *__restrict__ st, double *__restrict__ qpart,
    double *__restrict__ nrmpart, int64_t rows_per_wg, int64_t dyn_begin, int chunk, unsigned int *dyn) {
  using TA = typename PassTypes<MODE>::TA;
  using TC = typename PassTypes<MODE>::TC;
  constexpr int WR = kPassWaves / WC;
  constexpr int R = pass_rows(MODE, J * VEC);
  constexpr int COLS = kWave * VEC * J;  // columns per wave
  __shared__ double xch[WC > 1 ? 2 : 1][WC > 1 ? WR : 1][R][WC];
  __shared__ double qbuf[WR > 1 ? WC * COLS : 1];
  __shared__ double nbuf[kPassWaves];
  if (st->done) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int wc = wave % WC, wr = wave / WC;
  const int col0 = wc * COLS;
  const TC c_ap = static_cast<TC>(st->c_ap);
  const TC c_u = static_cast<TC>(st->c_u);

  TC preg[J][VEC], q[J][VEC];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int c = col0 + (j * kWave + lane) * VEC + e;
      preg[j][e] = c < n ? p[c] : TC(0);
      q[j][e] = TC(0);
    }

  __shared__ unsigned int next_chunk[2];
  double nrm = 0.0;
  // rows [i_begin, i_end), WR * R per step; for WC > 1 the caller separates
  // two calls by a barrier (the exchange buffer parity restarts)
  auto rows = [&](int64_t i_begin, int64_t i_end) {
  const int64_t nsteps = i_end > i_begin ? (i_end - i_begin + WR * R - 1) / (WR * R) : 0;
  auto load_step = [&](int64_t step, TA (&a)[R][J][VEC]) {
    const int64_t base = i_begin + step * (WR * R) + wr * R;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = base + r;
      const bool rv = row < i_end;
      const TA *arow = A + row * lda;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int c = col0 + (j * kWave + lane) * VEC;
        if (rv && c < n) {
          TA v[VEC];
          load_stream<TA, VEC>(arow + c, v);
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[r][j][e] = v[e];
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[r][j][e] = TA(0);
        }
      }
    }
  };
  auto compute_step = [&](int64_t step, TA (&a)[R][J][VEC]) {
    const int64_t base = i_begin + step * (WR * R) + wr * R;
    TC dot[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      TC s = TC(0);
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) s += static_cast<TC>(a[r][j][e]) * preg[j][e];
      dot[r] = wave_sum_u(s);
    }
    if constexpr (WC > 1) {
      const int parity = static_cast<int>(step & 1);
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) xch[parity][wr][r][wc] = static_cast<double>(dot[r]);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WC; ++w) s += xch[parity][wr][r][w];
        dot[r] = static_cast<TC>(s);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = base + r;
      if (row < i_end) {
        const TC uh = c_ap * dot[r] + c_u * static_cast<TC>(u_in[row]);
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
          for (int e = 0; e < VEC; ++e) q[j][e] += uh * static_cast<TC>(a[r][j][e]);
        if (wc == 0 && lane == 0) {
          u_out[row] = static_cast<typename PassTypes<MODE>::TUO>(uh);
          nrm += static_cast<double>(uh) * static_cast<double>(uh);
        }
      }
    }
  };
  // two steps in flight per wave: the loads of step s+1 are issued before
  // step s is reduced (512-thread workgroups leave the registers for it)
  TA a0[R][J][VEC], a1[R][J][VEC];
  if (nsteps > 0) load_step(0, a0);
  for (int64_t step = 0; step < nsteps; step += 2) {
    if (step + 1 < nsteps) load_step(step + 1, a1);
    compute_step(step, a0);
    if (step + 1 < nsteps) {
      if (step + 2 < nsteps) load_step(step + 2, a0);
      compute_step(step + 1, a1);
    }
  }
  };

  // The static range first, then claimed chunks.  One thread claims; each
  // claim is issued before the range in hand is processed and published at
  // the barrier that ends it (the first before the static range).
  const bool dynamic = dyn_begin < m;
  unsigned int claim = 0;
  if (dynamic && threadIdx.x == 0) claim = atomicAdd(dyn, 1u);
  const int64_t s_begin = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
  int64_t r0 = s_begin, r1 = min(min(m, dyn_begin), s_begin + rows_per_wg);
  for (int it = 0;; ++it) {
    if (it > 0 && threadIdx.x == 0) claim = atomicAdd(dyn, 1u);
    rows(r0, r1);
    if (!dynamic) break;
    if (threadIdx.x == 0) next_chunk[it & 1] = claim;
    __syncthreads();
    // the same LDS word in every lane: keep the range in scalar registers
    r0 = dyn_begin + static_cast<int64_t>(__builtin_amdgcn_readfirstlane(next_chunk[it & 1])) * chunk;
    if (r0 >= m) break;
    r1 = min(m, r0 + chunk);
  }

  // Per-workgroup partials: q (row groups combined in a fixed order through
  // LDS) and ||u||^2.
  double *qdst = qpart + static_cast<int64_t>(blockIdx.x) * n;
  if constexpr (WR > 1) {
    for (int g = 0; g < WR; ++g) {
      __syncthreads();
      if (wr == g) {
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const int cl = wc * COLS + (j * kWave + lane) * VEC + e;
            qbuf[cl] = (g == 0 ? 0.0 : qbuf[cl]) + static_cast<double>(q[j][e]);
          }
      }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n && c < WC * COLS; c += kPassThreads) qdst[c] = qbuf[c];
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int c = col0 + (j * kWave + lane) * VEC + e;
        if (c < n) qdst[c] = static_cast<double>(q[j][e]);
      }
  }
  if (lane == 0) nbuf[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kPassWaves; ++w) s += nbuf[w];
    nrmpart[blockIdx.x] = s;
    // every claim of this workgroup has returned (its value was used), so
    // the last workgroup here sees no further claims
    if (dynamic && atomicAdd(dyn + 1, 1u) == gridDim.x - 1) {
      atomicExch(dyn, 0u);
      atomicExch(dyn + 1, 0u);
    }
  }
}

// [fused-pass-end]

// --------------------------------------------------------------------------
// Explicit preconditioner M = R^-1 (the paper's choice, Sec. 3.2).  Formed
// once per solve; each iteration then applies M^T and M as wide GEMVs over
// the whole GPU instead of two chains of dependent triangular blocks.

// Upper triangle of M (n x n, column-major, ld n) by blocked back
// substitution of R X = I: for the C columns of this workgroup (all in
// diagonal block jb), X_jb = D_jb (the inverted diagonal block) and, for
// ib = jb-1 .. 0, X_ib = -D_ib sum_{kb > ib} R_{ib,kb} X_kb.  The columns
// being built live in LDS.  Each step is a 64 x K x C product followed by a
// 64 x 64 x C one; the K terms are split over the 16 waves (lane = row of the
// block, eight loads of R in flight per lane), so a step costs a few load
// latencies instead of K / 8 of them; partial sums are combined in a fixed
// order.  LDS: C n doubles of X and 16 * 64 * C partials.
constexpr int kInvThreads = 1024;
constexpr int kInvWaves = kInvThreads / kWave;

template <int C>
__global__ __launch_bounds__(kInvThreads) void tri_inverse_kernel(const double *__restrict__ R, int64_t ldr, int n,
                                                                  const double *__restrict__ Dup,
                                                                  double *__restrict__ M) {
  extern __shared__ unsigned char lds_raw[];
  double *X = reinterpret_cast<double *>(lds_raw);  // X[k + q n], q < C
  double *red = X + static_cast<size_t>(C) * n;     // red[(w 64 + r) C + q]; the w = 0 slots then hold the sums
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), w = t / kWave;
  const int c0 = static_cast<int>(blockIdx.x) * C;
  const int jb = c0 / kTrsvB;
  const int kend = min(n, (jb + 1) * kTrsvB);
  if (t < kWave * C) {  // X_jb = D_jb (columns of this workgroup)
    const int q = t / kWave, row = jb * kTrsvB + lane;
    const double *D = Dup + static_cast<int64_t>(jb) * kTrsvB * kTrsvB;
    if (row < n) X[row + q * n] = c0 + q < n ? D[lane + (c0 + q - jb * kTrsvB) * kTrsvB] : 0.0;
  }
  __syncthreads();
  for (int ib = jb - 1; ib >= 0; --ib) {
    const int row = ib * kTrsvB + lane;  // a full block: ib < jb
    const int k0 = (ib + 1) * kTrsvB;
    const int per = (kend - k0 + kInvWaves - 1) / kInvWaves;
    const int ka = min(kend, k0 + w * per), kb = min(kend, ka + per);
    double acc[C];
#pragma unroll
    for (int q = 0; q < C; ++q) acc[q] = 0.0;
    int k = ka;
    for (; k + 8 <= kb; k += 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) a[u] = R[row + static_cast<int64_t>(k + u) * ldr];
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int q = 0; q < C; ++q) acc[q] += a[u] * X[k + u + q * n];
    }
    for (; k < kb; ++k) {
      const double a = R[row + static_cast<int64_t>(k) * ldr];
#pragma unroll
      for (int q = 0; q < C; ++q) acc[q] += a * X[k + q * n];
    }
#pragma unroll
    for (int q = 0; q < C; ++q) red[(w * kWave + lane) * C + q] = acc[q];
    __syncthreads();
    if (t < kWave * C) {  // thread (r = lane, q = wave): sum over the waves, into the w = 0 slot
      const int q = w;
      double sum = 0.0;
      for (int ww = 0; ww < kInvWaves; ++ww) sum += red[(ww * kWave + lane) * C + q];
      red[lane * C + q] = sum;
    }
    __syncthreads();
    if (t < kWave * C) {  // X_ib = -D_ib T
      const int q = w;
      const double *D = Dup + static_cast<int64_t>(ib) * kTrsvB * kTrsvB;
      double x = 0.0;
#pragma unroll 16
      for (int qq = 0; qq < kTrsvB; ++qq) x -= D[lane + qq * kTrsvB] * red[qq * C + q];
      X[row + q * n] = c0 + q < n ? x : 0.0;
    }
    __syncthreads();
  }
  // write the columns out (rows 0 .. end of block jb; the rest of M's column
  // lies below the diagonal and is never read)
  for (int e = t; e < kend * C; e += kInvThreads) {
    const int k = e % kend, ql = e / kend;
    const int c = c0 + ql;
    if (c < n) M[k + static_cast<int64_t>(c) * n] = X[k + ql * n];
  }
}

// Columns per workgroup for M = R^-1: as many as fit in LDS (160 KiB per
// workgroup on gfx950, 1 KiB kept spare), at most 8.
int tri_inverse_cols(int n) {
  for (int c = 8; c > 1; c >>= 1)
    if (static_cast<size_t>(c) * (static_cast<size_t>(n) + kInvWaves * kWave) * sizeof(double) <= 159 * 1024)
      return c;
  return 1;
}

__global__ __launch_bounds__(256) void inverse_transpose_kernel(const double *__restrict__ M, int n,
                                                                double *__restrict__ Mt) {
  __shared__ double tile[32][33];
  trsv_transpose_tile(M, n, n, static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y), Mt, tile);
}

// q = sum over the pass partials, in two fixed-order levels: this kernel sums
// slice s (kQSlice consecutive partials) for 64 columns; the GEMV kernels sum
// the slices.
constexpr int kQSlice = 64;
__global__ __launch_bounds__(256) void q_slices_kernel(const double *__restrict__ qpart, int G, int n,
                                                       double *__restrict__ qs) {
  __shared__ double red[4][64];
  const int t = threadIdx.x;
  const int cl = t % 64, sub = t / 64;
  const int c = blockIdx.x * 64 + cl;
  const int g0 = blockIdx.y * kQSlice;
  const int g1 = min(G, g0 + kQSlice);
  double s = 0.0;
  if (c < n)
    for (int g = g0 + sub; g < g1; g += 4) s += qpart[static_cast<int64_t>(g) * n + c];
  red[sub][cl] = s;
  __syncthreads();
  if (sub == 0 && c < n) qs[static_cast<int64_t>(blockIdx.y) * n + c] = red[0][cl] + red[1][cl] + red[2][cl] + red[3][cl];
}

// beta = ||u_hat|| from the pass partials (fixed order, every workgroup the same).
__device__ __forceinline__ double beta_from_partials(const double *__restrict__ nrmpart, int G, double *scr) {
  double bsq = 0.0;
  for (int g = threadIdx.x; g < G; g += 1024) bsq += nrmpart[g];
  return sqrt(wg_sum(bsq, scr));
}

// v_hat = M^T q / beta - beta v (Alg. 2 in the App. D.4.1 order); one wave per
// entry j (column j of M, rows 0..j); per-workgroup partials of ||v_hat||^2.
__global__ __launch_bounds__(1024) void lsqr_mtq_kernel(const double *__restrict__ M, int n,
                                                        const double *__restrict__ qs, int nslices,
                                                        const double *__restrict__ nrmpart, int G,
                                                        const double *__restrict__ v, double *__restrict__ vh,
                                                        double *__restrict__ vpart, const LsqrState *st) {
  __shared__ double scr[16];
  __shared__ double q[kMaxN];
  __shared__ double wsum[16];
  if (st->done) return;
  const double beta = beta_from_partials(nrmpart, G, scr);
  const int t = threadIdx.x;
  for (int c = t; c < n; c += 1024) {
    double a = 0.0;
    for (int s = 0; s < nslices; ++s) a += qs[static_cast<int64_t>(s) * n + c];
    q[c] = a;
  }
  __syncthreads();
  const int lane = t & (kWave - 1), wave = t / kWave;
  const int j = blockIdx.x * 16 + wave;
  double sq = 0.0;
  if (j < n) {
    const double *__restrict__ col = M + static_cast<int64_t>(j) * n;
    double acc = 0.0;
    for (int k = lane; k <= j; k += kWave) acc += col[k] * q[k];
    acc = wave_sum_u(acc);
    const double vhj = beta > 0.0 ? acc / beta - (st->init ? 0.0 : beta * v[j]) : 0.0;
    if (lane == 0) vh[j] = vhj;
    sq = vhj * vhj;
  }
  if (lane == 0) wsum[wave] = sq;
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
    for (int w = 0; w < 16; ++w) a += wsum[w];
    vpart[blockIdx.x] = a;
  }
}

// alpha = ||v_hat||, v = v_hat / alpha, p = M v; one wave per entry r (row r
// of M = column r of M^T, rows r..n-1).  Workgroup 0 records beta, alpha.
__global__ __launch_bounds__(1024) void lsqr_mv_kernel(const double *__restrict__ Mt, int n,
                                                       const double *__restrict__ vh, const double *__restrict__ vpart,
                                                       int nvpart, const double *__restrict__ nrmpart, int G,
                                                       double *__restrict__ v, double *__restrict__ p,
                                                       float *__restrict__ p32, LsqrState *st) {
  __shared__ double scr[16];
  __shared__ double vs[kMaxN];
  if (st->done) return;
  const double beta = beta_from_partials(nrmpart, G, scr);
  const int t = threadIdx.x;
  double asq = 0.0;
  for (int k = t; k < nvpart; k += 1024) asq += vpart[k];
  const double alpha = beta > 0.0 ? sqrt(wg_sum(asq, scr)) : 0.0;
  const bool proceed = beta > 0.0 && alpha > 0.0;
  if (!proceed) {
    if (blockIdx.x == 0 && t == 0) {
      st->beta_new = beta;
      st->alpha_new = alpha;
      st->proceed = 0;
    }
    return;
  }
  const double ia = 1.0 / alpha;
  for (int c = t; c < n; c += 1024) vs[c] = vh[c] * ia;
  __syncthreads();
  const int lane = t & (kWave - 1), wave = t / kWave;
  const int rr = blockIdx.x * 16 + wave;
  if (rr < n) {
    const double *__restrict__ col = Mt + static_cast<int64_t>(rr) * n;
    double acc = 0.0;
    for (int k = rr + lane; k < n; k += kWave) acc += col[k] * vs[k];
    acc = wave_sum_u(acc);
    if (lane == 0) {
      p[rr] = acc;
      if (p32) p32[rr] = static_cast<float>(acc);
      v[rr] = vs[rr];
    }
  }
  if (blockIdx.x == 0 && t == 0) {
    st->beta_new = beta;
    st->alpha_new = alpha;
    st->proceed = 1;
  }
}

// Plane rotation, x and w updates, stopping test (one workgroup).
__global__ __launch_bounds__(kTrsvThreads) void lsqr_update_kernel(const double *p, double *__restrict__ w,
                                                                   double *__restrict__ x, int n, LsqrState *st) {
  if (st->done) return;
  upper_epilogue(n, p, w, x, st, nullptr);
}

// Fresh state for an LSQR run; clears the chain flags of the two solves.
__global__ void lsqr_init_state_kernel(LsqrState *st, double tol, int maxiter, int *flags, int nflags,
                                       int total_iters, int rel, unsigned int *dyn) {
  for (int i = threadIdx.x; i < nflags; i += blockDim.x) flags[i] = 0;
  if (threadIdx.x != 0) return;
  __hip_atomic_store(dyn, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(dyn + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
  st->alpha_new = st->beta_new = 0.0;
  st->c_ap = -1.0;
  st->c_u = 1.0;
  st->tol = tol;
  st->resid_est = st->normar_est = 0.0;
  st->iter = 0;
  st->maxiter = maxiter;
  st->done = 0;
  st->converged = 0;
  st->init = 1;
  st->proceed = 0;
  st->total_iters = total_iters;
  st->steps = 0;
  st->rel = rel;
}

// ||b|| into st->normb: per-workgroup partial sums, then a fixed-order sum
// by the last workgroup to finish.
__global__ __launch_bounds__(1024) void norm_kernel(const double *__restrict__ b, int64_t m, double *partial,
                                                    unsigned int *ticket, LsqrState *__restrict__ st) {
  __shared__ double scr[16];
  __shared__ bool last;
  double s = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 1024 + threadIdx.x; i < m;
       i += static_cast<int64_t>(gridDim.x) * 1024)
    s += b[i] * b[i];
  s = wg_sum(s, scr);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    double tot = 0.0;
    for (unsigned g = 0; g < gridDim.x; ++g)
      tot += __hip_atomic_load(&partial[g], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    st->normb = sqrt(tot);
    *ticket = 0;
  }
}

__global__ void copy_f64_kernel(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// --------------------------------------------------------------------------
// Pass configuration: columns per wave = 64 * VEC * J, WC waves across the
// columns.
struct PassCfg {
  int vec, j, wc;
};

template <int MODE>
PassCfg choose_pass(int n, int64_t lda, const void *A) {
  using TA = typename PassTypes<MODE>::TA;
  const int vmax = 16 / static_cast<int>(sizeof(TA));
  const bool aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % vmax == 0) && (n % vmax == 0);
  PassCfg c{aligned ? vmax : 1, 2, 1};
  // at most 16 elements of a row per lane (A values, p and q live in
  // registers); at most kPassWaves waves across a row (n <= 8192 needs 8)
  const int jmax = 16 / c.vec;
  const int per_j = kWave * c.vec;
  const int need = (n + per_j - 1) / per_j;  // J * WC needed
  if (need <= jmax) {
    int j = 2;
    while (j < need) j <<= 1;
    c.j = j;
    c.wc = 1;
  } else {
    c.j = jmax;
    int wc = 2;
    while (wc * jmax < need) wc <<= 1;
    c.wc = wc;
  }
  return c;
}

template <int MODE, int VEC, int J, int WC>
const void *pass_fn() {
  return reinterpret_cast<const void *>(&lsqr_pass_kernel<MODE, VEC, J, WC>);
}

template <int MODE, int VEC, int J>
const void *pick_wc(int wc) {
  switch (wc) {
    case 2: return pass_fn<MODE, VEC, J, 2>();
    case 4: return pass_fn<MODE, VEC, J, 4>();
    default: return pass_fn<MODE, VEC, J, 8>();  // kPassWaves
  }
}

// J that pick_vec instantiates for c (the host mirror of its choice).
int pass_j(const PassCfg &c) {
  const int jmax = 16 / c.vec;
  if (c.wc > 1) return jmax;
  if (c.j == 2 || c.j == 4 || (c.j == 8 && jmax >= 8)) return c.j;
  return jmax;
}

template <int MODE, int VEC>
const void *pick_vec(const PassCfg &c) {
  constexpr int JMAX = 16 / VEC;
  if (c.wc == 1) {
    switch (pass_j(c)) {
      case 2: return pass_fn<MODE, VEC, 2, 1>();
      case 4: return pass_fn<MODE, VEC, 4, 1>();
      case 8:
        if constexpr (JMAX >= 8) return pass_fn<MODE, VEC, 8, 1>();
        [[fallthrough]];
      default: return pass_fn<MODE, VEC, JMAX, 1>();
    }
  }
  return pick_wc<MODE, VEC, JMAX>(c.wc);
}

template <int MODE>
const void *pick_pass(const PassCfg &c) {
  constexpr int vmax = 16 / static_cast<int>(sizeof(typename PassTypes<MODE>::TA));
  return c.vec == 1 ? pick_vec<MODE, 1>(c) : pick_vec<MODE, vmax>(c);
}

std::mutex g_occ_mu;
std::unordered_map<const void *, int> g_occ;

int occupancy(const void *fn) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto it = g_occ.find(fn);
  if (it != g_occ.end()) return it->second;
  int blocks = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kPassThreads, 0) != hipSuccess || blocks < 1)
    blocks = 1;
  g_occ[fn] = blocks;
  return blocks;
}

struct PassPlan {
  const void *fn;
  int grid;
  int64_t rows_per_wg;  // static rows per workgroup
  int64_t dyn_begin;    // first row of the dynamically claimed tail
  int chunk;            // rows per claim
};

int max_grid(sap_ctx *ctx) { return ctx->num_cus * 2; }

// Rows one step of the kernel pick_pass returns for c covers: WR =
// kPassWaves / WC row groups of R rows.
int rows_per_step(int mode, const PassCfg &c) {
  return (kPassWaves / c.wc) * pass_rows(mode, pass_j(c) * c.vec);
}

// Share of the rows assigned statically (the rest is claimed in chunks),
// for passes over at least kDynamicMinBytes of A; shorter passes split the
// rows statically (the XCD imbalance is a few microseconds there, less than
// the claims cost).
constexpr double kStaticShare = 0.875;
constexpr int kStepsPerChunk = 4;
constexpr double kDynamicMinBytes = 512.0 * 1024 * 1024;

PassPlan plan_pass(sap_ctx *ctx, int mode, int64_t m, int n, int64_t lda, const void *A) {
  const void *fn;
  PassCfg c;
  const double a_bytes = static_cast<double>(m) * n * (mode == 0 ? 8.0 : 4.0);
  if (mode == 0) { c = choose_pass<0>(n, lda, A); fn = pick_pass<0>(c); }
  else if (mode == 1) { c = choose_pass<1>(n, lda, A); fn = pick_pass<1>(c); }
  else if (mode == 2) { c = choose_pass<2>(n, lda, A); fn = pick_pass<2>(c); }
  else { c = choose_pass<3>(n, lda, A); fn = pick_pass<3>(c); }
  int64_t grid = static_cast<int64_t>(ctx->num_cus) * std::min(2, occupancy(fn));
  const int64_t min_rows = 64;
  if (grid * min_rows > m) grid = (m + min_rows - 1) / min_rows;
  if (grid < 1) grid = 1;
  const int64_t step = rows_per_step(mode, c);
  if (a_bytes < kDynamicMinBytes) return PassPlan{fn, static_cast<int>(grid), (m + grid - 1) / grid, m, 0};
  const int64_t per_wg = static_cast<int64_t>(kStaticShare * static_cast<double>(m) / static_cast<double>(grid)) /
                         step * step;
  return PassPlan{fn, static_cast<int>(grid), per_wg, grid * per_wg, static_cast<int>(step * kStepsPerChunk)};
}

void launch_pass(sap_ctx *ctx, const PassPlan &pl, const void *A, int64_t lda, int64_t m, int n, const void *p,
                 const void *u_in, void *u_out, const LsqrState *st, double *qpart, double *nrmpart,
                 unsigned int *dyn, hipStream_t s) {
  int64_t lda_ = lda, m_ = m, rows = pl.rows_per_wg, dyn_begin = pl.dyn_begin;
  int n_ = n, chunk = pl.chunk;
  const void *A_ = A, *p_ = p, *ui = u_in, *st_ = st;
  void *uo = u_out, *qp = qpart, *np = nrmpart, *dy = dyn;
  void *args[] = {&A_, &lda_, &m_, &n_, &p_, &ui, &uo, &st_, &qp, &np, &rows, &dyn_begin, &chunk, &dy};
  hipEvent_t pb = prof_begin(ctx, s);
  const hipError_t e = hipLaunchKernel(pl.fn, dim3(pl.grid), dim3(kPassThreads), args, 0, s);
  if (e != hipSuccess) (void)e;  // reported by the hipGetLastError check after the batch
  prof_end(ctx, kProfPass, pb, s);
}

}  // namespace

size_t lsqr_workspace_bytes(sap_ctx *ctx, int64_t m, int n) {
  const size_t G = static_cast<size_t>(max_grid(ctx));
  const size_t nblk = static_cast<size_t>((n + kTrsvB - 1) / kTrsvB);
  size_t bytes = 256 * 32;                                // alignment slack
  bytes += sizeof(LsqrState);
  bytes += G * n * sizeof(double) + G * sizeof(double);  // partials
  bytes += 6 * static_cast<size_t>(n) * sizeof(double);  // v w p x0copy (+1 spare)
  bytes += 2 * static_cast<size_t>(m) * sizeof(double);  // u, two buffers
  bytes += (3 * nblk + 16) * sizeof(int) + 4096 * sizeof(double);                  // flags, err, norm partials
  bytes += 2 * sizeof(unsigned int);                                               // pass claim counters
  bytes += 2 * static_cast<size_t>(n) * n * sizeof(double);                        // M = R^-1 and M^T
  bytes += (static_cast<size_t>((G + kQSlice - 1) / kQSlice) + 2) * n * sizeof(double);  // q slices, v_hat
  bytes += static_cast<size_t>((n + 15) / 16 + 1) * sizeof(double);                // ||v_hat||^2 partials
  bytes += static_cast<size_t>(n) * (sizeof(float) + sizeof(double)) + 2 * sizeof(double);  // p32, xprev, norms
  bytes += trsv_factor_bytes(n);
  return bytes;
}

size_t trsv_workspace_bytes(int n) {
  return trsv_factor_bytes(n) + 8 * 256 + ((n + kTrsvB - 1) / kTrsvB + 8) * sizeof(int);
}

sap_status launch_trsv(sap_ctx *ctx, const double *R, int64_t ldr, int n, int trans, const double *rhs, double *x,
                       void *work, hipStream_t st) {
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "sap_trsv: n > 8192 is not supported");
  Carve cv(work);
  int *flags = cv.take<int>((n + kTrsvB - 1) / kTrsvB + 1);
  int *err = cv.take<int>(1);
  TrsvFactor f;
  trsv_factor_carve(f, cv, n);
  sap_status s = trsv_prepare(ctx, R, ldr, f, st);
  if (s != SAP_OK) return s;
  SAP_HIP_TRY(hipMemsetAsync(err, 0, sizeof(int), st));
  s = trsv_solve(ctx, f, trans == 0, rhs, x, flags, err, st);
  if (s != SAP_OK) return s;
  int herr = 0;
  SAP_HIP_TRY(hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st));
  SAP_HIP_TRY(hipStreamSynchronize(st));
  if (herr) return fail(ctx, SAP_EDEVICE, "sap_trsv: a block wait expired");
  return SAP_OK;
}

namespace {

// out[0] = ||x - xprev||, out[1] = ||x|| (fixed-order sums, one workgroup).
__global__ __launch_bounds__(1024) void delta_norm_kernel(const double *__restrict__ x, const double *__restrict__ xprev,
                                                          int n, double *__restrict__ out) {
  __shared__ double scr[16];
  double a = 0.0, b = 0.0;
  for (int c = threadIdx.x; c < n; c += 1024) {
    const double dx = x[c] - xprev[c];
    a += dx * dx;
    b += x[c] * x[c];
  }
  a = wg_sum(a, scr);
  b = wg_sum(b, scr);
  if (threadIdx.x == 0) {
    out[0] = sqrt(a);
    out[1] = sqrt(b);
  }
}

}  // namespace

namespace {

// The LSQR (and momentum) buffers carved from the workspace, in the order
// lsqr_workspace_bytes counts them.
struct LsqrBufs {
  LsqrState *st;
  double *qpart, *nrmpart, *v, *w, *p, *xin;
  // u alternates between two buffers: with several waves across a row
  // (n > 1024), every wave of the row reads u_in[i] while one of them writes
  // u_out[i], so a pass must not update u in place.  FP32 values in the
  // refinement form.
  double *ubuf[2];
  int *flags, *flags_x0, *err;
  unsigned int *ticket, *dyn;
  double *normpart, *M, *Mt, *qs, *vh, *vpart;
  float *p32;
  double *xprev, *dnorm;
  TrsvFactor f;
  int nblk, nslices, ngemv;
};

LsqrBufs carve_lsqr(sap_ctx *ctx, void *work, int64_t m, int n) {
  LsqrBufs B;
  Carve cv(work);
  B.nblk = (n + kTrsvB - 1) / kTrsvB;
  B.st = cv.take<LsqrState>(1);
  B.qpart = cv.take<double>(static_cast<size_t>(max_grid(ctx)) * n);
  B.nrmpart = cv.take<double>(max_grid(ctx));
  B.v = cv.take<double>(n);
  B.w = cv.take<double>(n);
  B.p = cv.take<double>(n);
  B.xin = cv.take<double>(n);
  B.ubuf[0] = cv.take<double>(m);
  B.ubuf[1] = cv.take<double>(m);
  B.flags = cv.take<int>(3 * B.nblk + 2);
  B.flags_x0 = B.flags + 2 * B.nblk;
  B.err = cv.take<int>(4);
  B.ticket = reinterpret_cast<unsigned int *>(B.err + 1);
  B.dyn = cv.take<unsigned int>(2);  // pass row-claim counters
  B.normpart = cv.take<double>(4096);
  B.nslices = (max_grid(ctx) + kQSlice - 1) / kQSlice;
  B.M = cv.take<double>(static_cast<size_t>(n) * n);
  B.Mt = cv.take<double>(static_cast<size_t>(n) * n);
  B.qs = cv.take<double>(static_cast<size_t>(B.nslices) * n);
  B.vh = cv.take<double>(n);
  B.ngemv = (n + 15) / 16;
  B.vpart = cv.take<double>(B.ngemv);
  B.p32 = cv.take<float>(n);
  B.xprev = cv.take<double>(n);
  B.dnorm = cv.take<double>(2);
  trsv_factor_carve(B.f, cv, n);
  return B;
}

// x0 (R^-1 z when z is given, else a copy of x0), then M = R^-1 and M^T.
sap_status setup_precond(sap_ctx *ctx, const double *R, int64_t ldr, const double *x0, const double *z, double *x,
                         LsqrBufs &B, int n, hipStream_t s) {
  sap_status sst = trsv_prepare(ctx, R, ldr, B.f, s);
  if (sst != SAP_OK) return sst;
  SAP_HIP_TRY(hipMemsetAsync(B.err, 0, 4 * sizeof(int), s));
  if (z) {
    // x0 = R^-1 z: the minimiser of ||S b - S A x|| (Alg. 1, initial guess)
    sst = trsv_solve(ctx, B.f, true, z, x, B.flags_x0, B.err, s);
    if (sst != SAP_OK) return sst;
  } else {
    // x0 may alias x: copy first.
    copy_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(x0, B.xin, n);
    copy_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(B.xin, x, n);
  }
  // M = R^-1 and its transpose (the columns a workgroup builds sit in LDS)
  const unsigned nt = static_cast<unsigned>((n + 31) / 32);
  const int ci = tri_inverse_cols(n);
  const size_t lds = static_cast<size_t>(ci) * (static_cast<size_t>(n) + kInvWaves * kWave) * sizeof(double);
  const unsigned gi = static_cast<unsigned>((n + ci - 1) / ci);
  switch (ci) {
    case 8: tri_inverse_kernel<8><<<gi, kInvThreads, lds, s>>>(R, ldr, n, B.f.Dup, B.M); break;
    case 4: tri_inverse_kernel<4><<<gi, kInvThreads, lds, s>>>(R, ldr, n, B.f.Dup, B.M); break;
    case 2: tri_inverse_kernel<2><<<gi, kInvThreads, lds, s>>>(R, ldr, n, B.f.Dup, B.M); break;
    default: tri_inverse_kernel<1><<<gi, kInvThreads, lds, s>>>(R, ldr, n, B.f.Dup, B.M); break;
  }
  inverse_transpose_kernel<<<dim3(nt, nt), 256, 0, s>>>(B.M, n, B.Mt);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

// ---- iteration batches -------------------------------------------------------
// A batch of iterations is captured once into a hipGraph and replayed: the
// launches of one batch are the same every time (the u buffers alternate an
// even number of times), so the captured graph is valid for as long as every
// value it bakes in is unchanged; the key lists them.  Capture runs on a
// context-owned stream (the caller's may be the null stream); the graph is
// launched on the caller's.  Timing mode (sap_profile_enable) records events
// around each pass, so it launches directly.
struct GraphKey {
  uint64_t v[32];
  int n = 0;
  void add(uint64_t x) { v[n++] = x; }
  void addp(const void *p) { add(static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p))); }
  void addd(double d) {
    uint64_t u;
    std::memcpy(&u, &d, sizeof u);
    add(u);
  }
  bool operator==(const GraphKey &o) const { return n == o.n && std::memcmp(v, o.v, sizeof(uint64_t) * n) == 0; }
};

struct BatchGraphs {
  struct Entry {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
  } e[4];
  int next = 0;
  hipStream_t cap = nullptr;
};

template <typename F>
hipGraphExec_t batch_graph(sap_ctx *ctx, const GraphKey &key, F &&launch) {
  if (ctx->profiling) return nullptr;
  auto *G = static_cast<BatchGraphs *>(ctx->batch_graphs);
  if (!G) {
    G = new BatchGraphs();
    ctx->batch_graphs = G;
  }
  for (auto &en : G->e)
    if (en.exec && en.key == key) return en.exec;
  if (!G->cap && hipStreamCreateWithFlags(&G->cap, hipStreamNonBlocking) != hipSuccess) {
    G->cap = nullptr;
    (void)hipGetLastError();
    return nullptr;
  }
  if (hipStreamBeginCapture(G->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  launch(G->cap);
  hipGraph_t g = nullptr;
  if (hipStreamEndCapture(G->cap, &g) != hipSuccess || !g) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess || !ex) {
    (void)hipGetLastError();
    return nullptr;
  }
  auto &slot = G->e[G->next];
  G->next = (G->next + 1) % 4;
  if (slot.exec) (void)hipGraphExecDestroy(slot.exec);
  slot.exec = ex;
  slot.key = key;
  return ex;
}

// Host view of one batch's end state (pinned, two slots).
struct BatchSlot {
  LsqrState st;
  int err;
};

// Run batches until the state reports done: batch k+1 is enqueued before the
// state of batch k is waited for, so the device does not idle on the host's
// read (a batch after `done` finds every kernel returning at once).  The
// last state read lands in *hs, the error word in *herr.
template <typename F>
sap_status run_batches(sap_ctx *ctx, hipGraphExec_t exec, F &&launch_direct, const LsqrState *st, const int *err,
                       int max_batches, LsqrState *hs, int *herr, hipStream_t s, const char *who) {
  auto *slots = static_cast<BatchSlot *>(ctx->pinned);
  auto enqueue = [&](int slot) -> hipError_t {
    if (exec) {
      const hipError_t e = hipGraphLaunch(exec, s);
      if (e != hipSuccess) return e;
    } else {
      launch_direct(s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&slots[slot].st, st, sizeof(LsqrState), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(&slots[slot].err, err, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(ctx->batch_ev[slot], s);
  };
  SAP_HIP_TRY(enqueue(0));
  for (int nbatch = 0;; ++nbatch) {
    const int cur = nbatch & 1;
    if (nbatch + 1 <= max_batches) SAP_HIP_TRY(enqueue(cur ^ 1));
    SAP_HIP_TRY(hipEventSynchronize(ctx->batch_ev[cur]));
    *hs = slots[cur].st;
    *herr = slots[cur].err;
    if (*herr) return fail(ctx, SAP_EDEVICE, std::string(who) + ": a triangular-solve wait expired");
    if (hs->done) return SAP_OK;
    if (nbatch + 1 > max_batches) return fail(ctx, SAP_EDEVICE, std::string(who) + ": device never reported completion");
  }
}

// ---- heavy-ball momentum (App. D.3) ----------------------------------------
// s = M^T q (q summed from the pass slices: q = A^T r, r = b - A x); one wave
// per entry j (column j of M, rows 0..j); per-workgroup partials of ||s||^2.
__global__ __launch_bounds__(1024) void hbm_mtq_kernel(const double *__restrict__ M, int n,
                                                       const double *__restrict__ qs, int nslices,
                                                       double *__restrict__ sv, double *__restrict__ spart,
                                                       LsqrState *st) {
  __shared__ double q[kMaxN];
  __shared__ double wsum[16];
  if (st->done) return;
  const int t = threadIdx.x;
  for (int c = t; c < n; c += 1024) {
    double a = 0.0;
    for (int k = 0; k < nslices; ++k) a += qs[static_cast<int64_t>(k) * n + c];
    q[c] = a;
  }
  __syncthreads();
  const int lane = t & (kWave - 1), wave = t / kWave;
  const int j = blockIdx.x * 16 + wave;
  double sq = 0.0;
  if (j < n) {
    const double *__restrict__ col = M + static_cast<int64_t>(j) * n;
    double acc = 0.0;
    for (int k = lane; k <= j; k += kWave) acc += col[k] * q[k];
    acc = wave_sum_u(acc);
    if (lane == 0) sv[j] = acc;
    sq = acc * acc;
  }
  if (lane == 0) wsum[wave] = sq;
  __syncthreads();
  if (t == 0) {
    double a = 0.0;
    for (int w = 0; w < 16; ++w) a += wsum[w];
    spart[blockIdx.x] = a;
    // step counter of the momentum iteration (read by hbm_step_kernel only,
    // which runs after this kernel; no workgroup here reads it)
    if (blockIdx.x == 0) st->iter += 1;
  }
}

// One step from x_t (t updates made): the stopping test on x_t when t >= 1
// (||r_t|| = 0, ||s_t|| <= tol ||r_t|| or ||r_t|| <= tol ||b||), or the cap
// t = maxiter; otherwise g = M s_t (the paper's g_{t+1}, formed from the
// residual), delta <- alpha g + beta delta and x <- x + delta, so that
// delta = x_{t+1} - x_t carries the momentum.  Every workgroup takes the same
// decision from the same partials; only workgroup 0 writes the state.
__global__ __launch_bounds__(1024) void hbm_step_kernel(const double *__restrict__ Mt, int n,
                                                        const double *__restrict__ sv,
                                                        const double *__restrict__ spart, int nspart,
                                                        const double *__restrict__ nrmpart, int G,
                                                        double alpha, double beta, double *__restrict__ delta,
                                                        double *__restrict__ x, LsqrState *st) {
  __shared__ double scr[16];
  __shared__ double ss[kMaxN];
  if (st->done) return;
  const int t = st->iter - 1;  // updates made: hbm_mtq_kernel advanced the counter for this step
  const double rn = beta_from_partials(nrmpart, G, scr);
  double a = 0.0;
  for (int k = threadIdx.x; k < nspart; k += 1024) a += spart[k];
  const double sn = sqrt(wg_sum(a, scr));
  const bool conv = t >= 1 && (rn == 0.0 || sn <= st->tol * rn || rn <= st->tol * st->normb);
  if (conv || t >= st->maxiter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->done = 1;
      st->converged = conv ? 1 : 0;
      st->total_iters = t;
      st->resid_est = rn;
      st->normar_est = sn;
    }
    return;
  }
  for (int c = threadIdx.x; c < n; c += 1024) ss[c] = sv[c];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int rr = blockIdx.x * 16 + wave;
  if (rr < n) {
    const double *__restrict__ col = Mt + static_cast<int64_t>(rr) * n;
    double acc = 0.0;
    for (int k = rr + lane; k < n; k += kWave) acc += col[k] * ss[k];
    acc = wave_sum_u(acc);
    if (lane == 0) {
      const double dl = alpha * acc + beta * delta[rr];
      delta[rr] = dl;
      x[rr] += dl;
    }
  }
}

__global__ void zero_f64_kernel(double *__restrict__ p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

// ---- s-step form (App. D.4.2) --------------------------------------------
// out = M in (or xacc += M in when xacc is non-null): one wave per row r,
// row r of M read as column r of M^T (entries r .. n-1).
__global__ __launch_bounds__(1024) void sstep_mv_kernel(const double *__restrict__ Mt, int n,
                                                        const double *__restrict__ in, double *__restrict__ out,
                                                        double *__restrict__ xacc) {
  __shared__ double v[kMaxN];
  for (int c = threadIdx.x; c < n; c += 1024) v[c] = in[c];
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int r = blockIdx.x * 16 + wave;
  if (r >= n) return;
  const double *__restrict__ col = Mt + static_cast<int64_t>(r) * n;
  double acc = 0.0;
  for (int k = r + lane; k < n; k += kWave) acc += col[k] * v[k];
  acc = wave_sum_u(acc);
  if (lane == 0) {
    if (xacc) xacc[r] += acc;
    else out[r] = acc;
  }
}

// The next Chebyshev basis vector: u_{k+1} = (Z u_k - c u_k)/h for k = 0,
// 2 (Z u_k - c u_k)/h - u_{k-1} after.
__global__ void sstep_cheb_kernel(int n, int k, double c, double h, const double *__restrict__ wk,
                                  const double *__restrict__ uk, const double *__restrict__ ukm1,
                                  double *__restrict__ unext) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double y = (wk[i] - c * uk[i]) / h;
  unext[i] = k == 0 ? y : 2.0 * y - ukm1[i];
}

// Gram entries, one workgroup each (fixed summation order): block (j, k < s)
// gives Graw[j + k s] = u_j . (Z u_k), block (j, s) gives g[j] = u_j . u_0.
__global__ __launch_bounds__(256) void sstep_gram_kernel(const double *__restrict__ U,
                                                         const double *__restrict__ W, int n, int s,
                                                         double *__restrict__ Graw, double *__restrict__ g) {
  __shared__ double scr[4];
  const int j = blockIdx.x, k = blockIdx.y;
  const double *__restrict__ a = U + static_cast<int64_t>(j) * n;
  const double *__restrict__ b = (k < s) ? W + static_cast<int64_t>(k) * n : U;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += a[i] * b[i];
  acc = wave_sum_u(acc);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) scr[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = scr[0] + scr[1] + scr[2] + scr[3];
    if (k < s) Graw[j + static_cast<int64_t>(k) * s] = t;
    else g[j] = t;
  }
}

// (U^T Z U) c = U^T r0 by Cholesky of the symmetrised Gram matrix, one
// thread (s <= kMaxSstep).  A pivot at or below 1e-12 of its diagonal entry
// stops the factorisation: the basis has become numerically dependent, and
// the system is solved on the steps before it (the rest of c is zero).
__global__ void sstep_solve_kernel(int s, const double *__restrict__ Graw, const double *__restrict__ g,
                                   double *__restrict__ c) {
  if (threadIdx.x != 0) return;
  double G[kMaxSstep * kMaxSstep], L[kMaxSstep * kMaxSstep], y[kMaxSstep];
  for (int j = 0; j < s; ++j)
    for (int k = 0; k < s; ++k) {
      G[j + k * s] = 0.5 * (Graw[j + k * s] + Graw[k + j * s]);
      L[j + k * s] = 0.0;
    }
  int kk = 0;
  for (int j = 0; j < s; ++j) {
    double dj = G[j + j * s];
    for (int i = 0; i < j; ++i) dj -= L[j + i * s] * L[j + i * s];
    if (!(dj > 1e-12 * G[j + j * s])) break;
    const double ljj = sqrt(dj);
    L[j + j * s] = ljj;
    for (int r = j + 1; r < s; ++r) {
      double v = G[r + j * s];
      for (int i = 0; i < j; ++i) v -= L[r + i * s] * L[j + i * s];
      L[r + j * s] = v / ljj;
    }
    kk = j + 1;
  }
  for (int j = 0; j < s; ++j) c[j] = 0.0;
  for (int j = 0; j < kk; ++j) {
    double v = g[j];
    for (int i = 0; i < j; ++i) v -= L[j + i * s] * y[i];
    y[j] = v / L[j + j * s];
  }
  for (int j = kk - 1; j >= 0; --j) {
    double v = y[j];
    for (int i = j + 1; i < kk; ++i) v -= L[i + j * s] * c[i];
    c[j] = v / L[j + j * s];
  }
}

// y = U c (n x s times s).
__global__ void sstep_combine_kernel(const double *__restrict__ U, int n, int s, const double *__restrict__ c,
                                     double *__restrict__ y) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double a = 0.0;
  for (int j = 0; j < s; ++j) a += U[i + static_cast<int64_t>(j) * n] * c[j];
  y[i] = a;
}

// out[0] = ||r|| from the pass partials, out[1] = ||M^T A^T r|| from the
// M^T q partials, out[2] = ||b|| (one workgroup, fixed order).
__global__ __launch_bounds__(1024) void sstep_norms_kernel(const double *__restrict__ nrmpart, int G,
                                                           const double *__restrict__ spart, int nsp,
                                                           const LsqrState *__restrict__ st,
                                                           double *__restrict__ out) {
  __shared__ double scr[16];
  const double rn = beta_from_partials(nrmpart, G, scr);
  double a = 0.0;
  for (int k = threadIdx.x; k < nsp; k += 1024) a += spart[k];
  const double fn = sqrt(wg_sum(a, scr));
  if (threadIdx.x == 0) {
    out[0] = rn;
    out[1] = fn;
    out[2] = st->normb;
  }
}

// The product state: every pass run with it forms u = A p (u_in unused).
__global__ void sstep_zstate_kernel(const LsqrState *__restrict__ src, LsqrState *__restrict__ dst) {
  if (threadIdx.x != 0) return;
  *dst = *src;
  dst->c_ap = 1.0;
  dst->c_u = 0.0;
  dst->done = 0;
}

}  // namespace


// Runs LSQR (Alg. 2) from x0 on A R^-1.  mode 0: A in FP64; mode 1: A
// stored in FP32, FP64 arithmetic throughout; mode 2: A stored in FP32,
// residual refinement: each outer step forms r = b - A x with FP64
// accumulation and solves min ||r - A delta|| by LSQR with FP32 products,
// accumulation and u until that problem's normal-equation residual has
// dropped by kInnerReduction or reached FP32 resolution; x += delta.  The
// refinement stops when ||delta|| <= tol ||x|| (the inner reduction makes
// the remaining error much smaller than the last correction), and gives up
// when a correction is no smaller than the one before (the FP32 inner solves
// cannot resolve the remaining error) or after max_refine steps.
sap_status run_lsqr(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *x0,
                    const double *z, double tol, int maxiter, int mode, int max_refine, double *x, sap_info *info,
                    void *work, hipStream_t s, const SparseA *sp) {
  constexpr double kInnerTol = 0x1p-23;  // FP32 resolution of the inner test
  const int64_t m = prob->m;
  const int n = prob->n;
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "LSQR: n > 8192 is not supported");
  const bool refine = mode == 2;
  if (sp && refine) return fail(ctx, SAP_EINVAL, "LSQR: the refinement form is not available for sparse A");
  PassPlan plan{}, plan_res{};
  if (sp) {
    plan.grid = csr_pass_grid(ctx, *sp);
    plan_res = plan;
  } else {
    plan = plan_pass(ctx, refine ? 2 : mode, m, n, prob->lda, prob->A);
    plan_res = refine ? plan_pass(ctx, 3, m, n, prob->lda, prob->A) : plan;
  }
  if (plan.grid > max_grid(ctx) || plan_res.grid > max_grid(ctx))
    return fail(ctx, SAP_EINVAL, "LSQR: internal grid larger than planned");
  LsqrBufs B = carve_lsqr(ctx, work, m, n);
  LsqrState *st = B.st;
  double *qpart = B.qpart, *nrmpart = B.nrmpart, *v = B.v, *w = B.w, *p = B.p;
  double *ubuf[2] = {B.ubuf[0], B.ubuf[1]};
  int ucur = 0;  // ubuf[ucur] holds the current u
  int *flags = B.flags, *err = B.err;
  unsigned int *ticket = B.ticket, *dyn = B.dyn;
  double *normpart = B.normpart, *M = B.M, *Mt = B.Mt, *qs = B.qs, *vh = B.vh, *vpart = B.vpart;
  float *p32 = B.p32;
  double *xprev = B.xprev, *dnorm = B.dnorm;
  const int nblk = B.nblk, ngemv = B.ngemv;
  sap_status sst = setup_precond(ctx, R, ldr, x0, z, x, B, n, s);
  if (sst != SAP_OK) return sst;
  lsqr_init_state_kernel<<<1, 256, 0, s>>>(st, refine ? kInnerTol : tol, maxiter, flags, 2 * nblk, 0,
                                           refine ? 1 : 0, dyn);
  const int ngrid = static_cast<int>(std::min<int64_t>(256, (m + 1023) / 1024));
  norm_kernel<<<ngrid, 1024, 0, s>>>(prob->b, m, normpart, ticket, st);
  SAP_HIP_TRY(hipGetLastError());

  // One iteration = pass over A; q from the pass partials; v_hat = M^T q /
  // beta - beta v; alpha, v, p = M v; rotation, x and w updates and the
  // stopping test.
  auto iteration = [&](const PassPlan &pl, const void *pv, const void *uin, hipStream_t ls) {
    const int G = pl.grid;
    const int qsl = (G + kQSlice - 1) / kQSlice;
    if (sp)
      launch_csr_pass(ctx, *sp, G, static_cast<const double *>(pv), static_cast<const double *>(uin), ubuf[ucur ^ 1],
                      st, qpart, nrmpart, ls);
    else
      launch_pass(ctx, pl, prob->A, prob->lda, m, n, pv, uin, ubuf[ucur ^ 1], st, qpart, nrmpart, dyn, ls);
    ucur ^= 1;
    q_slices_kernel<<<dim3((n + 63) / 64, qsl), 256, 0, ls>>>(qpart, G, n, qs);
    lsqr_mtq_kernel<<<ngemv, 1024, 0, ls>>>(M, n, qs, qsl, nrmpart, G, v, vh, vpart, st);
    lsqr_mv_kernel<<<ngemv, 1024, 0, ls>>>(Mt, n, vh, vpart, ngemv, nrmpart, G, v, p, refine ? p32 : nullptr, st);
    lsqr_update_kernel<<<1, kTrsvThreads, 0, ls>>>(p, w, x, n, st);
  };

  const int batch = 8;
  LsqrState hs{};
  int herr = 0;
  int refinements = 0;
  bool converged = false;
  double prev_delta = INFINITY;
  const int max_outer = refine ? (max_refine > 0 ? max_refine : 10) : 1;
  for (int outer = 0; outer < max_outer; ++outer) {
    if (outer > 0)
      lsqr_init_state_kernel<<<1, 256, 0, s>>>(st, kInnerTol, maxiter, flags, 0, hs.total_iters, 1, dyn);
    if (refine) copy_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(x, xprev, n);
    // Initialisation: beta_1 u_1 = b - A x (the pass with p = x, u_in = b);
    // in the refinement form this is the FP64-accumulated residual pass.
    iteration(plan_res, x, prob->b, s);
    SAP_HIP_TRY(hipGetLastError());
    if (refine) {
      ++refinements;
      SAP_HIP_TRY(hipMemcpyAsync(&hs, st, sizeof(LsqrState), hipMemcpyDeviceToHost, s));
      SAP_HIP_TRY(hipStreamSynchronize(s));
      if (hs.done) {  // breakdown: r or (A M)^T r is exactly zero, x is the solution
        converged = true;
        break;
      }
      if (hs.total_iters >= maxiter) break;
    }
    // Iterations in batches; one state read per batch.  The update kernel
    // sets `done` no later than iteration maxiter, so the batch count is
    // bounded.
    const int max_batches = maxiter / batch + 2;
    const void *pit = refine ? static_cast<const void *>(p32) : static_cast<const void *>(p);
    auto launch_batch = [&](hipStream_t ls) {
      for (int k = 0; k < batch; ++k) iteration(plan, pit, ubuf[ucur], ls);
    };
    GraphKey key;
    key.add(1);  // LSQR
    key.addp(work);
    key.addp(prob->A);
    key.add(static_cast<uint64_t>(prob->lda));
    key.add(static_cast<uint64_t>(m));
    key.add(static_cast<uint64_t>(n));
    key.add(static_cast<uint64_t>(mode));
    key.addp(x);
    key.add(static_cast<uint64_t>(ucur));
    key.addp(plan.fn);
    key.add(static_cast<uint64_t>(plan.grid));
    key.add(static_cast<uint64_t>(plan.rows_per_wg));
    key.add(static_cast<uint64_t>(plan.dyn_begin));
    key.add(static_cast<uint64_t>(plan.chunk));
    key.addp(sp ? sp->indptr : nullptr);
    key.addp(sp ? sp->indices : nullptr);
    key.addp(sp ? sp->values : nullptr);
    key.add(sp ? static_cast<uint64_t>(sp->nnz) : 0);
    key.add(sp ? static_cast<uint64_t>(sp->v_type) : 0);
    key.add(static_cast<uint64_t>(ctx->num_cus));
    hipGraphExec_t exec = batch_graph(ctx, key, launch_batch);
    sst = run_batches(ctx, exec, launch_batch, st, err, max_batches, &hs, &herr, s, "LSQR");
    if (sst != SAP_OK) return sst;
    if (!refine) {
      converged = hs.converged != 0;
      break;
    }
    delta_norm_kernel<<<1, 1024, 0, s>>>(x, xprev, n, dnorm);
    double hd[2] = {0.0, 0.0};
    SAP_HIP_TRY(hipMemcpyAsync(hd, dnorm, sizeof(hd), hipMemcpyDeviceToHost, s));
    SAP_HIP_TRY(hipStreamSynchronize(s));
    if (hd[0] <= tol * hd[1]) {
      converged = true;
      break;
    }
    if (hd[0] >= prev_delta || hs.total_iters >= maxiter) break;  // stagnated, or out of iterations
    prev_delta = hd[0];
  }
  if (info) {
    info->iters = hs.total_iters;
    info->refinements = refinements;
    info->resid_est = hs.resid_est;
    info->normar_est = hs.normar_est;
  }
  return converged ? SAP_OK : SAP_NOT_CONVERGED;
}

// Heavy-ball momentum (App. D.3) in place of LSQR, on the dense pass: each
// step is one fused pass (r = b - A x and q = A^T r), q from the slices,
// s = M^T q, then the test and the update with g = M s.  The paper writes the
// gradient as v - M M^T A^T A x with v = M M^T A^T b; forming r first gives
// the same vector without the cancellation of those two terms near x*.
sap_status run_hbm(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *z,
                   double tol, int maxiter, int mode, double alpha, double beta, double *x, sap_info *info,
                   void *work, hipStream_t s) {
  const int64_t m = prob->m;
  const int n = prob->n;
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "momentum: n > 8192 is not supported");
  if (mode != 0 && mode != 1) return fail(ctx, SAP_EINVAL, "momentum: mode must be FP64 or MIXED_FP32");
  const PassPlan plan = plan_pass(ctx, mode, m, n, prob->lda, prob->A);
  if (plan.grid > max_grid(ctx)) return fail(ctx, SAP_EINVAL, "momentum: internal grid larger than planned");
  LsqrBufs B = carve_lsqr(ctx, work, m, n);
  sap_status sst = setup_precond(ctx, R, ldr, nullptr, z, x, B, n, s);
  if (sst != SAP_OK) return sst;
  LsqrState *st = B.st;
  double *delta = B.w, *sv = B.vh;
  // c_ap = -1, c_u = 1: every pass forms r = b - A x
  lsqr_init_state_kernel<<<1, 256, 0, s>>>(st, tol, maxiter, B.flags, 2 * B.nblk, 0, 0, B.dyn);
  zero_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(delta, n);
  const int ngrid = static_cast<int>(std::min<int64_t>(256, (m + 1023) / 1024));
  norm_kernel<<<ngrid, 1024, 0, s>>>(prob->b, m, B.normpart, B.ticket, st);
  SAP_HIP_TRY(hipGetLastError());
  const int G = plan.grid;
  const int qsl = (G + kQSlice - 1) / kQSlice;
  const int batch = 8;
  const int max_batches = maxiter / batch + 2;
  LsqrState hs{};
  int herr = 0;
  auto launch_batch = [&](hipStream_t ls) {
    for (int k = 0; k < batch; ++k) {
      launch_pass(ctx, plan, prob->A, prob->lda, m, n, x, prob->b, B.ubuf[0], st, B.qpart, B.nrmpart, B.dyn, ls);
      q_slices_kernel<<<dim3((n + 63) / 64, qsl), 256, 0, ls>>>(B.qpart, G, n, B.qs);
      hbm_mtq_kernel<<<B.ngemv, 1024, 0, ls>>>(B.M, n, B.qs, qsl, sv, B.vpart, st);
      hbm_step_kernel<<<B.ngemv, 1024, 0, ls>>>(B.Mt, n, sv, B.vpart, B.ngemv, B.nrmpart, G, alpha, beta, delta, x,
                                                st);
    }
  };
  GraphKey key;
  key.add(2);  // momentum
  key.addp(work);
  key.addp(prob->A);
  key.addp(prob->b);
  key.add(static_cast<uint64_t>(prob->lda));
  key.add(static_cast<uint64_t>(m));
  key.add(static_cast<uint64_t>(n));
  key.add(static_cast<uint64_t>(mode));
  key.addp(x);
  key.addd(alpha);
  key.addd(beta);
  key.addp(plan.fn);
  key.add(static_cast<uint64_t>(plan.grid));
  key.add(static_cast<uint64_t>(plan.rows_per_wg));
  key.add(static_cast<uint64_t>(plan.dyn_begin));
  key.add(static_cast<uint64_t>(plan.chunk));
  key.add(static_cast<uint64_t>(ctx->num_cus));
  hipGraphExec_t exec = batch_graph(ctx, key, launch_batch);
  sst = run_batches(ctx, exec, launch_batch, st, B.err, max_batches, &hs, &herr, s, "momentum");
  if (sst != SAP_OK) return sst;
  if (info) {
    info->iters = hs.total_iters;
    info->resid_est = hs.resid_est;
    info->normar_est = hs.normar_est;
  }
  return hs.converged ? SAP_OK : SAP_NOT_CONVERGED;
}

size_t sstep_workspace_bytes(int n, int s) {
  return 16 * 256 + sizeof(LsqrState) + sizeof(double) * (2 * static_cast<size_t>(n) * s + n + s * s + 2 * s + 4);
}

// The s-step form of App. D.4.2 from x0 = R^-1 z: blocks of s Krylov steps.
// Per block, from the current x: the residual pass (u = b - A x, q = A^T u)
// and r0 = M^T q with ||r||, ||r0|| read back for the stopping test (after
// at least one block: ||r|| = 0, ||r0|| <= tol ||r|| or ||r|| <= tol ||b||);
// then the Chebyshev basis u_0 = r0, u_{k+1} from Z u_k = M^T A^T A M u_k,
// one fused pass each (p = M u_k, u = A p, q = A^T u), no inner products;
// G = U^T Z U and g = U^T r0 (s^2 + s dots); (G c = g) by Cholesky; x += M U c.
// s + 1 passes over A per block of s steps.  Blocks run while fewer than
// maxiter steps have been made.
sap_status run_sstep(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *z,
                     double tol, int maxiter, int mode, int s_steps, double lo, double hi, double *x, sap_info *info,
                     void *work, void *swork, hipStream_t s) {
  const int64_t m = prob->m;
  const int n = prob->n;
  const int S = s_steps;
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "s-step: n > 8192 is not supported");
  if (mode != 0 && mode != 1) return fail(ctx, SAP_EINVAL, "s-step: mode must be FP64 or MIXED_FP32");
  if (S < 1 || S > kMaxSstep || !(hi > lo)) return fail(ctx, SAP_EINVAL, "s-step: bad block size or interval");
  const PassPlan plan = plan_pass(ctx, mode, m, n, prob->lda, prob->A);
  if (plan.grid > max_grid(ctx)) return fail(ctx, SAP_EINVAL, "s-step: internal grid larger than planned");
  LsqrBufs B = carve_lsqr(ctx, work, m, n);
  sap_status sst = setup_precond(ctx, R, ldr, nullptr, z, x, B, n, s);
  if (sst != SAP_OK) return sst;
  Carve cv(swork);
  LsqrState *stz = cv.take<LsqrState>(1);
  double *U = cv.take<double>(static_cast<size_t>(n) * S);
  double *W = cv.take<double>(static_cast<size_t>(n) * S);
  double *y = cv.take<double>(n);
  double *Graw = cv.take<double>(static_cast<size_t>(S) * S);
  double *g = cv.take<double>(S);
  double *cc = cv.take<double>(S);
  double *dn = cv.take<double>(4);
  LsqrState *st = B.st;  // residual passes: c_ap = -1, c_u = 1
  lsqr_init_state_kernel<<<1, 256, 0, s>>>(st, tol, maxiter, B.flags, 2 * B.nblk, 0, 0, B.dyn);
  const int ngrid = static_cast<int>(std::min<int64_t>(256, (m + 1023) / 1024));
  norm_kernel<<<ngrid, 1024, 0, s>>>(prob->b, m, B.normpart, B.ticket, st);
  sstep_zstate_kernel<<<1, 64, 0, s>>>(st, stz);
  SAP_HIP_TRY(hipGetLastError());
  const int G = plan.grid;
  const int qsl = (G + kQSlice - 1) / kQSlice;
  const unsigned nv = static_cast<unsigned>((n + 255) / 256);
  const double cen = 0.5 * (hi + lo), half = 0.5 * (hi - lo);
  // r = b - A x, q = A^T r, out = M^T q (and its norm partials in B.vpart)
  auto product = [&](const double *pv, LsqrState *pst, double *out) {
    launch_pass(ctx, plan, prob->A, prob->lda, m, n, pv, prob->b, B.ubuf[0], pst, B.qpart, B.nrmpart, B.dyn, s);
    q_slices_kernel<<<dim3((n + 63) / 64, qsl), 256, 0, s>>>(B.qpart, G, n, B.qs);
    hbm_mtq_kernel<<<B.ngemv, 1024, 0, s>>>(B.M, n, B.qs, qsl, out, B.vpart, pst);
  };
  auto *hn = static_cast<double *>(ctx->pinned);  // rn, ||r0||, ||b||, error flag
  int steps = 0;
  bool conv = false;
  for (;;) {
    product(x, st, U);  // u_0 = r0 = M^T A^T (b - A x)
    sstep_norms_kernel<<<1, 1024, 0, s>>>(B.nrmpart, G, B.vpart, B.ngemv, st, dn);
    SAP_HIP_TRY(hipGetLastError());
    SAP_HIP_TRY(hipMemcpyAsync(hn, dn, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    SAP_HIP_TRY(hipMemcpyAsync(hn + 3, B.err, sizeof(int), hipMemcpyDeviceToHost, s));
    SAP_HIP_TRY(hipStreamSynchronize(s));
    if (*reinterpret_cast<const int *>(hn + 3)) return fail(ctx, SAP_EDEVICE, "s-step: a block wait expired");
    const double rn = hn[0], fn = hn[1], nb = hn[2];
    if (info) {
      info->resid_est = rn;
      info->normar_est = fn;
    }
    if (steps >= 1 && (rn == 0.0 || fn <= tol * rn || rn <= tol * nb)) {
      conv = true;
      break;
    }
    if (steps >= maxiter) break;
    for (int k = 0; k < S; ++k) {
      double *uk = U + static_cast<int64_t>(k) * n;
      sstep_mv_kernel<<<B.ngemv, 1024, 0, s>>>(B.Mt, n, uk, B.p, nullptr);  // p = M u_k
      product(B.p, stz, W + static_cast<int64_t>(k) * n);                   // Z u_k
      if (k + 1 < S)
        sstep_cheb_kernel<<<nv, 256, 0, s>>>(n, k, cen, half, W + static_cast<int64_t>(k) * n, uk,
                                             k > 0 ? uk - n : uk, uk + n);
    }
    sstep_gram_kernel<<<dim3(S, S + 1), 256, 0, s>>>(U, W, n, S, Graw, g);
    sstep_solve_kernel<<<1, 64, 0, s>>>(S, Graw, g, cc);
    sstep_combine_kernel<<<nv, 256, 0, s>>>(U, n, S, cc, y);
    sstep_mv_kernel<<<B.ngemv, 1024, 0, s>>>(B.Mt, n, y, nullptr, x);  // x += M U c
    SAP_HIP_TRY(hipGetLastError());
    steps += S;
  }
  if (info) info->iters = steps;
  return conv ? SAP_OK : SAP_NOT_CONVERGED;
}

void batch_graphs_free(sap_ctx *ctx) {
  auto *G = static_cast<BatchGraphs *>(ctx->batch_graphs);
  if (!G) return;
  for (auto &en : G->e)
    if (en.exec) (void)hipGraphExecDestroy(en.exec);
  if (G->cap) (void)hipStreamDestroy(G->cap);
  delete G;
  ctx->batch_graphs = nullptr;
}

}  // namespace sap
