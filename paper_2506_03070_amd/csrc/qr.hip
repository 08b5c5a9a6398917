// Blocked Householder QR of the sketch Y (d x ncols, column-major, FP64) on
// gfx950 (the factorization step of Alg. 1; the paper calls a vendor QR).
//
// Right-looking blocked algorithm (Golub & Van Loan 5.2.2) with the compact
// WY form Q = I - V T V^T of Schreiber & Van Loan (1989), one launch per
// panel of NB columns:
//   * every 512-thread workgroup owns a block of NB trailing columns, holds
//     its rows in registers (thread t owns rows t, t+512, ...), and applies
//     Q_k^T = I - V T^T V^T to it: W = V^T C is NB*NB workgroup-wide sums,
//     W2 = T^T W, C -= V W2; the block is read once and written once;
//   * workgroup 0's block is the next panel, which it factors on the spot
//     (look-ahead) into the other of two T buffers: per column one workgroup
//     reduction for the norm below the diagonal and one batched reduction that
//     gives both v_j^T C (the update of the panel columns to its right) and
//     V_{<j}^T v_j (the next column of T).
// Sign convention: LAPACK dlarfg, beta = -sign(alpha) ||(alpha, x)||.
#include <algorithm>

#include "common.h"
#include "qr_dev.h"

namespace sap {
namespace {

using namespace qr_dev;

// The first panel (columns 0 .. nb-1).  TH threads, S rows each.
template <int S, int NB, int TH>
__global__ __launch_bounds__(TH) void qr_first_panel_kernel(double *__restrict__ Y, int64_t ldy, int d, int nb,
                                                            double *__restrict__ tau, double *__restrict__ Tout) {
  __shared__ PanelShared<NB, TH> sh;
  double P[S][NB];
  load_block<S, NB, TH>(Y, ldy, 0, d, 0, nb, P);
  factor_panel<S, NB>(P, sh, nb, d, 0, 0, tau, Tout);
  store_block<S, NB, TH>(Y, ldy, 0, d, 0, nb, P);
}

// One step of the right-looking factorisation: every workgroup applies
// Q_k^T (panel k = columns k0 .. k0+nb-1) to its block of NB trailing
// columns; workgroup 0's block is panel k+1, which it then factors at once
// (look-ahead) into Tnext.
template <int S, int NB, int TH>
__global__ __launch_bounds__(TH) void qr_step_kernel(double *__restrict__ Y, int64_t ldy, int d, int ncols, int k0,
                                                     int nb, const double *__restrict__ Tcur,
                                                     double *__restrict__ Tnext, double *__restrict__ tau) {
  __shared__ PanelShared<NB, TH> sh;
  const int c0 = k0 + nb + static_cast<int>(blockIdx.x) * NB;
  const int ncb = min(NB, ncols - c0);
  const int dr = d - k0;
  double C[S][NB];
  load_block<S, NB, TH>(Y, ldy, k0, dr, c0, ncb, C);
  apply_panel_qt<S, NB>(Y, ldy, dr, k0, nb, Tcur, C, ncb, sh);
  if (blockIdx.x == 0) {
    // panel k+1 starts at row and column k1 = c0; rows k0..k1-1 ride along
    const int k1 = c0;
    factor_panel<S, NB>(C, sh, ncb, d - k1, k1 - k0, k1, tau, Tnext);
  }
  store_block<S, NB, TH>(Y, ldy, k0, dr, c0, ncb, C);
}

// Rank test on R's diagonal: deficient when min |R_kk| <= d * 2^-53 * max |R_kk|.
__global__ __launch_bounds__(1024) void rank_check_kernel(const double *__restrict__ R, int64_t ldr,
                                                          int n, int d, int *__restrict__ flag) {
  __shared__ double smax[16], smin[16];
  double mx = 0.0, mn = INFINITY;
  for (int k = threadIdx.x; k < n; k += 1024) {
    const double a = fabs(R[k + static_cast<int64_t>(k) * ldr]);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
  mx = wave_max(mx);
  mn = -wave_max(-mn);
  const int lane = threadIdx.x & 63, wave = threadIdx.x / 64;
  if (lane == 0) {
    smax[wave] = mx;
    smin[wave] = mn;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < 16; ++w) {
      mx = fmax(mx, smax[w]);
      mn = fmin(mn, smin[w]);
    }
    *flag = !(mn > static_cast<double>(d) * 0x1p-53 * mx);
  }
}

// ---- two-level blocking for wide sketches -----------------------------------
// Panels of kWy columns are factored by the kernels above (restricted to the
// panel); the rest of the matrix is then updated once per panel with the
// panel's compact WY form, Q_p^T C = C - V T^T (V^T C), as three tiled FP64
// products (W = V^T C with the rows split over workgroups, W2 = T^T W, and
// C -= V W2).  This reads and writes the trailing matrix once per kWy columns
// instead of once per NB columns.
constexpr int kWy = 64;        // panel width of the outer blocking
constexpr int kWyRows = 64;    // rows per LDS sub-chunk
constexpr int kWyTn = 32;      // trailing columns per workgroup
constexpr int kWyThreads = 256;

// V entry of the panel at (panel-relative row r, column i), from the
// factored panel stored in Y (unit diagonal implicit, zeros above).
__device__ __forceinline__ double wy_v(const double *__restrict__ Yp, int64_t ldy, int rows, int pw, int r, int i) {
  if (r >= rows || i >= pw || r < i) return 0.0;
  if (r == i) return 1.0;
  return Yp[r + static_cast<int64_t>(i) * ldy];
}

// Gp[s] = partial V^T V over row chunk s (kWy x kWy, column-major).
__global__ __launch_bounds__(kWyThreads) void qr_gram_kernel(const double *__restrict__ Yp, int64_t ldy, int rows,
                                                             int pw, int chunk, double *__restrict__ Gp) {
  __shared__ double Vs[kWyRows][kWy + 1];
  const int t = threadIdx.x;
  const int i = t % kWy, jg = t / kWy;  // 4 groups of 16 columns
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  const int r_begin = blockIdx.x * chunk;
  const int r_end = min(rows, r_begin + chunk);
  for (int r0 = r_begin; r0 < r_end; r0 += kWyRows) {
    __syncthreads();
    for (int e = t; e < kWyRows * kWy; e += kWyThreads) {
      const int rr = e % kWyRows, ii = e / kWyRows;
      const int r = r0 + rr;
      Vs[rr][ii] = r < r_end ? wy_v(Yp, ldy, rows, pw, r, ii) : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < kWyRows; ++rr) {
      const double vi = Vs[rr][i];
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[q] += vi * Vs[rr][jg * 16 + q];
    }
  }
  double *G = Gp + static_cast<int64_t>(blockIdx.x) * kWy * kWy;
#pragma unroll
  for (int q = 0; q < 16; ++q) G[i + (jg * 16 + q) * kWy] = acc[q];
}

// T of the panel (upper triangular, column-major kWy x kWy) from the Gram
// partials and tau (LAPACK dlarft, forward columnwise):
// T(i,i) = tau_i, T(0:i, i) = -tau_i T(0:i, 0:i) (V^T v_i)(0:i).
__global__ __launch_bounds__(kWyThreads) void qr_build_t_kernel(const double *__restrict__ Gp, int nparts, int pw,
                                                                const double *__restrict__ tau,
                                                                double *__restrict__ T) {
  __shared__ double G[kWy][kWy + 1];
  __shared__ double Ts[kWy][kWy + 1];
  const int t = threadIdx.x;
  for (int e = t; e < kWy * kWy; e += kWyThreads) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += Gp[static_cast<int64_t>(p) * kWy * kWy + e];
    G[e % kWy][e / kWy] = s;
    Ts[e % kWy][e / kWy] = 0.0;
  }
  __syncthreads();
  for (int i = 0; i < pw; ++i) {
    const double ti = tau[i];
    if (t < i) {
      double s = 0.0;
      for (int q = t; q < i; ++q) s += Ts[t][q] * G[q][i];
      Ts[t][i] = -ti * s;
    }
    if (t == 0) Ts[i][i] = ti;
    __syncthreads();
  }
  for (int e = t; e < kWy * kWy; e += kWyThreads) T[e] = Ts[e % kWy][e / kWy];
}

// Wp[s] = partial V^T C over row chunk s for trailing columns j0 .. j0+31
// (Wp: kWy x ntr per chunk, column-major).
__global__ __launch_bounds__(kWyThreads) void qr_wy_w_kernel(const double *__restrict__ Yp, int64_t ldy, int rows,
                                                             int pw, int ntr, int chunk, double *__restrict__ Wp) {
  __shared__ double Vs[kWyRows][kWy + 1];
  __shared__ double Cs[kWyRows][kWyTn + 1];
  const int t = threadIdx.x;
  const int i = t % kWy, jg = t / kWy;  // 4 groups of 8 columns
  const int j0 = blockIdx.x * kWyTn;
  const double *__restrict__ C = Yp + static_cast<int64_t>(pw) * ldy;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  const int r_begin = blockIdx.y * chunk;
  const int r_end = min(rows, r_begin + chunk);
  for (int r0 = r_begin; r0 < r_end; r0 += kWyRows) {
    __syncthreads();
    for (int e = t; e < kWyRows * kWy; e += kWyThreads) {
      const int rr = e % kWyRows, ii = e / kWyRows;
      const int r = r0 + rr;
      Vs[rr][ii] = r < r_end ? wy_v(Yp, ldy, rows, pw, r, ii) : 0.0;
    }
    for (int e = t; e < kWyRows * kWyTn; e += kWyThreads) {
      const int rr = e % kWyRows, jj = e / kWyRows;
      const int r = r0 + rr, j = j0 + jj;
      Cs[rr][jj] = (r < r_end && j < ntr) ? C[r + static_cast<int64_t>(j) * ldy] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < kWyRows; ++rr) {
      const double vi = Vs[rr][i];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] += vi * Cs[rr][jg * 8 + q];
    }
  }
  double *W = Wp + static_cast<int64_t>(blockIdx.y) * kWy * ntr;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int j = j0 + jg * 8 + q;
    if (j < ntr) W[i + static_cast<int64_t>(j) * kWy] = acc[q];
  }
}

// W2(:, j) = T^T sum_s Wp[s](:, j) for 4 columns per workgroup.
__global__ __launch_bounds__(kWyThreads) void qr_wy_t2_kernel(const double *__restrict__ Wp, int nparts, int ntr,
                                                              const double *__restrict__ T,
                                                              double *__restrict__ W2) {
  __shared__ double Ws[4][kWy];
  const int t = threadIdx.x;
  const int i = t % kWy, jj = t / kWy;
  const int j = blockIdx.x * 4 + jj;
  double s = 0.0;
  if (j < ntr)
    for (int p = 0; p < nparts; ++p) s += Wp[static_cast<int64_t>(p) * kWy * ntr + i + static_cast<int64_t>(j) * kWy];
  Ws[jj][i] = s;
  __syncthreads();
  if (j >= ntr) return;
  double a = 0.0;
  for (int l = 0; l <= i; ++l) a += T[l + i * kWy] * Ws[jj][l];
  W2[i + static_cast<int64_t>(j) * kWy] = a;
}

// C(r0:r0+64, j0:j0+32) -= V(r0:r0+64, :) W2(:, j0:j0+32).
__global__ __launch_bounds__(kWyThreads) void qr_wy_update_kernel(double *__restrict__ Yp, int64_t ldy, int rows,
                                                                  int pw, int ntr, const double *__restrict__ W2) {
  __shared__ double Vs[kWyRows][kWy + 1];
  __shared__ double Ws[kWy][kWyTn + 1];
  const int t = threadIdx.x;
  const int r0 = blockIdx.x * kWyRows, j0 = blockIdx.y * kWyTn;
  for (int e = t; e < kWyRows * kWy; e += kWyThreads) {
    const int rr = e % kWyRows, ii = e / kWyRows;
    Vs[rr][ii] = wy_v(Yp, ldy, rows, pw, r0 + rr, ii);
  }
  for (int e = t; e < kWy * kWyTn; e += kWyThreads) {
    const int ii = e % kWy, jj = e / kWy;
    const int j = j0 + jj;
    Ws[ii][jj] = (j < ntr && ii < pw) ? W2[ii + static_cast<int64_t>(j) * kWy] : 0.0;
  }
  __syncthreads();
  const int rr = t % kWyRows, jg = t / kWyRows;  // 4 groups of 8 columns
  const int r = r0 + rr;
  if (r >= rows) return;
  double acc[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  for (int ii = 0; ii < pw; ++ii) {
    const double v = Vs[rr][ii];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += v * Ws[ii][jg * 8 + q];
  }
  double *C = Yp + static_cast<int64_t>(pw) * ldy;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int j = j0 + jg * 8 + q;
    if (j < ntr) C[r + static_cast<int64_t>(j) * ldy] -= acc[q];
  }
}

template <int S, int NB, int TH>
sap_status qr_run(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                  hipStream_t st) {
  Carve cv(work);
  double *T[2] = {cv.take<double>(NB * NB), cv.take<double>(NB * NB)};
  const int kmax = rows < cols ? rows : cols;
  int nb = kmax < NB ? kmax : NB;
  qr_first_panel_kernel<S, NB, TH><<<1, TH, 0, st>>>(Y, ldy, rows, nb, tau, T[0]);
  SAP_HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int k0 = 0; k0 + nb < cols; k0 += NB) {
    const int trailing = cols - (k0 + nb);
    const int nblocks = (trailing + NB - 1) / NB;
    qr_step_kernel<S, NB, TH><<<nblocks, TH, 0, st>>>(Y, ldy, rows, cols, k0, nb, T[cur], T[1 - cur], tau);
    SAP_HIP_TRY(hipGetLastError());
    cur ^= 1;
    nb = (cols - (k0 + NB)) < NB ? (cols - (k0 + NB)) : NB;
  }
  return SAP_OK;
}

constexpr size_t kUnblockedBytes = 4 * 256 + 2 * sizeof(double) * 16 * 16;

sap_status qr_unblocked(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                        hipStream_t st) {
  // S rows per thread, NB columns per step, TH threads: the register blocks
  // (S * NB doubles per thread, twice: V and C) must fit in the 256 VGPRs a
  // lane keeps at 512 threads.  (1024-thread steps, S halved, measured ~20%
  // slower at 4000 x 1001: the steps are bound by barriers and cross-wave
  // sums, which more waves lengthen.)
  if (rows <= 512) return qr_run<1, 8, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 1024) return qr_run<2, 8, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 2048) return qr_run<4, 8, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 4096) return qr_run<8, 4, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 8192) return qr_run<16, 2, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 16384) return qr_run<32, 1, 512>(ctx, Y, ldy, rows, cols, tau, work, st);
  return fail(ctx, SAP_EINVAL, "sap_qr: more than 16384 rows is not supported");
}

// The two-level form pays off where the one-level steps are bound by the
// traffic of the trailing matrix (tall sketches, narrow NB); below that the
// one-level steps are bound by the panel's reduction latency, which the
// two-level form does not shorten.
bool use_blocked(int rows, int cols) { return cols > 3 * kWy && rows > 4096; }

int gram_parts(int prow) { return std::max(1, std::min(8, (prow + 1023) / 1024)); }
int round64(int x) { return (x + kWyRows - 1) / kWyRows * kWyRows; }
constexpr int kMaxSplits = 16;

sap_status qr_blocked(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                      hipStream_t st) {
  const int kmax = std::min(rows, cols);
  Carve cv(work);
  void *pwork = cv.take<char>(kUnblockedBytes);
  double *T = cv.take<double>(kWy * kWy);
  double *Gp = cv.take<double>(static_cast<size_t>(8) * kWy * kWy);
  double *Wp = cv.take<double>(static_cast<size_t>(kMaxSplits) * kWy * cols);
  double *W2 = cv.take<double>(static_cast<size_t>(kWy) * cols);
  for (int k = 0; k < kmax; k += kWy) {
    const int pw = std::min(kWy, kmax - k);
    const int prow = rows - k;
    double *Yp = Y + k + static_cast<int64_t>(k) * ldy;
    sap_status s = qr_unblocked(ctx, Yp, ldy, prow, pw, tau + k, pwork, st);
    if (s != SAP_OK) return s;
    const int ntr = cols - k - pw;
    if (ntr <= 0) continue;
    int gparts = gram_parts(prow);
    const int gchunk = round64((prow + gparts - 1) / gparts);
    gparts = (prow + gchunk - 1) / gchunk;
    qr_gram_kernel<<<gparts, kWyThreads, 0, st>>>(Yp, ldy, prow, pw, gchunk, Gp);
    qr_build_t_kernel<<<1, kWyThreads, 0, st>>>(Gp, gparts, pw, tau + k, T);
    const int ntiles = (ntr + kWyTn - 1) / kWyTn;
    int splits = std::max(1, std::min({kMaxSplits, (2 * ctx->num_cus + ntiles - 1) / ntiles, (prow + 255) / 256}));
    const int chunk = round64((prow + splits - 1) / splits);
    splits = (prow + chunk - 1) / chunk;
    qr_wy_w_kernel<<<dim3(ntiles, splits), kWyThreads, 0, st>>>(Yp, ldy, prow, pw, ntr, chunk, Wp);
    qr_wy_t2_kernel<<<(ntr + 3) / 4, kWyThreads, 0, st>>>(Wp, splits, ntr, T, W2);
    qr_wy_update_kernel<<<dim3((prow + kWyRows - 1) / kWyRows, ntiles), kWyThreads, 0, st>>>(Yp, ldy, prow, pw,
                                                                                            ntr, W2);
    SAP_HIP_TRY(hipGetLastError());
  }
  return SAP_OK;
}

}  // namespace

size_t qr_workspace_bytes(int rows, int cols) {
  size_t b = kUnblockedBytes;
  if (use_blocked(rows, cols))
    b += 8 * 256 + sizeof(double) * (static_cast<size_t>(kWy) * kWy * 9 +
                                     static_cast<size_t>(kMaxSplits + 1) * kWy * cols);
  return b;
}

sap_status launch_qr(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                     hipStream_t st) {
  if (use_blocked(rows, cols)) return qr_blocked(ctx, Y, ldy, rows, cols, tau, work, st);
  return qr_unblocked(ctx, Y, ldy, rows, cols, tau, work, st);
}

sap_status launch_rank_check(sap_ctx *ctx, const double *R, int64_t ldr, int n, int d, int *flag,
                             hipStream_t st) {
  rank_check_kernel<<<1, 1024, 0, st>>>(R, ldr, n, d, flag);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

}  // namespace sap
