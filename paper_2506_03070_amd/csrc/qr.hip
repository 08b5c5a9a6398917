// Blocked Householder QR of the sketch Y (d x ncols, column-major, FP64) on
// gfx950 (the factorization step of Alg. 1; the paper calls a vendor QR).
//
// Blocked Householder QR (Golub & Van Loan 5.2.2) with the compact WY form
// Q = I - V T V^T of Schreiber & Van Loan (1989), in one launch (the chained
// form): workgroup j, numbered in the order the workgroups start (an atomic
// ticket), owns columns NB j .. NB j + NB-1 (NB = 4 up to 4096 rows, 2 up to
// 8192, 1 up to 16384) and holds all their rows in registers for the whole
// factorisation (thread t owns rows t, t+512, ...).
//   * it applies panel k, Q_k^T = I - V T^T V^T (W = V^T C as NB*NB
//     workgroup-wide sums, W2 = T^T W, C -= V W2), as soon as panel k's owner
//     has published it: reflectors and T written through to the coherence
//     point shared by the XCDs, then a flag;
//   * it then factors its own panel, one workgroup reduction per column for
//     the norm below the diagonal and one batched reduction that gives both
//     v_j^T C (the update of the panel columns to its right) and V_{<j}^T v_j
//     (the next column of T), and publishes it.
// The trailing matrix never goes back to memory between panels and no launch
// boundary separates them: a panel's critical path is one block apply and one
// panel factorisation.  A workgroup only waits for workgroups that started
// before it, so the chain completes whatever number of them is resident.
// Sketches taller than 4096 rows and wider than 192 columns take the
// two-level form below: 64-column panels factored by the chained form, the
// trailing matrix updated on the FP64 matrix cores.
// Sign convention: LAPACK dlarfg, beta = -sign(alpha) ||(alpha, x)||.
#include <algorithm>

#include "common.h"
#include "qr_dev.h"
#include "trsv.h"

namespace sap {
namespace {

using namespace qr_dev;

// Chained QR: C <- (I - V T^T V^T) C for a block held at fixed rows (thread t
// holds rows t + TH s of the whole column block), with panel k's reflectors
// (columns k0 .. k0+nbp-1 of Y, rows from k0, unit diagonal implicit) and T
// read through the coherence point, since another workgroup wrote them
// during this launch.  Rows above the panel have V = 0 and are unchanged.
template <int S, int NB, int TH>
__device__ __forceinline__ void chain_apply_panel(const double *__restrict__ Y, int64_t ldy, int d, int k0, int nbp,
                                                  const double *__restrict__ T, double (&C)[S][NB], int ncb,
                                                  PanelShared<NB, TH> &sh) {
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  const double tload = t < NB * NB ? load_coherent(T + t) : 0.0;
  double V[S][NB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = t + TH * s;
    const int lr = r - k0;
    const int rr = min(max(r, k0), d - 1);  // in-range address; masked below
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const double y = load_coherent(Y + static_cast<int64_t>(k0 + min(i, nbp - 1)) * ldy + rr);
      V[s][i] = (i < nbp && lr >= 0 && r < d) ? vval(lr, i, y) : 0.0;
    }
  }
  if (t < NB * NB) sh.Tl[t] = tload;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < S; ++s) acc += V[s][i] * C[s][c];
      acc = wave_sum_u(acc);
      if (lane == 0) sh.red[wave][i * NB + c] = acc;
    }
  __syncthreads();
  if (t < NB * NB) {
    const int i = t / NB, c = t % NB;
    double s_ = 0.0;
    for (int l = 0; l <= i && l < nbp; ++l) {
      double wlc = 0.0;
      for (int w = 0; w < (TH / kWave); ++w) wlc += sh.red[w][l * NB + c];
      s_ += sh.Tl[l + i * NB] * wlc;
    }
    sh.W2[i][c] = (i < nbp && c < ncb) ? s_ : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < NB; ++i) acc += V[s][i] * sh.W2[i][c];
      C[s][c] -= acc;
    }
}

// A wait of the chain gives up after this many polls (a producer that never
// ran, which the start-ordered tickets rule out); the block is then NaN, which
// the rank test that follows every solve's QR reports as a non-finite R.
constexpr int kQrSpinLimit = 1 << 20;

// One launch of ceil(cols / NB) workgroups; w: the ticket word and one flag
// per panel, zero on entry; Tall: NB x NB per panel.
template <int S, int NB, int TH>
__global__ __launch_bounds__(TH) void qr_chain_kernel(double *__restrict__ Y, int64_t ldy, int d, int cols,
                                                      double *__restrict__ Tall, double *__restrict__ tau,
                                                      int *__restrict__ w) {
  __shared__ PanelShared<NB, TH> sh;
  __shared__ double Tsh[NB * NB];
  __shared__ int jsh, failed;
  const int t = threadIdx.x;
  if (t == 0) {
    jsh = atomicAdd(w, 1);
    failed = 0;
  }
  __syncthreads();
  const int j = jsh;
  int *flags = w + 1;
  const int c0 = j * NB;
  const int ncb = min(NB, cols - c0);
  double C[S][NB];
  load_block<S, NB, TH>(Y, ldy, 0, d, c0, ncb, C);
  for (int k = 0; k < j; ++k) {
    if (t == 0) {
      int spins = 0;
      while (__hip_atomic_load(flags + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < 1) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > kQrSpinLimit) {
          failed = 1;
          break;
        }
      }
    }
    __syncthreads();
    if (failed) break;  // uniform
    chain_apply_panel<S, NB, TH>(Y, ldy, d, k * NB, min(NB, cols - k * NB), Tall + k * NB * NB, C, ncb, sh);
  }
  if (failed) {
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int c = 0; c < NB; ++c) C[s][c] = __builtin_nan("");
  } else {
    factor_panel<S, NB>(C, sh, ncb, d - c0, c0, c0, tau, Tsh);
    __syncthreads();
    if (t < NB * NB) store_coherent(Tall + j * NB * NB + t, Tsh[t]);
  }
  double *__restrict__ base = Y + static_cast<int64_t>(c0) * ldy;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int r = t + TH * s;
    if (r < d) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < ncb) store_coherent(base + static_cast<int64_t>(c) * ldy + r, C[s][c]);
    }
  }
  publish_flag(flags + j, 1);
}

__global__ void qr_chain_zero_kernel(int *w, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) w[i] = 0;
}

// Rank test on R's diagonal: deficient (1) when min |R_kk| <= d * 2^-53 * max |R_kk|,
// 2 when an R_kk is not finite.
__global__ __launch_bounds__(1024) void rank_check_kernel(const double *__restrict__ R, int64_t ldr,
                                                          int n, int d, int *__restrict__ flag) {
  __shared__ double smax[16], smin[16];
  __shared__ int sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  double mx = 0.0, mn = INFINITY;
  bool bad = false;
  for (int k = threadIdx.x; k < n; k += 1024) {
    const double a = fabs(R[k + static_cast<int64_t>(k) * ldr]);
    bad = bad || !isfinite(a);
    mx = fmax(mx, a);
    mn = fmin(mn, a);
  }
  if (bad) atomicOr(&sbad, 1);
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
    // 2: a non-finite diagonal (non-finite A, or a chained-QR wait that expired)
    *flag = sbad ? 2 : !(mn > static_cast<double>(d) * 0x1p-53 * mx);
  }
}

// ---- two-level blocking for wide sketches -----------------------------------
// Panels of kWy columns are factored by the kernels above (restricted to the
// panel); the rest of the matrix is then updated once per panel with the
// panel's compact WY form, Q_p^T C = C - V T^T (V^T C), on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64):
//   W' = V^T [V C]   one pass over the panel's rows, split over workgroups;
//                    its first kWy columns are the Gram matrix G = V^T V;
//   W2 = T^T W       without forming T: T^-1 = diag(1 / tau) + the strict
//                    upper triangle of G (Puglisi; Joffrain et al., "UT
//                    transform"), so W2 solves (T^-1)^T W2 = W by forward
//                    substitution, one thread per column, as
//                    W2_i = tau_i (W_i - sum_{l<i} G_li W2_l) (tau_i = 0 drops
//                    reflector i, as LAPACK's T does);
//   C -= V W2        tiles of 64 x 64.
// This reads and writes the trailing matrix once per kWy columns instead of
// once per NB columns.
//
// Matrix-core lane layout (checked on the device): for D = A B + C with A
// 16 x 4, B 4 x 16, lane l holds A[l % 16][l / 16] and B[l / 16][l % 16],
// and register r of D holds D[l / 16 + 4 r][l % 16].
constexpr int kWy = 64;        // panel width of the outer blocking
constexpr int kWyRows = 64;    // rows per LDS sub-chunk / rows of an update tile
constexpr int kWyTn = 64;      // columns of a tile
constexpr int kWyThreads = 256;
constexpr int kLdsPad = kWy + 1;

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mfma_d4 mfma_f64(double a, double b, mfma_d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Staging of a 64-row slice of the panel's V (rows r0 .. r0+63, all kWy
// columns) and of 64 columns of B = [V C] into registers: thread t holds
// elements e = t + 256 q (q < 16), row e % 64 and column e / 64, so that
// the loads run down columns (contiguous) and are all issued before any is
// used.
constexpr int kStage = kWyRows * kWy / kWyThreads;  // 16

__device__ __forceinline__ void stage_v(const double *__restrict__ Yp, int64_t ldy, int r_end, int pw, int r0,
                                        double (&v)[kStage]) {
#pragma unroll
  for (int q = 0; q < kStage; ++q) {
    const int e = static_cast<int>(threadIdx.x) + kWyThreads * q;
    const int r = r0 + e % kWyRows, i = e / kWyRows;
    const bool in = r < r_end && i < pw;
    const double y = (in && r > i) ? Yp[r + static_cast<int64_t>(i) * ldy] : 0.0;
    v[q] = (in && r == i) ? 1.0 : y;
  }
}

__device__ __forceinline__ void stage_b(const double *__restrict__ Yp, int64_t ldy, int r_end, int pw, int nball,
                                        int r0, int j0, double (&v)[kStage]) {
#pragma unroll
  for (int q = 0; q < kStage; ++q) {
    const int e = static_cast<int>(threadIdx.x) + kWyThreads * q;
    const int r = r0 + e % kWyRows, j = j0 + e / kWyRows;
    const bool in = r < r_end && j < nball;
    // column j < pw of B is V's (unit diagonal, zeros above)
    const bool ld = in && (j >= pw || r > j);
    const double y = ld ? Yp[r + static_cast<int64_t>(j) * ldy] : 0.0;
    v[q] = (in && j < pw && r == j) ? 1.0 : y;
  }
}

__device__ __forceinline__ void unstage(double (*S)[kLdsPad], const double (&v)[kStage]) {
#pragma unroll
  for (int q = 0; q < kStage; ++q) {
    const int e = static_cast<int>(threadIdx.x) + kWyThreads * q;
    S[e % kWyRows][e / kWyRows] = v[q];
  }
}

// Wp[s][i][j] = sum over the rows of chunk s of V(r, i) B(r, j), B = [V C],
// for the 64 columns j0 .. j0+63 of B; row-major per chunk with leading
// dimension ldw.  Wave w takes i in [16 w, 16 w + 16) and the tile's four
// 16-column blocks.  The next 64-row slice is loaded into registers while
// the matrix cores work on the current one.
__global__ __launch_bounds__(kWyThreads) void qr_wy_w_kernel(const double *__restrict__ Yp, int64_t ldy, int rows,
                                                             int pw, int nball, int chunk, int64_t ldw,
                                                             double *__restrict__ Wp) {
  __shared__ double Vs[kWyRows][kLdsPad];
  __shared__ double Bs[kWyRows][kLdsPad];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int j0 = blockIdx.x * kWyTn;
  const int r_begin = blockIdx.y * chunk;
  const int r_end = min(rows, r_begin + chunk);
  mfma_d4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
  double rv[kStage], rb[kStage];
  stage_v(Yp, ldy, r_end, pw, r_begin, rv);
  stage_b(Yp, ldy, r_end, pw, nball, r_begin, j0, rb);
  for (int r0 = r_begin; r0 < r_end; r0 += kWyRows) {
    __syncthreads();
    unstage(Vs, rv);
    unstage(Bs, rb);
    __syncthreads();
    if (r0 + kWyRows < r_end) {
      stage_v(Yp, ldy, r_end, pw, r0 + kWyRows, rv);
      stage_b(Yp, ldy, r_end, pw, nball, r0 + kWyRows, j0, rb);
    }
#pragma unroll 4
    for (int kk = 0; kk < kWyRows; kk += 4) {
      const double a = Vs[kk + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[b] = mfma_f64(a, Bs[kk + (lane >> 4)][16 * b + (lane & 15)], acc[b]);
    }
  }
  double *W = Wp + static_cast<int64_t>(blockIdx.y) * kWy * ldw;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int j = j0 + 16 * b + (lane & 15);
    if (j >= nball) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * w + (lane >> 4) + 4 * r;
      W[static_cast<int64_t>(i) * ldw + j] = acc[b][r];
    }
  }
}

// Ws = sum of the chunk partials Wp[s] (s ascending), kWy x nball row-major.
__global__ __launch_bounds__(256) void qr_wy_sum_kernel(const double *__restrict__ Wp, int nparts, int64_t ldw,
                                                        int nball, double *__restrict__ Ws) {
  const int j = blockIdx.x * 256 + threadIdx.x, i = blockIdx.y;
  if (j >= nball) return;
  const double *src = Wp + static_cast<int64_t>(i) * ldw + j;
  const int64_t stride = static_cast<int64_t>(kWy) * ldw;
  double s = 0.0;
  int p = 0;
  for (; p + 4 <= nparts; p += 4) {
    const double a0 = src[p * stride], a1 = src[(p + 1) * stride], a2 = src[(p + 2) * stride],
                 a3 = src[(p + 3) * stride];
    s += a0;
    s += a1;
    s += a2;
    s += a3;
  }
  for (; p < nparts; ++p) s += src[p * stride];
  Ws[static_cast<int64_t>(i) * ldw + j] = s;
}

// W2[:, j] for the trailing columns j (one thread each) from Ws = V^T [V C]:
// G = V^T V is its first pw columns (every workgroup copies it to LDS), then
// W2_i = tau_i (W_i - sum_{l<i} G_li W2_l).  Indices i >= pw carry tau_i = 0
// (a narrower last panel).  W2 row-major kWy x ntr (leading dimension ntr).
__global__ __launch_bounds__(kWyThreads) void qr_wy_t2_kernel(const double *__restrict__ Ws, int64_t ldw, int pw,
                                                              int ntr, const double *__restrict__ tau,
                                                              double *__restrict__ W2) {
  __shared__ double G[kWy][kLdsPad];
  __shared__ double ts[kWy];
  const int t = threadIdx.x;
  for (int e = t; e < kWy * kWy; e += kWyThreads) {
    const int l = e / kWy, i = e % kWy;  // G[l][i]; l < i is used
    G[l][i] = (l < pw && i < pw) ? Ws[static_cast<int64_t>(l) * ldw + i] : 0.0;
  }
  if (t < kWy) ts[t] = t < pw ? tau[t] : 0.0;
  __syncthreads();
  const int j = blockIdx.x * kWyThreads + t;
  if (j >= ntr) return;
  const int64_t col = pw + j;
  double x[kWy];
#pragma unroll
  for (int i = 0; i < kWy; ++i) x[i] = Ws[static_cast<int64_t>(i) * ldw + col];
#pragma unroll
  for (int i = 0; i < kWy; ++i) {
    double s = x[i];
#pragma unroll
    for (int l = 0; l < i; ++l) s -= G[l][i] * x[l];
    x[i] = ts[i] * s;
  }
#pragma unroll
  for (int i = 0; i < kWy; ++i) W2[static_cast<int64_t>(i) * ntr + j] = x[i];
}

// C(r0:r0+64, j0:j0+64) -= V(r0:r0+64, :) W2(:, j0:j0+64), C = Yp(:, pw:).
// Computed as (W2^T V^T)^T so that the 16 lanes of a matrix-core output row
// run down a column of C (contiguous).  Wave w takes columns j0 + 16 w ..
// j0 + 16 w + 15 and the four 16-row blocks of the tile; its 16 values of C
// are loaded before the matrix-core loop.
__global__ __launch_bounds__(kWyThreads) void qr_wy_update_kernel(double *__restrict__ Yp, int64_t ldy, int rows,
                                                                  int pw, int ntr, const double *__restrict__ W2) {
  __shared__ double Vs[kWyRows][kLdsPad];
  __shared__ double Ws[kWy][kLdsPad];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r0 = blockIdx.x * kWyRows, j0 = blockIdx.y * kWyTn;
  {
    double rv[kStage], rw[kStage];
    stage_v(Yp, ldy, rows, pw, r0, rv);
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = t + kWyThreads * q;
      const int jj = e % kWyTn, ii = e / kWyTn;
      const int j = j0 + jj;
      rw[q] = (j < ntr && ii < pw) ? W2[static_cast<int64_t>(ii) * ntr + j] : 0.0;
    }
    unstage(Vs, rv);
#pragma unroll
    for (int q = 0; q < kStage; ++q) {
      const int e = t + kWyThreads * q;
      Ws[e / kWyTn][e % kWyTn] = rw[q];
    }
  }
  double *C = Yp + static_cast<int64_t>(pw) * ldy;
  double cv[4][4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int r = r0 + 16 * b + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + 16 * w + (lane >> 4) + 4 * q;
      cv[b][q] = (r < rows && j < ntr) ? C[r + static_cast<int64_t>(j) * ldy] : 0.0;
    }
  }
  __syncthreads();
  mfma_d4 acc[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = mfma_d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int kk = 0; kk < kWy; kk += 4) {
    const double a = Ws[kk + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = mfma_f64(a, Vs[16 * b + (lane & 15)][kk + (lane >> 4)], acc[b]);
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int r = r0 + 16 * b + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + 16 * w + (lane >> 4) + 4 * q;
      if (r < rows && j < ntr) C[r + static_cast<int64_t>(j) * ldy] = cv[b][q] - acc[b][q];
    }
  }
}

constexpr size_t kUnblockedBytes = 4 * 256 + 2 * sizeof(double) * 16 * 16;
// Workspace of the chained form for any NB <= 4: NB x NB of T per block and
// one ticket word plus one flag per block.
size_t chain_bytes(int cols) {
  const size_t c = static_cast<size_t>(cols);
  return 2 * 256 + sizeof(double) * 16 * ((c + 3) / 4) + sizeof(int) * (c + 1);
}

template <int S, int NB>
sap_status qr_chain(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                    hipStream_t st) {
  constexpr int TH = 512;
  if (rows > S * TH) return fail(ctx, SAP_EINVAL, "sap_qr: rows exceed the register block");
  const int nblk = (cols + NB - 1) / NB;
  Carve cv(work);
  double *Tall = cv.take<double>(static_cast<size_t>(NB) * NB * nblk);
  int *w = cv.take<int>(static_cast<size_t>(nblk) + 1);
  qr_chain_zero_kernel<<<1, 256, 0, st>>>(w, nblk + 1);
  SAP_HIP_TRY(hipGetLastError());
  qr_chain_kernel<S, NB, TH><<<nblk, TH, 0, st>>>(Y, ldy, rows, cols, Tall, tau, w);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

sap_status qr_unblocked(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                        hipStream_t st) {
  // S rows per thread, NB columns per block, 512 threads: the register
  // blocks (S * NB doubles per thread, twice: V and C) must fit in the 256
  // VGPRs a lane keeps at 512 threads.  (1024 threads with S halved measured
  // ~20% slower at 4000 x 1001: the panels are bound by barriers and
  // cross-wave sums, which more waves lengthen.)  4-column blocks up to 2048
  // rows as well: 8-column panels measured 20-25% slower there, twice the
  // dependent column reductions per panel.
  if (rows <= 512) return qr_chain<1, 4>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 1024) return qr_chain<2, 4>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 2048) return qr_chain<4, 4>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 4096) return qr_chain<8, 4>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 8192) return qr_chain<16, 2>(ctx, Y, ldy, rows, cols, tau, work, st);
  if (rows <= 16384) return qr_chain<32, 1>(ctx, Y, ldy, rows, cols, tau, work, st);
  return fail(ctx, SAP_EINVAL, "sap_qr: more than 16384 rows is not supported");
}

// The two-level form pays off where the one-level panels are bound by the
// trailing matrix (tall sketches, narrow NB); below that the one-level
// panels are bound by the panel's reduction latency, which the
// two-level form does not shorten.
bool use_blocked(int rows, int cols) { return cols > 3 * kWy && rows > 4096; }

int round64(int x) { return (x + kWyRows - 1) / kWyRows * kWyRows; }
constexpr int kMaxSplits = 16;

sap_status qr_blocked(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                      hipStream_t st) {
  const int kmax = std::min(rows, cols);
  const int64_t ldw = cols;  // >= kWy + the widest trailing part
  Carve cv(work);
  void *pwork = cv.take<char>(kUnblockedBytes + chain_bytes(kWy));
  double *Wp = cv.take<double>(static_cast<size_t>(kMaxSplits) * kWy * ldw);
  double *Wsum = cv.take<double>(static_cast<size_t>(kWy) * ldw);
  double *W2 = cv.take<double>(static_cast<size_t>(kWy) * cols);
  for (int k = 0; k < kmax; k += kWy) {
    const int pw = std::min(kWy, kmax - k);
    const int prow = rows - k;
    double *Yp = Y + k + static_cast<int64_t>(k) * ldy;
    sap_status s = qr_unblocked(ctx, Yp, ldy, prow, pw, tau + k, pwork, st);
    if (s != SAP_OK) return s;
    const int ntr = cols - k - pw;
    if (ntr <= 0) continue;
    const int nball = pw + ntr;
    const int ntiles = (nball + kWyTn - 1) / kWyTn;
    int splits = std::max(1, std::min({kMaxSplits, (2 * ctx->num_cus + ntiles - 1) / ntiles, (prow + 255) / 256}));
    const int chunk = round64((prow + splits - 1) / splits);
    splits = (prow + chunk - 1) / chunk;
    qr_wy_w_kernel<<<dim3(ntiles, splits), kWyThreads, 0, st>>>(Yp, ldy, prow, pw, nball, chunk, ldw, Wp);
    qr_wy_sum_kernel<<<dim3((nball + 255) / 256, kWy), 256, 0, st>>>(Wp, splits, ldw, nball, Wsum);
    qr_wy_t2_kernel<<<(ntr + kWyThreads - 1) / kWyThreads, kWyThreads, 0, st>>>(Wsum, ldw, pw, ntr, tau + k, W2);
    qr_wy_update_kernel<<<dim3((prow + kWyRows - 1) / kWyRows, (ntr + kWyTn - 1) / kWyTn), kWyThreads, 0, st>>>(
        Yp, ldy, prow, pw, ntr, W2);
    SAP_HIP_TRY(hipGetLastError());
  }
  return SAP_OK;
}

}  // namespace

size_t qr_workspace_bytes(int rows, int cols) {
  size_t b = kUnblockedBytes + chain_bytes(cols);
  if (use_blocked(rows, cols))
    b += 4 * 256 + sizeof(double) * static_cast<size_t>(kMaxSplits + 2) * kWy * cols;
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
