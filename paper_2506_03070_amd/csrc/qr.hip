// Blocked Householder QR of the sketch Y (d x ncols, column-major, FP64) on
// gfx950 (Alg. 1 "factor Q, R = QR(Y)"; the paper calls a vendor QR).
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
#include "common.h"
#include "qr_dev.h"

namespace sap {
namespace {

using namespace qr_dev;

// The first panel (columns 0 .. nb-1).
template <int S, int NB>
__global__ __launch_bounds__(kPanelThreads) void qr_first_panel_kernel(double *__restrict__ Y, int64_t ldy, int d,
                                                                       int nb, double *__restrict__ tau,
                                                                       double *__restrict__ Tout) {
  __shared__ PanelShared<NB> sh;
  double P[S][NB];
  load_block<S, NB>(Y, ldy, 0, d, 0, nb, P);
  factor_panel<S, NB>(P, sh, nb, d, 0, 0, tau, Tout);
  store_block<S, NB>(Y, ldy, 0, d, 0, nb, P);
}

// One step of the right-looking factorisation: every workgroup applies
// Q_k^T (panel k = columns k0 .. k0+nb-1) to its block of NB trailing
// columns; workgroup 0's block is panel k+1, which it then factors at once
// (look-ahead) into Tnext.
template <int S, int NB>
__global__ __launch_bounds__(kPanelThreads) void qr_step_kernel(double *__restrict__ Y, int64_t ldy, int d, int ncols,
                                                                int k0, int nb, const double *__restrict__ Tcur,
                                                                double *__restrict__ Tnext,
                                                                double *__restrict__ tau) {
  __shared__ PanelShared<NB> sh;
  const int c0 = k0 + nb + static_cast<int>(blockIdx.x) * NB;
  const int ncb = min(NB, ncols - c0);
  const int dr = d - k0;
  double C[S][NB];
  load_block<S, NB>(Y, ldy, k0, dr, c0, ncb, C);
  apply_panel_qt<S, NB>(Y, ldy, dr, k0, nb, Tcur, C, ncb, sh);
  if (blockIdx.x == 0) {
    // panel k+1 starts at row and column k1 = c0; rows k0..k1-1 ride along
    const int k1 = c0;
    factor_panel<S, NB>(C, sh, ncb, d - k1, k1 - k0, k1, tau, Tnext);
  }
  store_block<S, NB>(Y, ldy, k0, dr, c0, ncb, C);
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

struct QrShape {
  int s;   // rows per thread (512 threads)
  int nb;  // panel width = trailing block width
};

QrShape qr_shape(int rows) {
  // The register blocks (S * NB doubles per thread, twice: V and C) must fit
  // in the 256 VGPRs a 512-thread workgroup leaves each lane: S * NB <= 32.
  const int s = (rows + kPanelThreads - 1) / kPanelThreads;
  if (s <= 1) return {1, 8};
  if (s <= 2) return {2, 8};
  if (s <= 4) return {4, 8};
  if (s <= 8) return {8, 4};
  if (s <= 16) return {16, 2};
  return {32, 1};
}

template <int S, int NB>
sap_status qr_run(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                  hipStream_t st) {
  Carve cv(work);
  double *T[2] = {cv.take<double>(NB * NB), cv.take<double>(NB * NB)};
  const int kmax = rows < cols ? rows : cols;
  int nb = kmax < NB ? kmax : NB;
  qr_first_panel_kernel<S, NB><<<1, kPanelThreads, 0, st>>>(Y, ldy, rows, nb, tau, T[0]);
  SAP_HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int k0 = 0; k0 + nb < cols; k0 += NB) {
    const int trailing = cols - (k0 + nb);
    const int nblocks = (trailing + NB - 1) / NB;
    qr_step_kernel<S, NB><<<nblocks, kPanelThreads, 0, st>>>(Y, ldy, rows, cols, k0, nb, T[cur], T[1 - cur], tau);
    SAP_HIP_TRY(hipGetLastError());
    cur ^= 1;
    nb = (cols - (k0 + NB)) < NB ? (cols - (k0 + NB)) : NB;
  }
  return SAP_OK;
}

}  // namespace

size_t qr_workspace_bytes(int rows, int cols) {
  (void)rows;
  (void)cols;
  return 4 * 256 + 2 * sizeof(double) * 16 * 16;
}

sap_status launch_qr(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                     hipStream_t st) {
  const QrShape sh = qr_shape(rows);
  switch (sh.s) {
    case 1: return qr_run<1, 8>(ctx, Y, ldy, rows, cols, tau, work, st);
    case 2: return qr_run<2, 8>(ctx, Y, ldy, rows, cols, tau, work, st);
    case 4: return qr_run<4, 8>(ctx, Y, ldy, rows, cols, tau, work, st);
    case 8: return qr_run<8, 4>(ctx, Y, ldy, rows, cols, tau, work, st);
    case 16: return qr_run<16, 2>(ctx, Y, ldy, rows, cols, tau, work, st);
    default: break;
  }
  if (rows <= 32 * kPanelThreads) return qr_run<32, 1>(ctx, Y, ldy, rows, cols, tau, work, st);
  return fail(ctx, SAP_EINVAL, "sap_qr: more than 16384 rows is not supported");
}

sap_status launch_rank_check(sap_ctx *ctx, const double *R, int64_t ldr, int n, int d, int *flag,
                             hipStream_t st) {
  rank_check_kernel<<<1, 1024, 0, st>>>(R, ldr, n, d, flag);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

}  // namespace sap
