// Blocked Householder QR of the sketch Y (d x ncols, column-major, FP64) on
// gfx950 (Alg. 1 "factor Q, R = QR(Y)"; the paper calls a vendor QR).
//
// Right-looking blocked algorithm (Golub & Van Loan 5.2.2; compact WY form
// of Schreiber & Van Loan 1989):
//   for each panel of NB columns:
//     1. panel kernel (one 1024-thread workgroup): the panel's rows live in
//        registers (thread t owns rows t, t+1024, ...); each column needs one
//        workgroup reduction for its norm and one batched reduction that gives
//        both v_j^T C (the update of the columns to its right) and
//        V_{<j}^T v_j (the next column of the triangular factor T).
//        Sign convention: LAPACK dlarfg, beta = -sign(alpha) ||(alpha, x)||.
//     2. W_part = V^T C  over row splits (LDS-tiled, 256 threads);
//     3. W2 = T^T (sum of W_part)         (fixed-order reduction);
//     4. C -= V W2                        (LDS-tiled rank-NB update).
// Steps 2-4 apply Q^T = I - V T^T V^T to the trailing columns.
#include "common.h"

namespace sap {
namespace {

constexpr int kPanelThreads = 512;
constexpr int kPanelWaves = kPanelThreads / kWave;
constexpr int kTile = 64;

// Householder vector entry (implicit unit diagonal, zeros above) of panel
// column k at panel-relative row r; `y` is the stored panel value.
__device__ __forceinline__ double vval(int r, int k, double y) {
  return r > k ? y : (r == k ? 1.0 : 0.0);
}

// Shared state of the panel factorisation (LDS).
template <int NB>
struct PanelShared {
  double red[kPanelWaves][NB + 1];
  double bc[2];
  double Ts[NB][NB];
  double gdot[NB];
};

// Column J of the panel: reflector, update of columns J+1.. of the panel,
// column J of T.  J is a template parameter so that every register index of
// the panel P is static (no scratch).
template <int S, int NB, int J>
__device__ __forceinline__ void panel_column(double (&P)[S][NB], PanelShared<NB> &sh, int nb, int dr, int k0,
                                             double *__restrict__ tau) {
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  // --- norm of the part below the diagonal ---
  double part = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + kPanelThreads * s;
    if (lr > J && lr < dr) part += P[s][J] * P[s][J];
  }
  part = wave_sum_u(part);
  __syncthreads();  // previous readers of red/bc are done
  if (lane == 0) sh.red[wave][0] = part;
  if (t == J) sh.bc[0] = P[0][J];  // alpha: row J belongs to thread J (J < NB <= 1024)
  __syncthreads();
  double sq = 0.0;
#pragma unroll
  for (int w = 0; w < kPanelWaves; ++w) sq += sh.red[w][0];
  const double alpha = sh.bc[0];
  double tj, beta, scale;
  if (sq == 0.0) {
    tj = 0.0;
    beta = alpha;
    scale = 0.0;
  } else {
    const double nrm = sqrt(alpha * alpha + sq);
    beta = alpha >= 0.0 ? -nrm : nrm;
    tj = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + kPanelThreads * s;
    if (lr > J) P[s][J] *= scale;
    if (lr == J) P[s][J] = beta;
  }
  // --- dot_x = v_J^T (column x) for every x != J (x > J: update weights,
  //     x < J: V_{<J}^T v_J for the T factor) ---
  double dots[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    double acc = 0.0;
    if (x != J) {
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int lr = t + kPanelThreads * s;
        if (lr > J && lr < dr) acc += P[s][J] * P[s][x];
        else if (lr == J) acc += P[s][x];
      }
    }
    dots[x] = wave_sum_u(acc);
  }
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int x = 0; x < NB; ++x) sh.red[wave][x] = dots[x];
  }
  __syncthreads();
  if (t < NB) {
    double s_ = 0.0;
    for (int w = 0; w < kPanelWaves; ++w) s_ += sh.red[w][t];
    sh.gdot[t] = s_;
  }
  __syncthreads();
#pragma unroll
  for (int x = 0; x < NB; ++x) dots[x] = sh.gdot[x];
  // --- apply H_J to the columns right of J inside the panel ---
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + kPanelThreads * s;
    const double v = (lr > J) ? P[s][J] : (lr == J ? 1.0 : 0.0);
#pragma unroll
    for (int x = J + 1; x < NB; ++x)
      if (x < nb && lr >= J) P[s][x] -= tj * dots[x] * v;
  }
  // --- T(:, J) = [-tau_J T(0:J,0:J) V_{<J}^T v_J ; tau_J] (dlarft) ---
  if (t == 0) {
    for (int l = 0; l < J; ++l) {
      double acc = 0.0;
      for (int q = l; q < J; ++q) acc += sh.Ts[l][q] * sh.gdot[q];
      sh.Ts[l][J] = -tj * acc;
    }
    sh.Ts[J][J] = tj;
    tau[k0 + J] = tj;
  }
}

template <int S, int NB, int J>
__device__ __forceinline__ void panel_columns(double (&P)[S][NB], PanelShared<NB> &sh, int nb, int dr, int k0,
                                              double *__restrict__ tau) {
  if constexpr (J < NB) {
    if (J < nb) {  // nb is uniform: every thread reaches the same barriers
      panel_column<S, NB, J>(P, sh, nb, dr, k0, tau);
      panel_columns<S, NB, J + 1>(P, sh, nb, dr, k0, tau);
    }
  }
}

template <int S, int NB>
__global__ __launch_bounds__(kPanelThreads) void qr_panel_kernel(double *__restrict__ Y, int64_t ldy,
                                                                 int d, int k0, int nb,
                                                                 double *__restrict__ tau,
                                                                 double *__restrict__ Tout) {
  __shared__ PanelShared<NB> sh;
  const int t = threadIdx.x;
  const int dr = d - k0;

  // Columns >= nb are zero-filled so they stay inert.  Column bases are
  // wave-uniform (scalar registers); each lane adds one 32-bit row offset.
  double *const ybase = Y + k0 + static_cast<int64_t>(k0) * ldy;
  double P[S][NB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(t + kPanelThreads * s);
#pragma unroll
    for (int c = 0; c < NB; ++c)
      P[s][c] = (lr < static_cast<unsigned>(dr) && c < nb) ? ybase[static_cast<int64_t>(c) * ldy + lr] : 0.0;
  }
  if (t < NB * NB) sh.Ts[t / NB][t % NB] = 0.0;

  panel_columns<S, NB, 0>(P, sh, nb, dr, k0, tau);

  __syncthreads();
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(t + kPanelThreads * s);
    if (lr < static_cast<unsigned>(dr)) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) ybase[static_cast<int64_t>(c) * ldy + lr] = P[s][c];
    }
  }
  if (t < NB * NB) Tout[t] = sh.Ts[t % NB][t / NB];  // column-major NB x NB
}

// W_part[split][k][c] = sum over the split's rows of V[r][k] * C[r][c].
template <int NB>
__global__ __launch_bounds__(256) void qr_vtc_kernel(const double *__restrict__ Y, int64_t ldy, int d,
                                                     int k0, int nb, int c_begin, int nc,
                                                     int rows_per_split, double *__restrict__ Wp) {
  constexpr int CPT = NB >= 4 ? NB / 4 : 1;  // output columns per thread
  constexpr int TPK = kTile / CPT;           // threads per V column (NB * TPK <= 256)
  __shared__ double Vs[kTile][NB + 1];
  __shared__ double Cs[kTile][kTile + 1];  // [column][row]
  const int t = threadIdx.x;
  const int k = t / TPK, cq = t % TPK;
  const int cblk = blockIdx.x * kTile;
  const int split = blockIdx.y;
  const int dr = d - k0;
  const int r_begin = split * rows_per_split;
  const int r_end = min(dr, r_begin + rows_per_split);
  double acc[CPT];
#pragma unroll
  for (int q = 0; q < CPT; ++q) acc[q] = 0.0;

  for (int r0 = r_begin; r0 < r_end; r0 += kTile) {
    for (int e = t; e < kTile * kTile; e += 256) {
      const int cc = e / kTile, rr = e % kTile;
      const int r = r0 + rr, c = cblk + cc;
      Cs[cc][rr] = (r < r_end && c < nc) ? Y[(k0 + r) + static_cast<int64_t>(c_begin + c) * ldy] : 0.0;
    }
    for (int e = t; e < kTile * NB; e += 256) {
      const int kk = e / kTile, rr = e % kTile;
      const int r = r0 + rr;
      double v = 0.0;
      if (r < r_end && kk < nb)
        v = vval(r, kk, r > kk ? Y[(k0 + r) + static_cast<int64_t>(k0 + kk) * ldy] : 0.0);
      Vs[rr][kk] = v;
    }
    __syncthreads();
#pragma unroll 8
    for (int rr = 0; rr < kTile; ++rr) {
      const double v = k < NB ? Vs[rr][k] : 0.0;
#pragma unroll
      for (int q = 0; q < CPT; ++q) acc[q] += v * Cs[cq * CPT + q][rr];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < CPT; ++q) {
    const int c = cblk + cq * CPT + q;
    if (k < NB && c < nc) Wp[(static_cast<int64_t>(split) * NB + k) * nc + c] = acc[q];
  }
}

// W2[k][c] = sum_{l<=k} T[l][k] * (sum_split W_part[split][l][c]).
template <int NB>
__global__ __launch_bounds__(256) void qr_w2_kernel(const double *__restrict__ Wp, int nsplit, int nc,
                                                    int nb, const double *__restrict__ T,
                                                    double *__restrict__ W2) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  double w[NB];
#pragma unroll
  for (int l = 0; l < NB; ++l) {
    double s = 0.0;
    if (l < nb)
      for (int sp = 0; sp < nsplit; ++sp) s += Wp[(static_cast<int64_t>(sp) * NB + l) * nc + c];
    w[l] = s;
  }
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l <= k; ++l) s += T[l + k * NB] * w[l];
    W2[static_cast<int64_t>(k) * nc + c] = (k < nb) ? s : 0.0;
  }
}

// C[r][c] -= sum_k V[r][k] * W2[k][c] on a 64 x 64 tile.
template <int NB>
__global__ __launch_bounds__(256) void qr_update_kernel(double *__restrict__ Y, int64_t ldy, int d,
                                                        int k0, int nb, int c_begin, int nc,
                                                        const double *__restrict__ W2) {
  __shared__ double Vs[kTile][NB + 1];
  __shared__ double Ws[NB][kTile + 1];
  const int t = threadIdx.x;
  const int rblk = blockIdx.x * kTile, cblk = blockIdx.y * kTile;
  const int dr = d - k0;
  for (int e = t; e < kTile * NB; e += 256) {
    const int kk = e / kTile, rr = e % kTile;
    const int r = rblk + rr;
    double v = 0.0;
    if (r < dr && kk < nb) v = vval(r, kk, r > kk ? Y[(k0 + r) + static_cast<int64_t>(k0 + kk) * ldy] : 0.0);
    Vs[rr][kk] = v;
    const int c = cblk + rr;
    Ws[kk][rr] = (c < nc) ? W2[static_cast<int64_t>(kk) * nc + c] : 0.0;
  }
  __syncthreads();
  const int rr = t % kTile, cg = t / kTile;  // 4 groups of 16 columns
  const int r = rblk + rr;
  if (r >= dr) return;
  double v[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) v[k] = Vs[rr][k];
#pragma unroll 4
  for (int q = 0; q < kTile / 4; ++q) {
    const int cc = cg * (kTile / 4) + q;
    const int c = cblk + cc;
    if (c < nc) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < NB; ++k) s += v[k] * Ws[k][cc];
      Y[(k0 + r) + static_cast<int64_t>(c_begin + c) * ldy] -= s;
    }
  }
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
  int s;   // rows per thread in the panel kernel
  int nb;  // panel width
};

QrShape qr_shape(int rows) {
  // The register panel (S * NB doubles per thread) plus the per-column
  // temporaries must fit in the 256 VGPRs a 512-thread workgroup leaves each
  // lane; S * NB <= 32 does (larger products spill to scratch).
  const int s = (rows + kPanelThreads - 1) / kPanelThreads;
  if (s <= 1) return {1, 16};
  if (s <= 2) return {2, 16};
  if (s <= 4) return {4, 8};
  if (s <= 8) return {8, 4};
  if (s <= 16) return {16, 2};
  return {32, 1};
}

constexpr int kMaxSplits = 32;

template <int S, int NB>
sap_status qr_run(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                  hipStream_t st) {
  Carve cv(work);
  double *T = cv.take<double>(NB * NB);
  double *W2 = cv.take<double>(static_cast<size_t>(NB) * cols);
  double *Wp = cv.take<double>(static_cast<size_t>(kMaxSplits) * NB * cols);
  const int kmax = rows < cols ? rows : cols;
  for (int k0 = 0; k0 < kmax; k0 += NB) {
    const int nb = (kmax - k0) < NB ? (kmax - k0) : NB;
    qr_panel_kernel<S, NB><<<1, kPanelThreads, 0, st>>>(Y, ldy, rows, k0, nb, tau, T);
    SAP_HIP_TRY(hipGetLastError());
    const int c_begin = k0 + nb;
    const int nc = cols - c_begin;
    if (nc <= 0) continue;
    const int dr = rows - k0;
    const int cblocks = (nc + kTile - 1) / kTile;
    // enough row splits to give ~2 workgroups per CU, each >= 128 rows
    int nsplit = (2 * ctx->num_cus + cblocks - 1) / cblocks;
    nsplit = nsplit < 1 ? 1 : (nsplit > kMaxSplits ? kMaxSplits : nsplit);
    const int max_by_rows = (dr + 127) / 128;
    if (nsplit > max_by_rows) nsplit = max_by_rows < 1 ? 1 : max_by_rows;
    int rps = (dr + nsplit - 1) / nsplit;
    rps = (rps + kTile - 1) / kTile * kTile;
    nsplit = (dr + rps - 1) / rps;
    qr_vtc_kernel<NB><<<dim3(cblocks, nsplit), 256, 0, st>>>(Y, ldy, rows, k0, nb, c_begin, nc, rps, Wp);
    SAP_HIP_TRY(hipGetLastError());
    qr_w2_kernel<NB><<<(nc + 255) / 256, 256, 0, st>>>(Wp, nsplit, nc, nb, T, W2);
    SAP_HIP_TRY(hipGetLastError());
    qr_update_kernel<NB><<<dim3((dr + kTile - 1) / kTile, cblocks), 256, 0, st>>>(Y, ldy, rows, k0, nb,
                                                                               c_begin, nc, W2);
    SAP_HIP_TRY(hipGetLastError());
  }
  return SAP_OK;
}

}  // namespace

size_t qr_workspace_bytes(int rows, int cols) {
  const QrShape sh = qr_shape(rows);
  return 256 * 4 + sizeof(double) * (static_cast<size_t>(sh.nb) * sh.nb +
                                     static_cast<size_t>(sh.nb) * cols * (1 + kMaxSplits));
}

sap_status launch_qr(sap_ctx *ctx, double *Y, int64_t ldy, int rows, int cols, double *tau, void *work,
                     hipStream_t st) {
  const QrShape sh = qr_shape(rows);
  switch (sh.s) {
    case 1: return qr_run<1, 16>(ctx, Y, ldy, rows, cols, tau, work, st);
    case 2: return qr_run<2, 16>(ctx, Y, ldy, rows, cols, tau, work, st);
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
