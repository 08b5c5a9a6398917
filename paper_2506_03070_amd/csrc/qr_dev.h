// Device code of the blocked Householder QR (qr.hip), shared by the single
// and batched launches: register-block panel factorisation with the LAPACK
// dlarfg sign convention and the compact-WY block-reflector apply.
#pragma once

#include "common.h"

namespace sap {
namespace qr_dev {


constexpr int kPanelThreads = 512;
constexpr int kPanelWaves = kPanelThreads / kWave;

// Householder vector entry (implicit unit diagonal, zeros above) of panel
// column k at panel-relative row r; `y` is the stored value.
__device__ __forceinline__ double vval(int r, int k, double y) {
  return r > k ? y : (r == k ? 1.0 : 0.0);
}

// Shared state of the panel factorisation and the block-reflector apply (LDS).
template <int NB>
struct PanelShared {
  double red[kPanelWaves][NB * NB + 1];
  double bc[2];
  double Ts[NB][NB];
  double gdot[NB * NB];
  double W2[NB][NB];
};

// Rows: thread t holds panel-relative rows lr = t + 512 s - roff (s < S);
// rows with lr < 0 lie above the panel (they belong to R) and only ride along.

// Column J of the panel: reflector, update of columns J+1.. of the panel,
// column J of T.  J is a template parameter so that every register index of
// the panel P is static (no scratch).
template <int S, int NB, int J>
__device__ __forceinline__ void panel_column(double (&P)[S][NB], PanelShared<NB> &sh, int nb, int dr, int roff,
                                             int k0, double *__restrict__ tau) {
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  // --- norm of the part below the diagonal ---
  double part = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + kPanelThreads * s - roff;
    if (lr > J && lr < dr) part += P[s][J] * P[s][J];
  }
  part = wave_sum_u(part);
  __syncthreads();  // previous readers of red/bc are done
  if (lane == 0) sh.red[wave][0] = part;
#pragma unroll
  for (int s = 0; s < S; ++s)
    if (t + kPanelThreads * s - roff == J) sh.bc[0] = P[s][J];  // alpha
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
    const int lr = t + kPanelThreads * s - roff;
    if (lr > J && lr < dr) P[s][J] *= scale;
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
        const int lr = t + kPanelThreads * s - roff;
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
    const int lr = t + kPanelThreads * s - roff;
    const double v = (lr > J && lr < dr) ? P[s][J] : (lr == J ? 1.0 : 0.0);
#pragma unroll
    for (int x = J + 1; x < NB; ++x)
      if (x < nb) P[s][x] -= tj * dots[x] * v;
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
__device__ __forceinline__ void panel_columns(double (&P)[S][NB], PanelShared<NB> &sh, int nb, int dr, int roff,
                                              int k0, double *__restrict__ tau) {
  if constexpr (J < NB) {
    if (J < nb) {  // nb is uniform: every thread reaches the same barriers
      panel_column<S, NB, J>(P, sh, nb, dr, roff, k0, tau);
      panel_columns<S, NB, J + 1>(P, sh, nb, dr, roff, k0, tau);
    }
  }
}

// Factor the panel held in P (columns k0 .. k0+nb-1, rows from k0); writes
// tau and T (column-major NB x NB).
template <int S, int NB>
__device__ __forceinline__ void factor_panel(double (&P)[S][NB], PanelShared<NB> &sh, int nb, int dr, int roff,
                                             int k0, double *__restrict__ tau, double *__restrict__ Tout) {
  const int t = threadIdx.x;
  __syncthreads();
  if (t < NB * NB) sh.Ts[t / NB][t % NB] = 0.0;
  panel_columns<S, NB, 0>(P, sh, nb, dr, roff, k0, tau);
  __syncthreads();
  if (t < NB * NB) Tout[t] = sh.Ts[t % NB][t / NB];
}

// C <- (I - V T^T V^T) C for the block C[S][NB] (rows from k0), where V are
// the nbp Householder vectors stored in columns k0.. of Y (unit diagonal
// implicit) and T the panel's triangular factor (column-major NB x NB).
template <int S, int NB>
__device__ __forceinline__ void apply_panel_qt(const double *__restrict__ Y, int64_t ldy, int dr, int k0, int nbp,
                                               const double *__restrict__ T, double (&C)[S][NB], int ncb,
                                               PanelShared<NB> &sh) {
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  const double *__restrict__ vb = Y + k0 + static_cast<int64_t>(k0) * ldy;
  double V[S][NB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(t + kPanelThreads * s);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      double v = 0.0;
      if (i < nbp && lr < static_cast<unsigned>(dr)) v = vval(static_cast<int>(lr), i, lr > static_cast<unsigned>(i) ? vb[static_cast<int64_t>(i) * ldy + lr] : 0.0);
      V[s][i] = v;
    }
  }
  // W = V^T C  (NB x NB values, each a workgroup-wide sum)
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
    double s_ = 0.0;
    for (int w = 0; w < kPanelWaves; ++w) s_ += sh.red[w][t];
    sh.gdot[t] = s_;  // W[i][c] at i*NB + c
  }
  __syncthreads();
  // W2 = T^T W: W2[i][c] = sum_{l <= i} T[l][i] W[l][c]
  if (t < NB * NB) {
    const int i = t / NB, c = t % NB;
    double s_ = 0.0;
    for (int l = 0; l <= i && l < nbp; ++l) s_ += T[l + i * NB] * sh.gdot[l * NB + c];
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

template <int S, int NB>
__device__ __forceinline__ void load_block(const double *__restrict__ Y, int64_t ldy, int r0, int dr, int c0, int ncb,
                                           double (&C)[S][NB]) {
  const double *__restrict__ base = Y + r0 + static_cast<int64_t>(c0) * ldy;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(threadIdx.x + kPanelThreads * s);
#pragma unroll
    for (int c = 0; c < NB; ++c)
      C[s][c] = (lr < static_cast<unsigned>(dr) && c < ncb) ? base[static_cast<int64_t>(c) * ldy + lr] : 0.0;
  }
}

template <int S, int NB>
__device__ __forceinline__ void store_block(double *__restrict__ Y, int64_t ldy, int r0, int dr, int c0, int ncb,
                                            const double (&C)[S][NB]) {
  double *__restrict__ base = Y + r0 + static_cast<int64_t>(c0) * ldy;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(threadIdx.x + kPanelThreads * s);
    if (lr < static_cast<unsigned>(dr)) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < ncb) base[static_cast<int64_t>(c) * ldy + lr] = C[s][c];
    }
  }
}

}  // namespace qr_dev
}  // namespace sap
