// Device code of the blocked Householder QR, shared by the chained single QR
// (qr.hip) and the batched step launches (batch.hip): register-block panel
// factorisation with the LAPACK dlarfg sign convention, block loads and
// stores, and the compact-WY block-reflector apply of the batched steps.
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
// TH: threads of the workgroup (512 or 1024); thread t holds rows t + TH s.
template <int NB, int TH = kPanelThreads>
struct PanelShared {
  double red[TH / kWave][NB * NB + 1];  // per-wave partials of W = V^T C
  double W2[NB][NB];
  double cred[2][TH / kWave][NB];       // per-wave partials of one panel column, by column parity
  double ctot[2][2 * NB];                // its totals (0..NB-1) and row J of the panel (NB..2NB-1)
  double G[NB][NB];                      // G[J][q] = v_q^T v_J (q < J), for T
  double tauv[NB];
  double Tl[NB * NB];                    // T of the panel being applied
};

// Rows: thread t holds panel-relative rows lr = t + TH s - roff (s < S);
// rows with lr < 0 lie above the panel (they belong to R) and only ride along.

// Column J of the panel: reflector, update of columns J+1.. of the panel,
// and what column J of T needs (tau_J, V_{<J}^T v_J, kept in LDS).  One batched
// workgroup reduction per column: with a = column J below the diagonal,
// alpha its diagonal entry and v = [1; a / (alpha - beta)], every quantity
// the column needs follows from a^T a and a^T (column x) for all x and from
// row J of the panel: v^T (column x) = P[J][x] + (a^T column x) / (alpha - beta).
// J is a template parameter so that every register index of the panel P is
// static (no scratch).
template <int S, int NB, int J, int TH>
__device__ __forceinline__ void panel_column(double (&P)[S][NB], PanelShared<NB, TH> &sh, int nb, int dr, int roff,
                                             int k0, double *__restrict__ tau) {
  constexpr int B = J & 1;  // LDS buffers alternate between columns: one barrier fewer
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  // Straight-line code: masks instead of per-row branches (the column is
  // latency-bound, and every branch costs exec-mask bookkeeping).
  double acc[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) acc[x] = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + TH * s - roff;
    const double a = (lr > J && lr < dr) ? P[s][J] : 0.0;
#pragma unroll
    for (int x = 0; x < NB; ++x) acc[x] += a * P[s][x];
  }
  // row J of the panel is held by one thread: in its register row 0 whenever
  // J + roff < TH (every caller: roff <= NB), else found by selects with
  // static indices only
  if (J + roff < TH) {  // uniform
    if (J < dr && t == J + roff) {
#pragma unroll
      for (int x = 0; x < NB; ++x) sh.ctot[B][NB + x] = P[0][x];
    }
  } else {
    double rowv[NB];
    bool has_j = false;
#pragma unroll
    for (int x = 0; x < NB; ++x) rowv[x] = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int lr = t + TH * s - roff;
      const bool hit = lr == J && lr < dr;
      has_j = has_j || hit;
#pragma unroll
      for (int x = 0; x < NB; ++x) rowv[x] = hit ? P[s][x] : rowv[x];
    }
    if (has_j) {
#pragma unroll
      for (int x = 0; x < NB; ++x) sh.ctot[B][NB + x] = rowv[x];
    }
  }
#pragma unroll
  for (int x = 0; x < NB; ++x) acc[x] = wave_sum_u(acc[x]);
  if (lane == 0) {
#pragma unroll
    for (int x = 0; x < NB; ++x) sh.cred[B][wave][x] = acc[x];
  }
  __syncthreads();
  if (t < NB) {
    double s_ = 0.0;
    for (int w = 0; w < (TH / kWave); ++w) s_ += sh.cred[B][w][t];
    sh.ctot[B][t] = s_;
  }
  __syncthreads();
  const bool has_row = J < dr;  // uniform; a panel shorter than J+1 rows has no row J
  double tot[NB], row[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    tot[x] = sh.ctot[B][x];
    row[x] = has_row ? sh.ctot[B][NB + x] : 0.0;
  }
  const double alpha = row[J];
  const double sq = tot[J];
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
  // dots[x] = v^T (column x): x > J weights the update of column x, x < J
  // gives V_{<J}^T v for the T factor
  double dots[NB], wgt[NB];
#pragma unroll
  for (int x = 0; x < NB; ++x) {
    dots[x] = x == J ? 0.0 : row[x] + scale * tot[x];
    wgt[x] = (x > J && x < nb) ? tj * dots[x] : 0.0;
  }
  // column J becomes v below the diagonal and beta on it; H_J = I - tj v v^T
  // is applied to the panel columns right of J (v = 0 outside the panel rows
  // from J on, where the subtraction leaves the value unchanged)
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + TH * s - roff;
    const bool below = lr > J && lr < dr;
    const bool diag = lr == J;
    const double v = below ? P[s][J] * scale : (diag ? 1.0 : 0.0);
    P[s][J] = below ? v : (diag ? beta : P[s][J]);
#pragma unroll
    for (int x = J + 1; x < NB; ++x) P[s][x] -= wgt[x] * v;
  }
  // LDS only: a global store here would hold up the next column, since a
  // workgroup barrier waits for the wave's outstanding memory operations
  if (t == 0) {
    sh.tauv[J] = tj;
#pragma unroll
    for (int q = 0; q < J; ++q) sh.G[J][q] = dots[q];
  }
}

template <int S, int NB, int J, int TH>
__device__ __forceinline__ void panel_columns(double (&P)[S][NB], PanelShared<NB, TH> &sh, int nb, int dr, int roff,
                                              int k0, double *__restrict__ tau) {
  if constexpr (J < NB) {
    if (J < nb) {  // nb is uniform: every thread reaches the same barriers
      panel_column<S, NB, J, TH>(P, sh, nb, dr, roff, k0, tau);
      panel_columns<S, NB, J + 1, TH>(P, sh, nb, dr, roff, k0, tau);
    }
  }
}

// Factor the panel held in P (columns k0 .. k0+nb-1, rows from k0); writes
// tau and T (column-major NB x NB).  T follows the dlarft recurrence
// T(0:J, J) = -tau_J T(0:J, 0:J) V_{<J}^T v_J, T(J, J) = tau_J once all
// columns are done: row l of T depends only on its own earlier entries, so
// thread l builds row l.  Ends without a barrier (the tau and T stores stay
// in flight); a caller that reuses `sh` afterwards synchronises first.
template <int S, int NB, int TH>
__device__ __forceinline__ void factor_panel(double (&P)[S][NB], PanelShared<NB, TH> &sh, int nb, int dr, int roff,
                                             int k0, double *__restrict__ tau, double *__restrict__ Tout) {
  const int t = threadIdx.x;
  __syncthreads();  // earlier users of the shared buffers are done
  if (t < NB * NB) sh.G[t / NB][t % NB] = 0.0;
  if (t < NB) sh.tauv[t] = 0.0;
  panel_columns<S, NB, 0, TH>(P, sh, nb, dr, roff, k0, tau);  // its first barrier orders the zeroing
  __syncthreads();
  if (t < NB) {
    const int l = t;
    double row[NB];
#pragma unroll
    for (int J = 0; J < NB; ++J) {
      double a = 0.0;
#pragma unroll
      for (int q = 0; q < J; ++q)
        if (q >= l) a += row[q] * sh.G[J][q];
      row[J] = J < l ? 0.0 : (J == l ? sh.tauv[J] : -sh.tauv[J] * a);
      Tout[l + J * NB] = row[J];
    }
    if (l < nb) tau[k0 + l] = sh.tauv[l];
  }
}

// C <- (I - V T^T V^T) C for the block C[S][NB] (rows from k0), where V are
// the nbp Householder vectors stored in columns k0.. of Y (unit diagonal
// implicit) and T the panel's triangular factor (column-major NB x NB).
// Writes `sh` before its first barrier: no other use of `sh` may be pending.
template <int S, int NB, int TH>
__device__ __forceinline__ void apply_panel_qt(const double *__restrict__ Y, int64_t ldy, int dr, int k0, int nbp,
                                               const double *__restrict__ T, double (&C)[S][NB], int ncb,
                                               PanelShared<NB, TH> &sh) {
  if (nbp <= 0 || dr <= 0) return;  // uniform: no reflectors, nothing to apply
  const int t = threadIdx.x;
  const int lane = t & (kWave - 1), wave = t / kWave;
  const double *__restrict__ vb = Y + k0 + static_cast<int64_t>(k0) * ldy;
  const double tload = t < NB * NB ? T[t] : 0.0;  // in flight with the V loads
  // Every load is issued unconditionally from an in-range address (row and
  // column clamped, dr >= 1 and nbp >= 1) and masked afterwards: no branch
  // separates the loads.
  double V[S][NB];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int lr = t + TH * s;
    const int rr = min(lr, dr - 1);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const double y = vb[static_cast<int64_t>(min(i, nbp - 1)) * ldy + rr];
      V[s][i] = (i < nbp && lr < dr) ? vval(lr, i, y) : 0.0;
    }
  }
  if (t < NB * NB) sh.Tl[t] = tload;
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
  // W2 = T^T W: W2[i][c] = sum_{l <= i} T[l][i] W[l][c], each W[l][c] summed
  // over the waves by the thread that needs it (no separate pass for W)
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

// Loads rows r0 .. r0+dr-1 of columns c0 .. c0+ncb-1.  Addresses are
// clamped into the block, so the loads need no branches and no select waits
// for their data: a slot outside the block (row >= dr or column >= ncb) holds
// a copy of an entry inside it.  Every user masks those slots: the apply
// weights them by V = 0 and W2 = 0, the panel factorisation by its row and
// column masks, and store_block does not write them.
template <int S, int NB, int TH = kPanelThreads>
__device__ __forceinline__ void load_block(const double *__restrict__ Y, int64_t ldy, int r0, int dr, int c0, int ncb,
                                           double (&C)[S][NB]) {
  if (dr <= 0 || ncb <= 0) {  // uniform
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int c = 0; c < NB; ++c) C[s][c] = 0.0;
    return;
  }
  const double *__restrict__ base = Y + r0 + static_cast<int64_t>(c0) * ldy;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int rr = min(static_cast<int>(threadIdx.x) + TH * s, dr - 1);
#pragma unroll
    for (int c = 0; c < NB; ++c) C[s][c] = base[static_cast<int64_t>(min(c, ncb - 1)) * ldy + rr];
  }
}

template <int S, int NB, int TH = kPanelThreads>
__device__ __forceinline__ void store_block(double *__restrict__ Y, int64_t ldy, int r0, int dr, int c0, int ncb,
                                            const double (&C)[S][NB]) {
  double *__restrict__ base = Y + r0 + static_cast<int64_t>(c0) * ldy;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const unsigned lr = static_cast<unsigned>(threadIdx.x + TH * s);
    if (lr < static_cast<unsigned>(dr)) {
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < ncb) base[static_cast<int64_t>(c) * ldy + lr] = C[s][c];
    }
  }
}

}  // namespace qr_dev
}  // namespace sap
