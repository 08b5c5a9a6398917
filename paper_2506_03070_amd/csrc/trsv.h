// Blocked triangular solves with R (shared by the standalone solve and the
// LSQR iteration kernels).  See trsv.hip for the scheme.
#pragma once

#include "common.h"

namespace sap {

constexpr int kTrsvB = 64;                            // block size
constexpr int kTrsvThreads = 1024;                    // threads per block workgroup
constexpr int kTrsvGroups = kTrsvThreads / kTrsvB;    // column groups per block
constexpr int kTrsvCols = kTrsvB / kTrsvGroups;       // columns per thread per block

// Per-factorisation data of the chain solves: R (in place), the explicit
// transpose of its upper triangle, and the inverses of the diagonal blocks.
struct TrsvFactor {
  int n = 0;
  const double *R = nullptr;
  int64_t ldr = 0;
  double *Rt = nullptr;   // n x n, column-major; Rt(c, r) = R(r, c) for r <= c
  double *Dup = nullptr;  // nblk blocks of 64 x 64: inverses of R's diagonal blocks
  double *Dlo = nullptr;  // their transposes
};

size_t trsv_factor_bytes(int n);
void trsv_factor_carve(TrsvFactor &f, Carve &cv, int n);
sap_status trsv_prepare(sap_ctx *ctx, const double *R, int64_t ldr, TrsvFactor &f, hipStream_t st);
// z = R^-1 rhs (upper) or R^-T rhs (lower).  flags: nblk ints of workspace;
// err: device word, bit 1 set if a wait expired.
sap_status trsv_solve(sap_ctx *ctx, const TrsvFactor &f, bool upper, const double *rhs, double *x, int *flags,
                      int *err, hipStream_t st);

constexpr int kSpinLimit = 1 << 24;

// Cross-workgroup hand-off without whole-cache maintenance.  The solution
// entries and the flags are written and read with agent-scope relaxed
// atomics, which the gfx950 memory model makes coherent across the XCDs
// per access (no L2 writeback or invalidate).  Ordering: a producer waits
// until its own entry stores have completed (s_waitcnt vmcnt(0)) before it
// stores the flag; a consumer issues its entry loads only after its flag
// load has returned the awaited epoch.
__device__ __forceinline__ void store_coherent(double *p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_coherent(const double *p) {
  return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void wait_flag(const int *flag, int epoch, int *err) {
  if (threadIdx.x == 0) {
    int spins = 0;
    while (__hip_atomic_load(const_cast<int *>(flag), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kSpinLimit) {
        atomicOr(err, 2);
        break;
      }
    }
  }
  __syncthreads();
}

// Every wave calls this after its coherent stores; thread 0 then raises the flag.
__device__ __forceinline__ void publish_flag(int *flag, int epoch) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Solve for block b of the chain; rb (LDS, kTrsvB doubles) holds the
// right-hand side of the block on entry.  On exit z_b is in rb, in z, and
// announced through flags[b].  red: LDS of kTrsvGroups * kTrsvB doubles.
template <bool UP>
__device__ __forceinline__ void chain_block(const double *__restrict__ M, int64_t ldm, int n, const double *__restrict__ Dinv,
                            double *__restrict__ z, int *flags, int epoch, int b, double *rb, double *red,
                            int *err) {
  const int t = threadIdx.x;
  const int r = t % kTrsvB, g = t / kTrsvB;  // row of the block, column group
  const int nblk = (n + kTrsvB - 1) / kTrsvB;
  const int row = b * kTrsvB + r;
  double acc = 0.0;
  const int ndeps = UP ? (nblk - 1 - b) : b;
  for (int s = 0; s < ndeps; ++s) {
    const int j = UP ? (nblk - 1 - s) : s;  // production order
    double mv[kTrsvCols];
#pragma unroll
    for (int k = 0; k < kTrsvCols; ++k) {
      const int col = j * kTrsvB + g + kTrsvGroups * k;
      mv[k] = (row < n && col < n) ? M[row + static_cast<int64_t>(col) * ldm] : 0.0;
    }
    wait_flag(&flags[j], epoch, err);
#pragma unroll
    for (int k = 0; k < kTrsvCols; ++k) {
      const int col = j * kTrsvB + g + kTrsvGroups * k;
      const double zc = col < n ? load_coherent(z + col) : 0.0;
      acc += mv[k] * zc;
    }
  }
  red[g * kTrsvB + r] = acc;
  __syncthreads();
  if (t < kTrsvB) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kTrsvGroups; ++q) s += red[q * kTrsvB + t];
    rb[t] = rb[t] - s;
  }
  __syncthreads();
  // z_b = Dinv_b rb
  const double *D = Dinv + static_cast<int64_t>(b) * kTrsvB * kTrsvB;
  double acc2 = 0.0;
#pragma unroll
  for (int k = 0; k < kTrsvCols; ++k) {
    const int c = g + kTrsvGroups * k;
    acc2 += D[r + c * kTrsvB] * rb[c];
  }
  __syncthreads();
  red[g * kTrsvB + r] = acc2;
  __syncthreads();
  if (t < kTrsvB) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kTrsvGroups; ++q) s += red[q * kTrsvB + t];
    rb[t] = s;
    if (row < n) store_coherent(z + row, s);
  }
  publish_flag(&flags[b], epoch);
}

// Inverse of diagonal block b of R (upper) and its transpose (for R^T);
// 256 threads, column c of the inverse by back substitution of R_bb x = e_c.
struct TrsvPrepShared {
  double Rb[kTrsvB][kTrsvB + 1];
  double X[kTrsvB][kTrsvB + 1];  // X[row][col] = (R_bb^-1)(row, col)
};

__device__ __forceinline__ void trsv_invert_diag_block(const double *__restrict__ R, int64_t ldr, int n, int b,
                                                       double *__restrict__ Dup, double *__restrict__ Dlo,
                                                       TrsvPrepShared &sh) {
  const int k0 = b * kTrsvB;
  const int kn = min(kTrsvB, n - k0);
  for (int e = threadIdx.x; e < kTrsvB * kTrsvB; e += blockDim.x) {
    const int rr = e % kTrsvB, cc = e / kTrsvB;
    sh.Rb[rr][cc] = (rr < kn && cc < kn && rr <= cc) ? R[(k0 + rr) + static_cast<int64_t>(k0 + cc) * ldr] : 0.0;
    sh.X[rr][cc] = 0.0;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < kn) {
    sh.X[c][c] = 1.0 / sh.Rb[c][c];
    for (int rr = c - 1; rr >= 0; --rr) {
      double s = 0.0;
      for (int k = rr + 1; k <= c; ++k) s += sh.Rb[rr][k] * sh.X[k][c];
      sh.X[rr][c] = -s / sh.Rb[rr][rr];
    }
  }
  __syncthreads();
  double *du = Dup + static_cast<int64_t>(b) * kTrsvB * kTrsvB;
  double *dl = Dlo + static_cast<int64_t>(b) * kTrsvB * kTrsvB;
  for (int e = threadIdx.x; e < kTrsvB * kTrsvB; e += blockDim.x) {
    const int rr = e % kTrsvB, cc = e / kTrsvB;
    du[rr + cc * kTrsvB] = sh.X[rr][cc];  // col-major
    dl[rr + cc * kTrsvB] = sh.X[cc][rr];  // (R_bb^T)^-1 = (R_bb^-1)^T
  }
}

// One 32 x 32 tile of the transpose of R's upper triangle:
// Rt[c + r*n] = R[r + c*ldr] for r <= c (the strict lower triangle of Rt is
// never read by the chain and is left untouched).  256 threads.
__device__ __forceinline__ void trsv_transpose_tile(const double *__restrict__ R, int64_t ldr, int n, int tx_blk,
                                                    int ty_blk, double *__restrict__ Rt, double (&tile)[32][33]) {
  const int bx = tx_blk * 32, by = ty_blk * 32;  // tile of R: rows by.., cols bx..
  const int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  if (by > bx + 31) return;  // entirely below the diagonal (uniform per workgroup)
  for (int k = ty; k < 32; k += 8) {
    const int rr = by + tx, cc = bx + k;
    tile[k][tx] = (rr < n && cc < n) ? R[rr + static_cast<int64_t>(cc) * ldr] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    // Rt(row = bx + tx, col = by + k) = R(by + k, bx + tx)
    const int rr = bx + tx, cc = by + k;
    if (rr < n && cc < n && cc <= rr) Rt[rr + static_cast<int64_t>(cc) * n] = tile[tx][k];
  }
}

}  // namespace sap
