// Blocked triangular solves with the preconditioner factor R on gfx950
// (M = R^-1 of Alg. 1 applied without forming the inverse).
//
// The solve is split into 64-row blocks.  Block b is owned by one 1024-thread
// workgroup, which
//   1. streams the off-diagonal blocks M[b, j] of its block row into
//      registers before their solution pieces z_j exist,
//   2. waits, in production order, for each z_j it depends on (a flag written
//      with release semantics by the producing workgroup, read with acquire
//      semantics here), and subtracts M[b, j] z_j,
//   3. multiplies by the inverse of its 64 x 64 diagonal block (inverted once
//      per factorisation), and publishes z_b and its flag.
// Workgroup indices are assigned so that a workgroup only ever waits on
// workgroups with a smaller index, which the hardware dispatches first: the
// chain makes progress even when not every workgroup is resident.  Waits are
// bounded; on expiry an error word is set and the kernel finishes (the result
// is then discarded by the host).
//
// Upper solves (R x = v) read R in place.  Lower solves (R^T y = q) read an
// explicit transpose of R's upper triangle so that both directions stream
// contiguous 64-element column pieces.
#include <cmath>

#include "common.h"
#include "trsv.h"

namespace sap {

// ---------------------------------------------------------------------------
// Per-factorisation preparation: inverses of the diagonal blocks of R (upper,
// for R x = v) and of R^T (their transposes, for R^T y = q), and the explicit
// transpose of R's upper triangle.
__global__ __launch_bounds__(256) void trsv_prepare_kernel(const double *__restrict__ R, int64_t ldr, int n,
                                                           double *__restrict__ Dup, double *__restrict__ Dlo) {
  __shared__ TrsvPrepShared sh;
  trsv_invert_diag_block(R, ldr, n, static_cast<int>(blockIdx.x), Dup, Dlo, sh);
}

__global__ __launch_bounds__(256) void trsv_transpose_kernel(const double *__restrict__ R, int64_t ldr, int n,
                                                             double *__restrict__ Rt) {
  __shared__ double tile[32][33];
  trsv_transpose_tile(R, ldr, n, static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y), Rt, tile);
}

__global__ void trsv_zero_flags_kernel(int *flags, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) flags[i] = 0;
}

// Standalone solve: z = T^-1 rhs with T = R (UP) or R^T (lower, via Rt).
template <bool UP>
__global__ __launch_bounds__(kTrsvThreads) void trsv_solve_kernel(const double *__restrict__ M, int64_t ldm, int n,
                                                                  const double *__restrict__ Dinv,
                                                                  const double *__restrict__ rhs, double *z,
                                                                  int *flags, int *err) {
  __shared__ double rb[kTrsvB];
  __shared__ double red[kTrsvGroups * kTrsvB];
  const int nblk = (n + kTrsvB - 1) / kTrsvB;
  const int b = UP ? (nblk - 1 - static_cast<int>(blockIdx.x)) : static_cast<int>(blockIdx.x);
  if (threadIdx.x < kTrsvB) {
    const int row = b * kTrsvB + threadIdx.x;
    rb[threadIdx.x] = row < n ? rhs[row] : 0.0;
  }
  __syncthreads();
  chain_block<UP>(M, ldm, n, Dinv, z, flags, 1, b, rb, red, err);
}

size_t trsv_factor_bytes(int n) {
  const size_t nblk = static_cast<size_t>((n + kTrsvB - 1) / kTrsvB);
  return sizeof(double) * (2 * nblk * kTrsvB * kTrsvB + static_cast<size_t>(n) * n) + 4 * 256;
}

void trsv_factor_carve(TrsvFactor &f, Carve &cv, int n) {
  const size_t nblk = static_cast<size_t>((n + kTrsvB - 1) / kTrsvB);
  f.n = n;
  f.Dup = cv.take<double>(nblk * kTrsvB * kTrsvB);
  f.Dlo = cv.take<double>(nblk * kTrsvB * kTrsvB);
  f.Rt = cv.take<double>(static_cast<size_t>(n) * n);
}

sap_status trsv_prepare(sap_ctx *ctx, const double *R, int64_t ldr, TrsvFactor &f, hipStream_t st) {
  const int n = f.n;
  const int nblk = (n + kTrsvB - 1) / kTrsvB;
  f.R = R;
  f.ldr = ldr;
  trsv_prepare_kernel<<<nblk, 256, 0, st>>>(R, ldr, n, f.Dup, f.Dlo);
  const int nt = (n + 31) / 32;
  trsv_transpose_kernel<<<dim3(nt, nt), 256, 0, st>>>(R, ldr, n, f.Rt);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

sap_status trsv_solve(sap_ctx *ctx, const TrsvFactor &f, bool upper, const double *rhs, double *x, int *flags,
                      int *err, hipStream_t st) {
  const int n = f.n;
  const int nblk = (n + kTrsvB - 1) / kTrsvB;
  trsv_zero_flags_kernel<<<1, 256, 0, st>>>(flags, nblk);
  if (upper)
    trsv_solve_kernel<true><<<nblk, kTrsvThreads, 0, st>>>(f.R, f.ldr, n, f.Dup, rhs, x, flags, err);
  else
    trsv_solve_kernel<false><<<nblk, kTrsvThreads, 0, st>>>(f.Rt, n, n, f.Dlo, rhs, x, flags, err);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

}  // namespace sap
