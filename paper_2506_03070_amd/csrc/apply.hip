// Sketch apply Y = S [A b] on gfx950 (Alg. 1 "form Y = SA"; the paper calls a
// library sparse-times-dense product, Sec. 3).
//
// Design: A is read from HBM exactly once.  The output Y (d x ncols,
// column-major) is far larger than one CU's LDS, so each workgroup owns a
// narrow column tile of Y, Y[r_lo : r_lo + DR, c0 : c0 + NT], kept in LDS
// for its whole life, and streams its slice of the rows of A.  For every row
// i and every one of its zeta nonzeros (row idx[i][k], sign bit k) it adds
// +-A[i, c0:c0+NT] into the LDS rows with native ds_add_f64 / ds_add_f32.
// Workgroups that share a slice of rows are placed on the same XCD with
// adjacent column tiles, so the 128-byte lines of A and the sketch words they
// all read are served from that XCD's L2 after the first touch.  When there
// are too few column tiles to fill the chip, rows are split into slices whose
// partial tiles are summed (in a fixed order) by a second kernel.
#include <hip/hip_bf16.h>

#include <cmath>
#include <type_traits>

#include "common.h"

namespace sap {
namespace {

constexpr int kApplyThreads = 1024;
constexpr size_t kApplyLdsBytes = 160000;  // gfx950: up to 160 KB of LDS per workgroup
constexpr int kXcds = 8;

template <typename TA, typename TY>
__device__ __forceinline__ TY load_as(const TA *p) {
  if constexpr (std::is_same<TA, __hip_bfloat16>::value)
    return static_cast<TY>(__bfloat162float(*p));
  else
    return static_cast<TY>(*p);
}

// One work item = (column tile, row range of Y, slice of rows of A).
template <typename TA, typename TY, int NT, int ZT>
__global__ __launch_bounds__(kApplyThreads) void apply_lds_kernel(
    const int32_t *__restrict__ idx, const uint64_t *__restrict__ sign, int zeta,
    const TA *__restrict__ A, int64_t lda, const double *__restrict__ b, int64_t m, int n,
    int ncols, int d, int dr, int ntiles, int nranges, int nslices, int64_t rows_per_slice,
    TY *__restrict__ out, int64_t ldo, int64_t slice_stride, double h, int scale_now) {
  extern __shared__ unsigned char lds_raw[];
  TY *acc = reinterpret_cast<TY *>(lds_raw);

  // XCD-aware decode: hardware deals workgroup IDs round-robin over the 8
  // XCDs, so give each XCD a contiguous block of work items.
  const int total = ntiles * nranges * nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int w = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (w >= total) return;
  const int tile = w % ntiles;
  const int range = (w / ntiles) % nranges;
  const int slice = w / (ntiles * nranges);
  const int c0 = tile * NT;
  const int r_lo = range * dr;
  const int rows_here = min(dr, d - r_lo);
  const int64_t i_begin = static_cast<int64_t>(slice) * rows_per_slice;
  const int64_t i_end = min(m, i_begin + rows_per_slice);

  for (int e = threadIdx.x; e < rows_here * NT; e += kApplyThreads) acc[e] = TY(0);
  __syncthreads();

  const int zeta_n = ZT > 0 ? ZT : zeta;
  for (int64_t i = i_begin + threadIdx.x; i < i_end; i += kApplyThreads) {
    TY a[NT];
#pragma unroll
    for (int q = 0; q < NT; ++q) {
      const int c = c0 + q;
      a[q] = c < n ? load_as<TA, TY>(A + i * lda + c) : (c == n && c < ncols ? TY(b[i]) : TY(0));
    }
    const uint64_t sg = sign[i];
    const int32_t *row = idx + i * zeta_n;
#pragma unroll
    for (int k = 0; k < zeta_n; ++k) {
      const int r = row[k] - r_lo;
      if (static_cast<unsigned>(r) < static_cast<unsigned>(rows_here)) {
        const bool plus = (sg >> k) & 1ull;
        TY *dst = acc + r * NT;
#pragma unroll
        for (int q = 0; q < NT; ++q) atomicAdd(dst + q, plus ? a[q] : -a[q]);
      }
    }
  }
  __syncthreads();

  const TY scale = scale_now ? TY(h) : TY(1);
  TY *dst = out + static_cast<int64_t>(slice) * slice_stride;
  for (int e = threadIdx.x; e < rows_here * NT; e += kApplyThreads) {
    const int q = e / rows_here, r = e % rows_here;
    const int c = c0 + q;
    if (c < ncols) dst[(r_lo + r) + static_cast<int64_t>(c) * ldo] = acc[r * NT + q] * scale;
  }
}

// Y[r, c] = h * sum_s part[s][r + c*d], slices summed in ascending order.
template <typename TY>
__global__ __launch_bounds__(256) void apply_reduce_kernel(const TY *__restrict__ part, int nslices,
                                                           int64_t slice_stride, int d, int ncols,
                                                           TY *__restrict__ Y, int64_t ldy, double h) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (e >= static_cast<int64_t>(d) * ncols) return;
  const int r = static_cast<int>(e % d);
  const int c = static_cast<int>(e / d);
  TY s = TY(0);
  for (int k = 0; k < nslices; ++k) s += part[k * slice_stride + e];
  Y[r + static_cast<int64_t>(c) * ldy] = s * TY(h);
}

struct ApplyPlan {
  int nt, dr, ntiles, nranges, nslices;
  int64_t rows_per_slice;
};

ApplyPlan make_plan(int num_cus, int64_t m, int d, int ncols, size_t esize) {
  ApplyPlan p{};
  // Widest power-of-two tile (<= 16 columns) whose d rows fit in LDS.
  int nt = 16;
  while (nt > 1 && static_cast<size_t>(d) * nt * esize > kApplyLdsBytes) nt >>= 1;
  while (nt > 1 && (ncols + nt - 1) / nt < 2 * kXcds && nt > 2) nt >>= 1;  // keep several tiles
  p.nt = nt;
  const int64_t dr_max = static_cast<int64_t>(kApplyLdsBytes / (esize * nt));
  p.dr = static_cast<int>(d < dr_max ? d : dr_max);
  p.nranges = (d + p.dr - 1) / p.dr;
  p.ntiles = (ncols + nt - 1) / nt;
  const int items = p.ntiles * p.nranges;
  // One resident workgroup per CU (the tile fills most of the LDS).  Split the
  // rows of A into slices only when there are too few items to fill the chip,
  // and keep each slice at least 4096 rows long.
  int ns = 1;
  if (items < num_cus) ns = (num_cus + items - 1) / items;
  const int64_t max_slices = (m + 4095) / 4096;
  if (ns > max_slices) ns = static_cast<int>(max_slices < 1 ? 1 : max_slices);
  p.nslices = ns;
  p.rows_per_slice = (m + ns - 1) / ns;
  return p;
}

template <typename TA, typename TY, int NT>
void launch_nt(const ApplyPlan &p, const sps_sketch *S, const TA *A, int64_t lda, const double *b,
               int n, int ncols, TY *out, int64_t ldo, int64_t slice_stride, double h,
               int scale_now, hipStream_t st) {
  const int total = p.ntiles * p.nranges * p.nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const dim3 grid(static_cast<unsigned>(per_xcd * kXcds));
  const size_t lds = static_cast<size_t>(p.dr) * NT * sizeof(TY);
  if (S->zeta == 8)
    apply_lds_kernel<TA, TY, NT, 8><<<grid, kApplyThreads, lds, st>>>(
        S->idx, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.ntiles, p.nranges,
        p.nslices, p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
  else
    apply_lds_kernel<TA, TY, NT, 0><<<grid, kApplyThreads, lds, st>>>(
        S->idx, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.ntiles, p.nranges,
        p.nslices, p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
}

template <typename TA, typename TY>
sap_status apply_typed(sap_ctx *ctx, const sps_sketch *S, const TA *A, int64_t lda, const double *b,
                       int n, TY *Y, int64_t ldy, void *work, hipStream_t st) {
  const int ncols = n + (b != nullptr ? 1 : 0);
  const ApplyPlan p = make_plan(ctx->num_cus, S->m, S->d, ncols, sizeof(TY));
  const double h = 1.0 / std::sqrt(static_cast<double>(S->zeta));
  TY *out = Y;
  int64_t ldo = ldy, slice_stride = 0;
  int scale_now = 1;
  if (p.nslices > 1) {
    out = static_cast<TY *>(work);
    ldo = S->d;
    slice_stride = static_cast<int64_t>(S->d) * ncols;
    scale_now = 0;
  }
  switch (p.nt) {
    case 16: launch_nt<TA, TY, 16>(p, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, st); break;
    case 8: launch_nt<TA, TY, 8>(p, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, st); break;
    case 4: launch_nt<TA, TY, 4>(p, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, st); break;
    case 2: launch_nt<TA, TY, 2>(p, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, st); break;
    default: launch_nt<TA, TY, 1>(p, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, st); break;
  }
  SAP_HIP_TRY(hipGetLastError());
  if (p.nslices > 1) {
    const int64_t total = static_cast<int64_t>(S->d) * ncols;
    apply_reduce_kernel<TY><<<static_cast<unsigned>((total + 255) / 256), 256, 0, st>>>(
        out, p.nslices, slice_stride, S->d, ncols, Y, ldy, h);
    SAP_HIP_TRY(hipGetLastError());
  }
  return SAP_OK;
}

}  // namespace

size_t apply_workspace_bytes(sap_ctx *ctx, int64_t m, int d, int ncols, sap_dtype y_type) {
  const size_t es = (y_type == SAP_F64) ? 8 : 4;
  const ApplyPlan p = make_plan(ctx->num_cus, m, d, ncols, es);
  if (p.nslices <= 1) return 0;
  return static_cast<size_t>(p.nslices) * d * ncols * es;
}

sap_status launch_apply(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda,
                        sap_dtype a_type, const double *b, int n, void *Y, int64_t ldy,
                        sap_dtype y_type, void *work, hipStream_t st) {
  if (y_type == SAP_F64) {
    double *y = static_cast<double *>(Y);
    switch (a_type) {
      case SAP_F64: return apply_typed<double, double>(ctx, S, static_cast<const double *>(A), lda, b, n, y, ldy, work, st);
      case SAP_F32: return apply_typed<float, double>(ctx, S, static_cast<const float *>(A), lda, b, n, y, ldy, work, st);
      case SAP_BF16: return apply_typed<__hip_bfloat16, double>(ctx, S, static_cast<const __hip_bfloat16 *>(A), lda, b, n, y, ldy, work, st);
    }
  } else {
    float *y = static_cast<float *>(Y);
    switch (a_type) {
      case SAP_F64: return apply_typed<double, float>(ctx, S, static_cast<const double *>(A), lda, b, n, y, ldy, work, st);
      case SAP_F32: return apply_typed<float, float>(ctx, S, static_cast<const float *>(A), lda, b, n, y, ldy, work, st);
      case SAP_BF16: return apply_typed<__hip_bfloat16, float>(ctx, S, static_cast<const __hip_bfloat16 *>(A), lda, b, n, y, ldy, work, st);
    }
  }
  return fail(ctx, SAP_EINVAL, "sps_apply: unsupported dtype combination");
}

}  // namespace sap
