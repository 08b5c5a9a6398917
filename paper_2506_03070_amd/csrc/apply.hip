// Sketch apply Y = S [A b] on gfx950 (Alg. 1 "form Y = SA"; the paper calls a
// library sparse-times-dense product, Sec. 3).
//
// Design.  A is streamed from HBM once; every nonzero (i, k) of S adds
// +-A[i, :] into row idx[i][k] of Y.  Y (d x ncols, column-major) is far
// larger than one CU's LDS, so each workgroup owns a tile
// Y[r_lo : r_lo + DR, c0 : c0 + 16] in LDS for its whole life:
//   * 16 columns = one 128-byte piece of a row of A, so the 16 lanes that
//     serve one nonzero read one line and add into 16 consecutive LDS
//     doubles; a wave instruction serves 4 nonzeros and touches every bank
//     equally (no serialisation beyond the minimum for 512 bytes);
//   * the rows of Y are split into ranges of DR <= 1250 (FP64) rows so the
//     tile fits in 160 KB of LDS; a counting-sort pre-pass buckets the
//     nonzeros by range (kept in ascending-i order within each chunk), so a
//     workgroup walks only its own nonzeros;
//   * the workgroups of one column tile (all ranges) sit on the same XCD, so
//     the pieces of A that several ranges need come from that XCD's L2 after
//     the first touch;
//   * when there are too few tiles to fill the chip the nonzeros of a range
//     are split into slices whose partial tiles a second kernel sums in a
//     fixed order.
// The 1/sqrt(zeta) scale is applied once, after summation.
#include <hip/hip_bf16.h>

#include <cmath>
#include <type_traits>

#include "common.h"

namespace sap {
namespace {

constexpr int kApplyThreads = 1024;
constexpr int kApplyWaves = kApplyThreads / kWave;
constexpr int kTileCols = 16;                // columns per tile: one 128-byte row piece
constexpr int kGroups = kWave / kTileCols;   // nonzeros per wave instruction
constexpr int kUnroll = 8;                   // nonzeros in flight per lane
constexpr size_t kApplyLdsBytes = 160000;    // gfx950: up to 160 KB of LDS per workgroup
constexpr int kXcds = 8;
constexpr int kChunkRows = 8192;             // rows of A per bucketing chunk
constexpr int kMaxRanges = 64;

template <typename TA, typename TY>
__device__ __forceinline__ TY load_as(const TA *p) {
  if constexpr (std::is_same<TA, __hip_bfloat16>::value)
    return static_cast<TY>(__bfloat162float(*p));
  else
    return static_cast<TY>(*p);
}

// ---- bucketing of the nonzeros by row range of Y (counting sort) ----------
__global__ __launch_bounds__(256) void bucket_count_kernel(const int32_t *__restrict__ idx, int64_t m, int zeta,
                                                           int d, int dr, int nranges, int *__restrict__ counts) {
  __shared__ int hist[kMaxRanges];
  for (int k = threadIdx.x; k < nranges; k += 256) hist[k] = 0;
  __syncthreads();
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kChunkRows * zeta;
  const int64_t e1 = min(m * zeta, e0 + static_cast<int64_t>(kChunkRows) * zeta);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int r = idx[e];
    if (static_cast<unsigned>(r) < static_cast<unsigned>(d)) atomicAdd(&hist[r / dr], 1);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nranges; k += 256) counts[static_cast<int64_t>(blockIdx.x) * nranges + k] = hist[k];
}

// Exclusive offsets: range-major, chunk-minor.  start[range] = first entry
// of the range; offs[chunk][range] = first slot of that chunk's entries.
__global__ void bucket_scan_kernel(const int *__restrict__ counts, int nchunks, int nranges, int64_t *__restrict__ offs,
                                   int64_t *__restrict__ start) {
  if (threadIdx.x != 0) return;
  int64_t pos = 0;
  for (int r = 0; r < nranges; ++r) {
    start[r] = pos;
    for (int c = 0; c < nchunks; ++c) {
      offs[static_cast<int64_t>(c) * nranges + r] = pos;
      pos += counts[static_cast<int64_t>(c) * nranges + r];
    }
  }
  start[nranges] = pos;
}

// Entries are (row i, local row | sign << 31).  Within a chunk the slots of a
// range are claimed through LDS counters, so chunks are in ascending order of
// i but the order inside a (chunk, range) run is unspecified (the apply adds
// with LDS atomics, whose order is unspecified anyway).  Row indices outside
// [0, d) are ignored here and in the count.
__global__ __launch_bounds__(256) void bucket_scatter_kernel(const int32_t *__restrict__ idx,
                                                             const uint64_t *__restrict__ sign, int64_t m, int zeta,
                                                             int d, int dr, int nranges,
                                                             const int64_t *__restrict__ offs,
                                                             uint2 *__restrict__ list) {
  __shared__ unsigned long long cursor[kMaxRanges];
  for (int k = threadIdx.x; k < nranges; k += 256) cursor[k] = offs[static_cast<int64_t>(blockIdx.x) * nranges + k];
  __syncthreads();
  const int64_t e0 = static_cast<int64_t>(blockIdx.x) * kChunkRows * zeta;
  const int64_t e1 = min(m * zeta, e0 + static_cast<int64_t>(kChunkRows) * zeta);
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) {
    const int r = idx[e];
    if (static_cast<unsigned>(r) >= static_cast<unsigned>(d)) continue;
    const int rg = r / dr;
    const int64_t i = e / zeta;
    const int k = static_cast<int>(e - i * zeta);
    const unsigned s = static_cast<unsigned>((sign[i] >> k) & 1ull);
    const unsigned long long pos = atomicAdd(&cursor[rg], 1ull);
    list[pos] = make_uint2(static_cast<unsigned>(i), static_cast<unsigned>(r - rg * dr) | (s << 31));
  }
}

// ---- main kernel ---------------------------------------------------------
// One work item = (column tile, row range of Y, slice of that range's
// nonzeros).  BUCKETED: nonzeros come from the bucket list; otherwise (a
// single range) straight from idx/sign in order.
template <typename TA, typename TY, bool BUCKETED>
__global__ __launch_bounds__(kApplyThreads) void apply_tile_kernel(
    const int32_t *__restrict__ idx, const uint64_t *__restrict__ sign, int zeta, const uint2 *__restrict__ list,
    const int64_t *__restrict__ start, const TA *__restrict__ A, int64_t lda, const double *__restrict__ b,
    int64_t m, int n, int ncols, int d, int dr, int ntiles, int nranges, int nslices, TY *__restrict__ out,
    int64_t ldo, int64_t slice_stride, double h, int scale_now) {
  extern __shared__ unsigned char lds_raw[];
  TY *acc = reinterpret_cast<TY *>(lds_raw);

  // XCD-aware decode: workgroup IDs are dealt round-robin over the 8 XCDs;
  // give each XCD a contiguous block of work items (range fastest, then
  // tile, then slice) so that the ranges of a tile share an L2.
  const int total = ntiles * nranges * nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int w = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (w >= total) return;
  const int range = w % nranges;
  const int tile = (w / nranges) % ntiles;
  const int slice = w / (nranges * ntiles);
  const int c0 = tile * kTileCols;
  const int r_lo = range * dr;
  const int rows_here = min(dr, d - r_lo);

  for (int e = threadIdx.x; e < rows_here * kTileCols; e += kApplyThreads) acc[e] = TY(0);
  __syncthreads();

  int64_t e_begin, e_end;
  if constexpr (BUCKETED) {
    e_begin = start[range];
    e_end = start[range + 1];
  } else {
    e_begin = 0;
    e_end = m * zeta;
  }
  const int64_t cnt = e_end - e_begin;
  const int64_t per_slice = (cnt + nslices - 1) / nslices;
  const int64_t s_begin = e_begin + min(cnt, per_slice * slice);
  const int64_t s_end = e_begin + min(cnt, per_slice * (slice + 1));

  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / kTileCols, c = lane % kTileCols;
  const int col = c0 + c;
  const bool col_a = col < n;
  const bool col_b = (col == n) && (col < ncols);
  constexpr int kStride = kApplyWaves * kGroups * kUnroll;  // nonzeros per workgroup round
  for (int64_t base = s_begin + wave * (kGroups * kUnroll); base < s_end; base += kStride) {
    TY val[kUnroll];
    int rloc[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t e = base + u * kGroups + g;
      rloc[u] = -1;
      val[u] = TY(0);
      if (e < s_end) {
        int64_t i;
        int r;
        bool plus;
        if constexpr (BUCKETED) {
          const uint2 en = list[e];
          i = en.x;
          r = static_cast<int>(en.y & 0x7fffffffu);
          plus = (en.y >> 31) != 0;
        } else {
          i = e / zeta;
          const int k = static_cast<int>(e - i * zeta);
          r = idx[e];
          plus = ((sign[i] >> k) & 1ull) != 0;
        }
        TY a = TY(0);
        if (col_a) a = load_as<TA, TY>(A + i * lda + col);
        else if (col_b) a = static_cast<TY>(b[i]);
        val[u] = plus ? a : -a;
        rloc[u] = static_cast<unsigned>(r) < static_cast<unsigned>(rows_here) ? r : -1;
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (rloc[u] >= 0) atomicAdd(acc + rloc[u] * kTileCols + c, val[u]);
  }
  __syncthreads();

  const TY scale = scale_now ? TY(h) : TY(1);
  TY *dst = out + static_cast<int64_t>(slice) * slice_stride;
  for (int e = threadIdx.x; e < rows_here * kTileCols; e += kApplyThreads) {
    const int q = e / rows_here, r = e % rows_here;
    const int cc = c0 + q;
    if (cc < ncols) dst[(r_lo + r) + static_cast<int64_t>(cc) * ldo] = acc[r * kTileCols + q] * scale;
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
  int dr, ntiles, nranges, nslices, nchunks;
  bool bucketed;
};

ApplyPlan make_plan(int num_cus, int64_t m, int zeta, int d, int ncols, size_t esize) {
  ApplyPlan p{};
  const int dr_max = static_cast<int>(kApplyLdsBytes / (esize * kTileCols));
  p.nranges = (d + dr_max - 1) / dr_max;
  p.dr = (d + p.nranges - 1) / p.nranges;
  p.ntiles = (ncols + kTileCols - 1) / kTileCols;
  p.bucketed = p.nranges > 1;
  p.nchunks = static_cast<int>((m + kChunkRows - 1) / kChunkRows);
  const int items = p.ntiles * p.nranges;
  // One resident workgroup per CU (the tile fills most of the LDS).  Split
  // the nonzeros of a range into slices only when there are too few items
  // to fill the chip, keeping at least 64K nonzeros per slice.
  int ns = 1;
  if (items < num_cus) ns = (num_cus + items - 1) / items;
  const int64_t nnz_per_range = m * zeta / p.nranges;
  const int64_t max_slices = (nnz_per_range + 65535) / 65536;
  if (ns > max_slices) ns = static_cast<int>(max_slices < 1 ? 1 : max_slices);
  p.nslices = ns;
  return p;
}

size_t bucket_bytes(const ApplyPlan &p, int64_t m, int zeta) {
  if (!p.bucketed) return 0;
  return 4 * 256 + sizeof(uint2) * static_cast<size_t>(m) * zeta +
         (sizeof(int) + sizeof(int64_t)) * static_cast<size_t>(p.nchunks) * p.nranges +
         sizeof(int64_t) * (p.nranges + 1);
}

template <typename TA, typename TY>
sap_status apply_typed(sap_ctx *ctx, const sps_sketch *S, const TA *A, int64_t lda, const double *b, int n, TY *Y,
                       int64_t ldy, void *work, hipStream_t st) {
  const int ncols = n + (b != nullptr ? 1 : 0);
  const ApplyPlan p = make_plan(ctx->num_cus, S->m, S->zeta, S->d, ncols, sizeof(TY));
  if (p.nranges > kMaxRanges) return fail(ctx, SAP_EINVAL, "sps_apply: d too large");
  if (p.bucketed && S->m > static_cast<int64_t>(UINT32_MAX)) return fail(ctx, SAP_EINVAL, "sps_apply: m >= 2^32");
  const double h = 1.0 / std::sqrt(static_cast<double>(S->zeta));
  Carve cv(work);
  uint2 *list = nullptr;
  int64_t *start = nullptr;
  if (p.bucketed) {
    list = cv.take<uint2>(static_cast<size_t>(S->m) * S->zeta);
    int *counts = cv.take<int>(static_cast<size_t>(p.nchunks) * p.nranges);
    int64_t *offs = cv.take<int64_t>(static_cast<size_t>(p.nchunks) * p.nranges);
    start = cv.take<int64_t>(p.nranges + 1);
    bucket_count_kernel<<<p.nchunks, 256, 0, st>>>(S->idx, S->m, S->zeta, S->d, p.dr, p.nranges, counts);
    bucket_scan_kernel<<<1, 64, 0, st>>>(counts, p.nchunks, p.nranges, offs, start);
    bucket_scatter_kernel<<<p.nchunks, 256, 0, st>>>(S->idx, S->sign, S->m, S->zeta, S->d, p.dr, p.nranges, offs,
                                                      list);
    SAP_HIP_TRY(hipGetLastError());
  }
  TY *out = Y;
  int64_t ldo = ldy, slice_stride = 0;
  int scale_now = 1;
  if (p.nslices > 1) {
    out = cv.take<TY>(static_cast<size_t>(p.nslices) * S->d * ncols);
    ldo = S->d;
    slice_stride = static_cast<int64_t>(S->d) * ncols;
    scale_now = 0;
  }
  const int total = p.ntiles * p.nranges * p.nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const dim3 grid(static_cast<unsigned>(per_xcd * kXcds));
  const size_t lds = static_cast<size_t>(p.dr) * kTileCols * sizeof(TY);
  if (p.bucketed)
    apply_tile_kernel<TA, TY, true><<<grid, kApplyThreads, lds, st>>>(
        S->idx, S->sign, S->zeta, list, start, A, lda, b, S->m, n, ncols, S->d, p.dr, p.ntiles, p.nranges,
        p.nslices, out, ldo, slice_stride, h, scale_now);
  else
    apply_tile_kernel<TA, TY, false><<<grid, kApplyThreads, lds, st>>>(
        S->idx, S->sign, S->zeta, list, start, A, lda, b, S->m, n, ncols, S->d, p.dr, p.ntiles, p.nranges,
        p.nslices, out, ldo, slice_stride, h, scale_now);
  SAP_HIP_TRY(hipGetLastError());
  if (p.nslices > 1) {
    const int64_t tot = static_cast<int64_t>(S->d) * ncols;
    apply_reduce_kernel<TY><<<static_cast<unsigned>((tot + 255) / 256), 256, 0, st>>>(out, p.nslices, slice_stride,
                                                                                      S->d, ncols, Y, ldy, h);
    SAP_HIP_TRY(hipGetLastError());
  }
  return SAP_OK;
}

}  // namespace

size_t apply_workspace_bytes(sap_ctx *ctx, int64_t m, int zeta, int d, int ncols, sap_dtype y_type) {
  const size_t es = (y_type == SAP_F64) ? 8 : 4;
  const ApplyPlan p = make_plan(ctx->num_cus, m, zeta, d, ncols, es);
  size_t bytes = 8 * 256 + bucket_bytes(p, m, zeta);
  if (p.nslices > 1) bytes += static_cast<size_t>(p.nslices) * d * ncols * es;
  return bytes;
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
