// Sketch apply Y = S [A b] on gfx950 (the sketching step of Alg. 1; the paper calls a
// library sparse-times-dense product, Sec. 3).
//
// Design.  Column j of S has zeta nonzeros, so row i of [A b] is added, with
// sign, into zeta rows of Y.  A is streamed from HBM once; Y (d x ncols,
// column-major) does not fit in one CU's LDS, so it is cut into column
// strips:
//   * a workgroup owns Y[r_lo : r_lo + DR, c0 : c0 + W] in LDS for its whole
//     life, W the widest power of two (<= 32) with d * W elements in 160 KB,
//     so normally DR = d and one strip pass reads each element of A once;
//   * W lanes serve one row of A: they load its W-element piece once and add
//     it into the zeta target rows with LDS atomics (ds_add), so a wave
//     instruction serves 64 / W rows; the zeta row indices are read once per
//     row (same address for the W lanes: one broadcast);
//   * the strips that share a cache line of A (consecutive strips) run on the
//     same XCD, so a line fetched from HBM for one strip serves its
//     neighbours from that XCD's L2;
//   * when strips alone do not fill the chip, the rows of A are split into
//     slices whose partial strips a second kernel sums in a fixed order;
//   * only when even W = 1 does not fit (d > 20000 in FP64) are the rows of
//     Y split into ranges, each range skipping the nonzeros outside it.
// The 1/sqrt(zeta) scale is applied once, after summation.
#include <hip/hip_bf16.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common.h"

namespace sap {
namespace {

constexpr int kApplyThreads = 1024;
constexpr int kApplyWaves = kApplyThreads / kWave;
constexpr size_t kApplyLdsBytes = 160000;  // gfx950: up to 160 KB of LDS per workgroup
constexpr int kXcds = 8;
constexpr int kUnroll = 8;                 // rows in flight per lane group
constexpr int kMaxW = 32;
constexpr int64_t kMinSliceRows = 4096;

template <typename TA, typename TY>
__device__ __forceinline__ TY load_as(const TA *p) {
  if constexpr (std::is_same<TA, __hip_bfloat16>::value)
    return static_cast<TY>(__bfloat162float(*p));
  else
    return static_cast<TY>(*p);
}

// One work item = (strip, range, slice).
// FAST (one range, zeta = 8, idx 16-byte aligned): per row two 16-byte index
// loads, every load of a batch of rows issued before any add, and no
// branches: a row past the slice end adds zeros, and an index outside [0, d)
// adds into a spare LDS row that is never written out.  Otherwise the
// general path loads the indices four at a time and skips indices outside
// the range.
// C16 (with FAST): the row indices come from a 16-bit copy (idx16, 8 per row,
// one 16-byte load), for sketches that many strips re-read: C16 = 1 keeps the
// sign word, C16 = 2 (d <= 32767) reads each sign from bit 15 of its index,
// so a row costs the strips 16 bytes of sketch instead of 24.
// The strip fills the LDS, so a CU holds one workgroup (4 waves a SIMD);
// telling the compiler so lets it keep every load of a batch in flight
// instead of trading registers for an occupancy it never gets.
template <typename TA, typename TY, int W, bool FAST, int C16>
__global__ __launch_bounds__(kApplyThreads) __attribute__((amdgpu_waves_per_eu(1, 4))) void apply_strip_kernel(
    const int32_t *__restrict__ idx, const uint16_t *__restrict__ idx16, const uint64_t *__restrict__ sign,
    int zeta, const TA *__restrict__ A,
    int64_t lda, const double *__restrict__ b, int64_t m, int n, int ncols, int d, int dr, int nstrips,
    int nranges, int nslices, int64_t rows_per_slice, TY *__restrict__ out, int64_t ldo, int64_t slice_stride,
    double h, int scale_now) {
  extern __shared__ unsigned char lds_raw[];
  TY *acc = reinterpret_cast<TY *>(lds_raw);
  constexpr int RPW = kWave / W;  // rows per wave instruction

  // XCD-aware decode: workgroup IDs are dealt round-robin over the XCDs;
  // each XCD gets a contiguous block of work items, strip fastest.
  const int total = nstrips * nranges * nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const int w = (blockIdx.x % kXcds) * per_xcd + blockIdx.x / kXcds;
  if (w >= total) return;
  const int strip = w % nstrips;
  const int range = (w / nstrips) % nranges;
  const int slice = w / (nstrips * nranges);
  const int c0 = strip * W;
  const int r_lo = range * dr;
  const int rows_here = min(dr, d - r_lo);

  for (int e = threadIdx.x; e < (rows_here + (FAST ? 1 : 0)) * W; e += kApplyThreads) acc[e] = TY(0);
  __syncthreads();

  const int64_t i_begin = static_cast<int64_t>(slice) * rows_per_slice;
  const int64_t i_end = min(m, i_begin + rows_per_slice);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int g = lane / W, c = lane % W;
  const int col = c0 + c;
  const bool col_a = col < n;
  const bool col_b = (col == n) && (col < ncols);
  constexpr int64_t kStride = static_cast<int64_t>(kApplyWaves) * RPW * kUnroll;
  for (int64_t base = i_begin + wave * (RPW * kUnroll) + g; base < i_end; base += kStride) {
    if constexpr (FAST) {
      TY val[kUnroll];
      uint32_t sg[kUnroll];
      int4 ix[kUnroll][2];
      uint4 raw[kUnroll];  // 16-bit copy: decoded after every load of the batch is issued
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t i0 = base + u * RPW;
        const bool ok = i0 < i_end;
        const int64_t i = ok ? i0 : i_end - 1;
        TY a = TY(0);
        if (col_a) a = load_as<TA, TY>(A + i * lda + col);
        else if (col_b) a = static_cast<TY>(b[i]);
        val[u] = ok ? a : TY(0);
        if constexpr (C16 != 0) {
          raw[u] = *reinterpret_cast<const uint4 *>(idx16 + i * 8);
          if constexpr (C16 == 1) sg[u] = static_cast<uint32_t>(sign[i]);
        } else {
          sg[u] = static_cast<uint32_t>(sign[i]);
          const int4 *ip = reinterpret_cast<const int4 *>(idx + i * 8);
          ix[u][0] = ip[0];
          ix[u][1] = ip[1];
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        int rr[8];
        bool pos[8];
        if constexpr (C16 != 0) {
          const uint32_t wd[4] = {raw[u].x, raw[u].y, raw[u].z, raw[u].w};
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const uint32_t half = (k & 1) ? (wd[k >> 1] >> 16) : (wd[k >> 1] & 0xFFFFu);
            if constexpr (C16 == 2) {
              rr[k] = static_cast<int>(half & 0x7FFFu);
              pos[k] = (half & 0x8000u) != 0;
            } else {
              rr[k] = static_cast<int>(half);
              pos[k] = ((sg[u] >> k) & 1u) != 0;
            }
          }
        } else {
          rr[0] = ix[u][0].x; rr[1] = ix[u][0].y; rr[2] = ix[u][0].z; rr[3] = ix[u][0].w;
          rr[4] = ix[u][1].x; rr[5] = ix[u][1].y; rr[6] = ix[u][1].z; rr[7] = ix[u][1].w;
#pragma unroll
          for (int k = 0; k < 8; ++k) pos[k] = ((sg[u] >> k) & 1u) != 0;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int r = static_cast<unsigned>(rr[k]) < static_cast<unsigned>(d) ? rr[k] : d;
          const TY v = pos[k] ? val[u] : -val[u];
          atomicAdd(acc + r * W + c, v);
        }
      }
    } else {
#pragma unroll 2
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t i = base + u * RPW;
        if (i >= i_end) break;
        TY a = TY(0);
        if (col_a) a = load_as<TA, TY>(A + i * lda + col);
        else if (col_b) a = static_cast<TY>(b[i]);
        const uint64_t sg = sign[i];
        const int32_t *ri = idx + i * zeta;
        for (int k0 = 0; k0 < zeta; k0 += 4) {
          int rr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) rr[q] = (k0 + q < zeta) ? ri[k0 + q] : -1;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = rr[q] - r_lo;
            if (rr[q] >= 0 && static_cast<unsigned>(r) < static_cast<unsigned>(rows_here)) {
              const TY v = ((sg >> (k0 + q)) & 1ull) ? a : -a;
              atomicAdd(acc + r * W + c, v);
            }
          }
        }
      }
    }
  }
  __syncthreads();

  const TY scale = scale_now ? TY(h) : TY(1);
  TY *dst = out + static_cast<int64_t>(slice) * slice_stride;
  for (int e = threadIdx.x; e < rows_here * W; e += kApplyThreads) {
    const int q = e / rows_here, r = e % rows_here;
    const int cc = c0 + q;
    if (cc < ncols) dst[(r_lo + r) + static_cast<int64_t>(cc) * ldo] = acc[r * W + q] * scale;
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

// 16-bit copy of the row indices (zeta = 8, d <= 65535); an index outside
// [0, d) becomes the largest value of its field (>= d), which the apply adds
// into its spare row.  With d <= kPackSignMaxD the index takes bits 0-14 and
// the sign of the nonzero (bit k of the row's sign word) bit 15.
constexpr int kPackSignMaxD = 32767;

__global__ __launch_bounds__(256) void idx16_kernel(const int32_t *__restrict__ idx,
                                                    const uint64_t *__restrict__ sign, int64_t count, int d,
                                                    uint16_t *__restrict__ out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  const bool pack = d <= kPackSignMaxD;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < count; e += stride) {
    const int32_t v = idx[e];
    if (pack) {
      const uint32_t s = static_cast<uint32_t>(sign[e >> 3] >> (e & 7)) & 1u;
      out[e] = static_cast<uint16_t>((v >= 0 && v < d ? v : 0x7FFF) | (s << 15));
    } else {
      out[e] = static_cast<uint16_t>(v >= 0 && v < d ? v : 65535);
    }
  }
}

// The strips re-read every row's indices and sign word (40 bytes); past this
// many bytes of such re-reads the 16-bit copy (24 bytes a row) pays for itself.
constexpr double kCompactMinRereadBytes = 16e9;

struct ApplyPlan {
  int w, dr, nstrips, nranges, nslices;
  int64_t rows_per_slice;
};

ApplyPlan make_plan(int num_cus, int64_t m, int d, int ncols, size_t esize) {
  ApplyPlan p{};
  // columns of a full-height strip (plus one spare row)
  const size_t fit = kApplyLdsBytes / (esize * (static_cast<size_t>(d) + 1));
  int w = 1;
  while (w * 2 <= kMaxW && static_cast<size_t>(w * 2) <= fit) w *= 2;
  // no wider than the matrix needs
  while (w > 1 && w / 2 >= ncols) w /= 2;
  p.w = w;
  if (fit >= 1) {
    p.nranges = 1;
    p.dr = d;
  } else {
    const int dr_max = static_cast<int>(kApplyLdsBytes / esize) - 1;  // plus the spare row
    p.nranges = (d + dr_max - 1) / dr_max;
    p.dr = (d + p.nranges - 1) / p.nranges;
  }
  p.nstrips = (ncols + w - 1) / w;
  // One resident workgroup per CU when the strip fills the LDS; split the
  // rows into slices when the strips alone leave CUs idle.
  const int items = p.nstrips * p.nranges;
  int ns = 1;
  if (items < num_cus) ns = (num_cus + items - 1) / items;
  const int64_t max_slices = std::max<int64_t>(1, m / kMinSliceRows);
  if (ns > max_slices) ns = static_cast<int>(max_slices);
  p.rows_per_slice = (m + ns - 1) / ns;
  p.nslices = static_cast<int>((m + p.rows_per_slice - 1) / p.rows_per_slice);
  if (p.nslices < 1) p.nslices = 1;
  return p;
}

bool use_compact(const ApplyPlan &p, int64_t m, int zeta, int d) {
  return zeta == 8 && p.nranges == 1 && d <= 65535 &&
         static_cast<double>(p.nstrips) * static_cast<double>(m) * 40.0 >= kCompactMinRereadBytes;
}

template <typename TA, typename TY, int W>
void launch_strip(const ApplyPlan &p, dim3 grid, size_t lds, hipStream_t st, const sps_sketch *S, const TA *A,
                  int64_t lda, const double *b, int n, int ncols, TY *out, int64_t ldo, int64_t slice_stride,
                  double h, int scale_now, const uint16_t *idx16) {
  // The 16-bit copy is read with 16-byte loads whatever S->idx's alignment
  // (the copy is 256-byte aligned); the 32-bit indices only when S->idx is.
  const bool fast = S->zeta == 8 && p.nranges == 1 && (reinterpret_cast<uintptr_t>(S->idx) % 16 == 0);
  if (S->zeta == 8 && p.nranges == 1 && idx16 != nullptr && S->d <= kPackSignMaxD)
    apply_strip_kernel<TA, TY, W, true, 2><<<grid, kApplyThreads, lds, st>>>(
        S->idx, idx16, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.nstrips, p.nranges, p.nslices,
        p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
  else if (S->zeta == 8 && p.nranges == 1 && idx16 != nullptr)
    apply_strip_kernel<TA, TY, W, true, 1><<<grid, kApplyThreads, lds, st>>>(
        S->idx, idx16, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.nstrips, p.nranges, p.nslices,
        p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
  else if (fast)
    apply_strip_kernel<TA, TY, W, true, 0><<<grid, kApplyThreads, lds, st>>>(
        S->idx, nullptr, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.nstrips, p.nranges, p.nslices,
        p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
  else
    apply_strip_kernel<TA, TY, W, false, 0><<<grid, kApplyThreads, lds, st>>>(
        S->idx, nullptr, S->sign, S->zeta, A, lda, b, S->m, n, ncols, S->d, p.dr, p.nstrips, p.nranges, p.nslices,
        p.rows_per_slice, out, ldo, slice_stride, h, scale_now);
}

template <typename TA, typename TY>
sap_status apply_typed(sap_ctx *ctx, const sps_sketch *S, const TA *A, int64_t lda, const double *b, int n, TY *Y,
                       int64_t ldy, void *work, hipStream_t st) {
  const int ncols = n + (b != nullptr ? 1 : 0);
  const ApplyPlan p = make_plan(ctx->num_cus, S->m, S->d, ncols, sizeof(TY));
  const double h = 1.0 / std::sqrt(static_cast<double>(S->zeta));
  Carve cv(work);
  TY *out = Y;
  int64_t ldo = ldy, slice_stride = 0;
  int scale_now = 1;
  if (p.nslices > 1) {
    out = cv.take<TY>(static_cast<size_t>(p.nslices) * S->d * ncols);
    ldo = S->d;
    slice_stride = static_cast<int64_t>(S->d) * ncols;
    scale_now = 0;
  }
  const uint16_t *idx16 = nullptr;
  if (use_compact(p, S->m, S->zeta, S->d)) {
    uint16_t *c = cv.take<uint16_t>(static_cast<size_t>(S->m) * 8);
    const int64_t count = S->m * 8;
    const unsigned g = static_cast<unsigned>(std::min<int64_t>((count + 255) / 256, int64_t(ctx->num_cus) * 16));
    idx16_kernel<<<g, 256, 0, st>>>(S->idx, S->sign, count, S->d, c);
    SAP_HIP_TRY(hipGetLastError());
    idx16 = c;
  }
  const int total = p.nstrips * p.nranges * p.nslices;
  const int per_xcd = (total + kXcds - 1) / kXcds;
  const dim3 grid(static_cast<unsigned>(per_xcd * kXcds));
  const size_t lds = (static_cast<size_t>(p.dr) + 1) * p.w * sizeof(TY);
  switch (p.w) {
    case 1: launch_strip<TA, TY, 1>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
    case 2: launch_strip<TA, TY, 2>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
    case 4: launch_strip<TA, TY, 4>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
    case 8: launch_strip<TA, TY, 8>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
    case 16: launch_strip<TA, TY, 16>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
    default: launch_strip<TA, TY, 32>(p, grid, lds, st, S, A, lda, b, n, ncols, out, ldo, slice_stride, h, scale_now, idx16); break;
  }
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

// Scratch of sps_apply_noalloc: a file-scope device array, one copy per GPU
// the library runs on, held until the process ends.  Host code never uses
// its name as an address (on the host it names a stand-in, not device
// memory): apply_scratch_init looks up this device's copy once and the
// context keeps that address.
static __device__ __align__(256) unsigned char g_apply_scratch[kNoAllocScratchBytes];

sap_status apply_scratch_init(sap_ctx *ctx) {
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_apply_scratch));
  if (e != hipSuccess) return hip_fail(ctx, e, "hipGetSymbolAddress(apply scratch)");
  if (p == nullptr) return fail(ctx, SAP_EDEVICE, "apply scratch: no device address");
  ctx->apply_scratch = p;
  ctx->apply_scratch_bytes = kNoAllocScratchBytes;
  return SAP_OK;
}

size_t apply_workspace_bytes(sap_ctx *ctx, int64_t m, int zeta, int d, int ncols, sap_dtype y_type) {
  const size_t es = (y_type == SAP_F64) ? 8 : 4;
  const ApplyPlan p = make_plan(ctx->num_cus, m, d, ncols, es);
  size_t bytes = 8 * 256;
  if (p.nslices > 1) bytes += static_cast<size_t>(p.nslices) * d * ncols * es;
  if (use_compact(p, m, zeta, d)) bytes += static_cast<size_t>(m) * 8 * sizeof(uint16_t) + 256;
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
