// Sparse A in CSR form (Sec. 3 applies the sketch to sparse matrices, whose
// apply costs far less than a dense one; Table 1 holds sparse problems).
//
//   sketch apply : Y = S [A b] by columns.  The CSR matrix is first turned
//                  into CSC (per-workgroup column counts, a column-wise
//                  prefix over the workgroups, a scan that also plans the
//                  work items, then a scatter through LDS cursors), so that
//                  column j of Y, S A[:, j], is the sum over the column's
//                  entries (i, a) of a s_i.  A work item holds one column of
//                  Y (d doubles) in LDS and adds the zeta signed copies of
//                  each entry of a chunk of the column into it; a column of
//                  one chunk is written to Y directly, longer ones through
//                  partial columns summed in a fixed order.  The cost is
//                  O(zeta nnz + zeta m) adds (b is column n, a dense one),
//                  and nothing waits on the host.
//   LSQR pass    : the fused u <- c_ap (A p) + c_u u, q += u_i A[i, :] of the
//                  dense pass on the stored entries: L lanes share a row (L
//                  the power of two nearest the mean row length, at most 64),
//                  p and the workgroup's partial q sit in LDS, and every
//                  stored entry adds u_i a into q with one LDS add.
//
// The apply kernels stay in bounds for any CSR arrays (entry ranges are
// clamped to [0, nnz), rows and columns range-checked); a separate check
// raises a flag that the caller reads, so that garbage in gives an error,
// never a fault.  The LSQR pass relies on that check having passed.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace sap {
namespace {

constexpr int kCscThreads = 256;
constexpr int kCscGridMax = 1024;       // workgroups of the count and scatter passes
constexpr int kApplyColThreads = 1024;
constexpr int kApplyPer = 8;            // entries of a work item per thread (two rounds of four)
constexpr int kScatWin = 1024;         // rows of a scatter window
constexpr int64_t kApplyChunk = static_cast<int64_t>(kApplyColThreads) * kApplyPer;
constexpr int kPassThreadsS = 1024;

int csc_grid(int64_t m) { return static_cast<int>(std::clamp<int64_t>((m + 1023) / 1024, 1, kCscGridMax)); }

int64_t apply_items_max(const SparseA &A) { return A.nnz / kApplyChunk + A.n + A.m / kApplyChunk + 2; }

template <typename TV>
__device__ __forceinline__ double as_f64(TV v) { return static_cast<double>(v); }

__device__ __forceinline__ int64_t clamp_e(int64_t v, int64_t nnz) { return v < 0 ? 0 : (v > nnz ? nnz : v); }

// ---- argument check --------------------------------------------------------
// *bad = 1 unless indptr[0] = 0, indptr[m] = nnz, indptr is non-decreasing and
// every column index lies in [0, n).
__global__ __launch_bounds__(256) void csr_check_kernel(const int64_t *__restrict__ indptr,
                                                        const int32_t *__restrict__ indices, int64_t m, int n,
                                                        int64_t nnz, int *__restrict__ bad) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
  int f = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < m; i += stride)
    f |= indptr[i] > indptr[i + 1];
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; e < nnz; e += stride)
    f |= static_cast<unsigned>(indices[e]) >= static_cast<unsigned>(n);
  if (blockIdx.x == 0 && threadIdx.x == 0) f |= (indptr[0] != 0) | (indptr[m] != nnz);
  if (f) atomicOr(bad, 1);
}

__global__ void clear_int_kernel(int *p) { *p = 0; }

// ---- CSR -> CSC ------------------------------------------------------------
// Workgroup w takes rows [w R, (w+1) R) and counts its entries per column into
// cnt[w n + c].
__global__ __launch_bounds__(kCscThreads) void csc_count_kernel(const int64_t *__restrict__ indptr,
                                                                const int32_t *__restrict__ indices, int64_t m, int n,
                                                                int64_t nnz, int64_t rows_per_wg,
                                                                int *__restrict__ cnt) {
  extern __shared__ int lcnt[];
  for (int c = threadIdx.x; c < n; c += kCscThreads) lcnt[c] = 0;
  __syncthreads();
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg, r1 = min(m, r0 + rows_per_wg);
  if (r0 < r1) {
    const int64_t e0 = clamp_e(indptr[r0], nnz), e1 = clamp_e(indptr[r1], nnz);
    for (int64_t e = e0 + threadIdx.x; e < e1; e += kCscThreads) {
      const int c = indices[e];
      if (static_cast<unsigned>(c) < static_cast<unsigned>(n)) atomicAdd(lcnt + c, 1);
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < n; c += kCscThreads) cnt[static_cast<int64_t>(blockIdx.x) * n + c] = lcnt[c];
}

// Per column: exclusive prefix of the G workgroup counts, in place, and the
// column total.  A workgroup takes 64 columns (one a lane); its 16 waves take
// consecutive ranges of workgroups.
__global__ __launch_bounds__(1024) void csc_colprefix_kernel(int *__restrict__ cnt, int G, int n,
                                                             int64_t *__restrict__ tot) {
  __shared__ int64_t ws[16][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + lane;
  const int per = (G + 15) / 16;
  const int w0 = min(G, wv * per), w1 = min(G, w0 + per);
  int64_t s = 0;
  if (c < n)
    for (int w = w0; w < w1; ++w) s += cnt[static_cast<int64_t>(w) * n + c];
  ws[wv][lane] = s;
  __syncthreads();
  int64_t run = 0, total = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < wv) run += ws[k][lane];
    total += ws[k][lane];
  }
  if (c < n) {
    for (int w = w0; w < w1; ++w) {
      const int64_t at = static_cast<int64_t>(w) * n + c;
      const int v = cnt[at];
      cnt[at] = static_cast<int>(run);
      run += v;
    }
    if (wv == 0) tot[c] = total;
  }
}

__device__ __forceinline__ int64_t items_of(int64_t len) {
  return len <= 0 ? 1 : (len + kApplyChunk - 1) / kApplyChunk;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const T y = __shfl_up(v, off, 64);
    if (lane >= off) v += y;
  }
  return v;
}

// One workgroup: colptr = exclusive scan of the column totals, and the work
// plan: column c (c = n is b, of m entries) gets max(1, ceil(len / chunk))
// items, itemptr = exclusive scan of those counts.
__global__ __launch_bounds__(1024) void csc_scan_kernel(const int64_t *__restrict__ tot, int n, int64_t m,
                                                        int ncols, int64_t *__restrict__ colptr,
                                                        int64_t *__restrict__ itemptr) {
  __shared__ int64_t wa[16], wb[16];
  const int t = threadIdx.x, w = t >> 6;
  const int q = (ncols + 1023) / 1024;
  const int lo = min(ncols, t * q), hi = min(ncols, lo + q);
  int64_t oa = 0, ob = 0;
  for (int c = lo; c < hi; ++c) {
    const int64_t len = c < n ? tot[c] : m;
    if (c < n) oa += len;
    ob += items_of(len);
  }
  const int64_t ia = wave_incl_scan(oa), ib = wave_incl_scan(ob);
  if ((t & 63) == 63) {
    wa[w] = ia;
    wb[w] = ib;
  }
  __syncthreads();
  int64_t ra = ia - oa, rb = ib - ob, ta = 0, tb = 0;
  for (int k = 0; k < 16; ++k) {
    if (k < w) {
      ra += wa[k];
      rb += wb[k];
    }
    ta += wa[k];
    tb += wb[k];
  }
  for (int c = lo; c < hi; ++c) {
    const int64_t len = c < n ? tot[c] : m;
    if (c < n) {
      colptr[c] = ra;
      ra += len;
    }
    itemptr[c] = rb;
    rb += items_of(len);
  }
  if (t == 0) {
    colptr[n] = ta;
    itemptr[ncols] = tb;
  }
}

// items[itemptr[c] + k] = (c, k) for the items k of column c.
__global__ __launch_bounds__(256) void csc_items_kernel(const int64_t *__restrict__ itemptr, int ncols,
                                                        int64_t items_max, int2 *__restrict__ items) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= ncols) return;
  const int64_t w0 = itemptr[c], w1 = min(itemptr[c + 1], items_max);
  for (int64_t w = w0; w < w1; ++w) items[w] = make_int2(c, static_cast<int>(w - w0));
}

// Scatter: workgroup w places its entries at colptr[c] + its prefix in column
// c, through LDS cursors.  Its rows are taken in windows of kScatWin: the
// window's row starts go to LDS, a thread takes an entry and finds its row by
// binary search there.
template <typename TV>
__global__ __launch_bounds__(kCscThreads) void csc_scatter_kernel(const int64_t *__restrict__ indptr,
                                                                  const int32_t *__restrict__ indices,
                                                                  const TV *__restrict__ values, int64_t m, int n,
                                                                  int64_t nnz, int64_t rows_per_wg,
                                                                  const int *__restrict__ pre,
                                                                  const int64_t *__restrict__ colptr,
                                                                  int32_t *__restrict__ crow, TV *__restrict__ cval) {
  extern __shared__ int lcur[];
  __shared__ int64_t rs[kScatWin + 1];
  for (int c = threadIdx.x; c < n; c += kCscThreads) lcur[c] = pre[static_cast<int64_t>(blockIdx.x) * n + c];
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg, r1 = min(m, r0 + rows_per_wg);
  for (int64_t wr = r0; wr < r1; wr += kScatWin) {
    const int nr = static_cast<int>(min<int64_t>(kScatWin, r1 - wr));
    __syncthreads();  // cursors set; the previous window's searches done
    for (int t = threadIdx.x; t <= nr; t += kCscThreads) rs[t] = clamp_e(indptr[wr + t], nnz);
    __syncthreads();
    const int64_t E0 = rs[0], E1 = max(rs[0], rs[nr]);
    for (int64_t e = E0 + threadIdx.x; e < E1; e += kCscThreads) {
      int lo = 0, hi = nr;  // rs[lo] <= e < rs[hi] when the starts do not decrease
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rs[mid] <= e) lo = mid;
        else hi = mid;
      }
      const int c = indices[e];
      if (static_cast<unsigned>(c) >= static_cast<unsigned>(n)) continue;
      const int64_t pos = colptr[c] + atomicAdd(lcur + c, 1);
      if (pos < colptr[c + 1] && pos < nnz) {
        crow[pos] = static_cast<int32_t>(wr + lo);
        cval[pos] = values[e];
      }
    }
  }
}

// ---- apply by columns ------------------------------------------------------
// Work item w = (j, k): the k-th of the K near-equal parts of column j's
// entries (j = n: b, a dense column of m entries), K = max(1, ceil(len / C)).
// acc holds the column of Y plus one sink slot (index d) that takes the adds
// of padding lanes and out-of-range rows.  Z in {8, 12, 16, 24} loads a row's
// Z sketch rows as Z/4 16-byte words, R rows of A a round; Z = 0 takes any
// zeta.
template <int Z>
constexpr int apply_round() { return Z == 0 ? 4 : (Z <= 8 ? 4 : (Z <= 16 ? 2 : 1)); }

template <typename TV, int Z>
__global__ __launch_bounds__(kApplyColThreads) __attribute__((amdgpu_waves_per_eu(8)))  // two workgroups a CU
void csc_apply_kernel(
    const int64_t *__restrict__ itemptr, const int2 *__restrict__ items, const int64_t *__restrict__ colptr,
    const int32_t *__restrict__ crow, const TV *__restrict__ cval, const double *__restrict__ b, int64_t m, int n,
    int ncols, int64_t nnz, int d, int zeta, const int32_t *__restrict__ idx, const uint64_t *__restrict__ sign,
    double *__restrict__ part, double *__restrict__ Y, int64_t ldy, double h) {
  extern __shared__ double acc[];
  const int64_t w = blockIdx.x;
  if (w >= itemptr[ncols]) return;
  const int2 it = items[w];
  const int j = it.x;
  const int64_t K = itemptr[j + 1] - itemptr[j];
  for (int r = threadIdx.x; r <= d; r += kApplyColThreads) acc[r] = 0.0;
  __syncthreads();
  const int64_t base = (j < n) ? colptr[j] : 0;
  const int64_t end = (j < n) ? max(base, min(colptr[j + 1], nnz)) : m;
  const int64_t len = end - base;
  const int64_t e0 = base + len * it.y / K, e1 = base + len * (it.y + 1) / K;
  constexpr int kApplyRound = apply_round<Z>();
#pragma unroll 1
  for (int rd = 0; rd < kApplyPer / kApplyRound; ++rd) {
    int row[kApplyRound];  // m < 2^31
    double a[kApplyRound];
#pragma unroll
    for (int u = 0; u < kApplyRound; ++u) {
      const int64_t e = e0 + threadIdx.x + static_cast<int64_t>(rd * kApplyRound + u) * kApplyColThreads;
      int64_t i = -1;
      double v = 0.0;
      if (e < e1) {
        if (j < n) {
          i = crow[e];
          v = as_f64(cval[e]);
        } else {
          i = e;
          v = b[e];
        }
      }
      row[u] = (i >= 0 && i < m) ? static_cast<int>(i) : -1;
      a[u] = v;
    }
    if constexpr (Z > 0) {
      int4 ix[kApplyRound][Z / 4];
      uint32_t sg[kApplyRound];  // Z <= 32: the low word holds every sign
#pragma unroll
      for (int u = 0; u < kApplyRound; ++u) {
        const int64_t i = row[u] >= 0 ? row[u] : 0;
        const int4 *ip = reinterpret_cast<const int4 *>(idx + i * Z);  // 16-byte aligned: checked by the caller
#pragma unroll
        for (int q4 = 0; q4 < Z / 4; ++q4) ix[u][q4] = ip[q4];
        sg[u] = static_cast<uint32_t>(sign[i]);
      }
#pragma unroll
      for (int u = 0; u < kApplyRound; ++u) {
#pragma unroll
        for (int q4 = 0; q4 < Z / 4; ++q4) {
          const int rr[4] = {ix[u][q4].x, ix[u][q4].y, ix[u][q4].z, ix[u][q4].w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = (row[u] >= 0 && static_cast<unsigned>(rr[q]) < static_cast<unsigned>(d)) ? rr[q] : d;
            atomicAdd(acc + r, ((sg[u] >> (4 * q4 + q)) & 1u) ? a[u] : -a[u]);
          }
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < kApplyRound; ++u) {
        const int64_t i = row[u] >= 0 ? row[u] : 0;
        const uint64_t sg = sign[i];
        const int32_t *ri = idx + i * zeta;
        for (int k0 = 0; k0 < zeta; k0 += 4) {
          int rr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) rr[q] = ri[min(k0 + q, zeta - 1)];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const bool take =
                row[u] >= 0 && k0 + q < zeta && static_cast<unsigned>(rr[q]) < static_cast<unsigned>(d);
            atomicAdd(acc + (take ? rr[q] : d), ((sg >> (k0 + q)) & 1ull) ? a[u] : -a[u]);
          }
        }
      }
    }
  }
  __syncthreads();
  if (K == 1) {
    double *dst = Y + static_cast<int64_t>(j) * ldy;
    for (int r = threadIdx.x; r < d; r += kApplyColThreads) dst[r] = acc[r] * h;
  } else {
    double *dst = part + w * d;
    for (int r = threadIdx.x; r < d; r += kApplyColThreads) dst[r] = acc[r];
  }
}

// Y[r, j] = h * sum of the partial columns of j, in item order, for the
// columns of more than one item (grid: (ceil(d / 256), ncols)).
__global__ __launch_bounds__(256) void csc_reduce_kernel(const double *__restrict__ part,
                                                         const int64_t *__restrict__ itemptr, int d,
                                                         int64_t items_max, double *__restrict__ Y, int64_t ldy,
                                                         double h) {
  const int j = blockIdx.y;
  const int64_t w0 = itemptr[j], w1 = min(itemptr[j + 1], items_max);
  if (w1 - w0 <= 1) return;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= d) return;
  double s = 0.0;
  int64_t w = w0;
  for (; w + 8 <= w1; w += 8) {  // eight loads in flight, added in item order
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[(w + q) * d + r];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; w < w1; ++w) s += part[w * d + r];
  Y[r + static_cast<int64_t>(j) * ldy] = s * h;
}

// ---- fused LSQR pass -------------------------------------------------------
template <typename TV>
__global__ __launch_bounds__(kPassThreadsS) void csr_pass_kernel(
    const int64_t *__restrict__ indptr, const int32_t *__restrict__ indices, const TV *__restrict__ values,
    int64_t m, int n, int L, int64_t rows_per_wg, const double *__restrict__ p, const double *__restrict__ u_in,
    double *__restrict__ u_out, const LsqrState *__restrict__ st, double *__restrict__ qpart,
    double *__restrict__ nrmpart) {
  extern __shared__ double sh[];
  __shared__ double nsh[kPassThreadsS / kWave];
  if (st->done) return;
  double *ps = sh, *qs = sh + n;
  const double c_ap = st->c_ap, c_u = st->c_u;
  for (int c = threadIdx.x; c < n; c += kPassThreadsS) {
    ps[c] = p[c];
    qs[c] = 0.0;
  }
  __syncthreads();
  const int g = threadIdx.x / L, sub = threadIdx.x % L, groups = kPassThreadsS / L;
  const int64_t r0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg, r1 = min(m, r0 + rows_per_wg);
  double nrm = 0.0;
  // every lane runs the same number of row steps, so that the L lanes of a
  // row reduce together; a row's first L entries stay in registers between
  // the product and the q update
  const int64_t steps = (r1 - r0 + groups - 1) / groups;
  for (int64_t t = 0; t < steps; ++t) {
    const int64_t i = r0 + t * groups + g;
    const bool rv = i < r1;
    const int64_t e0 = rv ? indptr[i] : 0, e1 = rv ? indptr[i + 1] : 0;
    const int64_t ef = e0 + sub;
    const bool h0 = ef < e1;
    const double a0 = h0 ? as_f64(values[ef]) : 0.0;
    const int c0 = h0 ? indices[ef] : 0;
    double s = a0 * ps[c0];
    for (int64_t e = ef + L; e < e1; e += L) s += as_f64(values[e]) * ps[indices[e]];
    for (int off = L >> 1; off >= 1; off >>= 1) s += __shfl_xor(s, off, kWave);
    if (rv) {
      const double uh = c_ap * s + c_u * u_in[i];
      if (sub == 0) {
        u_out[i] = uh;
        nrm += uh * uh;
      }
      if (h0) atomicAdd(qs + c0, uh * a0);
      for (int64_t e = ef + L; e < e1; e += L) atomicAdd(qs + indices[e], uh * as_f64(values[e]));
    }
  }
  nrm = wave_sum(nrm);
  if ((threadIdx.x & (kWave - 1)) == 0) nsh[threadIdx.x / kWave] = nrm;
  __syncthreads();
  double *qd = qpart + static_cast<int64_t>(blockIdx.x) * n;
  for (int c = threadIdx.x; c < n; c += kPassThreadsS) qd[c] = qs[c];
  if (threadIdx.x == 0) {
    double sum = 0.0;
    for (int w = 0; w < kPassThreadsS / kWave; ++w) sum += nsh[w];
    nrmpart[blockIdx.x] = sum;
  }
}

size_t vsize(sap_dtype t) { return t == SAP_F32 ? 4 : 8; }

}  // namespace

// ---------------------------------------------------------------------------
size_t csr_apply_workspace_bytes(const SparseA &A, int d) {
  const int n = A.n, ncols = n + 1;
  const int64_t items_max = apply_items_max(A);
  size_t b = 16 * 256;
  b += static_cast<size_t>(csc_grid(A.m)) * n * sizeof(int);
  b += static_cast<size_t>(n) * sizeof(int64_t) + static_cast<size_t>(n + 1) * sizeof(int64_t);
  b += static_cast<size_t>(A.nnz) * (sizeof(int32_t) + vsize(A.v_type));
  b += static_cast<size_t>(ncols + 1) * sizeof(int64_t);
  b += static_cast<size_t>(items_max) * sizeof(int2);
  b += static_cast<size_t>(items_max) * d * sizeof(double);
  return b;
}

sap_status launch_csr_apply(sap_ctx *ctx, const sps_sketch *S, const SparseA &A, const double *b, double *Y,
                            int64_t ldy, int *bad, void *work, hipStream_t st) {
  const int n = A.n, d = S->d, zeta = S->zeta;
  const int64_t m = A.m;
  if (static_cast<size_t>(d + 1) * sizeof(double) > 160000)
    return fail(ctx, SAP_EINVAL, "sparse apply: d >= 20000 is not supported");
  if (static_cast<size_t>(n) * sizeof(int) > 64 * 1024) return fail(ctx, SAP_EINVAL, "sparse apply: n too large");
  const int64_t items_max = apply_items_max(A);
  if (items_max >= (int64_t(1) << 31)) return fail(ctx, SAP_EINVAL, "sparse apply: too many work items");
  const int ncols = n + (b ? 1 : 0);
  const int G = csc_grid(m);
  const int64_t rpw = (m + G - 1) / G;
  Carve cv(work);
  int *cnt = cv.take<int>(static_cast<size_t>(G) * n);
  int64_t *tot = cv.take<int64_t>(n);
  int64_t *colptr = cv.take<int64_t>(n + 1);
  int32_t *crow = cv.take<int32_t>(A.nnz);
  void *cval = cv.take<char>(A.nnz * vsize(A.v_type));
  int64_t *itemptr = cv.take<int64_t>(n + 2);
  int2 *items = cv.take<int2>(items_max);
  double *part = cv.take<double>(static_cast<size_t>(items_max) * d);
  const size_t lds_n = static_cast<size_t>(n) * sizeof(int);
  clear_int_kernel<<<1, 1, 0, st>>>(bad);
  csr_check_kernel<<<1024, 256, 0, st>>>(A.indptr, A.indices, m, n, A.nnz, bad);
  csc_count_kernel<<<G, kCscThreads, lds_n, st>>>(A.indptr, A.indices, m, n, A.nnz, rpw, cnt);
  csc_colprefix_kernel<<<(n + 63) / 64, 1024, 0, st>>>(cnt, G, n, tot);
  csc_scan_kernel<<<1, 1024, 0, st>>>(tot, n, m, ncols, colptr, itemptr);
  csc_items_kernel<<<(ncols + 255) / 256, 256, 0, st>>>(itemptr, ncols, items_max, items);
  if (A.v_type == SAP_F32)
    csc_scatter_kernel<float><<<G, kCscThreads, lds_n, st>>>(A.indptr, A.indices,
                                                             static_cast<const float *>(A.values), m, n, A.nnz, rpw,
                                                             cnt, colptr, crow, static_cast<float *>(cval));
  else
    csc_scatter_kernel<double><<<G, kCscThreads, lds_n, st>>>(A.indptr, A.indices,
                                                              static_cast<const double *>(A.values), m, n, A.nnz,
                                                              rpw, cnt, colptr, crow, static_cast<double *>(cval));
  SAP_HIP_TRY(hipGetLastError());
  const size_t lds_d = static_cast<size_t>(d + 1) * sizeof(double);
  const double h = 1.0 / std::sqrt(static_cast<double>(zeta));
  const unsigned ni = static_cast<unsigned>(items_max);
#define SAP_CSC_APPLY(TV, Z)                                                                                    \
  csc_apply_kernel<TV, Z><<<ni, kApplyColThreads, lds_d, st>>>(itemptr, items, colptr, crow,                     \
                                                               static_cast<const TV *>(cval), b, m, n, ncols,    \
                                                               A.nnz, d, zeta, S->idx, S->sign, part, Y, ldy, h)
  // Z-specialised kernels load 16-byte words of the index array
  const int zfast = (reinterpret_cast<uintptr_t>(S->idx) & 15) == 0 &&
                            (zeta == 8 || zeta == 12 || zeta == 16 || zeta == 24)
                        ? zeta
                        : 0;
  if (A.v_type == SAP_F32) {
    switch (zfast) {
      case 8: SAP_CSC_APPLY(float, 8); break;
      case 12: SAP_CSC_APPLY(float, 12); break;
      case 16: SAP_CSC_APPLY(float, 16); break;
      case 24: SAP_CSC_APPLY(float, 24); break;
      default: SAP_CSC_APPLY(float, 0);
    }
  } else {
    switch (zfast) {
      case 8: SAP_CSC_APPLY(double, 8); break;
      case 12: SAP_CSC_APPLY(double, 12); break;
      case 16: SAP_CSC_APPLY(double, 16); break;
      case 24: SAP_CSC_APPLY(double, 24); break;
      default: SAP_CSC_APPLY(double, 0);
    }
  }
#undef SAP_CSC_APPLY
  csc_reduce_kernel<<<dim3((d + 255) / 256, ncols), 256, 0, st>>>(part, itemptr, d, items_max, Y, ldy, h);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

int csr_pass_grid(sap_ctx *ctx, const SparseA &A) {
  const int64_t g = std::min<int64_t>(static_cast<int64_t>(ctx->num_cus) * 2, (A.m + 255) / 256);
  return static_cast<int>(std::max<int64_t>(1, g));
}

void launch_csr_pass(sap_ctx *ctx, const SparseA &A, int grid, const double *p, const double *u_in, double *u_out,
                     const LsqrState *st, double *qpart, double *nrmpart, hipStream_t s) {
  const double mean = A.m > 0 ? static_cast<double>(A.nnz) / static_cast<double>(A.m) : 1.0;
  int L = 1;
  while (L < 64 && L < mean) L <<= 1;
  const int64_t rpw = (A.m + grid - 1) / grid;
  const size_t lds = 2 * static_cast<size_t>(A.n) * sizeof(double);
  // rows of a workgroup: the groups of L lanes walk them in steps
  hipEvent_t pb = prof_begin(ctx, s);
  if (A.v_type == SAP_F32)
    csr_pass_kernel<float><<<grid, kPassThreadsS, lds, s>>>(A.indptr, A.indices, static_cast<const float *>(A.values),
                                                            A.m, A.n, L, rpw, p, u_in, u_out, st, qpart, nrmpart);
  else
    csr_pass_kernel<double><<<grid, kPassThreadsS, lds, s>>>(A.indptr, A.indices,
                                                             static_cast<const double *>(A.values), A.m, A.n, L, rpw,
                                                             p, u_in, u_out, st, qpart, nrmpart);
  prof_end(ctx, kProfPass, pb, s);
}

}  // namespace sap
