// Preconditioned LSQR (Alg. 2) on A M, M = R^-1, for gfx950.
//
// One iteration is three kernels on one stream, with no host round trip:
//   1. pass   : one sweep over A computing, for every row i,
//                 u_i <- c_ap (A p)_i + c_u u_i        (p = M v_t)
//               and accumulating q = A^T u and ||u||^2 from the same
//               registers.  This is the one-synchronisation reorganisation of
//               App. D.4.1: A^T is applied to the unnormalised u_hat, and the
//               scale 1/beta is folded into the next step, so A is read once
//               per iteration instead of twice.
//   2. reduce : fixed-order sum of the per-workgroup partials of q and ||u||^2.
//   3. step   : a single 1024-thread workgroup doing the O(n^2) and O(n) work:
//               v_hat = R^-T q / beta - beta v, alpha = ||v_hat||, v = v_hat/alpha,
//               p = R^-1 v (two blocked triangular solves), the Givens
//               recurrences, x += (phi/rho) w, w = p - (theta/rho) w, and the
//               convergence test.  All scalars stay in device memory.
// Kernels early-exit once the device `done` flag is set, so the host enqueues
// iterations in batches and reads the flag once per batch.
#include <cmath>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace sap {
namespace {

constexpr int kStepThreads = 1024;
constexpr int kStepWaves = kStepThreads / kWave;
constexpr int kTB = 64;  // triangular-solve block
constexpr int kMaxN = 8192;

// --------------------------------------------------------------------------
// Blocked triangular solve by one 1024-thread workgroup; xs (LDS, n doubles)
// holds the right-hand side on entry and the solution on exit.
//   trans = false: R x = rhs (back substitution, blocks from the bottom);
//   trans = true : R^T x = rhs (forward substitution, blocks from the top).
// The diagonal 64 x 64 block is solved by wave 0 with register broadcasts;
// the off-diagonal parts are coalesced column reads shared by all waves.
__device__ void wg_trsv(const double *__restrict__ R, int64_t ldr, int n, bool trans, double *xs,
                        double *Dblk) {
  const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  const int nblk = (n + kTB - 1) / kTB;
  for (int bi = 0; bi < nblk; ++bi) {
    const int kb = trans ? bi : nblk - 1 - bi;
    const int k0 = kb * kTB, kn = min(kTB, n - k0);
    if (trans && k0 > 0) {
      // xs[k0+j] -= R[0:k0, k0+j] . xs[0:k0]  (column k0+j of R is contiguous)
      for (int j = wave; j < kn; j += kStepWaves) {
        const double *col = R + static_cast<int64_t>(k0 + j) * ldr;
        double acc = 0.0;
        for (int l = lane; l < k0; l += kWave) acc += col[l] * xs[l];
        acc = wave_sum(acc);
        if (lane == 0) xs[k0 + j] -= acc;
      }
    }
    for (int e = t; e < kn * kTB; e += kStepThreads) {
      const int c = e / kTB, r = e % kTB;
      if (r < kn) Dblk[r * (kTB + 1) + c] = R[(k0 + r) + static_cast<int64_t>(k0 + c) * ldr];
    }
    __syncthreads();
    if (wave == 0) {
      double val = lane < kn ? xs[k0 + lane] : 0.0;
      if (!trans) {
        for (int j = kn - 1; j >= 0; --j) {
          const double rj = Dblk[lane * (kTB + 1) + j];
          const double xj = wave_bcast(val, j) / Dblk[j * (kTB + 1) + j];
          if (lane == j) val = xj;
          else if (lane < j) val -= rj * xj;
        }
      } else {
        for (int j = 0; j < kn; ++j) {
          const double rj = Dblk[j * (kTB + 1) + lane];
          const double xj = wave_bcast(val, j) / Dblk[j * (kTB + 1) + j];
          if (lane == j) val = xj;
          else if (lane > j && lane < kn) val -= rj * xj;
        }
      }
      if (lane < kn) xs[k0 + lane] = val;
    }
    __syncthreads();
    if (!trans && k0 > 0) {
      // xs[0:k0] -= R[0:k0, k0:k0+kn] xs[k0:k0+kn]
      for (int i = t; i < k0; i += kStepThreads) {
        double acc = 0.0;
        for (int c = 0; c < kn; ++c) acc += R[i + static_cast<int64_t>(k0 + c) * ldr] * xs[k0 + c];
        xs[i] -= acc;
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kStepThreads) void trsv_kernel(const double *__restrict__ R, int64_t ldr,
                                                             int n, int trans,
                                                             const double *__restrict__ rhs,
                                                             double *__restrict__ x) {
  extern __shared__ double lds[];
  double *xs = lds;
  double *Dblk = lds + n;
  for (int c = threadIdx.x; c < n; c += kStepThreads) xs[c] = rhs[c];
  __syncthreads();
  wg_trsv(R, ldr, n, trans != 0, xs, Dblk);
  for (int c = threadIdx.x; c < n; c += kStepThreads) x[c] = xs[c];
}

size_t trsv_lds_bytes(int n) { return sizeof(double) * (static_cast<size_t>(n) + kTB * (kTB + 1)); }

// --------------------------------------------------------------------------
// Fused pass.  MODE 0: A, accumulation and u in FP64.  MODE 1: A, p,
// accumulation and u in FP32 (inner iterations of the mixed form).  MODE 2:
// FP32 A with FP64 accumulation, u_in FP64 (b), u_out FP32 (the residual
// refinement pass of the mixed form).
template <int MODE>
struct PassTypes;
template <>
struct PassTypes<0> {
  using TA = double; using TC = double; using TUI = double; using TUO = double;
};
template <>
struct PassTypes<1> {
  using TA = float; using TC = float; using TUI = float; using TUO = float;
};
template <>
struct PassTypes<2> {
  using TA = float; using TC = double; using TUI = double; using TUO = float;
};

template <typename T, int V>
struct alignas(sizeof(T) * V) VecT {
  T e[V];
};

template <int MODE, int VEC, int J, int WC, int WR>
__global__ __launch_bounds__(kWave * WC * WR) void lsqr_pass_kernel(
    const typename PassTypes<MODE>::TA *__restrict__ A, int64_t lda, int64_t m, int n,
    const typename PassTypes<MODE>::TC *__restrict__ p,
    const typename PassTypes<MODE>::TUI *u_in, typename PassTypes<MODE>::TUO *u_out,
    const LsqrState *__restrict__ st, double *__restrict__ qpart, double *__restrict__ nrmpart,
    int64_t rows_per_wg) {
  using TA = typename PassTypes<MODE>::TA;
  using TC = typename PassTypes<MODE>::TC;
  constexpr int R = (J * VEC >= 16) ? 1 : (16 / (J * VEC) > 4 ? 4 : 16 / (J * VEC));
  constexpr int COLS = kWave * VEC * J;  // columns per wave
  __shared__ double xch[WC > 1 ? 2 : 1][R][WC];
  __shared__ double qbuf[WR > 1 ? COLS : 1];
  __shared__ double nbuf[WC * WR];
  if (st->done) return;

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int wc = wave % WC, wr = wave / WC;
  const int col0 = wc * COLS;
  const TC c_ap = static_cast<TC>(st->c_ap);
  const TC c_u = static_cast<TC>(st->c_u);

  TC preg[J][VEC], q[J][VEC];
#pragma unroll
  for (int j = 0; j < J; ++j)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int c = col0 + (j * kWave + lane) * VEC + e;
      preg[j][e] = c < n ? p[c] : TC(0);
      q[j][e] = TC(0);
    }

  const int64_t i_begin = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
  const int64_t i_end = min(m, i_begin + rows_per_wg);
  double nrm = 0.0;
  int parity = 0;
  for (int64_t base = i_begin + static_cast<int64_t>(wr) * R; base < i_end; base += static_cast<int64_t>(WR) * R) {
    TA a[R][J][VEC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = base + r;
      const bool rv = row < i_end;
      const TA *arow = A + row * lda;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int c = col0 + (j * kWave + lane) * VEC;
        if (rv && c < n) {
          const VecT<TA, VEC> v = *reinterpret_cast<const VecT<TA, VEC> *>(arow + c);
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[r][j][e] = v.e[e];
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) a[r][j][e] = TA(0);
        }
      }
    }
    TC dot[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      TC s = TC(0);
#pragma unroll
      for (int j = 0; j < J; ++j)
#pragma unroll
        for (int e = 0; e < VEC; ++e) s += static_cast<TC>(a[r][j][e]) * preg[j][e];
      dot[r] = wave_sum(s);
    }
    if constexpr (WC > 1) {
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < R; ++r) xch[parity][r][wc] = static_cast<double>(dot[r]);
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < WC; ++w) s += xch[parity][r][w];
        dot[r] = static_cast<TC>(s);
      }
      parity ^= 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = base + r;
      if (row < i_end) {
        const TC uh = c_ap * dot[r] + c_u * static_cast<TC>(u_in[row]);
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
          for (int e = 0; e < VEC; ++e) q[j][e] += uh * static_cast<TC>(a[r][j][e]);
        if (wc == 0 && lane == 0) {
          u_out[row] = static_cast<typename PassTypes<MODE>::TUO>(uh);
          nrm += static_cast<double>(uh) * static_cast<double>(uh);
        }
      }
    }
  }

  // Per-workgroup partials: q over this wave's columns (row groups combined in
  // a fixed order through LDS), ||u||^2 over all rows.
  double *qdst = qpart + static_cast<int64_t>(blockIdx.x) * n;
  if constexpr (WR > 1) {
    for (int g = 0; g < WR; ++g) {
      __syncthreads();
      if (wr == g) {
#pragma unroll
        for (int j = 0; j < J; ++j)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const int cl = (j * kWave + lane) * VEC + e;
            qbuf[cl] = (g == 0 ? 0.0 : qbuf[cl]) + static_cast<double>(q[j][e]);
          }
      }
    }
    __syncthreads();
    for (int cl = threadIdx.x; cl < COLS; cl += kWave * WC * WR) {
      const int c = col0 + cl;  // WC == 1 whenever WR > 1
      if (c < n) qdst[c] = qbuf[cl];
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int c = col0 + (j * kWave + lane) * VEC + e;
        if (c < n) qdst[c] = static_cast<double>(q[j][e]);
      }
  }
  if (lane == 0) nbuf[wave] = nrm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < WC * WR; ++w) s += nbuf[w];
    nrmpart[blockIdx.x] = s;
  }
}

// q[c] = sum_g qpart[g][c]; beta_sq = sum_g nrmpart[g]  (fixed order).
__global__ __launch_bounds__(256) void lsqr_reduce_kernel(const double *__restrict__ qpart,
                                                          const double *__restrict__ nrmpart, int G,
                                                          int n, double *__restrict__ q,
                                                          LsqrState *__restrict__ st) {
  __shared__ double sm[4][64];
  if (st->done) return;
  const int cl = threadIdx.x & 63, g0 = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  double s = 0.0;
  if (c < n)
    for (int g = g0; g < G; g += 4) s += qpart[static_cast<int64_t>(g) * n + c];
  sm[g0][cl] = s;
  __syncthreads();
  if (threadIdx.x < 64 && c < n) q[c] = ((sm[0][cl] + sm[1][cl]) + sm[2][cl]) + sm[3][cl];
  if (blockIdx.x == 0) {
    __syncthreads();
    double t = 0.0;
    for (int g = threadIdx.x; g < G; g += 256) t += nrmpart[g];
    // fixed-order: wave sums then wave 0 combines
    t = wave_sum(t);
    __shared__ double ws[4];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = t;
    __syncthreads();
    if (threadIdx.x == 0) st->beta_sq = ((ws[0] + ws[1]) + ws[2]) + ws[3];
  }
}

// --------------------------------------------------------------------------
// The O(n^2) part of an iteration (see the file comment).  p32 (nullable)
// receives an FP32 copy of p for the FP32 passes of the mixed form.
__global__ __launch_bounds__(kStepThreads) void lsqr_step_kernel(
    const double *__restrict__ R, int64_t ldr, int n, const double *__restrict__ q,
    double *__restrict__ v, double *__restrict__ w, double *__restrict__ x, double *__restrict__ p,
    float *__restrict__ p32, LsqrState *__restrict__ st, double outer_tol) {
  extern __shared__ double lds[];
  __shared__ double red[kStepWaves];
  double *xs = lds;
  double *Dblk = lds + n;
  if (st->done) return;
  const int t = threadIdx.x;
  const bool init = st->init != 0;
  const double beta = sqrt(st->beta_sq);
  const double rhobar_old = st->rhobar, phibar_old = st->phibar;

  double alpha = 0.0;
  if (beta > 0.0) {
    for (int c = t; c < n; c += kStepThreads) xs[c] = q[c];
    __syncthreads();
    wg_trsv(R, ldr, n, true, xs, Dblk);  // xs = R^-T A^T u_hat
    double part = 0.0;
    for (int c = t; c < n; c += kStepThreads) {
      const double vh = xs[c] / beta - (init ? 0.0 : beta * v[c]);
      xs[c] = vh;
      part += vh * vh;
    }
    alpha = sqrt(block_sum(part, red, kStepWaves));
  }
  const bool proceed = beta > 0.0 && alpha > 0.0;
  if (proceed) {
    for (int c = t; c < n; c += kStepThreads) {
      const double vn = xs[c] / alpha;
      xs[c] = vn;
      v[c] = vn;
    }
    __syncthreads();
    wg_trsv(R, ldr, n, false, xs, Dblk);  // xs = p_{t+1} = R^-1 v_{t+1}
  }

  if (init) {
    // beta_1 u_1 = b - A x0, alpha_1 v_1 = M^T A^T u_1, w_1 = M v_1.
    if (proceed) {
      for (int c = t; c < n; c += kStepThreads) {
        const double pc = xs[c];
        p[c] = pc;
        w[c] = pc;
        if (p32) p32[c] = static_cast<float>(pc);
      }
    }
    if (t == 0) {
      st->init = 0;
      st->phibar = beta;
      st->rhobar = alpha;
      st->alpha = alpha;
      st->beta = beta;
      st->resid_est = beta;
      st->normar_est = alpha * beta;
      st->c_ap = 1.0;
      st->c_u = beta > 0.0 ? -alpha / beta : 0.0;
      bool stop = !proceed || st->maxiter <= st->total_iters;
      bool conv = !proceed;
      if (outer_tol > 0.0 && (alpha <= outer_tol || beta <= outer_tol * st->normb)) stop = conv = true;
      st->converged = conv ? 1 : 0;
      st->done = stop ? 1 : 0;
    }
    return;
  }

  // Plane rotation (Alg. 2, line 7) with beta_{t+1}, alpha_{t+1}.
  const double rho = sqrt(rhobar_old * rhobar_old + beta * beta);
  const double cs = rhobar_old / rho, sn = beta / rho;
  const double theta = sn * alpha;
  const double rhobar = -cs * alpha;
  const double phi = cs * phibar_old;
  const double phibar = sn * phibar_old;
  const double fx = phi / rho, fw = theta / rho;
  for (int c = t; c < n; c += kStepThreads) {
    const double wc = w[c];
    x[c] += fx * wc;
    if (proceed) {
      const double pc = xs[c];
      p[c] = pc;
      if (p32) p32[c] = static_cast<float>(pc);
      w[c] = pc - fw * wc;
    }
  }
  if (t == 0) {
    st->iter += 1;
    st->total_iters += 1;
    st->rhobar = rhobar;
    st->phibar = phibar;
    st->alpha = alpha;
    st->beta = beta;
    st->c_ap = 1.0;
    st->c_u = beta > 0.0 ? -alpha / beta : 0.0;
    st->resid_est = phibar;
    st->normar_est = phibar * alpha * fabs(cs);
    const bool conv = !proceed || alpha * fabs(cs) <= st->tol || phibar <= st->tol * st->normb;
    st->converged = conv ? 1 : 0;
    st->done = (conv || st->total_iters >= st->maxiter) ? 1 : 0;
  }
}

__global__ void lsqr_init_state_kernel(LsqrState *st, double tol, int maxiter, int total_iters) {
  if (threadIdx.x != 0) return;
  st->alpha = st->beta = st->rhobar = st->phibar = 0.0;
  st->c_ap = -1.0;
  st->c_u = 1.0;
  st->beta_sq = 0.0;
  st->tol = tol;
  st->resid_est = st->normar_est = 0.0;
  st->iter = 0;
  st->maxiter = maxiter;
  st->done = 0;
  st->converged = 0;
  st->init = 1;
  st->total_iters = total_iters;
}

// ||b||^2 into st->normb (fixed-order two-level sum).
__global__ __launch_bounds__(1024) void norm_kernel(const double *__restrict__ b, int64_t m,
                                                    LsqrState *__restrict__ st) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 1024) s += b[i] * b[i];
  s = block_sum(s, red, 16);
  if (threadIdx.x == 0) st->normb = sqrt(s);
}

__global__ void copy_f64_kernel(const double *__restrict__ src, double *__restrict__ dst, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// --------------------------------------------------------------------------
// Pass configuration: columns per wave = 64 * VEC * J, WC waves across the
// columns, WR independent row groups per workgroup.
struct PassCfg {
  int vec, j, wc, wr;
};

template <int MODE>
PassCfg choose_pass(int n, int64_t lda, const void *A) {
  using TA = typename PassTypes<MODE>::TA;
  const int vmax = 16 / static_cast<int>(sizeof(TA));
  const bool aligned = (reinterpret_cast<uintptr_t>(A) % 16 == 0) && (lda % vmax == 0) && (n % vmax == 0);
  PassCfg c{aligned ? vmax : 1, 1, 1, 4};
  const int per_j = kWave * c.vec;
  int need = (n + per_j - 1) / per_j;  // J * WC needed
  if (need <= 8) {
    int j = 1;
    while (j < need) j <<= 1;
    c.j = j < 2 ? 2 : j;
    c.wc = 1;
    c.wr = 4;
  } else {
    c.j = 8;
    int wc = 1;
    while (wc * 8 < need) wc <<= 1;
    c.wc = wc;
    c.wr = 1;
  }
  return c;
}

struct PassLaunch {
  const void *fn;
  int threads;
};

template <int MODE, int VEC, int J, int WC, int WR>
PassLaunch pass_fn() {
  return PassLaunch{reinterpret_cast<const void *>(&lsqr_pass_kernel<MODE, VEC, J, WC, WR>), kWave * WC * WR};
}

template <int MODE, int VEC>
PassLaunch pick_vec(const PassCfg &c) {
  if (c.wc == 1) {
    switch (c.j) {
      case 2: return pass_fn<MODE, VEC, 2, 1, 4>();
      case 4: return pass_fn<MODE, VEC, 4, 1, 4>();
      default: return pass_fn<MODE, VEC, 8, 1, 4>();
    }
  }
  switch (c.wc) {
    case 2: return pass_fn<MODE, VEC, 8, 2, 1>();
    case 4: return pass_fn<MODE, VEC, 8, 4, 1>();
    default: return pass_fn<MODE, VEC, 8, 8, 1>();
  }
}

template <int MODE>
PassLaunch pick_pass(const PassCfg &c) {
  constexpr int vmax = 16 / static_cast<int>(sizeof(typename PassTypes<MODE>::TA));
  return c.vec == 1 ? pick_vec<MODE, 1>(c) : pick_vec<MODE, vmax>(c);
}

std::mutex g_occ_mu;
std::unordered_map<const void *, int> g_occ;

int occupancy(const void *fn, int threads) {
  std::lock_guard<std::mutex> lk(g_occ_mu);
  auto it = g_occ.find(fn);
  if (it != g_occ.end()) return it->second;
  int blocks = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, threads, 0) != hipSuccess || blocks < 1) blocks = 1;
  g_occ[fn] = blocks;
  return blocks;
}

struct PassPlan {
  PassLaunch launch;
  int grid;
  int64_t rows_per_wg;
};

PassPlan plan_pass(sap_ctx *ctx, int mode, int64_t m, int n, int64_t lda, const void *A) {
  PassCfg c;
  PassLaunch l;
  if (mode == 0) {
    c = choose_pass<0>(n, lda, A);
    l = pick_pass<0>(c);
  } else if (mode == 1) {
    c = choose_pass<1>(n, lda, A);
    l = pick_pass<1>(c);
  } else {
    c = choose_pass<2>(n, lda, A);
    l = pick_pass<2>(c);
  }
  const int occ = occupancy(l.fn, l.threads);
  int64_t grid = static_cast<int64_t>(ctx->num_cus) * occ;
  const int64_t min_rows = 16;
  if (grid * min_rows > m) grid = (m + min_rows - 1) / min_rows;
  if (grid < 1) grid = 1;
  PassPlan p{l, static_cast<int>(grid), (m + grid - 1) / grid};
  return p;
}

void launch_pass(sap_ctx *ctx, const PassPlan &pl, const void *A, int64_t lda, int64_t m, int n, const void *p,
                 const void *u_in, void *u_out, const LsqrState *st, double *qpart, double *nrmpart,
                 hipStream_t s) {
  int64_t lda_ = lda, m_ = m, rows = pl.rows_per_wg;
  int n_ = n;
  const void *A_ = A, *p_ = p, *ui = u_in, *st_ = st;
  void *uo = u_out, *qp = qpart, *np = nrmpart;
  void *args[] = {&A_, &lda_, &m_, &n_, &p_, &ui, &uo, &st_, &qp, &np, &rows};
  hipEvent_t pb = prof_begin(ctx, s);
  const hipError_t e = hipLaunchKernel(pl.launch.fn, dim3(pl.grid), dim3(pl.launch.threads), args, 0, s);
  if (e != hipSuccess) (void)e;  // reported by the hipGetLastError check after the batch
  prof_end(ctx, kProfPass, pb, s);
}

int max_grid(sap_ctx *ctx) { return ctx->num_cus * 16; }

}  // namespace

sap_status launch_trsv(sap_ctx *ctx, const double *R, int64_t ldr, int n, int trans, const double *rhs,
                       double *x, hipStream_t st) {
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "sap_trsv: n > 8192 is not supported");
  trsv_kernel<<<1, kStepThreads, trsv_lds_bytes(n), st>>>(R, ldr, n, trans, rhs, x);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

size_t lsqr_workspace_bytes(sap_ctx *ctx, int64_t m, int n, int mode) {
  const size_t G = static_cast<size_t>(max_grid(ctx));
  size_t bytes = 0;
  bytes += 256 * 16;                                     // alignment slack
  bytes += sizeof(LsqrState);
  bytes += G * n * sizeof(double) + G * sizeof(double);  // partials
  bytes += 5 * static_cast<size_t>(n) * sizeof(double);  // q v w p x0copy
  bytes += static_cast<size_t>(n) * sizeof(float);       // p32
  bytes += static_cast<size_t>(m) * (mode == 0 ? sizeof(double) : sizeof(float));  // u
  return bytes;
}

// Runs LSQR from x0 on A R^-1 (mode 0: FP64; mode 1/2: mixed form with FP64
// residual refinement around FP32 inner iterations).
sap_status run_lsqr(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr, const double *x0,
                    double tol, int maxiter, int mode, int max_refine, double inner_tol, double *x,
                    sap_info *info, void *work, hipStream_t s) {
  const int64_t m = prob->m;
  const int n = prob->n;
  if (n > kMaxN) return fail(ctx, SAP_EINVAL, "LSQR: n > 8192 is not supported");
  Carve cv(work);
  LsqrState *st = cv.take<LsqrState>(1);
  const int pass_mode_main = (mode == 0) ? 0 : 1;
  const PassPlan plan_main = plan_pass(ctx, pass_mode_main, m, n, prob->lda, prob->A);
  const PassPlan plan_ref = (mode == 0) ? plan_main : plan_pass(ctx, 2, m, n, prob->lda, prob->A);
  const int G = plan_main.grid > plan_ref.grid ? plan_main.grid : plan_ref.grid;
  if (G > max_grid(ctx)) return fail(ctx, SAP_EINVAL, "LSQR: internal grid larger than planned");
  double *qpart = cv.take<double>(static_cast<size_t>(max_grid(ctx)) * n);
  double *nrmpart = cv.take<double>(max_grid(ctx));
  double *q = cv.take<double>(n);
  double *v = cv.take<double>(n);
  double *w = cv.take<double>(n);
  double *p = cv.take<double>(n);
  double *xin = cv.take<double>(n);
  float *p32 = cv.take<float>(n);
  void *u = (mode == 0) ? static_cast<void *>(cv.take<double>(m)) : static_cast<void *>(cv.take<float>(m));

  const size_t step_lds = trsv_lds_bytes(n);
  // x0 may alias x: copy first.
  copy_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(x0, xin, n);
  copy_f64_kernel<<<(n + 255) / 256, 256, 0, s>>>(xin, x, n);
  lsqr_init_state_kernel<<<1, 64, 0, s>>>(st, mode == 0 ? tol : inner_tol, maxiter, 0);
  norm_kernel<<<1, 1024, 0, s>>>(prob->b, m, st);
  SAP_HIP_TRY(hipGetLastError());

  const int batch = 8;
  int refinements = 0;
  LsqrState hs{};
  const int max_outer = (mode == 0) ? 1 : (max_refine > 0 ? max_refine : 8) + 1;
  for (int outer = 0; outer < max_outer; ++outer) {
    if (outer > 0) {
      lsqr_init_state_kernel<<<1, 64, 0, s>>>(st, inner_tol, maxiter, hs.total_iters);
      SAP_HIP_TRY(hipGetLastError());
    }
    // Initialisation pass: u_hat_1 = b - A x (mode 2 in the mixed form: FP64
    // accumulation of the FP32 A; this is the residual refinement pass).
    const int init_mode = (mode == 0) ? 0 : 2;
    const PassPlan &pi = (mode == 0) ? plan_main : plan_ref;
    launch_pass(ctx, pi, prob->A, prob->lda, m, n, x, prob->b, u, st, qpart, nrmpart, s);
    lsqr_reduce_kernel<<<(n + 63) / 64, 256, 0, s>>>(qpart, nrmpart, pi.grid, n, q, st);
    lsqr_step_kernel<<<1, kStepThreads, step_lds, s>>>(R, ldr, n, q, v, w, x, p, mode == 0 ? nullptr : p32, st,
                                                      mode == 0 ? 0.0 : tol);
    SAP_HIP_TRY(hipGetLastError());
    if (mode != 0) ++refinements;
    // Iterations in batches; one flag read per batch.  The step kernel sets
    // `done` no later than iteration maxiter, so the batch count is bounded.
    const int max_batches = maxiter / batch + 2;
    for (int nbatch = 0;; ++nbatch) {
      if (nbatch > max_batches) return fail(ctx, SAP_EDEVICE, "LSQR: device never reported completion");
      for (int k = 0; k < batch; ++k) {
        if (mode == 0)
          launch_pass(ctx, plan_main, prob->A, prob->lda, m, n, p, u, u, st, qpart, nrmpart, s);
        else
          launch_pass(ctx, plan_main, prob->A, prob->lda, m, n, p32, u, u, st, qpart, nrmpart, s);
        lsqr_reduce_kernel<<<(n + 63) / 64, 256, 0, s>>>(qpart, nrmpart, plan_main.grid, n, q, st);
        lsqr_step_kernel<<<1, kStepThreads, step_lds, s>>>(R, ldr, n, q, v, w, x, p,
                                                          mode == 0 ? nullptr : p32, st, 0.0);
      }
      SAP_HIP_TRY(hipGetLastError());
      SAP_HIP_TRY(hipMemcpyAsync(&hs, st, sizeof(LsqrState), hipMemcpyDeviceToHost, s));
      SAP_HIP_TRY(hipStreamSynchronize(s));
      if (hs.done) break;
    }
    if (mode == 0) break;
    // Mixed form: the inner loop ended.  Converged at the outer level only if
    // the refinement pass itself said so (done at init with converged set).
    if (hs.converged && hs.iter == 0) break;
    if (hs.total_iters >= maxiter) break;
  }
  if (info) {
    info->iters = hs.total_iters;
    info->refinements = refinements;
    info->resid_est = hs.resid_est;
    info->normar_est = hs.normar_est;
  }
  if (mode == 0) return hs.converged ? SAP_OK : SAP_NOT_CONVERGED;
  return (hs.converged && hs.iter == 0) ? SAP_OK : SAP_NOT_CONVERGED;
}

}  // namespace sap
