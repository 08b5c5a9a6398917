// Device code of the LSQR iteration shared by the single and batched
// launches: the per-block reduction of the pass partials and the scalar
// epilogues of the two chain solves (lsqr.hip describes the iteration).
#pragma once

#include "common.h"
#include "trsv.h"

namespace sap {

constexpr double kInnerReduction = 1e-6;

// Sum over a 1024-thread workgroup, result in every thread (two barriers).
__device__ __forceinline__ double wg_sum(double v, double *scratch) {
  v = wave_sum_u(v);
  const int wave = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kTrsvThreads / kWave; ++w) s += scratch[w];
  return s;
}

struct LowerShared {
  double rb[kTrsvB];
  double red[kTrsvGroups * kTrsvB];
  double scr[kTrsvThreads / kWave];
};

// rb = block b of q = sum over the G pass partials (fixed order).
__device__ __forceinline__ void reduce_q_block(const double *__restrict__ qpart, int G, int n, int b,
                                               LowerShared &sh) {
  const int t = threadIdx.x;
  const int r = t % kTrsvB, g = t / kTrsvB;
  const int c = b * kTrsvB + r;
  double s = 0.0;
  if (c < n)
    for (int pidx = g; pidx < G; pidx += kTrsvGroups) s += qpart[static_cast<int64_t>(pidx) * n + c];
  sh.red[g * kTrsvB + r] = s;
  __syncthreads();
  if (t < kTrsvB) {
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < kTrsvGroups; ++q) a += sh.red[q * kTrsvB + t];
    sh.rb[t] = a;
  }
  __syncthreads();
}

// After y = R^-T q is complete: beta = ||u_hat||, v_hat = y/beta - beta v,
// alpha = ||v_hat||, v = v_hat/alpha (the bidiagonalisation step of Alg. 2,
// in the App. D.4.1 order).  One workgroup.
__device__ __forceinline__ void lower_epilogue(int n, int G, const double *__restrict__ nrmpart, double *y,
                                               double *__restrict__ v, LsqrState *st, LowerShared &sh) {
  const int t = threadIdx.x;
  double bsq = 0.0;
  for (int g = t; g < G; g += kTrsvThreads) bsq += nrmpart[g];
  const double beta = sqrt(wg_sum(bsq, sh.scr));
  const bool init = st->init != 0;
  double alpha = 0.0;
  if (beta > 0.0) {
    double part = 0.0;
    for (int c = t; c < n; c += kTrsvThreads) {
      const double vh = load_coherent(y + c) / beta - (init ? 0.0 : beta * v[c]);
      y[c] = vh;
      part += vh * vh;
    }
    alpha = sqrt(wg_sum(part, sh.scr));
  }
  const bool proceed = beta > 0.0 && alpha > 0.0;
  if (proceed)
    for (int c = t; c < n; c += kTrsvThreads) v[c] = y[c] / alpha;
  if (t == 0) {
    st->beta_new = beta;
    st->alpha_new = alpha;
    st->proceed = proceed ? 1 : 0;
  }
}

// After p = R^-1 v is complete: initialisation (w = p) or the plane rotation
// of Alg. 2, x += (phi/rho) w, w = p - (theta/rho) w, the stopping
// test and the coefficients of the next pass.  One workgroup.  When the
// solve finishes, *done_count (nullable) is incremented once.
__device__ __forceinline__ void upper_epilogue(int n, const double *p, double *__restrict__ w,
                                               double *__restrict__ x, LsqrState *st, int *done_count) {
  const int t = threadIdx.x;
  const bool init = st->init != 0;
  const bool proceed = st->proceed != 0;
  const double beta = st->beta_new, alpha = st->alpha_new;
  if (init) {
    // beta_1 u_1 = b - A x0, alpha_1 v_1 = M^T A^T u_1, w_1 = M v_1
    if (proceed)
      for (int c = t; c < n; c += kTrsvThreads) w[c] = load_coherent(p + c);
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
      st->normref = st->rel ? beta : st->normb;
      st->normar0 = alpha * beta;
      st->converged = conv ? 1 : 0;
      st->done = stop ? 1 : 0;
      st->steps += 1;
      if (stop && done_count) atomicAdd(done_count, 1);
    }
    return;
  }
  // plane rotation of Alg. 2 with beta_{t+1}, alpha_{t+1}
  const double rhobar_old = st->rhobar, phibar_old = st->phibar;
  const double rho = sqrt(rhobar_old * rhobar_old + beta * beta);
  const double cs = rhobar_old / rho, sn = beta / rho;
  const double theta = sn * alpha;
  const double rhobar = -cs * alpha;
  const double phi = cs * phibar_old;
  const double phibar = sn * phibar_old;
  const double fx = phi / rho, fw = theta / rho;
  for (int c = t; c < n; c += kTrsvThreads) {
    const double wc = w[c];
    x[c] += fx * wc;
    if (proceed) w[c] = load_coherent(p + c) - fw * wc;
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
    // Inner solves of the refinement form (rel) also stop once the normal-
    // equation residual of their own problem has dropped by kInnerReduction.
    const bool conv = !proceed || alpha * fabs(cs) <= st->tol || phibar <= st->tol * st->normref ||
                      (st->rel && phibar * alpha * fabs(cs) <= kInnerReduction * st->normar0);
    st->converged = conv ? 1 : 0;
    const bool stop = conv || st->total_iters >= st->maxiter;
    st->done = stop ? 1 : 0;
    st->steps += 1;
    if (stop && done_count) atomicAdd(done_count, 1);
  }
}

}  // namespace sap
