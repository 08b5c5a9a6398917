// Sparse sign sketch generation on gfx950 (Def. 2.2; rejection sampling of
// Sec. 3.1.2 and Alg. 3).
//
// One lane owns one column of S.  The zeta row indices live in registers:
// a fully unrolled bitonic network sorts them, neighbours are compared in
// registers, and only the positions that repeat their right neighbour are
// redrawn (Sec. 3.1.2 step (iii)).  The redraw loop is rare (probability
// 1 - prod_{k<zeta}(1 - k/d), eq. 3.2), so a wave diverges only on the few
// lanes that need it.  Random words come from Philox4x64-10 (Salmon et al.,
// SC'11) keyed by (seed, stream) with counter (column, round, group, k);
// bounded integers use Lemire's multiply-shift with rejection (2019).
#include "common.h"
#include "sketch_dev.h"

namespace sap {
namespace {

using namespace sketch_dev;

template <int ZMAX>
__global__ __launch_bounds__(256) void generate_kernel(int64_t m, int d, int zeta, uint64_t seed, uint64_t stream,
                                                       int32_t *__restrict__ idx, uint64_t *__restrict__ sign,
                                                       int *__restrict__ err) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  generate_column<ZMAX>(i, d, zeta, seed, stream, idx, sign, err);
}

}  // namespace

sap_status launch_generate(sap_ctx *ctx, const sps_sketch *S, int *err_word, hipStream_t st) {
  const int64_t m = S->m;
  const int threads = 256;
  const dim3 grid(static_cast<unsigned>((m + threads - 1) / threads));
  if (S->zeta <= 8)
    generate_kernel<8><<<grid, threads, 0, st>>>(m, S->d, S->zeta, S->seed, S->stream, S->idx,
                                                  S->sign, err_word);
  else if (S->zeta <= 16)
    generate_kernel<16><<<grid, threads, 0, st>>>(m, S->d, S->zeta, S->seed, S->stream, S->idx,
                                                   S->sign, err_word);
  else if (S->zeta <= 32)
    generate_kernel<32><<<grid, threads, 0, st>>>(m, S->d, S->zeta, S->seed, S->stream, S->idx,
                                                   S->sign, err_word);
  else
    generate_kernel<64><<<grid, threads, 0, st>>>(m, S->d, S->zeta, S->seed, S->stream, S->idx,
                                                   S->sign, err_word);
  SAP_HIP_TRY(hipGetLastError());
  return SAP_OK;
}

}  // namespace sap
