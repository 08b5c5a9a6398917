// Device code of the sparse sign sketch generator (Def. 2.2; rejection
// sampling of Sec. 3.1.2 and Alg. 3), shared by the single and batched
// launches.  One lane owns one column of S; see sketch.hip.
#pragma once

#include "common.h"

namespace sap {
namespace sketch_dev {


constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;
constexpr uint32_t kSentinel = 0xFFFFFFFFu;  // sorts after every real row (< 2^31)
constexpr int kMaxRounds = 1 << 16;

struct Block4 {
  uint64_t w[4];
};

__device__ __forceinline__ Block4 philox(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                         uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += kPhiloxW0;
      k1 += kPhiloxW1;
    }
    const uint64_t lo0 = kPhiloxM0 * c0, hi0 = __umul64hi(kPhiloxM0, c0);
    const uint64_t lo1 = kPhiloxM1 * c2, hi1 = __umul64hi(kPhiloxM1, c2);
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return Block4{{c0, c1, c2, c3}};
}

// Lemire: accept w when low64(w*d) >= (2^64 - d) mod d; the value is
// high64(w*d).  The modulo is only needed in the rare case low < d.
__device__ __forceinline__ bool lemire(uint64_t w, uint64_t d, uint32_t &out) {
  const uint64_t low = w * d;
  if (low < d) {
    const uint64_t threshold = (0ull - d) % d;
    if (low < threshold) return false;
  }
  out = static_cast<uint32_t>(__umul64hi(w, d));
  return true;
}

// U(i, r, j) given the k = 0 word; steps k = 1, 2, ... on rejection.
static __device__ __noinline__ uint32_t bounded_slow(uint64_t i, uint64_t r, int j, uint64_t d,
                                              uint64_t seed, uint64_t stream) {
  uint32_t v = 0;
  for (uint64_t k = 1;; ++k) {
    Block4 b = philox(i, r, static_cast<uint64_t>(j >> 2), k, seed, stream);
    if (lemire(b.w[j & 3], d, v)) return v;
  }
}

template <int N>
__device__ __forceinline__ void bitonic_sort(uint32_t (&c)[N]) {
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
      for (int a = 0; a < N; ++a) {
        const int b = a ^ j;
        if (b > a) {
          const uint32_t x = c[a], y = c[b];
          const uint32_t lo = x < y ? x : y, hi = x < y ? y : x;
          if ((a & k) == 0) {
            c[a] = lo;
            c[b] = hi;
          } else {
            c[a] = hi;
            c[b] = lo;
          }
        }
      }
    }
  }
}

// Column i of the sketch: zeta ascending distinct rows into idx[i*zeta ..]
// and the sign word into sign[i].
template <int ZMAX>
__device__ __forceinline__ void generate_column(int64_t i, int d, int zeta, uint64_t seed, uint64_t stream,
                                                int32_t *__restrict__ idx, uint64_t *__restrict__ sign,
                                                int *__restrict__ err) {
  const uint64_t col = static_cast<uint64_t>(i);
  const uint64_t dd = static_cast<uint64_t>(d);
  uint32_t c[ZMAX];

  // Round 0: zeta draws with replacement (step (i)).
#pragma unroll
  for (int g = 0; g < ZMAX / 4; ++g) {
    if (4 * g < zeta) {
      const Block4 b = philox(col, 0, static_cast<uint64_t>(g), 0, seed, stream);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = 4 * g + e;
        uint32_t v = kSentinel;
        if (j < zeta && !lemire(b.w[e], dd, v)) v = bounded_slow(col, 0, j, dd, seed, stream);
        c[j] = v;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) c[4 * g + e] = kSentinel;
    }
  }
  bitonic_sort<ZMAX>(c);

  // Rounds r >= 1: redraw every position equal to its right neighbour (steps
  // (ii)-(iv)), comparing on the sorted column before any replacement.
  for (int r = 1;; ++r) {
    bool dup[ZMAX];
    bool any = false;
#pragma unroll
    for (int j = 0; j < ZMAX; ++j) {
      dup[j] = (j + 1 < ZMAX) && (j + 1 < zeta) && (c[j] == c[j + 1]);
      any |= dup[j];
    }
    if (!any) break;
    if (r >= kMaxRounds) {
      atomicOr(err, 1);
      break;
    }
#pragma unroll
    for (int g = 0; g < ZMAX / 4; ++g) {
      const bool need = dup[4 * g] | dup[4 * g + 1] | dup[4 * g + 2] | dup[4 * g + 3];
      if (need) {
        const Block4 b = philox(col, static_cast<uint64_t>(r), static_cast<uint64_t>(g), 0, seed,
                                stream);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int j = 4 * g + e;
          if (dup[j]) {
            uint32_t v;
            if (!lemire(b.w[e], dd, v)) v = bounded_slow(col, static_cast<uint64_t>(r), j, dd, seed, stream);
            c[j] = v;
          }
        }
      }
    }
    bitonic_sort<ZMAX>(c);
  }

  int32_t *out = idx + i * zeta;
#pragma unroll
  for (int j = 0; j < ZMAX; ++j)
    if (j < zeta) out[j] = static_cast<int32_t>(c[j]);
  const Block4 s = philox(col, ~0ull, 0, 0, seed, stream);
  const uint64_t mask = (zeta >= 64) ? ~0ull : ((1ull << zeta) - 1ull);
  sign[i] = s.w[0] & mask;
}


}  // namespace sketch_dev
}  // namespace sap
