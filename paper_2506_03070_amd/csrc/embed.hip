// Embedding dimension and iteration-count estimate (Sec. 4.3).
//
// The sketch generation and apply cost little more for a larger d, while the
// QR of the d x (n+1) sketch grows as d n^2 and the LSQR iterations shrink
// with the rate sqrt(n/d) (eq. (4.1)).  Eq. (4.2) picks the d at which the
// two costs balance, through the Lambert W function.  Host-only code: no
// device work, no context.
#include <climits>
#include <cmath>
#include <cstdint>

#include "../../include/sap.h"

namespace sap {
namespace {

// Principal branch W(z), z >= 0: Halley's iteration on w e^w - z (Corless,
// Gonnet, Hare, Jeffrey, Knuth, "On the Lambert W function", Adv. Comput.
// Math. 5 (1996), Sec. 5), started at ln(1 + z), which lies within a factor
// of two of the root for every z >= 0; cubic convergence ends it in a few
// steps.
double lambert_w0(double z) {
  double w = std::log1p(z);
  for (int it = 0; it < 64; ++it) {
    const double ew = std::exp(w);
    const double f = w * ew - z;
    const double step = f / (ew * (w + 1.0) - (w + 2.0) * f / (2.0 * w + 2.0));
    w -= step;
    if (!(std::fabs(step) > 4e-16 * (1.0 + std::fabs(w)))) break;
  }
  return w;
}

}  // namespace
}  // namespace sap

extern "C" sap_status sap_embedding_dim(int64_t m, int32_t n, double eps, double cost_ratio, int32_t *d) {
  if (d == nullptr || n < 1 || m <= n || !(eps > 0.0 && eps < 1.0) || !(cost_ratio > 0.0) ||
      !std::isfinite(cost_ratio))
    return SAP_EINVAL;
  const double nn = static_cast<double>(n);
  const double z = cost_ratio * (-static_cast<double>(m) * std::log(eps)) / (nn * nn);
  if (!std::isfinite(z)) return SAP_EINVAL;
  const double dr = nn * std::exp(sap::lambert_w0(z));
  // at least n + 1 rows (the sketch of [A b] must be tall), at most m
  double hi = static_cast<double>(m);
  if (hi > static_cast<double>(INT32_MAX)) hi = static_cast<double>(INT32_MAX);
  double v = std::ceil(dr);
  if (!(v >= nn + 1.0)) v = nn + 1.0;
  if (v > hi) v = hi;
  *d = static_cast<int32_t>(v);
  return SAP_OK;
}

extern "C" sap_status sap_iteration_estimate(int32_t n, int32_t d, double eps, int32_t *iters) {
  if (iters == nullptr || n < 1 || d <= n || !(eps > 0.0 && eps < 1.0)) return SAP_EINVAL;
  const double t = 2.0 * std::log(eps) / std::log(static_cast<double>(n) / static_cast<double>(d));
  const double c = std::ceil(t);
  *iters = c >= static_cast<double>(INT32_MAX) ? INT32_MAX : static_cast<int32_t>(c);
  return SAP_OK;
}
