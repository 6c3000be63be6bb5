// Derivatives of u = M(r) f (vector-Jacobian product and divergence).
#include "rpyw_internal.h"

namespace rpyw {

size_t vjp_ws_bytes(int64_t N, int prec) { return (size_t)N * 64 * (prec == RPYW_FP32C ? 4 : 8) + 4096; }

int vjp(const double*, const double*, const double*, double*, double*, int64_t, double, double, int, Arena&,
        hipStream_t) {
    return RPYW_EINVAL;
}

int divergence(const double*, double*, int64_t, double, double, int, Arena&, hipStream_t) { return RPYW_EINVAL; }

}  // namespace rpyw
