// Lower-precision dense gradient paths (FP32, BF16 and split refinements).
#include "common.h"
#include "runtime.h"

namespace gwl {

size_t dense_lp_ws_bytes(const gwr::Grid&, const gwr::Grid&, int) { return 0; }

gw_status dense_lp(const gwr::Grid&, const gwr::Grid&, const double*, int64_t, double*, int64_t,
                   int, gwr::Arena&, hipStream_t, const double*, const double*) {
  return GW_EUNSUPPORTED;
}

}  // namespace gwl
