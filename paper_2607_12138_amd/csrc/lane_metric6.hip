// Instantiations of the per-lane element pass (elem_lane.h).
#include "elem_lane.h"

namespace bras {

int lane_metric6(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s) {
  return lane_dispatch<FORM_METRIC, 6, double, double>(c, R, in, nullptr, zb, s);
}

}  // namespace bras
