// Instantiations of the per-lane element pass (elem_lane.h): 3D metric form,
// scheduling variant 2.
#include "elem_lane.h"

namespace bras {

int lane_metric6_v2(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s) {
  return lane_dispatch<FORM_METRIC, 6, double, double, 13>(c, R, in, nullptr, zb, s);
}

}  // namespace bras
