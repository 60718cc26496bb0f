// Instantiations of the per-lane element pass (elem_lane.h).
#include "elem_lane.h"

namespace bras {

int lane_packed_f32(Ctx* c, int R, const InArgs& in, const float* ap, float* zb, hipStream_t s) {
  return lane_dispatch<FORM_PACKED, 0, float, float, 256>(c, R, in, ap, zb, s);
}

}  // namespace bras
