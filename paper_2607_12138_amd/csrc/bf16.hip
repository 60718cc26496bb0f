// Multi-right-hand-side BRAS apply with the element inverses in BF16 Gram-
// factor form on MFMA (gfx950).  Not built yet: bras_setup rejects BF16.
#include "internal.h"
#include "cg_common.h"

namespace bras {

int launch_bras_bf16(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                     const int* active) {
  (void)c; (void)x; (void)y; (void)R; (void)s; (void)dotv; (void)dotpart; (void)active;
  return fail(BRAS_EINVAL, "BF16 apply is not available in this build");
}

int cg_bras_bf16_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  (void)c; (void)cg; (void)R; (void)s;
  return fail(BRAS_EINVAL, "BF16 apply is not available in this build");
}

}  // namespace bras
