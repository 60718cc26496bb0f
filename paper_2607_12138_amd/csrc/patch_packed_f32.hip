// Patch-form operator passes (patch_kern.h): packed float32 inverses (BRAS).
#include "patch_kern.h"

namespace bras {

template <int NL, int OUT>
static int bras_k(Ctx* c, const PatchCall& pc, hipStream_t s) {
  return patch_launch<NL, FORM_PACKED, 0, float, OUT, false, 272>(c, pc, (const float*)c->ainv, nullptr, nullptr, 0, nullptr, s);
}

template <int NL>
static int by_out(Ctx* c, const PatchCall& pc, hipStream_t s) {
  if (pc.op == 1) {
    switch (pc.out) {
      case OUT_PLAIN: return bras_k<NL, OUT_PLAIN>(c, pc, s);
      case OUT_BRAS_CG: return bras_k<NL, OUT_BRAS_CG>(c, pc, s);
      case OUT_STAT: return bras_k<NL, OUT_STAT>(c, pc, s);
      default: break;
    }
  }
  return fail(BRAS_EINVAL, "patch pass: operator %d has no epilogue %d in this form", pc.op, pc.out);
}

int patch_packed_f32(Ctx* c, const PatchCall& pc, hipStream_t s) {
#define CASE(N) \
  case N: return by_out<N>(c, pc, s);
  switch (c->nl) {
    PATCH_VECTOR_NL(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no patch kernel", c->nl);
  }
#undef CASE
}

}  // namespace bras
