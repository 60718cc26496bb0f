// Patch-form operator passes (patch_kern.h): scaled H1 form (shared reference matrix times the element factor).
#include "patch_kern.h"

namespace bras {

template <int NL, int OUT>
static int bras_k(Ctx* c, const PatchCall& pc, hipStream_t s) {
  return patch_launch<NL, FORM_METRIC, 1, double, OUT, true, 13>(c, pc, (const double*)nullptr, c->refinv_pk, c->icoef, 1, c->invd, s);
}

template <int NL, int OUT>
static int mass_k(Ctx* c, const PatchCall& pc, hipStream_t s) {
  return patch_launch<NL, FORM_METRIC, 1, double, OUT, false, 13>(c, pc, (const double*)nullptr, c->ref_pk, c->coef, 1, nullptr, s);
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
  if (pc.op == 0) {
    switch (pc.out) {
      case OUT_PLAIN: return mass_k<NL, OUT_PLAIN>(c, pc, s);
      case OUT_MASS_CG: return mass_k<NL, OUT_MASS_CG>(c, pc, s);
      case OUT_RES: return mass_k<NL, OUT_RES>(c, pc, s);
      default: break;
    }
  }
  return fail(BRAS_EINVAL, "patch pass: operator %d has no epilogue %d in this form", pc.op, pc.out);
}

int patch_scaled(Ctx* c, const PatchCall& pc, hipStream_t s) {
#define CASE(N) \
  case N: return by_out<N>(c, pc, s);
  switch (c->nl) {
    PATCH_SCALED_NL(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no patch kernel", c->nl);
  }
#undef CASE
}

}  // namespace bras
