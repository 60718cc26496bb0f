// Dispatch of the patch-form operator passes (kernels: patch_kern.h; one
// translation unit per element form: patch_scaled.hip, patch_packed_f32.hip,
// patch_packed_f64.hip, patch_metric3.hip, patch_metric6.hip).
#include "patch_kern.h"

namespace bras {

bool patch_supported(int form, int prec, int nl) {
  if (prec == BRAS_BF16) return false;
  bool ok = false;
#define CASE(N) ok = ok || nl == N;
  if (form == BRAS_ELEM_SCALED_REF) {
    PATCH_SCALED_NL(CASE)
  } else {
    PATCH_VECTOR_NL(CASE)
  }
#undef CASE
  return ok;
}

bool patch_active(const Ctx* c, int R) { return c->pt.npatch > 0 && c->use_patch && R == 1; }

int patch_blocks(const Ctx* c) { return (int)(c->pt.npatch + (c->pt.ns > 0 ? c->pt.nb2 : 0)); }

size_t patch_workspace_bytes(const Ctx* c) {
  return sizeof(double) * (size_t)(c->pt.nspart > 0 ? c->pt.nspart : 1);
}

int patch_pass(Ctx* c, int op, int out, const InArgs& in, double* y, const double* dotv, double* dotpart,
               const CgArgs& cg, hipStream_t s, double* ws) {
  PatchCall pc;
  pc.op = op;
  pc.out = out;
  pc.in = in;
  pc.y = y;
  pc.dotv = dotv;
  pc.dotpart = dotpart;
  pc.cg = cg;
  pc.spart = ws ? ws : c->pt.part;
  if (c->form == BRAS_ELEM_SCALED_REF) return patch_scaled(c, pc, s);
  if (op == 1) return c->prec == BRAS_FP64 ? patch_packed_f64(c, pc, s) : patch_packed_f32(c, pc, s);
  if (c->mpack) return patch_packed_f64(c, pc, s);
  return c->nsym <= 3 ? patch_metric3(c, pc, s) : patch_metric6(c, pc, s);
}

}  // namespace bras
