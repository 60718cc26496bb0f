// Error reporting, introspection, options and the kernel-variant autotuner.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "internal.h"

namespace bras {

static thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_err[0] = '\0'; }

}  // namespace bras

using namespace bras;

extern "C" const char* bras_last_error(void) { return g_err; }

extern "C" int bras_info(bras_handle h, int what, int64_t* value_h) {
  clear_error();
  BRAS_CHECK(h && value_h, "null argument");
  Ctx* c = (Ctx*)h;
  switch (what) {
    case BRAS_INFO_N: *value_h = c->n; break;
    case BRAS_INFO_E: *value_h = c->E; break;
    case BRAS_INFO_NLOC: *value_h = c->nl; break;
    case BRAS_INFO_NBR: *value_h = c->nbr; break;
    case BRAS_INFO_PREC: *value_h = c->prec; break;
    case BRAS_INFO_FORM: *value_h = c->form; break;
    case BRAS_INFO_MAXRHS: *value_h = c->max_rhs; break;
    case BRAS_INFO_RESTARTS: *value_h = c->last_restarts; break;
    case BRAS_INFO_VARIANT: *value_h = c->variant; break;
    case BRAS_INFO_SOLVE_PATH: *value_h = c->last_path; break;
    case BRAS_INFO_PATCHES: *value_h = c->pt.npatch; break;
    case BRAS_INFO_PATCH_ON: *value_h = (c->pt.npatch > 0 && c->use_patch) ? 1 : 0; break;
    default: return fail(BRAS_EINVAL, "unknown info key %d", what);
  }
  return BRAS_OK;
}

extern "C" int bras_set_option(bras_handle h, int opt, double value) {
  clear_error();
  BRAS_CHECK(h, "null handle");
  Ctx* c = (Ctx*)h;
  switch (opt) {
    case BRAS_OPT_GRAPH_ITERS:
      BRAS_CHECK(value >= 1 && value <= 32, "graph iterations must be in 1..32");
      c->graph_iters = (int)value;
      break;
    case BRAS_OPT_MAX_RESTART:
      BRAS_CHECK(value >= 0 && value <= 100, "restarts must be in 0..100");
      c->max_restart = (int)value;
      break;
    case BRAS_OPT_VARIANT:
      BRAS_CHECK(value >= -1 && value < variant_count(c), "variant must be -1 or in 0..%d", variant_count(c) - 1);
      c->variant = (int)value;
      cg_free(c);   // captured CG graphs hold the previous kernels
      break;
    case BRAS_OPT_SMALL_CG:
      BRAS_CHECK(value == 0 || value == 1, "small-problem solver switch must be 0 or 1");
      c->small_cg = (int)value;
      break;
    case BRAS_OPT_PATCH:
      BRAS_CHECK(value == 0 || value == 1, "patch-form switch must be 0 or 1");
      c->use_patch = (int)value;
      cg_free(c);   // captured CG graphs and partial buffers follow the operator form
      break;
    case BRAS_OPT_FLEXIBLE:
      BRAS_CHECK(value == -1 || value == 0 || value == 1, "flexible-beta switch must be -1, 0 or 1");
      c->flexible_opt = (int)value;
      break;
    default: return fail(BRAS_EINVAL, "unknown option %d", opt);
  }
  return BRAS_OK;
}

extern "C" int bras_export(bras_handle h, int what, void* dst_d, void* stream) {
  clear_error();
  BRAS_CHECK(h && dst_d, "null argument");
  Ctx* c = (Ctx*)h;
  hipStream_t s = (hipStream_t)stream;
  switch (what) {
    case BRAS_EXPORT_MULT:
      BRAS_HIP(hipMemcpyAsync(dst_d, c->mult, sizeof(int32_t) * c->n, hipMemcpyDeviceToDevice, s));
      break;
    case BRAS_EXPORT_ROWPTR:
      BRAS_HIP(hipMemcpyAsync(dst_d, c->rowptr, sizeof(int32_t) * (c->n + 1), hipMemcpyDeviceToDevice, s));
      break;
    case BRAS_EXPORT_DIAG:
      BRAS_HIP(hipMemcpyAsync(dst_d, c->diag, sizeof(double) * c->n, hipMemcpyDeviceToDevice, s));
      break;
    case BRAS_EXPORT_SLOT: {
      // internal l*E + K -> the caller's K*n_loc + l, on the host, each row in
      // increasing order (the handle's element order may be patch-major)
      std::vector<int32_t> in(c->nbr), rp(c->n + 1), perm;
      std::vector<int64_t> out(c->nbr);
      BRAS_HIP(hipMemcpyAsync(in.data(), c->slot, sizeof(int32_t) * c->nbr, hipMemcpyDeviceToHost, s));
      BRAS_HIP(hipMemcpyAsync(rp.data(), c->rowptr, sizeof(int32_t) * (c->n + 1), hipMemcpyDeviceToHost, s));
      if (c->pt.perm) {
        perm.resize(c->E);
        BRAS_HIP(hipMemcpyAsync(perm.data(), c->pt.perm, sizeof(int32_t) * c->E, hipMemcpyDeviceToHost, s));
      }
      BRAS_HIP(hipStreamSynchronize(s));
      for (int64_t p = 0; p < c->nbr; ++p) {
        const int64_t l = in[p] / c->E, K = in[p] - l * c->E;
        out[p] = (perm.empty() ? K : (int64_t)perm[K]) * c->nl + l;
      }
      if (!perm.empty())
        for (int64_t i = 0; i < c->n; ++i) std::sort(out.begin() + rp[i], out.begin() + rp[i + 1]);
      BRAS_HIP(hipMemcpyAsync(dst_d, out.data(), sizeof(int64_t) * c->nbr, hipMemcpyHostToDevice, s));
      BRAS_HIP(hipStreamSynchronize(s));
      break;
    }
    default: return fail(BRAS_EINVAL, "unknown export key %d", what);
  }
  return BRAS_OK;
}

int bras::variant_count(const Ctx* c) {
  const bool metric6 = c->form == BRAS_ELEM_METRIC_REF && c->nsym > 3 && c->nl <= kLaneMaxNL;
  if (c->form == BRAS_ELEM_SCALED_REF) return 2;   // matrix-core / per-row FMA element pass
  return metric6 ? kMetricVariants : 1;
}

// Times mass apply + BRAS apply (one CG iteration's operator passes) for every
// candidate of this handle and keeps the fastest: the element-pass
// scheduling variants, and, when the handle has a patch plan and nrhs = 1,
// the patch form of the passes (whose kernels do not depend on the variant).
extern "C" int bras_autotune(bras_handle h, int nrhs, void* stream) {
  clear_error();
  BRAS_CHECK(h, "null handle");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs outside 1..max_rhs");
  const int nv = variant_count(c);
  const bool plan = c->pt.npatch > 0 && nrhs == 1;
  struct Cand {
    int patch, variant;
  };
  std::vector<Cand> cands;
  if (plan) cands.push_back({1, c->variant >= 0 ? c->variant : 0});
  for (int v = 0; v < nv; ++v) cands.push_back({0, v});
  if (cands.size() == 1) {
    c->variant = 0;
    return BRAS_OK;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t vec = sizeof(double) * (size_t)c->n * nrhs;
  double *x = nullptr, *y = nullptr;
  BRAS_HIP(hipMalloc((void**)&x, vec));
  if (hipMalloc((void**)&y, vec) != hipSuccess) {
    (void)hipFree(x);
    return fail(BRAS_ENOMEM, "autotune workspace allocation failed");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int st = BRAS_OK;
  if (hipMemsetAsync(x, 0, vec, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    st = fail(BRAS_EHIP, "autotune set-up failed");
  float best = 1e30f;
  Cand pick = cands[0];
  for (size_t k = 0; k < cands.size() && st == BRAS_OK; ++k) {
    c->use_patch = cands[k].patch;
    c->variant = cands[k].variant;
    auto pass = [&]() {
      int r = launch_mass(c, x, y, nrhs, s, nullptr, nullptr, nullptr);
      return r ? r : launch_bras(c, x, y, nrhs, s, nullptr, nullptr, nullptr);
    };
    for (int w = 0; w < 2 && st == BRAS_OK; ++w) st = pass();
    if (st) break;
    (void)hipEventRecord(e0, s);
    for (int rep = 0; rep < 10 && st == BRAS_OK; ++rep) st = pass();
    (void)hipEventRecord(e1, s);
    (void)hipEventSynchronize(e1);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best) {
      best = ms;
      pick = cands[k];
    }
  }
  c->use_patch = plan ? pick.patch : 1;
  c->variant = pick.variant;
  cg_free(c);   // captured CG graphs hold the previous kernels
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(x);
  (void)hipFree(y);
  return st;
}
