// BRAS apply for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid hipMalloc): the
// same kernels as bras_apply, with the broken-vector workspace taken from a
// fixed device array of this file instead of the handle's own buffer.
//
// The array is a host-side symbol: its device address is obtained once per
// device with hipGetSymbolAddress (at bras_setup, with that device current)
// and only that address is ever passed to kernels.  Every call on a device
// shares the array; the element pass overwrites every entry the reduce reads,
// so nothing needs clearing between calls, but two calls that overlap on one
// device (different streams, no ordering) race on it.
#include <mutex>

#include "internal.h"

namespace bras {

constexpr size_t kScratchBytes = BRAS_NOALLOC_SCRATCH_BYTES;   // per device, held until the process ends
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of the scratch array on `dev` (which must be current).
int scratch_init(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(BRAS_EINVAL, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(BRAS_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  if (out) *out = g_scratch_ptr[dev];
  return BRAS_OK;
}

}  // namespace bras

using namespace bras;

extern "C" int bras_apply_noalloc(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream) {
  clear_error();
  BRAS_CHECK(h, "null handle");
  BRAS_CHECK(x_d && y_d, "null vector");
  BRAS_CHECK(x_d != y_d, "x and y must be distinct buffers");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs %d outside 1..max_rhs=%d", nrhs, c->max_rhs);
  int dev = -1;
  BRAS_HIP(hipGetDevice(&dev));
  BRAS_CHECK(dev == c->device, "the handle belongs to device %d, device %d is current", c->device, dev);
  const size_t need = broken_bytes(c, nrhs);
  BRAS_CHECK(need <= kScratchBytes,
             "bras_apply_noalloc needs %zu bytes of workspace for %d column(s) (%lld broken DOFs), above its "
             "fixed %zu-byte array; use bras_apply",
             need, nrhs, (long long)c->nbr, kScratchBytes);
  void* ws = nullptr;
  int st = scratch_init(dev, &ws);   // set at bras_setup: no runtime call beyond a lookup here
  if (st) return st;
  return launch_bras(c, x_d, y_d, nrhs, (hipStream_t)stream, nullptr, nullptr, nullptr, ws);
}
