// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bras.h"

namespace bras {

// ---- error reporting (thread-local message, status codes of bras.h) -------
int fail(int code, const char* fmt, ...);
void clear_error();

#define BRAS_HIP(call)                                                           \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return ::bras::fail(BRAS_EHIP, "%s failed: %s (%s:%d)", #call,              \
                          hipGetErrorString(e_), __FILE__, __LINE__);            \
  } while (0)

#define BRAS_CHECK(cond, ...)                                                    \
  do {                                                                           \
    if (!(cond)) return ::bras::fail(BRAS_EINVAL, __VA_ARGS__);                  \
  } while (0)

// ---- host finite-element helpers (host_mesh.cpp, host_fe.cpp) -------------
int element_counts(int family, int dim, int degree, int* n_loc, int counts[4]);
int nsym_of(int dim);

// ---- device state ---------------------------------------------------------
// Broken vectors live in "element-fastest" order: slot (K, l) is at l*E + K, so
// a thread owning element K touches consecutive addresses across a wavefront.

struct CgState;   // pcg.hip

struct Ctx {
  int device = 0;
  int64_t n = 0, E = 0, nbr = 0;
  int nl = 0;
  int form = 0, nsym = 0, prec = 0, max_rhs = 1;
  int variant = -1;          // apply kernel variant (-1: default)
  int graph_iters = 8;
  int max_restart = 8;
  int64_t last_restarts = 0;

  // maps
  int32_t* l2gT = nullptr;   // [nl][E]
  int32_t* mult = nullptr;   // [n]
  double* invd = nullptr;    // [n]
  int32_t* rowptr = nullptr; // [n+1]
  int32_t* slot = nullptr;   // [nbr] internal broken index l*E + K, rows ascending by K*nl + l

  // element data
  double* ref = nullptr;     // SCALED_REF: Mhat [nl*nl]; METRIC_REF: S [nsym][nl*nl]
  double* refinv = nullptr;  // SCALED_REF: Mhat^-1 [nl*nl]
  double* coef = nullptr;    // SCALED_REF: c_K [E]; METRIC_REF: G [nsym][E]; EXPLICIT: packed M_K [npack][E]
  double* icoef = nullptr;   // SCALED_REF: 1 / c_K [E]
  void* ainv = nullptr;      // METRIC/EXPLICIT: folded inverse, packed lower [npack][E] in prec,
                             // or (BF16) the Gram factor in MFMA tile layout
  size_t ainv_bytes = 0;
  double* diag = nullptr;    // diag(M) [n]
  double* invdiag = nullptr; // [n]

  // workspace
  void* zb = nullptr;        // broken vector, nbr * max_rhs float64 (viewed as float32 by reduced-precision passes)
  double* partial = nullptr; // reduction partials
  int* flag = nullptr;       // device error flag / element index
  CgState* cg = nullptr;
  hipStream_t s_int = nullptr;
};

inline int npack_of(int nl) { return nl * (nl + 1) / 2; }

// Launch helpers (apply.hip).  dotv/dotpart (optional): accumulate y . dotv
// into per-block partial sums [blocks][nrhs]; active (optional): per-column
// flags, columns with active[r] == 0 are skipped.
int launch_bras(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                const int* active);
int launch_mass(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                const int* active);
int launch_jacobi(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                  const int* active);
int launch_bras_bf16(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv,
                     double* dotpart, const int* active);
int reduce_blocks(Ctx* c, int nrhs);
void cg_free(Ctx* c);

// setup internals (setup.hip)
int element_setup(Ctx* c, const double* elem_d, hipStream_t s);

}  // namespace bras
