// Internal declarations shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/bras.h"
#include "patch.h"

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
// Broken vectors (and every per-element table) are stored local-index-major:
// slot (K, l) is at l*E + K (times nrhs columns, column fastest), so the 64
// lanes of a wavefront, one element each, touch consecutive addresses.

struct CgState;   // pcg.hip

struct Ctx {
  int device = 0;
  int ncu = 1;               // compute units of the device
  int64_t n = 0, E = 0, nbr = 0;
  int nl = 0;
  int form = 0, nsym = 0, prec = 0, max_rhs = 1;
  int variant = -1;          // element-pass scheduling variant (-1: built-in choice)
  int graph_iters = 32;      // most CG / stationary iterations launched between two host checks
  int max_restart = 8;
  int small_cg = 1;          // solve eligible small problems in one work-group (pcg_small.hip)
  int use_patch = 1;         // one-column operator passes in patch form when the handle has a plan (patch.hip)
  int patch_xcd = 1;         // patch passes: each XCD takes a contiguous run of patches (BRAS_PATCH_XCD=0: round robin)
  int flexible_opt = -1;     // BRAS-PCG beta: -1 flexible for BF16 inverses only, 0 never, 1 for FP32 / BF16
  int bf16_direct = 1;       // BF16 plain applies write single-copy DOFs from the element pass (BRAS_BF16_DIRECT=0: off)
  int bf16_grid = 0;         // BF16 element pass with that epilogue: persistent work-groups (0: other precisions)
  int bf16_grid_plain = 0;   // BF16 element pass without it (one input vector)
  int bf16_grid_x2 = 0;      // BF16 element pass with input r - alpha q (CG)
  int32_t* l2g_dir = nullptr;   // [E][n_loc] l2g with bit 31 set on single-copy DOFs (BF16 with the epilogue)
  int ip_mode = 0;           // 1 while a patch-form solve runs: operator passes address vectors in the
                             // internal DOF numbering of the patch plan (PatchDev::ip2g)
  int last_path = 0;         // path of the last pcg_solve: 0 multi-pass, 1 one work-group
  int64_t last_restarts = 0;

  // maps
  int32_t* l2g = nullptr;    // [E][nl]
  int32_t* mult = nullptr;   // [n]
  double* invd = nullptr;    // [n]
  int32_t* rowptr = nullptr; // [n+1]
  int32_t* chunk = nullptr;  // [nchunk+1] first DOF of each reduce chunk (<= 512 rows, <= 2048 copies)
  int64_t nchunk = 0;
  int32_t* slot = nullptr;   // [nbr] internal index l*E + K of each copy, rows ordered by K*nl + l

  // element data
  double* ref = nullptr;     // SCALED_REF: Mhat [nl*nl]; METRIC_REF: S [nsym][nl*nl]
  double* refinv = nullptr;  // SCALED_REF: Mhat^-1 [nl*nl]
  double* coef = nullptr;    // SCALED_REF: c_K [E]; METRIC_REF: G [nsym][E]
  double* icoef = nullptr;   // SCALED_REF: 1 / c_K [E]
  void* ainv = nullptr;      // METRIC/EXPLICIT: folded inverse, packed lower [npack][E] in prec,
                             // or (BF16) the Gram factor, packed lower, element-major [E][npack]
  size_t ainv_bytes = 0;
  int agroup = 0;            // layout of ainv (packed_group; 0 = element-major, also for the BF16 factor)
  int mgroup = 0;            // layout of mpack
  double* symtab = nullptr;  // METRIC_REF, n_loc <= kLaneMaxNL: pair tables packed [npack][sym_stride(nsym)]
  double* mpack = nullptr;   // packed float64 M_K [npack][E] for the mass pass (EXPLICIT, or METRIC with
                             // n_loc > kLaneMaxNL)
  PatchDev pt;               // patch plan (npatch == 0: none); element order is then patch-major
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

// Largest n_loc whose element passes keep a whole element in one lane's registers.
constexpr int kLaneMaxNL = 36;
// Scheduling variants of the 3D metric-form mass pass offered to bras_autotune.
constexpr int kMetricVariants = 3;
// Packed per-element matrices (q = i(i+1)/2 + j, i >= j) are stored either
// in groups of g consecutive entries (g = 16 bytes / entry size, for the
// per-lane pass, n_loc <= kLaneMaxNL): entry (q, K) at ((q / g) * E + K) * g
// + q % g, the entry count padded to a multiple of g; or element-major (g = 0,
// for the per-element passes): entry (q, K) at K * npack + q.
inline int packed_group(int nl, size_t esz) { return nl <= kLaneMaxNL ? (int)(16 / esz) : 0; }
inline size_t packed_slots(int nl, int g) {
  return g == 0 ? (size_t)npack_of(nl) : (size_t)((npack_of(nl) + g - 1) / g) * g;
}
__host__ __device__ inline int64_t packed_at(int q, int64_t K, int64_t E, int g, int npk) {
  return g == 0 ? K * npk + q : ((int64_t)(q / g) * E + K) * g + q % g;
}
// Row stride of the packed pair tables: 3 (up to 3 pairs, 2D) or 6 (3D), zero padded.
inline int sym_stride(int nsym) { return nsym <= 3 ? 3 : 6; }

// Launch helpers (apply.hip).  dotv/dotpart (optional): accumulate y . dotv
// into per-block partial sums [blocks][nrhs]; active (optional): per-column
// flags, columns with active[r] == 0 are skipped.
// ws (optional): broken-vector workspace of at least broken_bytes(c, nrhs)
// bytes to use instead of the handle's own
int launch_bras(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                const int* active, void* ws = nullptr);
int launch_mass(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                const int* active);
int launch_jacobi(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv, double* dotpart,
                  const int* active);
int launch_bras_bf16(Ctx* c, const double* x, double* y, int nrhs, hipStream_t s, const double* dotv,
                     double* dotpart, const int* active, void* zb);
// bytes of broken-vector workspace one BRAS apply of nrhs columns uses
size_t broken_bytes(const Ctx* c, int nrhs);
int reduce_blocks(Ctx* c, int nrhs);   // blocks (= partials per column) of a reduce pass
int reduce_chunk_blocks(const Ctx* c, int nrhs);   // work-groups of the transpose-map reduce
// plain BF16 applies of nrhs columns write single-copy DOFs from the element pass (bf16.hip)
inline bool bf16_bypass(const Ctx* c, int nrhs) { return c->l2g_dir && nrhs <= 32; }
int bf16_setup(Ctx* c, hipStream_t s);   // persistent grids and flagged map of the BF16 element pass
int vector_blocks(Ctx* c, int nrhs);   // blocks of a grid-stride vector pass (grid * 256 % nrhs == 0)
void cg_free(Ctx* c);

// Fused CG passes (apply.hip, bf16.hip): see cg_common.h for CgArgs.
struct CgArgs;
int cg_mass_step(Ctx* c, const CgArgs& cg, int nrhs, hipStream_t s);
int cg_precond_step(Ctx* c, int pc, const CgArgs& cg, int nrhs, hipStream_t s);
int cg_bras_bf16_step(Ctx* c, const CgArgs& cg, int nrhs, hipStream_t s);
// Stationary iterations (apply.hip): r = b - M x (partial r.r); d = a d + c C r, x += d
int st_mass_step(Ctx* c, const CgArgs& cg, int nrhs, hipStream_t s);
int st_precond_step(Ctx* c, int pc, const CgArgs& cg, int nrhs, hipStream_t s);
struct InArgs;
InArgs precond_input(const CgArgs& cg, int nrhs);
int bf16_stat_step(Ctx* c, const CgArgs& cg, const InArgs& in, int nrhs, hipStream_t s);   // bf16.hip
int precond_consumer_blocks(Ctx* c, int pc, int nrhs);
int metric_variant(const Ctx* c);   // apply.hip
int variant_count(const Ctx* c);    // scheduling variants of this handle's element passes
// reduce passes over a float32 broken vector (apply.hip)
int reduce_float_plain(Ctx* c, const float* zb, double* y, int nrhs, hipStream_t s, const double* dotv,
                       double* dotpart, int skip1);
int reduce_float_cg(Ctx* c, const float* zb, int nrhs, hipStream_t s, const CgArgs& cg);
int reduce_float_stat(Ctx* c, const float* zb, int nrhs, hipStream_t s, const CgArgs& cg);

// Single work-group PCG (pcg_small.hip): scaled H1 form, float64, one
// column, n <= kSmallMaxN, 16 n + 10 n_br <= kSmallLdsBytes (its LDS: two
// vectors, the broken vector, 16-bit transpose map), maxit <= kSmallMaxIt.
constexpr int kSmallMaxN = 2048;
constexpr int kSmallLdsBytes = 160000;
constexpr int kSmallMaxIt = 100000;
bool small_cg_eligible(const Ctx* c, int nrhs, int maxit);
int launch_small_cg(Ctx* c, int pc, const double* b, double* x, double rtol, int maxit, double* sc, int* ic,
                    hipStream_t s);
// damped fixed point / Chebyshev with the coefficient table coef [2][cap]
int launch_small_stationary(Ctx* c, int pc, const double* b, double* x, double rtol, int maxit, const double* coef,
                            int cap, double* sc, int* ic, hipStream_t s);

// fixed workspace of bras_apply_noalloc (noalloc.hip): its device address on
// dev (current), looked up once per device
int scratch_init(int dev, void** out);

// Patch form of the one-column operator passes (patch.hip): op 0 mass, 1
// BRAS; out one of OUT_* (cg_common.h); ws (optional) replaces the handle's
// buffer of shared-DOF partial sums (patch_workspace_bytes).  Dot partials:
// patch_blocks per column.
bool patch_supported(int form, int prec, int nl);
bool patch_active(const Ctx* c, int nrhs);
int patch_blocks(const Ctx* c);
size_t patch_workspace_bytes(const Ctx* c);
int patch_pass(Ctx* c, int op, int out, const InArgs& in, double* y, const double* dotv, double* dotpart,
               const CgArgs& cg, hipStream_t s, double* ws = nullptr);

// setup internals (setup.hip)
int element_setup(Ctx* c, const double* elem_d, hipStream_t s);

}  // namespace bras
