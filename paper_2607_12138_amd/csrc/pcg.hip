// Preconditioned conjugate gradients (Section 3), one independent CG per
// column, entirely on the device:
//
//   x = x0; r = b - M x; z = C r; p = 0; beta = 0; rho = r.z
//   repeat: p = z + beta p; q = M p; alpha = rho / p.q;
//           x += alpha p; r -= alpha q; stop when ||r|| <= rtol ||r_0||
//           (or after maxit products M p); z = C r; rho' = r.z;
//           beta = rho'/rho; rho = rho'
//
// Each iteration is two fused operator passes (apply.hip; for one column on
// a handle with a patch plan, each pass is a patch pass and a boundary-DOF
// pass, patch_kern.h, run on vectors permuted into the plan's internal DOF
// numbering) and one or two one-block kernels:
//   mass pass    element pass on z + beta p, reduce pass writes q and the new
//                p and the p.q partials;
//   alpha        alpha = rho / p.q, in a one-block kernel on large meshes or
//                in the prologue of the next pass's work-groups on small ones;
//   precond pass element pass on r - alpha q (BRAS), reduce pass updates x and
//                r, writes z and the r.r, r.z partials (Jacobi / none: one
//                vector pass);
//   finish       one block: ||r||, the stopping test, beta and rho.
// Scalars and convergence flags stay in device memory; every dot product is
// a fixed-order two-stage reduction, so results are bitwise reproducible.
// Iterations are captured into hipGraphs of 1, 2, 4, 8, 16 and 32
// iterations; columns that have stopped are skipped by every kernel, and the
// host reads the flags only between graph launches.  When the stored BRAS
// inverses are BF16 (FP32 with BRAS_OPT_FLEXIBLE 1) the flexible beta = r_new.(z_new - z_old)/rho_old
// is used and, at exit, CG restarts from x while the true residual is above
// the tolerance.  The fixed-point and Chebyshev iterations at the end of this
// file share the passes and the graph machinery.  Small single-column
// problems of the scaled H1 form run the same iteration in one work-group
// instead (pcg_small.hip).
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "internal.h"
#include "block_reduce.h"
#include "cg_common.h"

namespace bras {

constexpr int kBS = 256;
constexpr int kNumGraphs = 6;   // 1, 2, 4, 8, 16, 32 iterations


struct CgState {
  int R = 0;
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double* sc = nullptr;      // [S_NSC][R], followed in the same allocation by
  int* ic = nullptr;         // [I_NIC][R]
  double* part[4] = {nullptr, nullptr, nullptr, nullptr};   // partials [blocks][R]: r.r, r.z, r.z_old, p.q
  double* sc_host = nullptr; // pinned copy of sc and ic (same layout)
  int* ic_host = nullptr;
  double* stcoef = nullptr;  // stationary iterations: a_k [cap], then c_k [cap]
  int stcoef_cap = 0;
  struct Key {
    int kind, pc, flexible, maxit;   // kind 0: CG, 1: stationary iteration
    bool operator<(const Key& o) const {
      if (kind != o.kind) return kind < o.kind;
      if (pc != o.pc) return pc < o.pc;
      if (flexible != o.flexible) return flexible < o.flexible;
      return maxit < o.maxit;
    }
  };
  std::map<Key, std::vector<hipGraphExec_t>> graphs;
};

// r = b - q (q = M x), partial r.r
__global__ void __launch_bounds__(kBS) k_residual(int64_t n, int R, const double* __restrict__ b,
                                                  const double* __restrict__ q, double* __restrict__ r,
                                                  double* __restrict__ partial) {
  __shared__ double sh[kBS];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double dot = 0.0;
  for (int64_t t = t0; t < n * R; t += stride) {
    const double v = b[t] - q[t];
    r[t] = v;
    dot = fma(v, v, dot);
  }
  sh[threadIdx.x] = dot;
  block_partials(sh, R, partial);
}

// Start (or restart) of CG.  restart == 0: r_0 norm and target are set from
// this residual.  Columns already within target are stopped.
__global__ void __launch_bounds__(kBS) k_fin_init(int nb, int R, const double* __restrict__ part,
                                                  double* __restrict__ sc, int* __restrict__ ic, double rtol,
                                                  int restart) {
  __shared__ double sh[kBS], rr_s[256];
  block_sums_all(part, nb, R, rr_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    const double rr = rr_s[col];
    const double nrm = sqrt(rr);
    if (!restart) {
      sc[S_R0 * R + col] = nrm;
      sc[S_TARGET * R + col] = rtol * nrm;
      ic[I_ITERS * R + col] = 0;
    }
    sc[S_RR * R + col] = rr;
    const double r0 = sc[S_R0 * R + col];
    sc[S_RELRES * R + col] = r0 > 0.0 ? nrm / r0 : 0.0;
    if (!isfinite(nrm)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else if (nrm <= sc[S_TARGET * R + col] || nrm == 0.0) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_OK;
    } else {
      ic[I_ACTIVE * R + col] = 1;
      ic[I_STATUS * R + col] = ST_RUN;
    }
  }
}

// rho = r.z after the first preconditioner application (p = 0, beta = 0).
__global__ void __launch_bounds__(kBS) k_fin_rz(int nb, int R, const double* __restrict__ part,
                                                double* __restrict__ sc, int* __restrict__ ic) {
  __shared__ double sh[kBS], rz_s[256];
  block_sums_all(part, nb, R, rz_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    if (!ic[I_ACTIVE * R + col]) continue;
    const double rz = rz_s[col];
    sc[S_RZ * R + col] = rz;
    sc[S_BETA * R + col] = 0.0;
    if (!(rz > 0.0) || !isfinite(rz)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    }
  }
}

__global__ void __launch_bounds__(kBS) k_set_int(int* __restrict__ v, int n, int value) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) v[t] = value;
}

__global__ void __launch_bounds__(kBS) k_zero(int64_t n, double* __restrict__ v) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = t0; t < n; t += stride) v[t] = 0.0;
}

// alpha = rho / p.q for every running column (one block); used instead of the
// consumers' prologue when every consumer work-group re-reading the partials
// would cost more than this extra launch
__global__ void __launch_bounds__(kBS) k_fin_alpha(int nb, int R, const double* __restrict__ part,
                                                   double* __restrict__ sc, int* __restrict__ ic) {
  __shared__ double sh[kBS], pq_s[256];
  block_sums_all(part, nb, R, pq_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    if (!ic[I_ACTIVE * R + col]) continue;
    const double pq = pq_s[col];
    if (!(pq > 0.0) || !isfinite(pq)) {
      sc[S_ALPHA * R + col] = 0.0;
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else {
      sc[S_ALPHA * R + col] = sc[S_RZ * R + col] / pq;
    }
  }
}

// partial sums the alpha prologues of one iteration may re-read before a
// separate alpha kernel is cheaper
constexpr double kPrologueReadsMax = 4.0e6;

// convergence test, beta and rho after the preconditioner pass of an iteration
__global__ void __launch_bounds__(kBS) k_fin_iter(int nb, int R, const double* __restrict__ p0,
                                                  const double* __restrict__ p1, const double* __restrict__ p2,
                                                  double* __restrict__ sc, int* __restrict__ ic, int flexible,
                                                  int maxit) {
  __shared__ double sh[kBS], rr[256], rz[256], rzo[256];
  finish_iteration(p0, p1, p2, nb, R, sc, ic, flexible, maxit, sh, rr, rz, rzo);
}

// true residual norm at exit: relres = ||b - M x|| / ||r_0||
__global__ void __launch_bounds__(kBS) k_fin_true(int nb, int R, const double* __restrict__ part,
                                                  double* __restrict__ sc) {
  __shared__ double sh[kBS], rr_s[256];
  block_sums_all(part, nb, R, rr_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    const double r0 = sc[S_R0 * R + col];
    sc[S_RELRES * R + col] = r0 > 0.0 ? sqrt(rr_s[col]) / r0 : 0.0;
  }
}

void cg_free(Ctx* c) {
  CgState* g = c->cg;
  if (!g) return;
  for (auto& kv : g->graphs)
    for (auto ge : kv.second) (void)hipGraphExecDestroy(ge);
  double* bufs[] = {g->b, g->x, g->r, g->z, g->p, g->q, g->sc, g->part[0], g->part[1], g->part[2], g->part[3],
                    g->stcoef};
  for (double* p : bufs)
    if (p) (void)hipFree(p);
  if (g->sc_host) (void)hipHostFree(g->sc_host);   // ic and ic_host live in the sc blocks
  delete g;
  c->cg = nullptr;
}

// Vectors into / out of the internal DOF numbering of a patch plan:
// in: dst[i] = src[ip2g[i]]; out: dst[ip2g[i]] = src[i].
__global__ void __launch_bounds__(kBS) k_perm_in(int64_t n, const int32_t* __restrict__ ip2g,
                                                 const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[ip2g[i]];
}
__global__ void __launch_bounds__(kBS) k_perm_out(int64_t n, const int32_t* __restrict__ ip2g,
                                                  const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[ip2g[i]] = src[i];
}

// A solve's vectors (b, x) enter the CG state, and x leaves it, in the
// caller's numbering or, when the one-column passes run in patch form, in the
// plan's internal numbering (c->ip_mode is set for the duration of the solve,
// including graph capture).
struct SolveNumbering {
  Ctx* c;
  bool ip;
  SolveNumbering(Ctx* c_, int R) : c(c_), ip(patch_active(c_, R)) { c->ip_mode = ip ? 1 : 0; }
  ~SolveNumbering() { c->ip_mode = 0; }
  int in(const double* src, double* dst, size_t bytes, hipStream_t s) const {
    if (!ip) {
      BRAS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
      return BRAS_OK;
    }
    k_perm_in<<<(unsigned)((c->n + kBS - 1) / kBS), kBS, 0, s>>>(c->n, c->pt.ip2g, src, dst);
    BRAS_HIP(hipGetLastError());
    return BRAS_OK;
  }
  int out(const double* src, double* dst, size_t bytes, hipStream_t s) const {
    if (!ip) {
      BRAS_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
      return BRAS_OK;
    }
    k_perm_out<<<(unsigned)((c->n + kBS - 1) / kBS), kBS, 0, s>>>(c->n, c->pt.ip2g, src, dst);
    BRAS_HIP(hipGetLastError());
    return BRAS_OK;
  }
};

static size_t state_bytes(int R) { return sizeof(double) * S_NSC * R + sizeof(int) * I_NIC * R; }

static int cg_alloc(Ctx* c, int R) {
  if (c->cg && c->cg->R == R) return BRAS_OK;
  cg_free(c);
  CgState* g = new CgState();
  c->cg = g;
  g->R = R;
  const size_t vec = sizeof(double) * (size_t)c->n * R;
  double** vs[] = {&g->b, &g->x, &g->r, &g->z, &g->p, &g->q};
  for (double** v : vs)
    if (hipMalloc((void**)v, vec) != hipSuccess) return fail(BRAS_ENOMEM, "CG workspace allocation failed");
  // scalars and flags in one block (one copy reads both back)
  if (hipMalloc((void**)&g->sc, state_bytes(R)) != hipSuccess) return fail(BRAS_ENOMEM, "CG scalar allocation failed");
  g->ic = (int*)(g->sc + S_NSC * R);
  const int nb_r = reduce_blocks(c, R), nb_v = vector_blocks(c, R);
  const int nb = nb_r > nb_v ? nb_r : nb_v;
  for (int k = 0; k < 4; ++k)
    if (hipMalloc((void**)&g->part[k], sizeof(double) * (size_t)nb * R) != hipSuccess)
      return fail(BRAS_ENOMEM, "CG partial allocation failed");
  if (hipHostMalloc((void**)&g->sc_host, state_bytes(R), hipHostMallocDefault) != hipSuccess)
    return fail(BRAS_ENOMEM, "pinned host allocation failed");
  g->ic_host = (int*)(g->sc_host + S_NSC * R);
  return BRAS_OK;
}

__global__ void __launch_bounds__(kBS) k_identity_dot(int64_t n, int R, const double* __restrict__ r,
                                                      double* __restrict__ z, double* __restrict__ partial,
                                                      const int* __restrict__ active) {
  __shared__ double sh[kBS];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int col = (int)(t0 % R);
  double d = 0.0;
  if (!active || active[col])
    for (int64_t t = t0; t < n * R; t += stride) {
      z[t] = r[t];
      d = fma(r[t], r[t], d);
    }
  sh[threadIdx.x] = d;
  block_partials(sh, R, partial);
}

static int precond(Ctx* c, int pc, const double* r, double* z, int R, hipStream_t s, double* part, const int* active) {
  if (pc == BRAS_PC_BRAS) return launch_bras(c, r, z, R, s, r, part, active);
  if (pc == BRAS_PC_JACOBI) return launch_jacobi(c, r, z, R, s, r, part, active);
  // identity preconditioner: z = r, partial r.r
  k_identity_dot<<<vector_blocks(c, R), kBS, 0, s>>>(c->n, R, r, z, part, active);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// partials per column written by the preconditioner pass (and its start-up apply)
static int precond_blocks(Ctx* c, int pc, int R) {
  return pc == BRAS_PC_BRAS ? reduce_blocks(c, R) : vector_blocks(c, R);
}

static CgArgs cg_args(Ctx* c, int flexible, int maxit) {
  CgState* g = c->cg;
  CgArgs a;
  a.x = g->x;
  a.r = g->r;
  a.p = g->p;
  a.z = g->z;
  a.q = g->q;
  a.sc = g->sc;
  a.ic = g->ic;
  a.flexible = flexible;
  a.maxit = maxit;
  return a;
}

// One CG iteration (enqueued on s; also used under stream capture).
static int iteration(Ctx* c, int pc, int flexible, int maxit, hipStream_t s) {
  CgState* g = c->cg;
  const int R = g->R;
  CgArgs m = cg_args(c, flexible, maxit);
  m.part0 = g->part[3];                       // p.q partials
  int st = cg_mass_step(c, m, R, s);
  if (st) return st;
  CgArgs pcg = cg_args(c, flexible, maxit);
  pcg.part0 = g->part[0];                     // r.r
  pcg.part1 = g->part[1];                     // r.z
  pcg.part2 = g->part[2];                     // r.z_old (flexible)
  const int anb = reduce_blocks(c, R);
  if ((double)precond_consumer_blocks(c, pc, R) * anb * R > kPrologueReadsMax) {
    k_fin_alpha<<<1, kBS, 0, s>>>(anb, R, g->part[3], g->sc, g->ic);
    BRAS_HIP(hipGetLastError());
  } else {
    pcg.apart = g->part[3];
    pcg.anb = anb;
  }
  if ((st = cg_precond_step(c, pc, pcg, R, s))) return st;
  k_fin_iter<<<1, kBS, 0, s>>>(precond_blocks(c, pc, R), R, g->part[0], g->part[1], g->part[2], g->sc, g->ic,
                               flexible, maxit);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int start(Ctx* c, int pc, double rtol, int restart, hipStream_t s) {
  CgState* g = c->cg;
  const int R = g->R;
  const int nbv = vector_blocks(c, R);
  int st;
  if ((st = launch_mass(c, g->x, g->q, R, s, nullptr, nullptr, nullptr))) return st;
  k_residual<<<nbv, kBS, 0, s>>>(c->n, R, g->b, g->q, g->r, g->part[1]);
  k_fin_init<<<1, kBS, 0, s>>>(nbv, R, g->part[1], g->sc, g->ic, rtol, restart);
  int* active = g->ic + I_ACTIVE * R;
  if ((st = precond(c, pc, g->r, g->z, R, s, g->part[0], active))) return st;
  k_fin_rz<<<1, kBS, 0, s>>>(precond_blocks(c, pc, R), R, g->part[0], g->sc, g->ic);
  k_zero<<<nbv, kBS, 0, s>>>(c->n * R, g->p);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int read_state(Ctx* c, hipStream_t s) {
  CgState* g = c->cg;
  BRAS_HIP(hipMemcpyAsync(g->sc_host, g->sc, state_bytes(g->R), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  return BRAS_OK;
}

// Graphs of 1, 2, 4, ... iterations of one kind, captured on the idle
// internal stream before any work is queued.
template <typename F>
static int capture_graphs(Ctx* c, CgState::Key key, F one_iteration, std::vector<hipGraphExec_t>** out) {
  CgState* g = c->cg;
  auto it = g->graphs.find(key);
  if (it != g->graphs.end()) {
    *out = &it->second;
    return BRAS_OK;
  }
  std::vector<hipGraphExec_t> v;
  hipStream_t s = c->s_int;
  for (int k = 0; k < kNumGraphs; ++k) {
    const int iters = 1 << k;
    BRAS_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int st = BRAS_OK;
    for (int i = 0; i < iters && st == BRAS_OK; ++i) st = one_iteration(s);
    hipGraph_t graph;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (st) return st;
    if (e != hipSuccess) return fail(BRAS_EHIP, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ge;
    e = hipGraphInstantiate(&ge, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(BRAS_EHIP, "graph instantiation failed: %s", hipGetErrorString(e));
    v.push_back(ge);
  }
  g->graphs[key] = v;
  *out = &g->graphs[key];
  return BRAS_OK;
}

static int get_graphs(Ctx* c, int pc, int flexible, int maxit, std::vector<hipGraphExec_t>** out) {
  return capture_graphs(c, CgState::Key{0, pc, flexible, maxit},
                        [&](hipStream_t s) { return iteration(c, pc, flexible, maxit, s); }, out);
}

// Launch graphs for about `chunk` more iterations (binary decomposition).
static int launch_chunk(std::vector<hipGraphExec_t>& graphs, int chunk, hipStream_t s) {
  for (int k = kNumGraphs - 1; k >= 0; --k)
    if (chunk & (1 << k)) {
      hipError_t e = hipGraphLaunch(graphs[k], s);
      if (e != hipSuccess) return fail(BRAS_EHIP, "hipGraphLaunch failed: %s", hipGetErrorString(e));
    }
  return BRAS_OK;
}

// Iterations launched after the start of a solve before the host first
// looks at the flags (an iteration of a stopped column costs only launches).
constexpr int kFirstChunk = 8;

// Iterations to launch before the host looks at the flags again: enough to
// reach the target at the slowest running column's observed rate (1..32).
static int predict_chunk(CgState* g, int R, int maxit, int cap) {
  int any = 0, max_it = 0;
  double worst = 0.0;
  for (int col = 0; col < R; ++col) {
    if (!g->ic_host[I_ACTIVE * R + col]) continue;
    any = 1;
    const int it = g->ic_host[I_ITERS * R + col];
    max_it = it > max_it ? it : max_it;
    const double rel = g->sc_host[S_RELRES * R + col];
    const double tgt = g->sc_host[S_TARGET * R + col] / g->sc_host[S_R0 * R + col];
    if (it > 0 && rel > 0.0 && rel < 1.0) {
      const double rate = std::log(rel) / it;   // per-iteration log reduction (< 0)
      const double need = std::log(tgt / rel) / rate;
      if (need > worst) worst = need;
    } else if (4.0 > worst) {
      worst = 4.0;
    }
  }
  if (!any) return 0;
  int chunk = (int)std::ceil(worst);
  if (chunk < 1) chunk = 1;
  if (chunk > cap) chunk = cap;
  if (chunk > maxit - max_it + 1) chunk = maxit - max_it + 1;
  return chunk < 1 ? 1 : chunk;
}

}  // namespace bras

using namespace bras;

static int report(Ctx* c, int R, double rtol, int maxit, int* iters_h, double* relres_h, bool cg = true);

extern "C" int pcg_solve(bras_handle h, int pc, const double* b_d, double* x_d, int nrhs, double rtol, int maxit,
                         int* iters_h, double* relres_h, void* stream) {
  clear_error();
  BRAS_CHECK(h && b_d && x_d, "null argument");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(pc == BRAS_PC_NONE || pc == BRAS_PC_JACOBI || pc == BRAS_PC_BRAS, "unknown preconditioner %d", pc);
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs %d outside 1..max_rhs=%d", nrhs, c->max_rhs);
  BRAS_CHECK(rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
  BRAS_CHECK(maxit >= 1, "maxit must be >= 1");
  int st = cg_alloc(c, nrhs);
  if (st) return st;
  CgState* g = c->cg;
  hipStream_t us = (hipStream_t)stream, s = c->s_int;
  const size_t vec = sizeof(double) * (size_t)c->n * nrhs;
  // graphs are captured on the idle internal stream before any work is queued
  // flexible beta: BF16 inverses (a perturbation at the 2^-9 level), or FP32
  // on request; FP32 inverses are a fixed symmetric matrix applied with
  // float32 rounding (2^-24), for which the standard beta keeps the counts
  const int flexible = (pc != BRAS_PC_BRAS || c->prec == BRAS_FP64)
                           ? 0
                           : (c->flexible_opt >= 0 ? c->flexible_opt : (c->prec == BRAS_BF16 ? 1 : 0));
  // small single-column problems: the whole solve in one work-group, on the
  // caller's stream (no graphs, so no internal stream)
  if (small_cg_eligible(c, nrhs, maxit)) {
    c->last_path = 1;
    c->last_restarts = 0;
    if ((st = launch_small_cg(c, pc, b_d, x_d, rtol, maxit, g->sc, g->ic, us))) return st;
    if ((st = read_state(c, us))) return st;
    return report(c, nrhs, rtol, maxit, iters_h, relres_h);
  }
  c->last_path = 0;
  const SolveNumbering num(c, nrhs);
  std::vector<hipGraphExec_t>* graphs = nullptr;
  if ((st = get_graphs(c, pc, flexible, maxit, &graphs))) return st;
  // order the internal stream after the caller's prior work
  hipEvent_t ev;
  BRAS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  BRAS_HIP(hipEventRecord(ev, us));
  BRAS_HIP(hipStreamWaitEvent(s, ev, 0));
  if ((st = num.in(b_d, g->b, vec, s)) || (st = num.in(x_d, g->x, vec, s))) {
    (void)hipEventDestroy(ev);
    return st;
  }
  const int R = nrhs;
  const int nb = vector_blocks(c, R);
  int restarts = 0;
  int restart_mode = 0;
  while (true) {
    if ((st = start(c, pc, rtol, restart_mode, s))) break;
    // a first chunk without a host check (columns already within tolerance
    // or at maxit skip its iterations), then the remaining iterations
    // predicted from the observed rate
    const int first = kFirstChunk < c->graph_iters ? kFirstChunk : c->graph_iters;
    if ((st = launch_chunk(*graphs, first < maxit ? first : maxit, s))) break;
    if ((st = read_state(c, s))) break;
    while (true) {
      const int chunk = predict_chunk(g, R, maxit, c->graph_iters);
      if (chunk == 0) break;
      if ((st = launch_chunk(*graphs, chunk, s))) break;
      if ((st = read_state(c, s))) break;
    }
    if (st) break;
    // true residual
    if ((st = launch_mass(c, g->x, g->q, R, s, nullptr, nullptr, nullptr))) break;
    k_residual<<<nb, kBS, 0, s>>>(c->n, R, g->b, g->q, g->z, g->part[1]);
    k_fin_true<<<1, kBS, 0, s>>>(nb, R, g->part[1], g->sc);
    // x goes out with this check (one host wait); a restart writes it again
    if ((st = num.out(g->x, x_d, vec, s))) break;
    if ((st = read_state(c, s))) break;
    bool again = false;
    for (int col = 0; col < R; ++col)
      if (g->ic_host[I_STATUS * R + col] == ST_OK && g->sc_host[S_RELRES * R + col] > rtol &&
          g->ic_host[I_ITERS * R + col] < maxit)
        again = true;
    if (!again || restarts >= c->max_restart) break;
    ++restarts;
    restart_mode = 1;
  }
  c->last_restarts = restarts;
  if (st == BRAS_OK) {
    BRAS_HIP(hipEventRecord(ev, s));
    BRAS_HIP(hipStreamWaitEvent(us, ev, 0));
    BRAS_HIP(hipStreamSynchronize(s));
  }
  (void)hipEventDestroy(ev);
  if (st) return st;
  return report(c, R, rtol, maxit, iters_h, relres_h);
}

// Per-column results of the last solve (host copies of the state): iteration
// counts, true relative residuals, and the status code of the call.
static int report(Ctx* c, int R, double rtol, int maxit, int* iters_h, double* relres_h, bool cg) {
  CgState* g = c->cg;
  int result = BRAS_OK;
  int true_miss = -1;
  for (int col = 0; col < R; ++col) {
    if (iters_h) iters_h[col] = g->ic_host[I_ITERS * R + col];
    const double rel = g->sc_host[S_RELRES * R + col];
    if (relres_h) relres_h[col] = rel;
    const int cs = g->ic_host[I_STATUS * R + col];
    if (cs == ST_BREAK) result = BRAS_EBREAKDOWN;
    else if (cs == ST_NOCONV && result == BRAS_OK) result = BRAS_ENOCONV;
    else if (cs == ST_OK && !(rel <= rtol) && true_miss < 0) true_miss = col;
  }
  if (result == BRAS_EBREAKDOWN)
    return fail(result, cg ? "PCG breakdown (p.q <= 0, r.z <= 0 or non-finite values)" : "non-finite residual");
  if (result == BRAS_ENOCONV)
    return fail(result, "%sdid not reach rtol=%g within maxit=%d", cg ? "PCG " : "", rtol, maxit);
  if (true_miss >= 0)
    return fail(BRAS_ENOCONV, "column %d: true relative residual %.3e above rtol=%g after %lld restart(s)", true_miss,
                g->sc_host[S_RELRES * R + true_miss], rtol, (long long)c->last_restarts);
  return BRAS_OK;
}

// ===========================================================================
// Stationary iterations with the same operators (Section 3): the damped
// fixed point u_{k+1} = u_k + omega C (f - M u_k) and the Chebyshev
// semi-iteration on a spectral interval [lmin, lmax] of C M, both written as
//     r_k = f - M u_k;  stop if ||r_k|| <= rtol ||r_0||;
//     d_k = a_k d_{k-1} + c_k C r_k;  u_{k+1} = u_k + d_k
// with coefficient sequences computed on the host (fixed point: a_k = 0,
// c_k = omega; Chebyshev: the three-term recurrence of the Chebyshev
// polynomials on [lmin, lmax]).  No dot products other than ||r_k||.
// ===========================================================================
namespace bras {

// start: r_0 norm and target; coefficients of update 0
__global__ void __launch_bounds__(kBS) k_st_init(int nb, int R, const double* __restrict__ part,
                                                 double* __restrict__ sc, int* __restrict__ ic, double rtol,
                                                 const double* __restrict__ coef, int cap) {
  __shared__ double sh[kBS], rr_s[256];
  block_sums_all(part, nb, R, rr_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    const double nrm = sqrt(rr_s[col]);
    sc[S_R0 * R + col] = nrm;
    sc[S_TARGET * R + col] = rtol * nrm;
    sc[S_RELRES * R + col] = nrm > 0.0 ? 1.0 : 0.0;
    ic[I_ITERS * R + col] = 0;
    if (!isfinite(nrm)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else if (nrm == 0.0) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_OK;
    } else {
      ic[I_ACTIVE * R + col] = 1;
      ic[I_STATUS * R + col] = ST_RUN;
      sc[S_ALPHA * R + col] = coef[0];
      sc[S_BETA * R + col] = coef[cap];
    }
  }
}

// after update k (= iters so far + 1): residual test, next coefficients
__global__ void __launch_bounds__(kBS) k_st_fin(int nb, int R, const double* __restrict__ part,
                                                double* __restrict__ sc, int* __restrict__ ic,
                                                const double* __restrict__ coef, int cap, int maxit) {
  __shared__ double sh[kBS], rr_s[256];
  block_sums_all(part, nb, R, rr_s, sh);
  for (int col = threadIdx.x; col < R; col += kBS) {
    if (!ic[I_ACTIVE * R + col]) continue;
    const int it = ic[I_ITERS * R + col] + 1;
    ic[I_ITERS * R + col] = it;
    const double nrm = sqrt(rr_s[col]);
    sc[S_RR * R + col] = rr_s[col];
    sc[S_RELRES * R + col] = nrm / sc[S_R0 * R + col];
    if (!isfinite(nrm)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else if (nrm <= sc[S_TARGET * R + col]) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_OK;
    } else if (it >= maxit) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_NOCONV;
    } else {
      sc[S_ALPHA * R + col] = coef[it];
      sc[S_BETA * R + col] = coef[cap + it];
    }
  }
}

static CgArgs st_args(Ctx* c) {
  CgState* g = c->cg;
  CgArgs a;
  a.x = g->x;
  a.r = g->r;
  a.p = g->p;   // d
  a.b = g->b;
  a.sc = g->sc;
  a.ic = g->ic;
  a.part0 = g->part[0];
  return a;
}

static int st_iteration(Ctx* c, int pc, int maxit, hipStream_t s) {
  CgState* g = c->cg;
  const int R = g->R;
  CgArgs a = st_args(c);
  int st = st_precond_step(c, pc, a, R, s);
  if (st) return st;
  if ((st = st_mass_step(c, a, R, s))) return st;
  k_st_fin<<<1, kBS, 0, s>>>(reduce_blocks(c, R), R, g->part[0], g->sc, g->ic, g->stcoef, g->stcoef_cap, maxit);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// Common driver; ca, cc: host coefficient sequences of length maxit.
static int stationary(Ctx* c, int pc, const std::vector<double>& ca, const std::vector<double>& cc,
                      const double* b_d, double* x_d, int nrhs, double rtol, int maxit, int* iters_h,
                      double* relres_h, void* stream) {
  int st = cg_alloc(c, nrhs);
  if (st) return st;
  CgState* g = c->cg;
  hipStream_t us = (hipStream_t)stream, s = c->s_int;
  const int R = nrhs;
  const size_t vec = sizeof(double) * (size_t)c->n * R;
  if (g->stcoef_cap < maxit) {
    // a larger table moves: drop the stationary graphs that point at the old one
    for (auto it = g->graphs.begin(); it != g->graphs.end();) {
      if (it->first.kind == 1) {
        for (auto ge : it->second) (void)hipGraphExecDestroy(ge);
        it = g->graphs.erase(it);
      } else {
        ++it;
      }
    }
    if (g->stcoef) (void)hipFree(g->stcoef);
    g->stcoef = nullptr;
    g->stcoef_cap = 0;
    if (hipMalloc((void**)&g->stcoef, sizeof(double) * 2 * (size_t)maxit) != hipSuccess)
      return fail(BRAS_ENOMEM, "coefficient table allocation failed");
    g->stcoef_cap = maxit;
  }
  std::vector<double> tab(2 * (size_t)g->stcoef_cap, 0.0);
  for (int k = 0; k < maxit; ++k) {
    tab[k] = ca[k];
    tab[g->stcoef_cap + k] = cc[k];
  }
  // small single-column problems: the whole iteration in one work-group, on
  // the caller's stream
  if (small_cg_eligible(c, nrhs, maxit)) {
    c->last_path = 1;
    BRAS_HIP(hipMemcpyAsync(g->stcoef, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, us));
    if ((st = launch_small_stationary(c, pc, b_d, x_d, rtol, maxit, g->stcoef, g->stcoef_cap, g->sc, g->ic, us)))
      return st;
    if ((st = read_state(c, us))) return st;
    return report(c, R, rtol, maxit, iters_h, relres_h, false);
  }
  c->last_path = 0;
  const SolveNumbering num(c, nrhs);
  std::vector<hipGraphExec_t>* graphs = nullptr;
  if ((st = capture_graphs(c, CgState::Key{1, pc, 0, maxit}, [&](hipStream_t ss) { return st_iteration(c, pc, maxit, ss); },
                           &graphs)))
    return st;
  hipEvent_t ev;
  BRAS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  BRAS_HIP(hipEventRecord(ev, us));
  BRAS_HIP(hipStreamWaitEvent(s, ev, 0));
  BRAS_HIP(hipMemcpyAsync(g->stcoef, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, s));
  if ((st = num.in(b_d, g->b, vec, s)) || (st = num.in(x_d, g->x, vec, s))) {
    (void)hipEventDestroy(ev);
    return st;
  }
  const int nbv = vector_blocks(c, R);
  k_zero<<<nbv, kBS, 0, s>>>(c->n * R, g->p);
  k_set_int<<<1, kBS, 0, s>>>(g->ic + I_ACTIVE * R, R, 1);   // every column takes part in the first residual
  BRAS_HIP(hipGetLastError());
  CgArgs a = st_args(c);
  if ((st = st_mass_step(c, a, R, s)) == BRAS_OK) {
    k_st_init<<<1, kBS, 0, s>>>(reduce_blocks(c, R), R, g->part[0], g->sc, g->ic, rtol, g->stcoef, g->stcoef_cap);
    // as in pcg_solve: a first chunk before the first host check
    const int first = kFirstChunk < c->graph_iters ? kFirstChunk : c->graph_iters;
    st = launch_chunk(*graphs, first < maxit ? first : maxit, s);
    if (st == BRAS_OK) st = read_state(c, s);
  }
  while (st == BRAS_OK) {
    const int chunk = predict_chunk(g, R, maxit, c->graph_iters);
    if (chunk == 0) break;
    if ((st = launch_chunk(*graphs, chunk, s))) break;
    st = read_state(c, s);
  }
  if (st == BRAS_OK) {
    st = num.out(g->x, x_d, vec, s);
    (void)hipEventRecord(ev, s);
    (void)hipStreamWaitEvent(us, ev, 0);
    (void)hipStreamSynchronize(s);
  }
  (void)hipEventDestroy(ev);
  if (st) return st;
  return report(c, R, rtol, maxit, iters_h, relres_h, false);
}

static int check_stationary(bras_handle h, int pc, const double* b_d, double* x_d, int nrhs, double rtol, int maxit) {
  BRAS_CHECK(h && b_d && x_d, "null argument");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(pc == BRAS_PC_JACOBI || pc == BRAS_PC_BRAS, "preconditioner must be BRAS_PC_JACOBI or BRAS_PC_BRAS");
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs %d outside 1..max_rhs=%d", nrhs, c->max_rhs);
  BRAS_CHECK(rtol > 0.0 && rtol < 1.0, "rtol must be in (0, 1)");
  BRAS_CHECK(maxit >= 1 && maxit <= 1000000, "maxit must be in 1..1e6");
  return BRAS_OK;
}

// y = a x (grid-stride)
__global__ void __launch_bounds__(kBS) k_scale(int64_t n, double a, const double* __restrict__ x,
                                               double* __restrict__ y) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = t0; t < n; t += stride) y[t] = a * x[t];
}

// partial sums of x . y per block
__global__ void __launch_bounds__(kBS) k_dot(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
                                             double* __restrict__ partial) {
  __shared__ double sh[kBS];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double d = 0.0;
  for (int64_t t = t0; t < n; t += stride) d = fma(x[t], y[t], d);
  sh[threadIdx.x] = d;
  block_partials(sh, 1, partial);
}

static int host_sum(const double* part_d, int nb, hipStream_t s, double* out) {
  std::vector<double> h(nb);
  BRAS_HIP(hipMemcpyAsync(h.data(), part_d, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  double v = 0.0;
  for (int b = 0; b < nb; ++b) v += h[b];   // fixed order
  *out = v;
  return BRAS_OK;
}

}  // namespace bras

extern "C" int bras_lambda_max(bras_handle h, int pc, const double* v0_d, int iters, double* lambda_h,
                               void* stream) {
  clear_error();
  BRAS_CHECK(h && v0_d && lambda_h, "null argument");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(pc == BRAS_PC_JACOBI || pc == BRAS_PC_BRAS, "preconditioner must be BRAS_PC_JACOBI or BRAS_PC_BRAS");
  BRAS_CHECK(iters >= 1, "iters must be >= 1");
  int st = cg_alloc(c, 1);
  if (st) return st;
  CgState* g = c->cg;
  hipStream_t us = (hipStream_t)stream, s = c->s_int;
  hipEvent_t ev;
  BRAS_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  BRAS_HIP(hipEventRecord(ev, us));
  BRAS_HIP(hipStreamWaitEvent(s, ev, 0));
  const int nbv = vector_blocks(c, 1);
  const int nbq = reduce_blocks(c, 1);
  const int nbw = pc == BRAS_PC_BRAS ? reduce_blocks(c, 1) : vector_blocks(c, 1);
  double vv = 0.0, lam = 0.0;
  // v = v0 / ||v0||   (v in g->x, q = M v in g->q, w = C q in g->z)
  k_dot<<<nbv, kBS, 0, s>>>(c->n, v0_d, v0_d, g->part[0]);
  st = host_sum(g->part[0], nbv, s, &vv);
  if (st == BRAS_OK && !(vv > 0.0 && std::isfinite(vv))) st = fail(BRAS_EINVAL, "start vector must be nonzero and finite");
  if (st == BRAS_OK) k_scale<<<nbv, kBS, 0, s>>>(c->n, 1.0 / std::sqrt(vv), v0_d, g->x);
  for (int k = 0; k < iters && st == BRAS_OK; ++k) {
    double qv = 0.0, wq = 0.0, ww = 0.0;
    if ((st = launch_mass(c, g->x, g->q, 1, s, g->x, g->part[0], nullptr))) break;
    st = pc == BRAS_PC_BRAS ? launch_bras(c, g->q, g->z, 1, s, g->q, g->part[1], nullptr)
                            : launch_jacobi(c, g->q, g->z, 1, s, g->q, g->part[1], nullptr);
    if (st) break;
    k_dot<<<nbv, kBS, 0, s>>>(c->n, g->z, g->z, g->part[2]);
    if ((st = host_sum(g->part[0], nbq, s, &qv)) || (st = host_sum(g->part[1], nbw, s, &wq)) ||
        (st = host_sum(g->part[2], nbv, s, &ww)))
      break;
    if (!(qv > 0.0) || !(ww > 0.0) || !std::isfinite(wq)) {
      st = fail(BRAS_EBREAKDOWN, "power iteration broke down (non-positive or non-finite products)");
      break;
    }
    lam = wq / qv;
    k_scale<<<nbv, kBS, 0, s>>>(c->n, 1.0 / std::sqrt(ww), g->z, g->x);
  }
  (void)hipEventRecord(ev, s);
  (void)hipStreamWaitEvent(us, ev, 0);
  (void)hipStreamSynchronize(s);
  (void)hipEventDestroy(ev);
  if (st) return st;
  *lambda_h = lam;
  return BRAS_OK;
}

extern "C" int fixed_point_solve(bras_handle h, int pc, double omega, const double* b_d, double* x_d, int nrhs,
                                 double rtol, int maxit, int* iters_h, double* relres_h, void* stream) {
  clear_error();
  int st = check_stationary(h, pc, b_d, x_d, nrhs, rtol, maxit);
  if (st) return st;
  BRAS_CHECK(omega > 0.0 && std::isfinite(omega), "omega must be positive");
  std::vector<double> ca(maxit, 0.0), cc(maxit, omega);
  return stationary((Ctx*)h, pc, ca, cc, b_d, x_d, nrhs, rtol, maxit, iters_h, relres_h, stream);
}

extern "C" int chebyshev_solve(bras_handle h, int pc, double lmin, double lmax, const double* b_d, double* x_d,
                               int nrhs, double rtol, int maxit, int* iters_h, double* relres_h, void* stream) {
  clear_error();
  int st = check_stationary(h, pc, b_d, x_d, nrhs, rtol, maxit);
  if (st) return st;
  BRAS_CHECK(lmin > 0.0 && lmax > lmin && std::isfinite(lmax), "need 0 < lmin < lmax");
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  std::vector<double> ca(maxit, 0.0), cc(maxit, 0.0);
  cc[0] = 1.0 / theta;
  double rho = 1.0 / sigma;
  for (int k = 1; k < maxit; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    ca[k] = rn * rho;
    cc[k] = 2.0 * rn / delta;
    rho = rn;
  }
  return stationary((Ctx*)h, pc, ca, cc, b_d, x_d, nrhs, rtol, maxit, iters_h, relres_h, stream);
}
