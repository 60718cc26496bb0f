// Whole preconditioned CG solve (Section 3) of a small single-column problem
// in one work-group.  The multi-pass solver spends most of a small solve on
// kernel launches and host round trips (six launches per iteration); here
// every step of every iteration runs inside one kernel of 1024 threads,
// separated by work-group barriers, with everything an iteration touches on
// chip:
//   LDS        the two vectors that are gathered (p, and d^-1 r for BRAS),
//              the broken vector zb [n_loc][E], and the transpose map as
//              16-bit slots (up to 160 KiB in all);
//   registers  each thread's own DOFs' x, r, z, q, b, d^-1, diag(M)^-1, and
//              its elements' coefficients c_K, 1/c_K (and, for small n_loc,
//              their map entries).
//
// Scope: the scaled H1 form (M_K = c_K Mhat, M_K^-1 = Mhat^-1 / c_K,
// eq. piola_mass_pullbacks), float64, one column; size limits in
// small_cg_eligible.
//
// Each operator is the element pass and the transpose-map reduce of the
// multi-pass path, in the same arithmetic order (eq. mhatinvbras_def for
// BRAS): thread t owns elements t, t + 1024, ... and forms
// z_K,l = ck_K * sum_j A[l][j] v[pi(K, j)] (j ascending) into zb, then owns
// DOFs t, t + 1024, ... and sums their copies in transpose-map order.  The
// iteration is the one of pcg.hip (same stopping test, breakdown tests and
// status codes; relres at exit from the true residual).  Dot products are
// per-thread sums, a butterfly within each wavefront and the wavefront sums
// in order: a fixed order, so results are reproducible.
#include <cmath>

#include "internal.h"
#include "cg_common.h"

namespace bras {

namespace {

constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / 64;
constexpr int kPerThread = (kSmallMaxN + kSmallThreads - 1) / kSmallThreads;   // own DOFs
constexpr int kLdsDoubles = kSmallLdsBytes / 8;

// elements per thread for each n_loc, enough for the element counts the LDS
// budget admits on the structured meshes (e.g. 2048 triangles of P1, 3072
// tetrahedra of P1); checked on the host
template <int NL>
constexpr int elems_per_thread() {
  return NL == 4 ? 3 : (NL <= 15 ? 2 : 1);
}
// map entries kept in registers across the solve when they are few
template <int NL>
constexpr bool map_in_registers() {
  return NL * elems_per_thread<NL>() <= 16;
}
// gathered element inputs held in registers during a product (small n_loc);
// otherwise every product row re-reads them from LDS
template <int NL>
constexpr bool inputs_in_registers() {
  return NL <= 15;
}

struct SmallOp {
  int E = 0, n = 0, nbr = 0;
  const int32_t* l2g = nullptr;     // [E][NL]
  const int32_t* rowptr = nullptr;  // [n+1]
  const int32_t* slot = nullptr;    // [n_br] l * E + K
  const double* ref = nullptr;      // Mhat [NL][NL]
  const double* coef = nullptr;     // c_K [E]
  const double* refinv = nullptr;   // Mhat^-1 [NL][NL]
  const double* icoef = nullptr;    // 1 / c_K [E]
  const double* invd = nullptr;     // 1 / d_i [n]
  const double* invdiag = nullptr;  // 1 / M_ii [n]
};

// A value that every lane holds, moved to scalar registers (the CG scalars
// and the loop control derived from them then stay scalar).
__device__ inline double uniform(double v) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(bits & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(bits >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums of a and b over the work-group, the same values in every thread.
// Contains two barriers, so LDS writes made before the call are visible
// after it.
__device__ inline void wg_sum2(double& a, double& b, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = a;
    red[kSmallWaves + (threadIdx.x >> 6)] = b;
  }
  __syncthreads();
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int w = 0; w < kSmallWaves; ++w) {
    sa += red[w];
    sb += red[kSmallWaves + w];
  }
  __syncthreads();
  a = uniform(sa);
  b = uniform(sb);
}

template <int NL>
struct Elems {
  static constexpr int EPT = elems_per_thread<NL>();
  static constexpr int MR = map_in_registers<NL>() ? NL : 1;
  double c[EPT], ic[EPT];   // c_K, 1 / c_K
  int32_t m[EPT][MR];       // map entries (when kept in registers)
};

// zb[l][K] = ck_K * sum_j A[l][j] v[pi(K, j)] for the thread's elements;
// A is indexed uniformly (scalar loads)
template <int NL, bool INV>
__device__ inline void elem_pass(const SmallOp& o, const Elems<NL>& el, const double* __restrict__ A,
                                 const double* v, double* zb) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < Elems<NL>::EPT; ++e) {
    const int K = t + e * kSmallThreads;
    if (K < o.E) {
      int32_t m[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        if constexpr (map_in_registers<NL>())
          m[j] = el.m[e][j];
        else
          m[j] = o.l2g[(int64_t)K * NL + j];
      }
      const double ck = INV ? el.ic[e] : el.c[e];
      if constexpr (inputs_in_registers<NL>()) {
        double w[NL];
#pragma unroll
        for (int j = 0; j < NL; ++j) w[j] = v[m[j]];
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < NL; ++j) acc = fma(A[l * NL + j], w[j], acc);
          zb[l * o.E + K] = acc * ck;
        }
      } else {
        for (int l = 0; l < NL; ++l) {
          double acc = 0.0;
#pragma unroll
          for (int j = 0; j < NL; ++j) acc = fma(A[l * NL + j], v[m[j]], acc);
          zb[l * o.E + K] = acc * ck;
        }
      }
    }
  }
}

// y_k = sum of the copies of the thread's k-th DOF, in transpose-map order
__device__ inline void reduce_pass(const int (&r0)[kPerThread], const int (&r1)[kPerThread],
                                   const unsigned short* slot, const double* zb, double (&y)[kPerThread]) {
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    double s = 0.0;
    for (int p = r0[k]; p < r1[k]; ++p) s += zb[slot[p]];
    y[k] = s;
  }
}

// z = C r for the thread's DOFs; returns the thread's part of r.z.  Called
// after a barrier that follows the last reads of sv and zb.
template <int NL>
__device__ inline double precond(const SmallOp& o, const Elems<NL>& el, int pc, const int (&r0)[kPerThread],
                                 const int (&r1)[kPerThread], const unsigned short* slot, double* sv, double* zb,
                                 const double (&r)[kPerThread], const double (&dinv)[kPerThread],
                                 const double (&jinv)[kPerThread], double (&z)[kPerThread]) {
  const int t = threadIdx.x;
  if (pc == BRAS_PC_BRAS) {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int i = t + k * kSmallThreads;
      if (i < o.n) sv[i] = r[k] * dinv[k];
    }
    __syncthreads();
    elem_pass<NL, true>(o, el, o.refinv, sv, zb);
    __syncthreads();
    reduce_pass(r0, r1, slot, zb, z);
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) z[k] *= dinv[k];
  } else {
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) z[k] = pc == BRAS_PC_JACOBI ? jinv[k] * r[k] : r[k];
  }
  double rzp = 0.0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if (t + k * kSmallThreads < o.n) rzp = fma(z[k], r[k], rzp);
  return rzp;
}

// Set-up shared by the solvers: the transpose map into LDS, the thread's
// element data and own-DOF values into registers, sv = x (no barrier).
template <int NL>
__device__ inline void small_setup(const SmallOp& o, const double* xio, unsigned short* slot, double* sv,
                                   Elems<NL>& el, int (&r0)[kPerThread], int (&r1)[kPerThread],
                                   double (&x)[kPerThread], double (&dinv)[kPerThread], double (&jinv)[kPerThread]) {
  const int t = threadIdx.x;
  for (int p = t; p < o.nbr; p += kSmallThreads) slot[p] = (unsigned short)o.slot[p];
#pragma unroll
  for (int e = 0; e < Elems<NL>::EPT; ++e) {
    const int K = t + e * kSmallThreads;
    const int Kc = K < o.E ? K : 0;
    el.c[e] = o.coef[Kc];
    el.ic[e] = o.icoef[Kc];
#pragma unroll
    for (int j = 0; j < Elems<NL>::MR; ++j) el.m[e][j] = map_in_registers<NL>() ? o.l2g[(int64_t)Kc * NL + j] : 0;
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int i = t + k * kSmallThreads;
    const bool own = i < o.n;
    const int ii = own ? i : 0;
    r0[k] = own ? o.rowptr[ii] : 0;
    r1[k] = own ? o.rowptr[ii + 1] : 0;
    x[k] = own ? xio[ii] : 0.0;
    dinv[k] = o.invd[ii];
    jinv[k] = o.invdiag[ii];
    if (own) sv[i] = x[k];
  }
}

// One work-group.  xio: initial guess on entry, solution on exit.  Writes
// sc / ic (one column) as the multi-pass solver leaves them.
template <int NL>
__global__ void __launch_bounds__(kSmallThreads) k_cg_small(SmallOp o, int pc, const double* __restrict__ bg,
                                                            double* __restrict__ xio, double rtol, int maxit,
                                                            double* __restrict__ sc, int* __restrict__ ic) {
  __shared__ double lds[kLdsDoubles];
  __shared__ double red[2 * kSmallWaves];
  const int t = threadIdx.x, n = o.n;
  double* pv = lds;                      // p [n]
  double* sv = lds + n;                  // d^-1 r, or x for M x [n]
  double* zb = lds + 2 * n;              // [n_loc][E]
  unsigned short* slot = (unsigned short*)(lds + 2 * n + o.nbr);   // [n_br]
  Elems<NL> el;
  int r0[kPerThread], r1[kPerThread];
  double x[kPerThread], r[kPerThread], z[kPerThread], q[kPerThread], dinv[kPerThread], jinv[kPerThread];
  small_setup<NL>(o, xio, slot, sv, el, r0, r1, x, dinv, jinv);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    r[k] = z[k] = q[k] = 0.0;
    if (t + k * kSmallThreads < n) pv[t + k * kSmallThreads] = 0.0;
  }
  __syncthreads();
  // r_0 = b - M x_0
  elem_pass<NL, false>(o, el, o.ref, sv, zb);
  __syncthreads();
  reduce_pass(r0, r1, slot, zb, q);
  double rr = 0.0, dummy = 0.0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    r[k] = t + k * kSmallThreads < n ? bg[t + k * kSmallThreads] - q[k] : 0.0;
    rr = fma(r[k], r[k], rr);
  }
  wg_sum2(rr, dummy, red);
  const double rn0 = sqrt(rr), target = rtol * rn0;
  int status = ST_RUN, it = 0;
  double rz = 0.0, beta = 0.0;
  if (!isfinite(rn0)) status = ST_BREAK;
  else if (rn0 <= target || rn0 == 0.0) status = ST_OK;
  if (status == ST_RUN) {
    rz = precond<NL>(o, el, pc, r0, r1, slot, sv, zb, r, dinv, jinv, z);
    wg_sum2(rz, dummy, red);
    if (!(rz > 0.0) || !isfinite(rz)) status = ST_BREAK;
  }
  while (status == ST_RUN) {
    // p = z + beta p; q = M p; alpha = rho / p.q
    double pn[kPerThread];
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int i = t + k * kSmallThreads;
      pn[k] = 0.0;
      if (i < n) {
        pn[k] = fma(beta, pv[i], z[k]);
        pv[i] = pn[k];
      }
    }
    __syncthreads();
    elem_pass<NL, false>(o, el, o.ref, pv, zb);
    __syncthreads();
    reduce_pass(r0, r1, slot, zb, q);
    double pq = 0.0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) pq = fma(pn[k], q[k], pq);
    wg_sum2(pq, dummy, red);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = ST_BREAK;
      break;
    }
    const double alpha = rz / pq;
    // x += alpha p; r -= alpha q; z = C r
    double rrp = 0.0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      r[k] = fma(-alpha, q[k], r[k]);
      x[k] = fma(alpha, pn[k], x[k]);
      rrp = fma(r[k], r[k], rrp);
    }
    double rzp = precond<NL>(o, el, pc, r0, r1, slot, sv, zb, r, dinv, jinv, z);
    wg_sum2(rrp, rzp, red);
    // stopping test, beta, rho
    ++it;
    const double nrm = sqrt(rrp);
    if (!isfinite(nrm)) status = ST_BREAK;
    else if (nrm <= target) status = ST_OK;
    else if (it >= maxit) status = ST_NOCONV;
    else if (!(rzp > 0.0) || !isfinite(rzp)) status = ST_BREAK;
    else {
      beta = rzp / rz;
      rz = rzp;
    }
  }
  // true residual at exit
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int i = t + k * kSmallThreads;
    if (i < n) {
      sv[i] = x[k];
      xio[i] = x[k];
    }
  }
  __syncthreads();
  elem_pass<NL, false>(o, el, o.ref, sv, zb);
  __syncthreads();
  reduce_pass(r0, r1, slot, zb, q);
  double tr = 0.0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const double v = t + k * kSmallThreads < n ? bg[t + k * kSmallThreads] - q[k] : 0.0;
    tr = fma(v, v, tr);
  }
  wg_sum2(tr, dummy, red);
  if (t == 0) {
    sc[S_R0] = rn0;
    sc[S_TARGET] = target;
    sc[S_RZ] = rz;
    sc[S_RR] = tr;
    sc[S_RELRES] = rn0 > 0.0 ? sqrt(tr) / rn0 : 0.0;
    ic[I_ITERS] = it;
    ic[I_STATUS] = status;
    ic[I_ACTIVE] = 0;
  }
}

// Stationary iteration (Section 3) in one work-group, the iteration of the
// multi-pass stationary driver:
//   r_0 = b - M x_0;  stop if ||r_k|| <= rtol ||r_0||;
//   d_k = a_k d_{k-1} + c_k C r_k;  x_{k+1} = x_k + d_k;  r_{k+1} = b - M x_{k+1}
// with the coefficient table coef[0 .. cap) = a_k, coef[cap ..) = c_k.
template <int NL>
__global__ void __launch_bounds__(kSmallThreads) k_st_small(SmallOp o, int pc, const double* __restrict__ bg,
                                                            double* __restrict__ xio, double rtol, int maxit,
                                                            const double* __restrict__ coef, int cap,
                                                            double* __restrict__ sc, int* __restrict__ ic) {
  __shared__ double lds[kLdsDoubles];
  __shared__ double red[2 * kSmallWaves];
  const int t = threadIdx.x, n = o.n;
  double* sv = lds + n;                  // x for M x, or d^-1 r
  double* zb = lds + 2 * n;              // [n_loc][E]
  unsigned short* slot = (unsigned short*)(lds + 2 * n + o.nbr);   // [n_br]
  Elems<NL> el;
  int r0[kPerThread], r1[kPerThread];
  double x[kPerThread], r[kPerThread], d[kPerThread], b[kPerThread], q[kPerThread], dinv[kPerThread],
      jinv[kPerThread];
  small_setup<NL>(o, xio, slot, sv, el, r0, r1, x, dinv, jinv);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int i = t + k * kSmallThreads;
    b[k] = i < n ? bg[i] : 0.0;
    d[k] = 0.0;
  }
  __syncthreads();
  // r = b - M x (sv holds x; called after a barrier that follows the writes
  // of sv and the last reads of zb); returns the thread's part of r.r
  auto residual = [&]() {
    elem_pass<NL, false>(o, el, o.ref, sv, zb);
    __syncthreads();
    reduce_pass(r0, r1, slot, zb, q);
    double rr = 0.0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      r[k] = b[k] - q[k];
      rr = fma(r[k], r[k], rr);
    }
    return rr;
  };
  double rr = residual(), dummy = 0.0;
  wg_sum2(rr, dummy, red);
  const double rn0 = sqrt(rr), target = rtol * rn0;
  int status = ST_RUN, it = 0;
  double relres = rn0 > 0.0 ? 1.0 : 0.0;
  if (!isfinite(rn0)) status = ST_BREAK;
  else if (rn0 == 0.0) status = ST_OK;
  while (status == ST_RUN) {
    const double a = coef[it], c = coef[cap + it];
    // d = a d + c C r; x += d
    if (pc == BRAS_PC_BRAS) {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) {
        const int i = t + k * kSmallThreads;
        if (i < n) sv[i] = r[k] * dinv[k];
      }
      __syncthreads();
      elem_pass<NL, true>(o, el, o.refinv, sv, zb);
      __syncthreads();
      reduce_pass(r0, r1, slot, zb, q);
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) d[k] = fma(a, d[k], c * (q[k] * dinv[k]));
    } else {
#pragma unroll
      for (int k = 0; k < kPerThread; ++k) d[k] = fma(a, d[k], c * (r[k] * jinv[k]));
    }
    // (every thread has passed the barrier after the element pass that read
    // sv, so sv can take x)
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      const int i = t + k * kSmallThreads;
      x[k] = x[k] + d[k];
      if (i < n) sv[i] = x[k];
    }
    __syncthreads();
    double rrp = residual();
    wg_sum2(rrp, dummy, red);
    ++it;
    const double nrm = sqrt(rrp);
    relres = nrm / rn0;
    if (!isfinite(nrm)) status = ST_BREAK;
    else if (nrm <= target) status = ST_OK;
    else if (it >= maxit) status = ST_NOCONV;
    rr = rrp;
  }
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    const int i = t + k * kSmallThreads;
    if (i < n) xio[i] = x[k];
  }
  if (t == 0) {
    sc[S_R0] = rn0;
    sc[S_TARGET] = target;
    sc[S_RR] = rr;
    sc[S_RELRES] = relres;
    ic[I_ITERS] = it;
    ic[I_STATUS] = status;
    ic[I_ACTIVE] = 0;
  }
}

}  // namespace

// the H1 element sizes of degrees 1-4 (2D: 3, 6, 10, 15; 3D: 4, 10, 20, 35)
#define SMALL_NL_CASES(X) X(3) X(4) X(6) X(10) X(15) X(20) X(35)

static int small_elems_per_thread(int nl) {
#define CASE(N) \
  case N: return elems_per_thread<N>();
  switch (nl) {
    SMALL_NL_CASES(CASE)
    default: return 0;
  }
#undef CASE
}

bool small_cg_eligible(const Ctx* c, int nrhs, int maxit) {
  const int ept = small_elems_per_thread(c->nl);
  return c->small_cg && nrhs == 1 && c->form == BRAS_ELEM_SCALED_REF && c->prec == BRAS_FP64 && ept > 0 &&
         c->n >= 1 && c->n <= kSmallMaxN && c->E <= (int64_t)ept * kSmallThreads && c->nbr <= 65535 &&
         16 * c->n + 10 * c->nbr <= kSmallLdsBytes && maxit <= kSmallMaxIt;
}

static SmallOp small_op(const Ctx* c) {
  SmallOp o;
  o.E = (int)c->E;
  o.n = (int)c->n;
  o.nbr = (int)c->nbr;
  o.l2g = c->l2g;
  o.rowptr = c->rowptr;
  o.slot = c->slot;
  o.ref = c->ref;
  o.coef = c->coef;
  o.refinv = c->refinv;
  o.icoef = c->icoef;
  o.invd = c->invd;
  o.invdiag = c->invdiag;
  return o;
}

int launch_small_cg(Ctx* c, int pc, const double* b, double* x, double rtol, int maxit, double* sc, int* ic,
                    hipStream_t s) {
  BRAS_CHECK(small_cg_eligible(c, 1, maxit), "problem not eligible for the single work-group solver");
  const SmallOp o = small_op(c);
#define CASE(N)                                                                  \
  case N:                                                                        \
    k_cg_small<N><<<1, kSmallThreads, 0, s>>>(o, pc, b, x, rtol, maxit, sc, ic); \
    break;
  switch (c->nl) {
    SMALL_NL_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no single work-group solver", c->nl);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

int launch_small_stationary(Ctx* c, int pc, const double* b, double* x, double rtol, int maxit, const double* coef,
                            int cap, double* sc, int* ic, hipStream_t s) {
  BRAS_CHECK(small_cg_eligible(c, 1, maxit) && cap >= maxit, "problem not eligible for the single work-group solver");
  const SmallOp o = small_op(c);
#define CASE(N)                                                                                \
  case N:                                                                                      \
    k_st_small<N><<<1, kSmallThreads, 0, s>>>(o, pc, b, x, rtol, maxit, coef, cap, sc, ic);    \
    break;
  switch (c->nl) {
    SMALL_NL_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no single work-group solver", c->nl);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

}  // namespace bras
