// Operator application: the BRAS inverse D^-1 P^T M_br^-1 P D^-1 (eqs.
// mhatinvbras_def, mass_and_bras_element_sums), the conforming mass
// M = P^T M_br P (eq. M_PMbrP), diag(M)^-1, and the density gradient.
//
// Every operator is two passes:
//   element pass  one thread per (element K, column r): gather the K-th
//                 element's entries of x (optionally times D^-1), multiply by
//                 the element matrix, write the broken result z_K to the
//                 broken vector in element-fastest order (slot l*E + K), so a
//                 wavefront's stores are contiguous;
//   reduce pass   one thread per (conforming DOF i, column r): sum the broken
//                 copies of i in the fixed order of the transpose map, scale
//                 (D^-1 for BRAS), optionally accumulate a dot product with a
//                 second vector into per-block partial sums (deterministic
//                 tree in LDS, no atomics).
// Vectors with several columns are [n][R] (column fastest): the R threads of
// one element read R consecutive doubles per gathered DOF.
#include <cmath>

#include "internal.h"
#include "block_reduce.h"

namespace bras {

constexpr int kBS = 256;
constexpr int kMaxReduceBlocks = 2048;

// ---------------------------------------------------------------------------
// element passes
// ---------------------------------------------------------------------------

// Shared reference matrix (affine H1): z_K = coef_K * A (w_K), w_K = (s x)[pi_K].
template <int NL, bool SCALE_IN>
__global__ void __launch_bounds__(kBS) k_scaled_elem(int64_t E, int R, const int32_t* __restrict__ l2gT,
                                                     const double* __restrict__ x, const double* __restrict__ invd,
                                                     const double* __restrict__ A, const double* __restrict__ coefK,
                                                     double* __restrict__ zb, const int* __restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * R) return;
  const int64_t K = t / R;
  const int r = (int)(t - K * R);
  if (active && !active[r]) return;
  double w[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    const int32_t i = l2gT[(int64_t)j * E + K];
    double v = x[(int64_t)i * R + r];
    if (SCALE_IN) v *= invd[i];
    w[j] = v;
  }
  const double s = coefK[K];
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j) acc = fma(A[i * NL + j], w[j], acc);
    zb[((int64_t)i * E + K) * R + r] = s * acc;
  }
}

// Per-element packed symmetric matrix (lower triangle, SoA [q][E]):
// z_K = A_K w_K with w_K = x[pi_K], in precision T.
template <int NL, typename T, typename ZT>
__global__ void __launch_bounds__(kBS) k_packed_elem(int64_t E, int R, const int32_t* __restrict__ l2gT,
                                                     const double* __restrict__ x, const T* __restrict__ ap,
                                                     ZT* __restrict__ zb, const int* __restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * R) return;
  const int64_t K = t / R;
  const int r = (int)(t - K * R);
  if (active && !active[r]) return;
  T w[NL], z[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) {
    w[j] = (T)x[(int64_t)l2gT[(int64_t)j * E + K] * R + r];
    z[j] = (T)0;
  }
  int q = 0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j, ++q) {
      const T a = ap[(int64_t)q * E + K];
      z[i] = fma(a, w[j], z[i]);
      if (j < i) z[j] = fma(a, w[i], z[j]);
    }
  }
#pragma unroll
  for (int i = 0; i < NL; ++i) zb[((int64_t)i * E + K) * R + r] = (ZT)z[i];
}

// Metric reference tables (Piola): z_K = sum_p G_p,K S_p w_K, float64.
template <int NL>
__global__ void __launch_bounds__(kBS) k_metric_elem(int64_t E, int R, int nsym, const int32_t* __restrict__ l2gT,
                                                     const double* __restrict__ x, const double* __restrict__ S,
                                                     const double* __restrict__ Gsoa, double* __restrict__ zb,
                                                     const int* __restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * R) return;
  const int64_t K = t / R;
  const int r = (int)(t - K * R);
  if (active && !active[r]) return;
  double w[NL], g[6];
#pragma unroll
  for (int j = 0; j < NL; ++j) w[j] = x[(int64_t)l2gT[(int64_t)j * E + K] * R + r];
  for (int p = 0; p < 6; ++p) g[p] = p < nsym ? Gsoa[(int64_t)p * E + K] : 0.0;
#pragma unroll
  for (int i = 0; i < NL; ++i) {
    double acc = 0.0;
    for (int p = 0; p < nsym; ++p) {
      double sp = 0.0;
#pragma unroll
      for (int j = 0; j < NL; ++j) sp = fma(S[(p * NL + i) * NL + j], w[j], sp);
      acc = fma(g[p], sp, acc);
    }
    zb[((int64_t)i * E + K) * R + r] = acc;
  }
}

// Generic element pass for any n_loc: one wavefront per (element, column);
// the gathered vector is staged in LDS, lane i computes row i.
// kind 0: shared reference (A = ref, coefficient coefK[K], optional D^-1 in);
// kind 1: packed per-element (T); kind 2: metric tables.
template <typename T, typename ZT>
__global__ void __launch_bounds__(64) k_generic_elem(int kind, int64_t E, int R, int nl, int nsym,
                                                     const int32_t* __restrict__ l2gT, const double* __restrict__ x,
                                                     const double* __restrict__ invd, const double* __restrict__ A,
                                                     const double* __restrict__ coefK, const T* __restrict__ ap,
                                                     const double* __restrict__ Gsoa, ZT* __restrict__ zb,
                                                     const int* __restrict__ active) {
  __shared__ double w[96];
  const int64_t t = blockIdx.x;
  const int64_t K = t / R;
  const int r = (int)(t - K * R);
  if (active && !active[r]) return;
  for (int j = threadIdx.x; j < nl; j += 64) {
    const int32_t i = l2gT[(int64_t)j * E + K];
    double v = x[(int64_t)i * R + r];
    if (kind == 0 && invd) v *= invd[i];
    w[j] = v;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nl; i += 64) {
    double acc = 0.0;
    if (kind == 0) {
      for (int j = 0; j < nl; ++j) acc = fma(A[i * nl + j], w[j], acc);
      acc *= coefK[K];
    } else if (kind == 1) {
      for (int j = 0; j < nl; ++j) {
        const int a = i > j ? i : j, b = i > j ? j : i;
        acc += (double)ap[((int64_t)a * (a + 1) / 2 + b) * E + K] * (double)(T)w[j];
      }
    } else {
      for (int p = 0; p < nsym; ++p) {
        double sp = 0.0;
        for (int j = 0; j < nl; ++j) sp = fma(A[((int64_t)p * nl + i) * nl + j], w[j], sp);
        acc = fma(Gsoa[(int64_t)p * E + K], sp, acc);
      }
    }
    zb[((int64_t)i * E + K) * R + r] = (ZT)acc;
  }
}

// ---------------------------------------------------------------------------
// reduce pass with optional fused dot product
// ---------------------------------------------------------------------------
template <typename ZT>
__global__ void __launch_bounds__(kBS) k_reduce(int64_t n, int R, const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ slot, const ZT* __restrict__ zb,
                                                const double* __restrict__ scale, double* __restrict__ y,
                                                const double* __restrict__ dotv, double* __restrict__ partial,
                                                const int* __restrict__ active) {
  __shared__ double sh[kBS];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;   // a multiple of R
  const int r = (int)(t0 % R);
  double dot = 0.0;
  if (!active || active[r]) {
    for (int64_t t = t0; t < n * R; t += stride) {
      const int64_t i = t / R;
      double acc = 0.0;
      const int32_t a = rowptr[i], b = rowptr[i + 1];
      for (int32_t p = a; p < b; ++p) acc += (double)zb[(int64_t)slot[p] * R + r];
      if (scale) acc *= scale[i];
      y[t] = acc;
      if (dotv) dot = fma(acc, dotv[t], dot);
    }
  }
  if (!partial) return;
  sh[threadIdx.x] = dot;
  block_partials(sh, R, partial);
}

// y = s .* x (diagonal scaling) with optional fused dot product y . dotv
__global__ void __launch_bounds__(kBS) k_diag_scale(int64_t n, int R, const double* __restrict__ s,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    const double* __restrict__ dotv, double* __restrict__ partial,
                                                    const int* __restrict__ active) {
  __shared__ double sh[kBS];
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int r = (int)(t0 % R);
  double dot = 0.0;
  if (!active || active[r]) {
    for (int64_t t = t0; t < n * R; t += stride) {
      const double v = x[t] * s[t / R];
      y[t] = v;
      if (dotv) dot = fma(v, dotv[t], dot);
    }
  }
  if (!partial) return;
  sh[threadIdx.x] = dot;
  block_partials(sh, R, partial);
}

// g_K = -dcoef_K sum_r lam_K,r^T Mhat x_K,r  (density gradient, affine H1)
template <int NL>
__global__ void __launch_bounds__(kBS) k_rho_grad(int64_t E, int R, const int32_t* __restrict__ l2gT,
                                                  const double* __restrict__ x, const double* __restrict__ lam,
                                                  const double* __restrict__ Mhat, const double* __restrict__ dcoef,
                                                  double* __restrict__ g) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= E) return;
  double tot = 0.0;
  for (int r = 0; r < R; ++r) {
    double w[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) w[j] = x[(int64_t)l2gT[(int64_t)j * E + K] * R + r];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < NL; ++j) acc = fma(Mhat[i * NL + j], w[j], acc);
      tot = fma(lam[(int64_t)l2gT[(int64_t)i * E + K] * R + r], acc, tot);
    }
  }
  g[K] = -dcoef[K] * tot;
}

__global__ void __launch_bounds__(kBS) k_rho_grad_generic(int64_t E, int R, int nl, const int32_t* __restrict__ l2gT,
                                                          const double* __restrict__ x, const double* __restrict__ lam,
                                                          const double* __restrict__ Mhat,
                                                          const double* __restrict__ dcoef, double* __restrict__ g) {
  const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= E) return;
  double tot = 0.0;
  for (int r = 0; r < R; ++r)
    for (int i = 0; i < nl; ++i) {
      double acc = 0.0;
      for (int j = 0; j < nl; ++j) acc += Mhat[i * nl + j] * x[(int64_t)l2gT[(int64_t)j * E + K] * R + r];
      tot += lam[(int64_t)l2gT[(int64_t)i * E + K] * R + r] * acc;
    }
  g[K] = -dcoef[K] * tot;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n) { return (unsigned)((n + kBS - 1) / kBS); }

int reduce_blocks(Ctx* c, int R) {
  int64_t want = (c->n * R + kBS - 1) / kBS;
  int64_t nb = want < kMaxReduceBlocks ? want : kMaxReduceBlocks;
  if (nb < 1) nb = 1;
  // grid * kBS must be a multiple of R so that each thread keeps one column
  while (((int64_t)nb * kBS) % R) ++nb;
  return (int)nb;
}

#define SCALED_CASES(X) X(3) X(4) X(6) X(10) X(15) X(20) X(21) X(28) X(35)
#define PACKED_CASES(X) X(3) X(4) X(6) X(8) X(10) X(15) X(20) X(24)
#define METRIC_CASES(X) X(3) X(4) X(6) X(8) X(15) X(20)

static int scaled_elem(Ctx* c, const double* x, bool bras_in, const double* A, const double* coefK, int R,
                       hipStream_t s, const int* active) {
  double* zb = (double*)c->zb;
  const int64_t work = c->E * R;
#define CASE(N)                                                                                                  \
  case N:                                                                                                        \
    if (bras_in)                                                                                                 \
      k_scaled_elem<N, true><<<nblk(work), kBS, 0, s>>>(c->E, R, c->l2gT, x, c->invd, A, coefK, zb, active);     \
    else                                                                                                         \
      k_scaled_elem<N, false><<<nblk(work), kBS, 0, s>>>(c->E, R, c->l2gT, x, c->invd, A, coefK, zb, active);    \
    break;
  if (c->variant != 1) {
    switch (c->nl) {
      SCALED_CASES(CASE)
      default:
        k_generic_elem<double, double><<<(unsigned)work, 64, 0, s>>>(0, c->E, R, c->nl, 0, c->l2gT, x,
                                                                     bras_in ? c->invd : nullptr, A, coefK, nullptr,
                                                                     nullptr, zb, active);
    }
  } else {
    k_generic_elem<double, double><<<(unsigned)work, 64, 0, s>>>(0, c->E, R, c->nl, 0, c->l2gT, x,
                                                                 bras_in ? c->invd : nullptr, A, coefK, nullptr,
                                                                 nullptr, zb, active);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

template <typename T, typename ZT>
static int packed_elem(Ctx* c, const double* x, const T* ap, ZT* zb, int R, hipStream_t s, const int* active) {
  const int64_t work = c->E * R;
#define CASE(N) \
  case N: k_packed_elem<N, T, ZT><<<nblk(work), kBS, 0, s>>>(c->E, R, c->l2gT, x, ap, zb, active); break;
  if (c->variant != 1) {
    switch (c->nl) {
      PACKED_CASES(CASE)
      default:
        k_generic_elem<T, ZT><<<(unsigned)work, 64, 0, s>>>(1, c->E, R, c->nl, 0, c->l2gT, x, nullptr, nullptr,
                                                            nullptr, ap, nullptr, zb, active);
    }
  } else {
    k_generic_elem<T, ZT><<<(unsigned)work, 64, 0, s>>>(1, c->E, R, c->nl, 0, c->l2gT, x, nullptr, nullptr, nullptr,
                                                        ap, nullptr, zb, active);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int metric_elem(Ctx* c, const double* x, int R, hipStream_t s, const int* active) {
  const int64_t work = c->E * R;
  double* zb = (double*)c->zb;
#define CASE(N)                                                                                                  \
  case N:                                                                                                        \
    k_metric_elem<N><<<nblk(work), kBS, 0, s>>>(c->E, R, c->nsym, c->l2gT, x, c->ref, c->coef, zb, active);      \
    break;
  if (c->variant != 1) {
    switch (c->nl) {
      METRIC_CASES(CASE)
      default:
        k_generic_elem<double, double><<<(unsigned)work, 64, 0, s>>>(2, c->E, R, c->nl, c->nsym, c->l2gT, x, nullptr,
                                                                     c->ref, nullptr, nullptr, c->coef, zb, active);
    }
  } else {
    k_generic_elem<double, double><<<(unsigned)work, 64, 0, s>>>(2, c->E, R, c->nl, c->nsym, c->l2gT, x, nullptr,
                                                                 c->ref, nullptr, nullptr, c->coef, zb, active);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

template <typename ZT>
static int reduce(Ctx* c, const ZT* zb, const double* scale, double* y, int R, hipStream_t s, const double* dotv,
                  double* partial, const int* active) {
  k_reduce<ZT><<<reduce_blocks(c, R), kBS, 0, s>>>(c->n, R, c->rowptr, c->slot, zb, scale, y, dotv, partial, active);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// The mass pass is float64 throughout (it defines the problem being solved).
int launch_mass(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                const int* active) {
  int st;
  double* zb = (double*)c->zb;
  if (c->form == BRAS_ELEM_SCALED_REF) {
    if ((st = scaled_elem(c, x, false, c->ref, c->coef, R, s, active))) return st;
  } else if (c->form == BRAS_ELEM_METRIC_REF) {
    if ((st = metric_elem(c, x, R, s, active))) return st;
  } else {
    if ((st = packed_elem<double, double>(c, x, c->coef, zb, R, s, active))) return st;
  }
  return reduce<double>(c, zb, nullptr, y, R, s, dotv, dotpart, active);
}

int launch_bras(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                const int* active) {
  int st;
  if (c->form == BRAS_ELEM_SCALED_REF) {
    if ((st = scaled_elem(c, x, true, c->refinv, c->icoef, R, s, active))) return st;
    return reduce<double>(c, (const double*)c->zb, c->invd, y, R, s, dotv, dotpart, active);
  }
  if (c->prec == BRAS_FP64) {
    if ((st = packed_elem<double, double>(c, x, (const double*)c->ainv, (double*)c->zb, R, s, active))) return st;
    return reduce<double>(c, (const double*)c->zb, nullptr, y, R, s, dotv, dotpart, active);
  }
  if (c->prec == BRAS_FP32) {
    if ((st = packed_elem<float, float>(c, x, (const float*)c->ainv, (float*)c->zb, R, s, active))) return st;
    return reduce<float>(c, (const float*)c->zb, nullptr, y, R, s, dotv, dotpart, active);
  }
  return launch_bras_bf16(c, x, y, R, s, dotv, dotpart, active);
}

int launch_jacobi(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                  const int* active) {
  k_diag_scale<<<reduce_blocks(c, R), kBS, 0, s>>>(c->n, R, c->invdiag, x, y, dotv, dotpart, active);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

}  // namespace bras

using namespace bras;

static int check_apply(bras_handle h, const double* x, double* y, int nrhs) {
  BRAS_CHECK(h, "null handle");
  BRAS_CHECK(x && y, "null vector");
  BRAS_CHECK(x != y, "x and y must be distinct buffers");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs %d outside 1..max_rhs=%d", nrhs, c->max_rhs);
  return BRAS_OK;
}

extern "C" int bras_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream) {
  clear_error();
  int st = check_apply(h, x_d, y_d, nrhs);
  if (st) return st;
  return launch_bras((Ctx*)h, x_d, y_d, nrhs, (hipStream_t)stream, nullptr, nullptr, nullptr);
}

extern "C" int mass_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream) {
  clear_error();
  int st = check_apply(h, x_d, y_d, nrhs);
  if (st) return st;
  return launch_mass((Ctx*)h, x_d, y_d, nrhs, (hipStream_t)stream, nullptr, nullptr, nullptr);
}

extern "C" int jacobi_apply(bras_handle h, const double* x_d, double* y_d, int nrhs, void* stream) {
  clear_error();
  int st = check_apply(h, x_d, y_d, nrhs);
  if (st) return st;
  return launch_jacobi((Ctx*)h, x_d, y_d, nrhs, (hipStream_t)stream, nullptr, nullptr, nullptr);
}

extern "C" int bras_rho_grad(bras_handle h, const double* x_d, const double* lam_d, const double* dcoef_d,
                             double* g_d, int nrhs, void* stream) {
  clear_error();
  BRAS_CHECK(h && x_d && lam_d && dcoef_d && g_d, "null argument");
  Ctx* c = (Ctx*)h;
  BRAS_CHECK(c->form == BRAS_ELEM_SCALED_REF, "bras_rho_grad needs the SCALED_REF form");
  BRAS_CHECK(nrhs >= 1 && nrhs <= c->max_rhs, "nrhs %d outside 1..max_rhs", nrhs);
  hipStream_t s = (hipStream_t)stream;
  const unsigned nb = (unsigned)((c->E + kBS - 1) / kBS);
#define CASE(N) \
  case N: k_rho_grad<N><<<nb, kBS, 0, s>>>(c->E, nrhs, c->l2gT, x_d, lam_d, c->ref, dcoef_d, g_d); break;
  switch (c->nl) {
    SCALED_CASES(CASE)
    default:
      k_rho_grad_generic<<<nb, kBS, 0, s>>>(c->E, nrhs, c->nl, c->l2gT, x_d, lam_d, c->ref, dcoef_d, g_d);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}
