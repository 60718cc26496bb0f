// Setup kernels: element geometry, map validation and transpose, the exact
// element inverses, diag(M), and the bras_setup / bras_update entry points.
//
// The transpose map (conforming DOF -> its broken copies) is a CSR built by
// counting, a scan and a per-row sort, so every later reduction over the
// copies of a DOF runs in one fixed order (no floating-point atomics).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace bras {

// ---------------------------------------------------------------------------
// geometry: pullback coefficients (eq. piola_mass_pullbacks)
// ---------------------------------------------------------------------------
__global__ void k_geometry(int family, int dim, const double* __restrict__ X, const int32_t* __restrict__ cells,
                           int64_t E, int64_t nvert, const double* __restrict__ rho, double* __restrict__ out,
                           int nsym) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= E) return;
  const int nv = dim + 1;
  double J[3][3] = {{0}};
  const int32_t* c = cells + K * nv;
  for (int i = 0; i < nv; ++i)
    if (c[i] < 0 || c[i] >= nvert) {
      // invalid vertex id: a NaN coefficient makes setup fail with ENOTSPD
      const int cnt = (family == BRAS_H1 || family == BRAS_H1_BERNSTEIN) ? 1 : nsym;
      for (int p = 0; p < cnt; ++p) out[K * cnt + p] = __longlong_as_double(0x7ff8000000000000LL);
      return;
    }
  for (int i = 0; i < dim; ++i)
    for (int a = 0; a < dim; ++a) J[a][i] = X[(int64_t)c[i + 1] * dim + a] - X[(int64_t)c[0] * dim + a];
  double det;
  if (dim == 2)
    det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  else
    det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
          J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  const double adet = fabs(det);
  const double r = rho ? rho[K] : 1.0;
  if (family == BRAS_H1 || family == BRAS_H1_BERNSTEIN) {
    out[K] = r * adet;
    return;
  }
  double G[3][3];
  if (family == BRAS_HDIV || family == BRAS_HDIV2) {
    // J^T J / |det J|
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b) {
        double s = 0;
        for (int q = 0; q < dim; ++q) s += J[q][a] * J[q][b];
        G[a][b] = r * s / adet;
      }
  } else {
    // |det J| J^-1 J^-T ; J^-1 = adj(J)/det
    double A[3][3];
    if (dim == 2) {
      A[0][0] = J[1][1]; A[0][1] = -J[0][1];
      A[1][0] = -J[1][0]; A[1][1] = J[0][0];
    } else {
      A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
      A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
      A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
      A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
      A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
      A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    }
    // J^-1 J^-T = A A^T / det^2, times |det| -> A A^T / |det|
    for (int a = 0; a < dim; ++a)
      for (int b = 0; b < dim; ++b) {
        double s = 0;
        for (int q = 0; q < dim; ++q) s += A[a][q] * A[b][q];
        G[a][b] = r * s / adet;
      }
  }
  int p = 0;
  for (int a = 0; a < dim; ++a)
    for (int b = a; b < dim; ++b) out[K * nsym + p++] = G[a][b];
}

// ---------------------------------------------------------------------------
// maps
// ---------------------------------------------------------------------------
// Per element: range and distinctness checks, copy, counts.
__global__ void k_map_check(const int32_t* __restrict__ l2g, int64_t E, int nl, int64_t n,
                            int32_t* __restrict__ l2g_out, int32_t* __restrict__ cnt, int* __restrict__ flag) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= E) return;
  const int32_t* row = l2g + K * nl;
  bool ok = true;
  for (int l = 0; l < nl; ++l) {
    int32_t i = row[l];
    if (i < 0 || i >= n) {
      ok = false;
      break;
    }
    for (int m = 0; m < l; ++m)
      if (row[m] == i) ok = false;
  }
  if (!ok) {
    atomicMin(flag, (int)K);
    return;
  }
  for (int l = 0; l < nl; ++l) {
    l2g_out[K * nl + l] = row[l];
    atomicAdd(cnt + row[l], 1);   // integer: exact and order independent
  }
}

__global__ void k_mult(const int32_t* __restrict__ cnt, int64_t n, double* __restrict__ invd, int* __restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int d = cnt[i];
  if (d <= 0) {
    atomicMin(flag, (int)i);
    invd[i] = 0.0;
  } else {
    invd[i] = 1.0 / (double)d;
  }
}

// Exclusive scan of int32 counts, three passes (block scan, scan of block
// sums in one block, add).
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;

__global__ void k_scan_local(const int32_t* __restrict__ in, int64_t n, int32_t* __restrict__ out,
                             int32_t* __restrict__ bsum) {
  __shared__ int32_t s[kScanBlock];
  const int64_t base = ((int64_t)blockIdx.x * kScanBlock + threadIdx.x) * kScanItems;
  int32_t v[kScanItems];
  int32_t tot = 0;
  for (int q = 0; q < kScanItems; ++q) {
    int64_t i = base + q;
    v[q] = i < n ? in[i] : 0;
    tot += v[q];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int32_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  int32_t run = s[threadIdx.x] - tot;
  for (int q = 0; q < kScanItems; ++q) {
    int64_t i = base + q;
    if (i < n) out[i] = run;
    run += v[q];
  }
  if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = s[kScanBlock - 1];
}

__global__ void k_scan_sums(int32_t* __restrict__ bsum, int64_t nb, int32_t* __restrict__ total) {
  if (threadIdx.x != 0) return;
  int32_t run = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int32_t t = bsum[b];
    bsum[b] = run;
    run += t;
  }
  *total = run;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ bsum) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] += bsum[i / ((int64_t)kScanBlock * kScanItems)];
}

__global__ void k_fill_slots(const int32_t* __restrict__ l2g, int64_t nbr, const int32_t* __restrict__ rowptr,
                             int32_t* __restrict__ fill, int32_t* __restrict__ key) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nbr) return;
  int32_t i = l2g[t];
  int32_t pos = rowptr[i] + atomicAdd(fill + i, 1);
  key[pos] = (int32_t)t;   // canonical broken index K*nl + l
}

// Sort each row by canonical broken index K*nl + l, then store the internal
// local-index-major index l*E + K of each copy.
__global__ void k_sort_rows(const int32_t* __restrict__ rowptr, int64_t n, int nl, int64_t E,
                            int32_t* __restrict__ key, int32_t* __restrict__ slot) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t a = rowptr[i], b = rowptr[i + 1];
  for (int32_t p = a + 1; p < b; ++p) {
    int32_t v = key[p];
    int32_t q = p - 1;
    while (q >= a && key[q] > v) {
      key[q + 1] = key[q];
      --q;
    }
    key[q + 1] = v;
  }
  for (int32_t p = a; p < b; ++p) {
    const int32_t k = key[p];
    const int32_t K = k / nl, l = k - K * nl;
    slot[p] = (int32_t)((int64_t)l * E + K);
  }
}

// S [nsym][nl][nl] (symmetric pair tables) -> packed lower [q][ss], q = i(i+1)/2 + j,
// entries p >= nsym zero
__global__ void k_pack_sym(const double* __restrict__ S, int nl, int nsym, int ss, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t npk = (int64_t)nl * (nl + 1) / 2;
  if (t >= npk * ss) return;
  const int q = (int)(t / ss), p = (int)(t % ss);
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= q) ++i;
  const int j = q - i * (i + 1) / 2;
  out[t] = p < nsym ? S[(int64_t)p * nl * nl + i * nl + j] : 0.0;
}

// rows of per-element data into the internal (patch-major) element order:
// out[K][i] = in[perm[K]][i]
__global__ void k_permute_rows(const double* __restrict__ in, const int32_t* __restrict__ perm, int64_t E, int w,
                               double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * w) return;
  const int64_t K = t / w, i = t - K * w;
  out[t] = in[(int64_t)perm[K] * w + i];
}

// dst[i] = src[map[i]] (a vector in the internal DOF numbering of a patch plan)
__global__ void k_gather_vec(const double* __restrict__ src, const int32_t* __restrict__ map, int64_t n,
                             double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[map[i]];
}

// AoS [E][nsym] -> SoA [nsym][E]
__global__ void k_transpose_coef(const double* __restrict__ in, int64_t E, int nsym, double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= E * nsym) return;
  int64_t K = t / nsym, p = t % nsym;
  out[p * E + K] = in[t];
}

// ---------------------------------------------------------------------------
// element data
// ---------------------------------------------------------------------------
__global__ void k_scaled_coef(const double* __restrict__ c, int64_t E, double* __restrict__ coef,
                              double* __restrict__ icoef, int* __restrict__ flag) {
  int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= E) return;
  double v = c[K];
  if (!(v > 0.0) || !isfinite(v)) {
    atomicMin(flag, (int)K);
    v = 1.0;
  }
  coef[K] = v;
  icoef[K] = 1.0 / v;
}

// One work-group (one wavefront) per element: form M_K in LDS, Cholesky
// M_K = L L^T, X = L^-1 in place, and store the folded inverse
//   Atil = D_K^-1 M_K^-1 D_K^-1 = D_K^-1 X^T X D_K^-1   (packed lower, SoA)
// or, for the Gram-factor form, Gtil = X D_K^-1 (lower triangular), so that
// Atil = Gtil^T Gtil.  Only the lower triangle of A is used.
// mode: 0 = metric tables (S [nsym][nl*nl], G SoA), 1 = explicit row-major M_K.
template <typename T>
__device__ inline T cast_out(double v);
template <>
__device__ inline double cast_out<double>(double v) { return v; }
template <>
__device__ inline float cast_out<float>(double v) { return (float)v; }
template <>
__device__ inline __bf16 cast_out<__bf16>(double v) { return (__bf16)(float)v; }   // float64 -> float32 -> bfloat16, each to nearest even

__device__ inline void unpack_lower(int q, int& i, int& j) {
  int r = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= q) ++r;
  while (r * (r + 1) / 2 > q) --r;
  i = r;
  j = q - r * (r + 1) / 2;
}

template <typename T>
__global__ void __launch_bounds__(64) k_elem_factor(int mode, int64_t E, int nl, int nsym,
                                                    const double* __restrict__ S, const double* __restrict__ Gsoa,
                                                    const double* __restrict__ Mexp, const int32_t* __restrict__ l2g,
                                                    const double* __restrict__ invd, double* __restrict__ diagb,
                                                    double* __restrict__ mpack, int mg, T* __restrict__ out, int og,
                                                    int gram, int* __restrict__ flag) {
  extern __shared__ double lds[];
  double* A = lds;               // lower triangle, packed: entry (i, j), i >= j, at i(i+1)/2 + j
  double* g = A + nl * (nl + 1) / 2;   // nsym (<= 6)
  double* dinv = g + 8;          // nl
  __shared__ int bad;
  const int64_t K = blockIdx.x;
  const int t = threadIdx.x, nt = blockDim.x;
  const int npk = nl * (nl + 1) / 2;   // packed lower triangle (layout: packed_at)
  if (t == 0) bad = 0;
  if (mode == 0 && t < nsym) g[t] = Gsoa[(int64_t)t * E + K];
  for (int l = t; l < nl; l += nt) dinv[l] = invd[l2g[K * nl + l]];
  __syncthreads();
  const int nn = nl * nl;
  auto P = [](int i, int j) { return i * (i + 1) / 2 + j; };
  for (int q = t; q < npk; q += nt) {
    int i, j;
    unpack_lower(q, i, j);
    double v;
    if (mode == 0) {
      v = 0.0;
      for (int p = 0; p < nsym; ++p) v += g[p] * S[(int64_t)p * nn + i * nl + j];
    } else {
      v = Mexp[K * nn + i * nl + j];
    }
    A[P(i, j)] = v;
    if (mpack) mpack[packed_at(q, K, E, mg, npk)] = v;
    if (i == j) diagb[(int64_t)i * E + K] = v;
  }
  __syncthreads();
  // right-looking Cholesky
  for (int j = 0; j < nl; ++j) {
    const double piv = A[P(j, j)];
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (t == 0) bad = 1;
      break;
    }
    const double ljj = sqrt(piv);
    for (int i = j + 1 + t; i < nl; i += nt) A[P(i, j)] /= ljj;
    __syncthreads();
    if (t == 0) A[P(j, j)] = ljj;
    const int m = nl - j - 1;
    for (int q = t; q < m * (m + 1) / 2; q += nt) {
      int ii, kk;
      unpack_lower(q, ii, kk);
      const int i = j + 1 + ii, k = j + 1 + kk;
      A[P(i, k)] -= A[P(i, j)] * A[P(k, j)];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (t == 0) atomicMin(flag, (int)K);
    return;
  }
  // X = L^-1 in place, columns from the last: X_ij = -(sum_{k=j+1..i} X_ik L_kj) / L_jj
  for (int j = nl - 1; j >= 0; --j) {
    const double ljj = A[P(j, j)];
    double v[2] = {0.0, 0.0};
    int c = 0;
    for (int i = j + 1 + t; i < nl; i += nt, ++c) {
      double s = 0.0;
      for (int k = j + 1; k <= i; ++k) s += A[P(i, k)] * A[P(k, j)];
      v[c] = -s / ljj;
    }
    __syncthreads();
    c = 0;
    for (int i = j + 1 + t; i < nl; i += nt, ++c) A[P(i, j)] = v[c];
    if (t == 0) A[P(j, j)] = 1.0 / ljj;
    __syncthreads();
  }
  if (gram) {
    // element-major: the BF16 element pass reads one element per work-group
    for (int q = t; q < npk; q += nt) {
      int i, j;
      unpack_lower(q, i, j);
      out[K * npk + q] = cast_out<T>(A[P(i, j)] * dinv[j]);
    }
    return;
  }
  // Atil_ij = dinv_i dinv_j sum_{k >= i} X_ki X_kj  (i >= j)
  for (int q = t; q < npk; q += nt) {
    int i, j;
    unpack_lower(q, i, j);
    double s = 0.0;
    for (int k = i; k < nl; ++k) s += A[P(k, i)] * A[P(k, j)];
    out[packed_at(q, K, E, og, npk)] = cast_out<T>(s * dinv[i] * dinv[j]);
  }
}

// Inverse of one small SPD matrix (the shared reference matrix of affine H1),
// by one thread in global memory: L (work, lower) then Minv = L^-T L^-1.
__global__ void k_small_inverse(const double* __restrict__ M, int nl, double* __restrict__ L,
                                double* __restrict__ Minv, int* __restrict__ flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int q = 0; q < nl * nl; ++q) L[q] = M[q];
  for (int j = 0; j < nl; ++j) {
    double piv = L[j * nl + j];
    for (int k = 0; k < j; ++k) piv -= L[j * nl + k] * L[j * nl + k];
    if (!(piv > 0.0) || !isfinite(piv)) {
      *flag = 0;
      return;
    }
    const double ljj = sqrt(piv);
    L[j * nl + j] = ljj;
    for (int i = j + 1; i < nl; ++i) {
      double s = L[i * nl + j];
      for (int k = 0; k < j; ++k) s -= L[i * nl + k] * L[j * nl + k];
      L[i * nl + j] = s / ljj;
    }
  }
  // X = L^-1 into the strict upper part's mirror: store X column-major in Minv
  for (int c = 0; c < nl; ++c) {
    for (int i = 0; i < nl; ++i) Minv[c * nl + i] = 0.0;
    Minv[c * nl + c] = 1.0 / L[c * nl + c];
    for (int i = c + 1; i < nl; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += L[i * nl + k] * Minv[c * nl + k];
      Minv[c * nl + i] = -s / L[i * nl + i];
    }
  }
  // L <- X^T X (symmetric), then copy to Minv
  for (int i = 0; i < nl; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < nl; ++k) s += Minv[i * nl + k] * Minv[j * nl + k];
      L[i * nl + j] = s;
      L[j * nl + i] = s;
    }
  for (int q = 0; q < nl * nl; ++q) Minv[q] = L[q];
}

// diag(M)_i = sum over the broken copies of DOF i of the element diagonals,
// in the fixed order of the transpose map.
__global__ void k_diag_scaled(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ slot, int64_t n,
                              int64_t E, const double* __restrict__ coef, const double* __restrict__ Mhat, int nl,
                              double* __restrict__ diag, double* __restrict__ invdiag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    const int64_t idx = slot[p];
    const int64_t l = idx / E, K = idx - l * E;
    s += coef[K] * Mhat[l * nl + l];
  }
  diag[i] = s;
  invdiag[i] = 1.0 / s;
}

__global__ void k_diag_broken(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ slot, int64_t n,
                              const double* __restrict__ diagb, double* __restrict__ diag, double* __restrict__ invdiag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) s += diagb[slot[p]];
  diag[i] = s;
  invdiag[i] = 1.0 / s;
}

__global__ void k_fill_int(int* p, int64_t n, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static int read_flag(Ctx* c, hipStream_t s, int* out) {
  BRAS_HIP(hipMemcpyAsync(out, c->flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  return BRAS_OK;
}

static int reset_flag(Ctx* c, hipStream_t s) {
  k_fill_int<<<1, 64, 0, s>>>(c->flag, 1, 0x7fffffff);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int element_setup_ordered(Ctx* c, const double* elem_d, hipStream_t s);
static int element_setup_permuted(Ctx* c, const double* elem_d, hipStream_t s);

// Element data (caller's order) -> element inverses and diag(M), and the
// internal-numbering copy of diag(M)^-1 when the handle has a patch plan.
int element_setup(Ctx* c, const double* elem_d, hipStream_t s) {
  const int st = element_setup_permuted(c, elem_d, s);
  if (st || !c->pt.invdiag_ip) return st;
  k_gather_vec<<<blocks_for(c->n, 256), 256, 0, s>>>(c->invdiag, c->pt.ip2g, c->n, c->pt.invdiag_ip);
  BRAS_HIP(hipGetLastError());
  BRAS_HIP(hipStreamSynchronize(s));
  return BRAS_OK;
}

// The caller's number of internal element K (errors name the caller's element).
static int caller_element(const Ctx* c, int K) {
  if (!c->pt.perm || K < 0 || K >= c->E) return K;
  int32_t u = K;
  if (hipMemcpy(&u, c->pt.perm + K, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess) return K;
  return u;
}

// Element data arrive in the caller's element order; with a patch plan the
// handle's order is patch-major, so they are permuted first.
static int element_setup_permuted(Ctx* c, const double* elem_d, hipStream_t s) {
  if (!c->pt.perm) return element_setup_ordered(c, elem_d, s);
  const int w = c->form == BRAS_ELEM_SCALED_REF ? 1 : (c->form == BRAS_ELEM_METRIC_REF ? c->nsym : c->nl * c->nl);
  struct Tmp {
    double* p = nullptr;
    ~Tmp() {
      if (p) (void)hipFree(p);
    }
  } tmp;
  if (hipMalloc((void**)&tmp.p, sizeof(double) * (size_t)c->E * w) != hipSuccess)
    return fail(BRAS_ENOMEM, "element data permutation buffer allocation failed");
  k_permute_rows<<<blocks_for(c->E * w, 256), 256, 0, s>>>(elem_d, c->pt.perm, c->E, w, tmp.p);
  BRAS_HIP(hipGetLastError());
  const int st = element_setup_ordered(c, tmp.p, s);
  (void)hipStreamSynchronize(s);   // tmp is read by the kernels just queued
  return st;
}

static int element_setup_ordered(Ctx* c, const double* elem_d, hipStream_t s) {
  const int64_t E = c->E;
  const int nl = c->nl;
  int st;
  if ((st = reset_flag(c, s))) return st;
  if (c->form == BRAS_ELEM_SCALED_REF) {
    k_scaled_coef<<<blocks_for(E, 256), 256, 0, s>>>(elem_d, E, c->coef, c->icoef, c->flag);
    BRAS_HIP(hipGetLastError());
    int f;
    if ((st = read_flag(c, s, &f))) return st;
    if (f != 0x7fffffff)
      return fail(BRAS_ENOTSPD, "element %d: coefficient c_K must be positive and finite", caller_element(c, f));
    k_diag_scaled<<<blocks_for(c->n, 256), 256, 0, s>>>(c->rowptr, c->slot, c->n, E, c->coef, c->ref, nl, c->diag,
                                                        c->invdiag);
    BRAS_HIP(hipGetLastError());
    BRAS_HIP(hipStreamSynchronize(s));
    return BRAS_OK;
  }
  const double* G = nullptr;
  const double* Mexp = nullptr;
  int mode;
  if (c->form == BRAS_ELEM_METRIC_REF) {
    k_transpose_coef<<<blocks_for(E * c->nsym, 256), 256, 0, s>>>(elem_d, E, c->nsym, c->coef);
    BRAS_HIP(hipGetLastError());
    G = c->coef;
    mode = 0;
  } else {
    Mexp = elem_d;
    mode = 1;
  }
  double* mpack = c->mpack;   // non-null when the mass pass reads packed M_K
  size_t lds = sizeof(double) * (npack_of(nl) + 8 + nl);
  const int gram = c->prec == BRAS_BF16 ? 1 : 0;
  if (lds > 64 * 1024) return fail(BRAS_EINVAL, "n_loc %d too large for the element factorisation", nl);
  // broken diagonal of M_K, freed on every path below
  struct Scratch {
    double* p = nullptr;
    ~Scratch() {
      if (p) (void)hipFree(p);
    }
  } diag_scratch;
  BRAS_HIP(hipMalloc((void**)&diag_scratch.p, sizeof(double) * c->nbr));
  double* diagb = diag_scratch.p;
  if (c->prec == BRAS_FP64)
    k_elem_factor<double><<<(unsigned)E, 64, lds, s>>>(mode, E, nl, c->nsym, c->ref, G, Mexp, c->l2g, c->invd, diagb,
                                                        mpack, c->mgroup, (double*)c->ainv, c->agroup, 0, c->flag);
  else if (c->prec == BRAS_FP32)
    k_elem_factor<float><<<(unsigned)E, 64, lds, s>>>(mode, E, nl, c->nsym, c->ref, G, Mexp, c->l2g, c->invd, diagb,
                                                       mpack, c->mgroup, (float*)c->ainv, c->agroup, 0, c->flag);
  else
    k_elem_factor<__bf16><<<(unsigned)E, 64, lds, s>>>(mode, E, nl, c->nsym, c->ref, G, Mexp, c->l2g, c->invd, diagb,
                                                        mpack, c->mgroup, (__bf16*)c->ainv, c->agroup, gram,
                                                        c->flag);
  BRAS_HIP(hipGetLastError());
  k_diag_broken<<<blocks_for(c->n, 256), 256, 0, s>>>(c->rowptr, c->slot, c->n, diagb, c->diag, c->invdiag);
  BRAS_HIP(hipGetLastError());
  int f;
  st = read_flag(c, s, &f);   // synchronises s, so the scratch can be freed on return
  if (st) return st;
  if (f != 0x7fffffff)
    return fail(BRAS_ENOTSPD, "element %d: mass matrix is not symmetric positive definite", caller_element(c, f));
  return BRAS_OK;
}

static void free_ctx(Ctx* c) {
  if (!c) return;
  void* ptrs[] = {c->l2g, c->mult, c->invd, c->rowptr, c->chunk, c->slot, c->ref, c->refinv, c->coef, c->icoef, c->ainv,
                  c->symtab, c->mpack, c->diag, c->invdiag, c->zb, c->partial, c->flag, c->l2g_dir,
                  c->pt.perm, c->pt.pe, c->pt.pd, c->pt.pnl, c->pt.pdof, c->pt.code, c->pt.sbase, c->pt.srp,
                  c->pt.spos, c->pt.sdof, c->pt.part, c->pt.ip2g, c->pt.pidx, c->pt.invd_ip, c->pt.invdiag_ip};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  cg_free(c);
  if (c->s_int) (void)hipStreamDestroy(c->s_int);
  delete c;
}

template <typename T>
static int dalloc(T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
  if (e != hipSuccess) return fail(BRAS_ENOMEM, "hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
  return BRAS_OK;
}

}  // namespace bras

using namespace bras;

// Patch plan of the handle (host partition of the validated map), the map in
// patch-major element order, and the device copy of the plan.  Skipped for
// element forms without a patch kernel, for the scaled H1 form unless
// BRAS_PATCH_SCALED=1, and when BRAS_PATCH=0 is set in the environment;
// BRAS_PATCH_ELEMS / BRAS_PATCH_DOFS change the patch size and DOF cap.
static int patch_setup(Ctx* c, hipStream_t s) {
  const char* env = getenv("BRAS_PATCH");
  if (env && atoi(env) == 0) return BRAS_OK;
  if (!patch_supported(c->form, c->prec, c->nl)) return BRAS_OK;
  // scaled H1: the element / reduce passes are faster on the meshes measured
  // (the element-pass matrix-core product there); the patch form on request
  if (c->form == BRAS_ELEM_SCALED_REF) {
    const char* e = getenv("BRAS_PATCH_SCALED");
    if (!e || atoi(e) == 0) return BRAS_OK;
  }
  // the matrix-core pass of the scaled H1 form holds two 16-element column
  // tiles per wavefront above n_loc 20 (patches of at most 128 elements)
  int P = (c->form == BRAS_ELEM_SCALED_REF && c->nl > 20) ? 128 : kPatchElems, D = kPatchMaxDofs;
  if (const char* e = getenv("BRAS_PATCH_ELEMS")) P = atoi(e);
  if (const char* e = getenv("BRAS_PATCH_DOFS")) D = atoi(e);
  if (const char* e = getenv("BRAS_PATCH_XCD")) c->patch_xcd = atoi(e) != 0;
  if (P < 1 || P > kPatchBlock) return fail(BRAS_EINVAL, "BRAS_PATCH_ELEMS must be in 1..%d", kPatchBlock);
  if (D < 1 || D > 65536) return fail(BRAS_EINVAL, "BRAS_PATCH_DOFS must be in 1..65536");
  const int64_t n = c->n, E = c->E, nl = c->nl, nbr = c->nbr;
  std::vector<int32_t> l2g(nbr), mult(n);
  BRAS_HIP(hipMemcpyAsync(l2g.data(), c->l2g, sizeof(int32_t) * nbr, hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipMemcpyAsync(mult.data(), c->mult, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  PatchPlan plan;
  if (build_patch_plan(n, E, (int)nl, l2g.data(), mult.data(), P, D, &plan) != 0) return BRAS_OK;
  std::vector<int32_t> il2g(nbr);
  for (int64_t K = 0; K < E; ++K)
    for (int l = 0; l < nl; ++l) il2g[K * nl + l] = l2g[(int64_t)plan.perm[K] * nl + l];
  PatchDev& pt = c->pt;
  auto up = [&](auto** dst, const auto& v) -> int {
    typedef typename std::remove_reference<decltype(v[0])>::type T;
    const size_t cnt = v.size() > 0 ? v.size() : 1;
    if (hipMalloc((void**)dst, sizeof(T) * cnt) != hipSuccess)
      return fail(BRAS_ENOMEM, "patch plan allocation failed");
    if (!v.empty() && hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess)
      return fail(BRAS_EHIP, "patch plan copy failed");
    return BRAS_OK;
  };
  int st;
  if ((st = up(&pt.perm, plan.perm)) || (st = up(&pt.pe, plan.pe)) || (st = up(&pt.pd, plan.pd)) ||
      (st = up(&pt.pnl, plan.pnl)) || (st = up(&pt.pdof, plan.pdof)) || (st = up(&pt.code, plan.code)) ||
      (st = up(&pt.sbase, plan.sbase)) || (st = up(&pt.srp, plan.srp)) || (st = up(&pt.spos, plan.spos)) ||
      (st = up(&pt.sdof, plan.sdof)) || (st = up(&pt.ip2g, plan.ip2g)) || (st = up(&pt.pidx, plan.pidx)))
    return st;
  pt.nloc_total = plan.nloc_total;
  if (hipMalloc((void**)&pt.invd_ip, sizeof(double) * n) != hipSuccess ||
      hipMalloc((void**)&pt.invdiag_ip, sizeof(double) * n) != hipSuccess)
    return fail(BRAS_ENOMEM, "patch plan allocation failed");
  k_gather_vec<<<blocks_for(n, 256), 256, 0, s>>>(c->invd, pt.ip2g, n, pt.invd_ip);
  BRAS_HIP(hipGetLastError());
  BRAS_HIP(hipMemcpy(c->l2g, il2g.data(), sizeof(int32_t) * nbr, hipMemcpyHostToDevice));
  pt.ns = (int64_t)plan.sdof.size();
  pt.nspart = (int64_t)plan.spos.size();
  if (hipMalloc((void**)&pt.part, sizeof(double) * (size_t)(pt.nspart > 0 ? pt.nspart : 1)) != hipSuccess)
    return fail(BRAS_ENOMEM, "patch partial-sum buffer allocation failed");
  const int64_t nb2 = (pt.ns + kPatchSharedPerBlock - 1) / kPatchSharedPerBlock;
  pt.nb2 = (int)(nb2 < kPatchSharedBlocks ? (nb2 > 0 ? nb2 : 1) : kPatchSharedBlocks);
  pt.lbits = plan.lbits;
  pt.maxrank = plan.maxrank;
  pt.maxdofs = plan.maxdofs;
  for (int64_t q = 0; q < plan.npatch; ++q) pt.maxelems = std::max(pt.maxelems, plan.pe[q + 1] - plan.pe[q]);
  pt.npatch = plan.npatch;   // last: the plan is complete
  return BRAS_OK;
}

extern "C" int bras_geometry(int family, int dim, int64_t nvert, const double* coords_d, int64_t ncell,
                             const int32_t* cells_d, const double* rho_d, double* elem_d, void* stream) {
  clear_error();
  BRAS_CHECK(dim == 2 || dim == 3, "dim must be 2 or 3");
  BRAS_CHECK(family >= BRAS_H1 && family <= BRAS_HDIV2, "unknown family %d", family);
  BRAS_CHECK(coords_d && cells_d && elem_d, "null pointer argument");
  BRAS_CHECK(nvert > 0 && ncell > 0, "empty mesh");
  hipStream_t s = (hipStream_t)stream;
  k_geometry<<<(unsigned)((ncell + 255) / 256), 256, 0, s>>>(family, dim, coords_d, cells_d, ncell, nvert, rho_d,
                                                             elem_d, nsym_of(dim));
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

extern "C" int bras_setup(bras_handle* h, int64_t n, int64_t E, int n_loc, const int32_t* l2g_d, int form,
                          const double* ref_d, const double* elem_d, int nsym, int apply_prec, int max_rhs,
                          void* stream) {
  clear_error();
  BRAS_CHECK(h, "null handle pointer");
  *h = nullptr;
  BRAS_CHECK(n > 0 && E > 0 && n_loc > 0, "sizes must be positive (n=%lld E=%lld n_loc=%d)", (long long)n,
             (long long)E, n_loc);
  BRAS_CHECK(n_loc <= 120, "n_loc %d above the supported maximum 120", n_loc);
  BRAS_CHECK(E * n_loc < (1LL << 31) && n < (1LL << 31), "problem too large for int32 maps");
  BRAS_CHECK(l2g_d && elem_d, "null map or element data");
  BRAS_CHECK(form == BRAS_ELEM_EXPLICIT || form == BRAS_ELEM_SCALED_REF || form == BRAS_ELEM_METRIC_REF,
             "unknown element form %d", form);
  BRAS_CHECK(form == BRAS_ELEM_EXPLICIT || ref_d, "reference tables required for this form");
  BRAS_CHECK(form != BRAS_ELEM_METRIC_REF || (nsym >= 1 && nsym <= 6), "nsym must be in 1..6 for METRIC_REF");
  BRAS_CHECK(apply_prec == BRAS_FP64 || apply_prec == BRAS_FP32 || apply_prec == BRAS_BF16, "unknown precision %d",
             apply_prec);
  BRAS_CHECK(!(apply_prec == BRAS_BF16 && form == BRAS_ELEM_SCALED_REF), "BF16 requires METRIC_REF or EXPLICIT");
  BRAS_CHECK(!(apply_prec != BRAS_FP64 && form == BRAS_ELEM_SCALED_REF), "SCALED_REF applies in FP64 only");
  BRAS_CHECK(max_rhs >= 1 && max_rhs <= 256, "max_rhs must be in 1..256");
  BRAS_CHECK((uint64_t)n * (uint64_t)max_rhs * 8u < (1ull << 32),
             "n * max_rhs * 8 bytes must stay below 4 GiB (a conforming block vector)");
  hipStream_t s = (hipStream_t)stream;
  Ctx* c = new Ctx();
  int st = BRAS_OK;
#define TRY(x)                 \
  do {                         \
    if ((st = (x)) != BRAS_OK) { \
      free_ctx(c);             \
      return st;               \
    }                          \
  } while (0)
  c->n = n;
  c->E = E;
  c->nl = n_loc;
  c->nbr = E * n_loc;
  c->form = form;
  c->nsym = form == BRAS_ELEM_METRIC_REF ? nsym : 0;
  c->prec = apply_prec;
  c->max_rhs = max_rhs;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
    delete c;
    return fail(BRAS_EHIP, "device query failed");
  }
  if (hipStreamCreateWithFlags(&c->s_int, hipStreamNonBlocking) != hipSuccess) {
    delete c;
    return fail(BRAS_EHIP, "hipStreamCreateWithFlags failed");
  }
  // device address of the fixed workspace of bras_apply_noalloc, once per device
  TRY(scratch_init(c->device, nullptr));
  TRY(dalloc(&c->l2g, c->nbr));
  TRY(dalloc(&c->mult, n));
  TRY(dalloc(&c->invd, n));
  TRY(dalloc(&c->rowptr, n + 1));
  TRY(dalloc(&c->slot, c->nbr));
  TRY(dalloc(&c->flag, 4));
  TRY(dalloc(&c->diag, n));
  TRY(dalloc(&c->invdiag, n));
  // maps
  k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>(c->mult, n, 0);
  if ((st = reset_flag(c, s))) { free_ctx(c); return st; }
  k_map_check<<<blocks_for(E, 256), 256, 0, s>>>(l2g_d, E, n_loc, n, c->l2g, c->mult, c->flag);
  if (hipGetLastError() != hipSuccess) { free_ctx(c); return fail(BRAS_EHIP, "map check launch failed"); }
  int f;
  TRY(read_flag(c, s, &f));
  if (f != 0x7fffffff) {
    free_ctx(c);
    return fail(BRAS_EINVAL, "element %d: local-to-global entries out of range or repeated", f);
  }
  TRY(reset_flag(c, s));
  k_mult<<<blocks_for(n, 256), 256, 0, s>>>(c->mult, n, c->invd, c->flag);
  TRY(read_flag(c, s, &f));
  if (f != 0x7fffffff) {
    free_ctx(c);
    return fail(BRAS_EINVAL, "DOF %d has no broken copy (P must have full column rank)", f);
  }
  TRY(patch_setup(c, s));
  {
    const int64_t per = (int64_t)kScanBlock * kScanItems;
    const int64_t nb = (n + per - 1) / per;
    int32_t* bsum = nullptr;
    int32_t* fill = nullptr;
    int32_t* key = nullptr;
    TRY(dalloc(&bsum, nb + 1));
    TRY(dalloc(&fill, n));
    TRY(dalloc(&key, c->nbr));
    k_scan_local<<<(unsigned)nb, kScanBlock, 0, s>>>(c->mult, n, c->rowptr, bsum);
    k_scan_sums<<<1, 64, 0, s>>>(bsum, nb, c->rowptr + n);
    k_scan_add<<<blocks_for(n, 256), 256, 0, s>>>(c->rowptr, n, bsum);
    k_fill_int<<<blocks_for(n, 256), 256, 0, s>>>(fill, n, 0);
    k_fill_slots<<<blocks_for(c->nbr, 256), 256, 0, s>>>(c->l2g, c->nbr, c->rowptr, fill, key);
    k_sort_rows<<<blocks_for(n, 256), 256, 0, s>>>(c->rowptr, n, n_loc, E, key, c->slot);
    hipError_t e = hipGetLastError();
    (void)hipStreamSynchronize(s);
    (void)hipFree(bsum);
    (void)hipFree(fill);
    (void)hipFree(key);
    if (e != hipSuccess) { free_ctx(c); return fail(BRAS_EHIP, "transpose-map kernels failed: %s", hipGetErrorString(e)); }
  }
  {
    // reduce chunks: consecutive rows, at most 512 rows and 2048 broken
    // copies each (a longer single row gets a chunk of its own)
    std::vector<int32_t> rp(n + 1);
    if (hipMemcpy(rp.data(), c->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess) {
      free_ctx(c);
      return fail(BRAS_EHIP, "copy of the transpose map failed");
    }
    std::vector<int32_t> ch;
    ch.push_back(0);
    int64_t i = 0;
    while (i < n) {
      int rows = 0;
      int64_t cnt = 0;
      while (i < n && rows < 512 && (rows == 0 || cnt + (rp[i + 1] - rp[i]) <= 2048)) {
        cnt += rp[i + 1] - rp[i];
        ++i;
        ++rows;
      }
      ch.push_back((int32_t)i);
    }
    c->nchunk = (int64_t)ch.size() - 1;
    TRY(dalloc(&c->chunk, ch.size()));
    if (hipMemcpy(c->chunk, ch.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice) != hipSuccess) {
      free_ctx(c);
      return fail(BRAS_EHIP, "copy of the reduce chunks failed");
    }
  }
  // element data
  const int nn = n_loc * n_loc;
  if (form == BRAS_ELEM_SCALED_REF) {
    TRY(dalloc(&c->ref, nn));
    TRY(dalloc(&c->refinv, nn));
    TRY(dalloc(&c->coef, E));
    TRY(dalloc(&c->icoef, E));
    if (hipMemcpyAsync(c->ref, ref_d, sizeof(double) * nn, hipMemcpyDeviceToDevice, s) != hipSuccess) {
      free_ctx(c);
      return fail(BRAS_EHIP, "copy of reference table failed");
    }
    TRY(reset_flag(c, s));
    double* work = nullptr;
    TRY(dalloc(&work, nn));
    k_small_inverse<<<1, 64, 0, s>>>(c->ref, n_loc, work, c->refinv, c->flag);
    st = read_flag(c, s, &f);
    (void)hipFree(work);
    if (st) { free_ctx(c); return st; }
    if (f != 0x7fffffff) { free_ctx(c); return fail(BRAS_ENOTSPD, "reference mass matrix is not SPD"); }
  } else {
    if (form == BRAS_ELEM_METRIC_REF) {
      TRY(dalloc(&c->ref, (size_t)c->nsym * nn));
      if (hipMemcpyAsync(c->ref, ref_d, sizeof(double) * c->nsym * nn, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        free_ctx(c);
        return fail(BRAS_EHIP, "copy of reference tables failed");
      }
      TRY(dalloc(&c->coef, (size_t)c->nsym * E));
      // the mass pass rebuilds M_K from packed pair tables when one lane can
      // hold an element, otherwise it reads a packed float64 copy of M_K
      if (n_loc <= kLaneMaxNL) {
        const int ss = sym_stride(c->nsym);
        const int64_t cnt = (int64_t)npack_of(n_loc) * ss;
        TRY(dalloc(&c->symtab, (size_t)cnt));
        k_pack_sym<<<blocks_for(cnt, 256), 256, 0, s>>>(c->ref, n_loc, c->nsym, ss, c->symtab);
        if (hipGetLastError() != hipSuccess) { free_ctx(c); return fail(BRAS_EHIP, "pair table packing failed"); }
      } else {
        c->mgroup = 0;   // element-major, read by the per-element pass
        TRY(dalloc(&c->mpack, (size_t)npack_of(n_loc) * E));
      }
    } else {
      c->mgroup = packed_group(n_loc, sizeof(double));
      const size_t cnt = packed_slots(n_loc, c->mgroup) * E;
      TRY(dalloc(&c->mpack, cnt));
      if (hipMemsetAsync(c->mpack, 0, sizeof(double) * cnt, s) != hipSuccess) {
        free_ctx(c);
        return fail(BRAS_EHIP, "clearing packed element matrices failed");
      }
    }
    size_t esz = apply_prec == BRAS_FP64 ? 8 : (apply_prec == BRAS_FP32 ? 4 : 2);
    c->agroup = apply_prec == BRAS_BF16 ? 0 : packed_group(n_loc, esz);
    c->ainv_bytes = esz * packed_slots(n_loc, c->agroup) * E;
    TRY(dalloc((char**)&c->ainv, c->ainv_bytes));
    if (hipMemsetAsync(c->ainv, 0, c->ainv_bytes, s) != hipSuccess) {
      free_ctx(c);
      return fail(BRAS_EHIP, "clearing packed element inverses failed");
    }
  }
  TRY(element_setup(c, elem_d, s));
  if (apply_prec == BRAS_BF16) TRY(bf16_setup(c, s));
  // workspace
  size_t zbytes = sizeof(double) * (size_t)c->nbr * max_rhs;
  TRY(dalloc((char**)&c->zb, zbytes));
  TRY(dalloc(&c->partial, (size_t)(c->nchunk + 1024) * max_rhs));
  if (hipStreamSynchronize(s) != hipSuccess) { free_ctx(c); return fail(BRAS_EHIP, "setup synchronisation failed"); }
#undef TRY
  *h = (bras_handle)c;
  return BRAS_OK;
}

extern "C" int bras_update(bras_handle h, const double* elem_d, void* stream) {
  clear_error();
  BRAS_CHECK(h && elem_d, "null argument");
  Ctx* c = (Ctx*)h;
  hipStream_t s = (hipStream_t)stream;
  int st = element_setup(c, elem_d, s);
  if (st) return st;
  BRAS_HIP(hipStreamSynchronize(s));
  return BRAS_OK;
}

extern "C" int bras_destroy(bras_handle h) {
  clear_error();
  if (!h) return BRAS_OK;
  Ctx* c = (Ctx*)h;
  (void)hipDeviceSynchronize();
  free_ctx(c);
  return BRAS_OK;
}
