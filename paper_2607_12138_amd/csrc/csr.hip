// Assembled operators: the CSR forms of M and M_bras^-1 (eq.
// mass_and_bras_element_sums; both share the sparsity of M) built on the
// device from the element data the handle holds, and a CSR product.
//
// Row i holds every DOF of every element containing a copy of DOF i.  Entry
// (i, j) is the sum, over the copies (K, l) of i in transpose-map order, of
// the element entry for (l, m) with pi(K, m) = j:
//   mass: M_K[l][m]
//   BRAS: d_i^-1 (M_K^-1)[l][m] d_j^-1   (the stored folded inverses, or for
//         the scaled H1 form d_i^-1 c_K^-1 Mhat^-1[l][m] d_j^-1)
// so the sums are taken in one fixed order, whatever the launch shape.
#include "internal.h"

namespace bras {
namespace {

constexpr int kCsrCap = 2048;   // candidate columns d_i * n_loc of one row

struct ElemView {
  int form, prec, nl, nsym;
  int64_t E;
  const double* ref;      // SCALED: Mhat; METRIC: S [nsym][nl*nl]
  const double* refinv;   // SCALED: Mhat^-1
  const double* coef;     // SCALED: c_K; METRIC: G [nsym][E]
  const double* icoef;    // SCALED: 1 / c_K
  const double* invd;     // d_i^-1
  const double* mpack;    // packed M_K (EXPLICIT, or METRIC with n_loc > 36)
  int mgroup;
  const void* ainv;       // folded inverses (FP64 / FP32)
  int agroup;
};

__device__ inline int packed_index(int l, int m) {
  const int a = l > m ? l : m, b = l > m ? m : l;
  return a * (a + 1) / 2 + b;
}

__device__ inline double mass_entry(const ElemView& v, int64_t K, int l, int m) {
  if (v.form == BRAS_ELEM_SCALED_REF) return v.coef[K] * v.ref[l * v.nl + m];
  const int npk = v.nl * (v.nl + 1) / 2;
  if (v.mpack) return v.mpack[packed_at(packed_index(l, m), K, v.E, v.mgroup, npk)];
  double s = 0.0;
  for (int p = 0; p < v.nsym; ++p) s += v.coef[(int64_t)p * v.E + K] * v.ref[(int64_t)p * v.nl * v.nl + l * v.nl + m];
  return s;
}

__device__ inline double bras_entry(const ElemView& v, int64_t K, int l, int m, int64_t i, int32_t j) {
  if (v.form == BRAS_ELEM_SCALED_REF) return v.invd[i] * v.icoef[K] * v.refinv[l * v.nl + m] * v.invd[j];
  const int npk = v.nl * (v.nl + 1) / 2;
  const int64_t at = packed_at(packed_index(l, m), K, v.E, v.agroup, npk);
  return v.prec == BRAS_FP64 ? ((const double*)v.ainv)[at] : (double)((const float*)v.ainv)[at];
}

// One work-group (one wavefront) per row, rows grid-strided: gather the
// candidate columns of row i, sort them (bitonic, in LDS), then count the
// distinct ones (fill == 0) or write them with their summed values.
template <int OP>
__global__ void __launch_bounds__(64) k_csr_rows(int fill, ElemView v, int64_t n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ slot, const int32_t* __restrict__ l2g,
                                                 int32_t* __restrict__ cnt, const int64_t* __restrict__ crow,
                                                 int32_t* __restrict__ col, double* __restrict__ val) {
  __shared__ int32_t cand[kCsrCap];
  __shared__ int32_t ucol[kCsrCap];
  __shared__ double acc[kCsrCap];
  const int t = threadIdx.x;
  const int nl = v.nl;
  const int64_t E = v.E;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const int32_t p0 = rowptr[i];
    const int nc = rowptr[i + 1] - p0;
    const int m = nc * nl;             // the host checked m <= kCsrCap
    int m2 = 1;
    while (m2 < m) m2 <<= 1;
    for (int q = t; q < m2; q += 64) {
      int32_t cv = 0x7fffffff;
      if (q < m) {
        const int pc = q / nl, j = q - pc * nl;
        const int32_t s = slot[p0 + pc];
        const int64_t K = s % E;
        cv = l2g[K * nl + j];
      }
      cand[q] = cv;
    }
    __syncthreads();
    for (int k = 2; k <= m2; k <<= 1)
      for (int jj = k >> 1; jj > 0; jj >>= 1) {
        for (int q = t; q < m2; q += 64) {
          const int pq = q ^ jj;
          if (pq > q) {
            const int32_t a = cand[q], b = cand[pq];
            if ((a > b) == ((q & k) == 0)) {
              cand[q] = b;
              cand[pq] = a;
            }
          }
        }
        __syncthreads();
      }
    int u = 0;   // distinct columns, compacted in ascending order
    for (int q0 = 0; q0 < m; q0 += 64) {
      const int q = q0 + t;
      const bool head = q < m && (q == 0 || cand[q] != cand[q - 1]);
      const uint64_t mask = __ballot(head);
      if (head) ucol[u + __popcll(mask & ((1ull << t) - 1ull))] = cand[q];
      u += __popcll(mask);
    }
    __syncthreads();
    if (!fill) {
      if (t == 0) cnt[i] = u;
      continue;
    }
    for (int q = t; q < u; q += 64) acc[q] = 0.0;
    __syncthreads();
    for (int pc = 0; pc < nc; ++pc) {
      const int32_t s = slot[p0 + pc];
      const int64_t l = s / E, K = s - l * E;
      // the DOFs of one element are distinct: no two lanes share a position
      for (int j = t; j < nl; j += 64) {
        const int32_t cj = l2g[K * nl + j];
        int lo = 0, hi = u - 1;
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (ucol[mid] < cj) lo = mid + 1; else hi = mid;
        }
        acc[lo] += OP == BRAS_OP_MASS ? mass_entry(v, K, (int)l, j) : bras_entry(v, K, (int)l, j, i, cj);
      }
      __syncthreads();
    }
    const int64_t o = crow[i];
    for (int q = t; q < u; q += 64) {
      col[o + q] = ucol[q];
      val[o + q] = acc[q];
    }
    __syncthreads();
  }
}

// y = A x, 16 lanes per row (rows grid-strided), each lane a strided part of
// the row, then a fixed butterfly over the 16 lanes: the same order for every
// launch shape.
__global__ void __launch_bounds__(256) k_csr_spmv(int64_t n, const int64_t* __restrict__ rowptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  const int g = threadIdx.x & 15;
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 4);
  for (int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 4) + (threadIdx.x >> 4); i < n; i += stride) {
    double s = 0.0;
    const int64_t p1 = rowptr[i + 1];
    for (int64_t p = rowptr[i] + g; p < p1; p += 16) s = fma(val[p], x[col[p]], s);
    for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
    if (g == 0) y[i] = s;
  }
}

int view_of(const Ctx* c, ElemView* v) {
  if (c->form != BRAS_ELEM_SCALED_REF && c->prec == BRAS_BF16)
    return fail(BRAS_EINVAL, "assembled BRAS needs FP64 or FP32 element inverses (the handle stores BF16 Gram factors)");
  *v = ElemView{c->form, c->prec, c->nl, c->nsym, c->E, c->ref, c->refinv, c->coef, c->icoef, c->invd,
                c->mpack, c->mgroup, c->ainv, c->agroup};
  return BRAS_OK;
}

int max_candidates(const Ctx* c, hipStream_t s, int64_t* out) {
  std::vector<int32_t> mult(c->n);
  BRAS_HIP(hipMemcpyAsync(mult.data(), c->mult, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  int32_t mx = 0;
  for (int32_t m : mult) mx = m > mx ? m : mx;
  *out = (int64_t)mx * c->nl;
  return BRAS_OK;
}

__global__ void __launch_bounds__(256) k_csr_diag(int64_t n, const double* __restrict__ invdiag,
                                                  int64_t* __restrict__ rowptr, int32_t* __restrict__ col,
                                                  double* __restrict__ val) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
    rowptr[i] = i;
    if (i < n) {
      col[i] = (int32_t)i;
      val[i] = invdiag[i];
    }
  }
}

unsigned row_grid(const Ctx* c) {
  const int64_t want = (int64_t)c->ncu * 32;
  return (unsigned)(c->n < want ? c->n : want);
}

}  // namespace
}  // namespace bras

using namespace bras;

extern "C" int bras_csr_rowptr(bras_handle h, int64_t* rowptr_d, int64_t* nnz_h, void* stream) {
  clear_error();
  BRAS_CHECK(h && rowptr_d && nnz_h, "null argument");
  Ctx* c = (Ctx*)h;
  hipStream_t s = (hipStream_t)stream;
  int64_t mc;
  int st = max_candidates(c, s, &mc);
  if (st) return st;
  BRAS_CHECK(mc <= kCsrCap, "a row has %lld candidate columns (multiplicity x n_loc); at most %d are supported",
             (long long)mc, kCsrCap);
  ElemView v;
  if ((st = view_of(c, &v))) return st;
  int32_t* cnt = nullptr;
  BRAS_HIP(hipMalloc((void**)&cnt, sizeof(int32_t) * c->n));
  k_csr_rows<BRAS_OP_MASS><<<row_grid(c), 64, 0, s>>>(0, v, c->n, c->rowptr, c->slot, c->l2g, cnt, nullptr,
                                                       nullptr, nullptr);
  hipError_t e = hipGetLastError();
  std::vector<int32_t> hc(c->n);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * c->n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(cnt);
  if (e != hipSuccess) return fail(BRAS_EHIP, "CSR row count failed: %s", hipGetErrorString(e));
  std::vector<int64_t> rp(c->n + 1);
  rp[0] = 0;
  for (int64_t i = 0; i < c->n; ++i) rp[i + 1] = rp[i] + hc[i];
  BRAS_CHECK(rp[c->n] < ((int64_t)1 << 31), "the assembled operator has %lld entries; at most 2^31 - 1 are supported",
             (long long)rp[c->n]);
  BRAS_HIP(hipMemcpyAsync(rowptr_d, rp.data(), sizeof(int64_t) * (c->n + 1), hipMemcpyHostToDevice, s));
  BRAS_HIP(hipStreamSynchronize(s));
  *nnz_h = rp[c->n];
  return BRAS_OK;
}

extern "C" int bras_csr_assemble(bras_handle h, int op, const int64_t* rowptr_d, int32_t* col_d, double* val_d,
                                 void* stream) {
  clear_error();
  BRAS_CHECK(h && rowptr_d && col_d && val_d, "null argument");
  BRAS_CHECK(op == BRAS_OP_MASS || op == BRAS_OP_BRAS, "unknown operator %d", op);
  Ctx* c = (Ctx*)h;
  hipStream_t s = (hipStream_t)stream;
  int64_t mc;
  int st = max_candidates(c, s, &mc);
  if (st) return st;
  BRAS_CHECK(mc <= kCsrCap, "a row has %lld candidate columns; at most %d are supported", (long long)mc, kCsrCap);
  ElemView v;
  if ((st = view_of(c, &v))) return st;
  if (op == BRAS_OP_MASS)
    k_csr_rows<BRAS_OP_MASS><<<row_grid(c), 64, 0, s>>>(1, v, c->n, c->rowptr, c->slot, c->l2g, nullptr, rowptr_d,
                                                         col_d, val_d);
  else
    k_csr_rows<BRAS_OP_BRAS><<<row_grid(c), 64, 0, s>>>(1, v, c->n, c->rowptr, c->slot, c->l2g, nullptr, rowptr_d,
                                                         col_d, val_d);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

extern "C" int bras_csr_jacobi(bras_handle h, int64_t* rowptr_d, int32_t* col_d, double* val_d, void* stream) {
  clear_error();
  BRAS_CHECK(h && rowptr_d && col_d && val_d, "null argument");
  Ctx* c = (Ctx*)h;
  const int64_t blocks = (c->n + 256) / 256;
  const int64_t want = (int64_t)c->ncu * 8;
  k_csr_diag<<<(unsigned)(blocks < want ? blocks : want), 256, 0, (hipStream_t)stream>>>(c->n, c->invdiag, rowptr_d,
                                                                                        col_d, val_d);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

extern "C" int bras_csr_apply(int64_t n, const int64_t* rowptr_d, const int32_t* col_d, const double* val_d,
                              const double* x_d, double* y_d, void* stream) {
  clear_error();
  BRAS_CHECK(n >= 0, "negative size");
  if (n == 0) return BRAS_OK;
  BRAS_CHECK(rowptr_d && col_d && val_d && x_d && y_d, "null argument");
  BRAS_CHECK(x_d != y_d, "x and y must not overlap");
  int dev = 0, ncu = 1;
  BRAS_HIP(hipGetDevice(&dev));
  BRAS_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t want = (int64_t)ncu * 16, need = (n + 15) / 16;
  k_csr_spmv<<<(unsigned)(need < want ? need : want), 256, 0, (hipStream_t)stream>>>(n, rowptr_d, col_d, val_d, x_d,
                                                                                    y_d);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}
