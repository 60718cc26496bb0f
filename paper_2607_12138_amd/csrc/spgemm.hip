// Sparse products for the Schur-complement approximations of Section 4:
// -St = C + G Mt^-1 G^T (eq. approx_positive_schur_general) is sparse when
// Mt^-1 is (M_bras^-1 has the sparsity of M), and is formed from the
// assembled operator as two products, (G Mt^-1) G^T, with the transpose of G.
//
// C = A B (CSR, int64 row pointers, int32 columns ascending and distinct
// within each row, float64 values): one wavefront per row of C.  The
// candidates of row i (the entries of the B rows that row i of A selects)
// are keyed (column, candidate index) in LDS and sorted (bitonic); the
// distinct columns are counted, or each sums its products in candidate
// order, i.e. in the order of A's columns, so the result does not depend on
// the launch shape.  Every step is parallel over the wavefront: a wave scan
// of the B row lengths, independent loads of all products.  Rows past 1024
// A entries or candidates (by default; up to 2048 can stay in LDS) are
// sorted in device memory instead, in batches, by a stable radix sort that
// keeps the candidate order within a column: the same sums, bit for bit.
//
// A^T: a stable radix sort of the entries by column (hipCUB), so each row of
// A^T lists A's rows in ascending order; exact (no arithmetic).
#include <cstdlib>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace bras {
namespace {

constexpr int kGemmCap = 2048;    // candidate products of one row of C
constexpr int kGemmSmall = 1024;  // rows up to this many run with half the LDS (twice the work-groups per CU)

// Rows with more candidates or A entries than this take the sort in device
// memory.  Default kGemmSmall: on the Schur products of 48^3 N1curl_2 and
// 24^3 P3 the sort forms the rows between 1024 and 2048 candidates about
// 2.4x faster than the kGemmCap variant at 3 work-groups per CU, and lower
// limits gain nothing on G Mt^-1 and lose on (G Mt^-1) G^T.  The
// environment variable BRAS_SPGEMM_LDS_MAX (0 .. kGemmCap) sets another.
int lds_max() {
  const char* e = std::getenv("BRAS_SPGEMM_LDS_MAX");
  if (!e || !*e) return kGemmSmall;
  const long long v = std::atoll(e);
  return v < 0 ? 0 : (v > kGemmCap ? kGemmCap : (int)v);
}

// Bitonic sort of key[0 .. m2) (m2 a power of two, at most kGemmCap) by one
// wavefront: every stage first loads all of this lane's pairs, then
// compares and stores, so a stage costs one LDS round trip, not one per pair.
template <int CAP, typename K>
__device__ inline void wave_bitonic(K* key, int m2) {
  constexpr int kPer = CAP / 64;
  const int t = threadIdx.x;
  for (int kk = 2; kk <= m2; kk <<= 1)
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      K xa[kPer], xb[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int q = t + 64 * u, pq = q ^ jj;
        if (q < m2 && pq > q) {
          xa[u] = key[q];
          xb[u] = key[pq];
        }
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int q = t + 64 * u, pq = q ^ jj;
        if (q < m2 && pq > q && ((xa[u] > xb[u]) == ((q & kk) == 0))) {
          key[q] = xb[u];
          key[pq] = xa[u];
        }
      }
      __syncthreads();
    }
}

// Two variants: CAP = kGemmSmall (half the LDS) takes the rows with at most
// kGemmSmall A entries and candidates, and raises flag[1] for the others;
// CAP = kGemmCap takes exactly those others.  Malformed rows raise flag[0];
// rows beyond lmax (A entries or candidates) are left to the sort in device
// memory, and the small variant raises flag[2] for them.
template <int CAP, int FILL, typename K>
__global__ void __launch_bounds__(64) k_spgemm(int64_t m, int64_t k, const int64_t* __restrict__ a_rp,
                                               const int32_t* __restrict__ a_col, const double* __restrict__ a_val,
                                               const int64_t* __restrict__ b_rp, const int32_t* __restrict__ b_col,
                                               const double* __restrict__ b_val, int32_t* __restrict__ cnt,
                                               const int64_t* __restrict__ c_rp, int32_t* __restrict__ c_col,
                                               double* __restrict__ c_val, int* __restrict__ flag, int lmax) {
  // (column << SH) | candidate index, sorted: 32-bit keys when every column
  // of B fits in 32 - SH bits (the host decides), else 64-bit
  constexpr int SH = sizeof(K) == 8 ? 32 : (CAP == 1024 ? 10 : 11);
  static_assert(sizeof(K) == 8 || (1 << SH) >= CAP, "candidate index bits");
  constexpr K kQmask = (K)(((uint64_t)1 << SH) - 1);
  __shared__ K key[CAP];
  __shared__ int32_t pre[CAP + 1];   // prefix sums of the selected B row lengths
  __shared__ int32_t bst[CAP];       // start of each selected B row
  __shared__ int16_t own[CAP];       // the A entry (index in the row) of each candidate
  __shared__ double prod[CAP];       // products, in sorted order
  const int t = threadIdx.x;
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const int64_t p0 = a_rp[i];
    const int64_t na64 = a_rp[i + 1] - p0;
    // validation before any candidate is read (all lanes, uniform result):
    // row pointers of A and of the selected B rows inside [0, nnz] and
    // non-decreasing, A's columns indexing rows of B; lengths summed by a
    // wave scan, 64 entries at a time, until they pass lmax <= kGemmCap (a
    // long row, validated in full by the sort's own pass)
    const int64_t annz = a_rp[m], bnnz = b_rp[k];
    bool ok = na64 >= 0 && p0 >= 0 && p0 + na64 <= annz;
    bool longrow = ok && na64 > lmax;   // sorted in device memory instead
    int tot = 0;
    bool big = ok && na64 > CAP;   // past this variant's tables: stop writing them
    if (ok && !longrow) {
      const int na = (int)na64;
      bool bad = false;
      if (t == 0 && !big) pre[0] = 0;
      for (int c0 = 0; c0 < na && tot <= lmax; c0 += 64) {
        const int p = c0 + t;
        int len = 0;
        if (p < na) {
          const int32_t a = a_col[p0 + p];
          if (a < 0 || a >= k) {
            bad = true;
          } else {
            const int64_t b0 = b_rp[a], b1 = b_rp[a + 1];
            if (b0 < 0 || b1 < b0 || b1 > bnnz) {
              bad = true;
            } else {
              len = (int)(b1 - b0 < (int64_t)kGemmCap + 1 ? b1 - b0 : (int64_t)kGemmCap + 1);
              if (!big) bst[p] = (int32_t)b0;
            }
          }
        }
        int x = len;   // inclusive scan over the wave
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
          const int y = __shfl_up(x, off, 64);
          if (t >= off) x += y;
        }
        if (p < na && !big && tot + x <= CAP) pre[p + 1] = tot + x;
        tot += __shfl(x, 63, 64);
        if (tot > CAP) big = true;
      }
      ok = __ballot(bad) == 0;
      longrow = ok && tot > lmax;
    }
    if (!ok || longrow) {
      if (t == 0) {
        if (!ok) flag[0] = 1;
        else if (CAP == kGemmSmall) flag[2] = 1;
        if (!FILL) cnt[i] = 0;
      }
      __syncthreads();
      continue;
    }
    const bool needs_large = na64 > kGemmSmall || tot > kGemmSmall;
    if (needs_large != (CAP == kGemmCap)) {
      // the other variant's row
      if (t == 0 && needs_large) flag[1] = 1;
      __syncthreads();
      continue;
    }
    __syncthreads();
    const int na = (int)na64, mt = tot;
    int m2 = 1;
    while (m2 < mt) m2 <<= 1;
    // owner of each candidate: A entry p covers candidates pre[p] .. pre[p+1)
    for (int p = t; p < na; p += 64)
      for (int q = pre[p]; q < pre[p + 1]; ++q) own[q] = (int16_t)p;
    __syncthreads();
    for (int q = t; q < m2; q += 64) {
      K kv = ~(K)0;
      if (q < mt) {
        const int pa = own[q];
        const uint32_t cj = (uint32_t)b_col[(int64_t)bst[pa] + (q - pre[pa])];
        kv = ((K)cj << SH) | (K)q;
      }
      key[q] = kv;
    }
    __syncthreads();
    wave_bitonic<CAP, K>(key, m2);
    // distinct columns: the heads of runs of equal column
    int u = 0;
    for (int q0 = 0; q0 < mt; q0 += 64) {
      const int q = q0 + t;
      const bool head = q < mt && (q == 0 || (key[q] >> SH) != (key[q - 1] >> SH));
      u += __popcll(__ballot(head));
    }
    if (!FILL) {
      if (t == 0) cnt[i] = u;
      __syncthreads();
      continue;
    }
    // the output row must have exactly the counted length inside [0, nnz(C)]
    const int64_t o = c_rp[i];
    if (o < 0 || c_rp[i + 1] - o != u || c_rp[i + 1] > c_rp[m]) {
      if (t == 0) flag[0] = 1;
      __syncthreads();
      continue;
    }
    // products of every candidate (independent loads), in sorted order
    for (int r = t; r < mt; r += 64) {
      const int q = (int)(key[r] & kQmask);
      const int pa = own[q];
      prod[r] = a_val[p0 + pa] * b_val[(int64_t)bst[pa] + (q - pre[pa])];
    }
    __syncthreads();
    // each head sums its run in candidate order (A's column order)
    int base = 0;
    for (int q0 = 0; q0 < mt; q0 += 64) {
      const int q = q0 + t;
      const bool head = q < mt && (q == 0 || (key[q] >> SH) != (key[q - 1] >> SH));
      const uint64_t mask = __ballot(head);
      if (head) {
        const K cbits = key[q] >> SH;
        double s = prod[q];
        for (int r = q + 1; r < mt && (key[r] >> SH) == cbits; ++r) s += prod[r];
        const int64_t at = o + base + __popcll(mask & ((1ull << t) - 1ull));
        c_col[at] = (int32_t)(uint32_t)cbits;
        c_val[at] = s;
      }
      base += __popcll(mask);
    }
    __syncthreads();
  }
}

// row index of every entry; rows whose pointers leave [0, nnz] or decrease
// raise the flag and write nothing
__global__ void __launch_bounds__(256) k_row_of(int64_t m, int64_t nnz, const int64_t* __restrict__ rp,
                                                int32_t* __restrict__ rowof, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int64_t r0 = rp[i], r1 = rp[i + 1];
    if (r0 < 0 || r1 < r0 || r1 > nnz) {
      flag[0] = 1;
      continue;
    }
    for (int64_t p = r0; p < r1; ++p) rowof[p] = (int32_t)i;
  }
}

__global__ void __launch_bounds__(256) k_iota(int64_t nnz, int32_t* __restrict__ idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += stride) idx[p] = (int32_t)p;
}

__global__ void __launch_bounds__(256) k_gather_t(int64_t nnz, const int32_t* __restrict__ perm,
                                                  const int32_t* __restrict__ rowof, const double* __restrict__ val,
                                                  int32_t* __restrict__ col_t, double* __restrict__ val_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nnz; r += stride) {
    const int32_t p = perm[r];
    col_t[r] = rowof[p];
    val_t[r] = val[p];
  }
}

// rp_t[j] = number of sorted keys below j, j = 0..n
__global__ void __launch_bounds__(256) k_col_starts(int64_t n, const int32_t* __restrict__ keys, int64_t nnz,
                                                    int64_t* __restrict__ rp_t) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j <= n; j += stride) {
    int64_t lo = 0, hi = nnz;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if ((int64_t)keys[mid] < j) lo = mid + 1; else hi = mid;
    }
    rp_t[j] = lo;
  }
}

// Rows of C = A B past the LDS limit (A entries or candidate products): their
// candidates are written to device memory keyed by column, one segment per
// row, sorted by a stable segmented radix sort over the bits the widest
// column of B uses, so each column's products keep their candidate order,
// and each run of equal keys is summed in that order: the same result, bit
// for bit, as the LDS variants give a shorter row.

// One thread per row of A: validation in full, and len[i] = the candidate
// count of a long row (0 included), -1 for the other rows.
__global__ void __launch_bounds__(256) k_long_len(int64_t m, int64_t k, const int64_t* __restrict__ a_rp,
                                                  const int32_t* __restrict__ a_col,
                                                  const int64_t* __restrict__ b_rp, int64_t* __restrict__ len,
                                                  int* __restrict__ flag, int lmax) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t annz = a_rp[m], bnnz = b_rp[k];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int64_t p0 = a_rp[i], p1 = a_rp[i + 1];
    bool bad = p0 < 0 || p1 < p0 || p1 > annz;
    int64_t tot = 0;
    for (int64_t p = p0; !bad && p < p1; ++p) {
      const int32_t a = a_col[p];
      if (a < 0 || a >= k) {
        bad = true;
        break;
      }
      const int64_t b0 = b_rp[a], b1 = b_rp[a + 1];
      if (b0 < 0 || b1 < b0 || b1 > bnnz) {
        bad = true;
        break;
      }
      tot += b1 - b0;
    }
    if (bad) flag[0] = 1;
    len[i] = (!bad && (p1 - p0 > lmax || tot > lmax)) ? tot : -1;
  }
}

// One wavefront per row of the batch: row rows[r]'s candidates, in candidate
// order, at off[r] .. off[r+1): key the column, value the product.
template <int FILL>
__global__ void __launch_bounds__(64) k_long_expand(int nb, const int32_t* __restrict__ rows,
                                                    const int64_t* __restrict__ off, const int64_t* __restrict__ a_rp,
                                                    const int32_t* __restrict__ a_col, const double* __restrict__ a_val,
                                                    const int64_t* __restrict__ b_rp, const int32_t* __restrict__ b_col,
                                                    const double* __restrict__ b_val, uint32_t* __restrict__ key,
                                                    double* __restrict__ val) {
  const int t = threadIdx.x;
  for (int r = blockIdx.x; r < nb; r += gridDim.x) {
    const int64_t i = rows[r], p1 = a_rp[i + 1], end = off[r + 1];
    int64_t at = off[r];
    for (int64_t p = a_rp[i]; p < p1; ++p) {
      const int32_t a = a_col[p];
      const int64_t b0 = b_rp[a], n = b_rp[a + 1] - b0;
      const double av = FILL ? a_val[p] : 0.0;
      for (int64_t q = t; q < n && at + q < end; q += 64) {
        key[at + q] = (uint32_t)b_col[b0 + q];
        if (FILL) val[at + q] = av * b_val[b0 + q];
      }
      at += n;
    }
  }
}

// One wavefront per row of the batch over its sorted candidates: the count
// of distinct keys, or (fill) each run summed in order and written, in
// column order, at c_rp[row].  An output row of another length raises the
// flag and writes nothing.
template <int FILL>
__global__ void __launch_bounds__(64) k_long_runs(int64_t m, int nb, const int32_t* __restrict__ rows,
                                                  const int64_t* __restrict__ off, const uint32_t* __restrict__ key,
                                                  const double* __restrict__ val, int32_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ c_rp, int32_t* __restrict__ c_col,
                                                  double* __restrict__ c_val, int* __restrict__ flag) {
  const int t = threadIdx.x;
  for (int r = blockIdx.x; r < nb; r += gridDim.x) {
    const int64_t i = rows[r], q0 = off[r], q1 = off[r + 1];
    int64_t u = 0;
    for (int64_t c = q0; c < q1; c += 64) {
      const int64_t q = c + t;
      u += __popcll(__ballot(q < q1 && (q == q0 || key[q] != key[q - 1])));
    }
    if (!FILL) {
      if (t == 0) cnt[i] = (int32_t)u;
      continue;
    }
    const int64_t o = c_rp[i];
    if (o < 0 || c_rp[i + 1] - o != u || c_rp[i + 1] > c_rp[m]) {
      if (t == 0) flag[0] = 1;
      continue;
    }
    int64_t base = 0;
    for (int64_t c = q0; c < q1; c += 64) {
      const int64_t q = c + t;
      const bool head = q < q1 && (q == q0 || key[q] != key[q - 1]);
      const uint64_t mask = __ballot(head);
      if (head) {
        const uint32_t kq = key[q];
        double sum = val[q];
        for (int64_t x = q + 1; x < q1 && key[x] == kq; ++x) sum += val[x];
        const int64_t at = o + base + __popcll(mask & ((1ull << t) - 1ull));
        c_col[at] = (int32_t)kq;
        c_val[at] = sum;
      }
      base += __popcll(mask);
    }
  }
}

unsigned grid_of(int64_t work, int per_cu);

// C = A + B (both m x n): one thread per row merges the two ascending column
// lists; an entry present in both is a + b.  Rows with malformed pointers
// (or, when filling, an output row whose length differs from the merge)
// raise the flag and write nothing.
template <int FILL>
__global__ void __launch_bounds__(256) k_csr_add(int64_t m, const int64_t* __restrict__ a_rp,
                                                 const int32_t* __restrict__ a_col, const double* __restrict__ a_val,
                                                 const int64_t* __restrict__ b_rp, const int32_t* __restrict__ b_col,
                                                 const double* __restrict__ b_val, int32_t* __restrict__ cnt,
                                                 const int64_t* __restrict__ c_rp, int32_t* __restrict__ c_col,
                                                 double* __restrict__ c_val, int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t annz = a_rp[m], bnnz = b_rp[m];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += stride) {
    const int64_t a0 = a_rp[i], a1 = a_rp[i + 1], b0 = b_rp[i], b1 = b_rp[i + 1];
    if (a0 < 0 || a1 < a0 || a1 > annz || b0 < 0 || b1 < b0 || b1 > bnnz) {
      flag[0] = 1;
      if (!FILL) cnt[i] = 0;
      continue;
    }
    int64_t o = 0, lim = 0;
    if (FILL) {
      o = c_rp[i];
      lim = c_rp[i + 1];
      if (o < 0 || lim < o || lim > c_rp[m]) {
        flag[0] = 1;
        continue;
      }
    }
    int64_t pa = a0, pb = b0, u = 0;
    while (pa < a1 || pb < b1) {
      const int32_t ca = pa < a1 ? a_col[pa] : 0x7fffffff, cb = pb < b1 ? b_col[pb] : 0x7fffffff;
      int32_t cc;
      double v = 0.0;
      if (ca < cb || pb >= b1) {
        cc = ca;
        if (FILL) v = a_val[pa];
        ++pa;
      } else if (cb < ca || pa >= a1) {
        cc = cb;
        if (FILL) v = b_val[pb];
        ++pb;
      } else {
        cc = ca;
        if (FILL) v = a_val[pa] + b_val[pb];
        ++pa;
        ++pb;
      }
      if (FILL) {
        if (o + u >= lim) break;   // the output row is too short: flagged below
        c_col[o + u] = cc;
        c_val[o + u] = v;
      }
      ++u;
    }
    if (!FILL) cnt[i] = (int32_t)u;
    else if (o + u != lim || pa < a1 || pb < b1) flag[0] = 1;
  }
}

// Both variants of a pass (the large one only when the small one left rows);
// *bad: a malformed or over-long row was found.
template <int FILL>
int long_rows(int64_t m, int64_t k, const int64_t* a_rp, const int32_t* a_col, const double* a_val,
              const int64_t* b_rp, const int32_t* b_col, const double* b_val, int32_t* cnt, const int64_t* c_rp,
              int32_t* c_col, double* c_val, int* flag_d, hipStream_t s, int lmax, uint32_t maxcol, int* bad);

int max_col(int64_t k, const int64_t* b_rp, const int32_t* b_col, hipStream_t s, uint32_t* out);

template <int FILL>
int spgemm_pass(int64_t m, int64_t k, const int64_t* a_rp, const int32_t* a_col, const double* a_val,
                const int64_t* b_rp, const int32_t* b_col, const double* b_val, int32_t* cnt, const int64_t* c_rp,
                int32_t* c_col, double* c_val, int* flag_d, hipStream_t s, int* bad) {
  int hf[3] = {0, 0, 0};
  BRAS_HIP(hipMemsetAsync(flag_d, 0, 3 * sizeof(int), s));
  const int lmax = lds_max();
  uint32_t maxcol = 0;
  int st = max_col(k, b_rp, b_col, s, &maxcol);
  if (st) return st;
  // 32-bit LDS keys when (column << index bits) | index stays below the
  // padding key 2^32 - 1 for every column
  if (maxcol < (1u << 22) - 1u)
    k_spgemm<kGemmSmall, FILL, uint32_t><<<grid_of(m, 32), 64, 0, s>>>(m, k, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                                                      cnt, c_rp, c_col, c_val, flag_d, lmax);
  else
    k_spgemm<kGemmSmall, FILL, uint64_t><<<grid_of(m, 32), 64, 0, s>>>(m, k, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                                                      cnt, c_rp, c_col, c_val, flag_d, lmax);
  BRAS_HIP(hipGetLastError());
  BRAS_HIP(hipMemcpyAsync(hf, flag_d, 3 * sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  if (!hf[0] && hf[1]) {
    if (maxcol < (1u << 21) - 1u)
      k_spgemm<kGemmCap, FILL, uint32_t><<<grid_of(m, 16), 64, 0, s>>>(m, k, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                                                      cnt, c_rp, c_col, c_val, flag_d, lmax);
    else
      k_spgemm<kGemmCap, FILL, uint64_t><<<grid_of(m, 16), 64, 0, s>>>(m, k, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                                                      cnt, c_rp, c_col, c_val, flag_d, lmax);
    BRAS_HIP(hipGetLastError());
    BRAS_HIP(hipMemcpyAsync(hf, flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
    BRAS_HIP(hipStreamSynchronize(s));
  }
  if (!hf[0] && hf[2])
    return long_rows<FILL>(m, k, a_rp, a_col, a_val, b_rp, b_col, b_val, cnt, c_rp, c_col, c_val, flag_d, s, lmax,
                           maxcol, bad);
  *bad = hf[0];
  return BRAS_OK;
}

unsigned grid_of(int64_t work, int per_cu) {
  int dev = 0, ncu = 1;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    ncu = 1;
  const int64_t want = (int64_t)ncu * per_cu;
  const int64_t g = work < want ? work : want;
  return (unsigned)(g < 1 ? 1 : g);
}

// Frees what it holds at scope exit (the entry points return on every error).
struct DevBufs {
  std::vector<void*> p;
  template <typename T>
  int get(T** out, size_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count ? count * sizeof(T) : 1) != hipSuccess) return fail(BRAS_ENOMEM, "device allocation failed");
    p.push_back(q);
    *out = (T*)q;
    return BRAS_OK;
  }
  ~DevBufs() {
    for (void* q : p) (void)hipFree(q);
  }
};

// The widest column of B, as unsigned (0 for an empty B).
int max_col(int64_t k, const int64_t* b_rp, const int32_t* b_col, hipStream_t s, uint32_t* out) {
  int64_t bnnz = 0;
  BRAS_HIP(hipMemcpyAsync(&bnnz, b_rp + k, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  *out = 0;
  if (bnnz <= 0) return BRAS_OK;
  BRAS_CHECK(bnnz < (1LL << 31), "B has %lld entries; at most 2^31 - 1 are supported", (long long)bnnz);
  DevBufs tmp;
  uint32_t* mx_d = nullptr;
  char* red_tmp = nullptr;
  size_t rbytes = 0;
  int st;
  const uint32_t* ucol = reinterpret_cast<const uint32_t*>(b_col);
  BRAS_HIP(hipcub::DeviceReduce::Max(nullptr, rbytes, ucol, mx_d, (int)bnnz, s));
  if ((st = tmp.get(&mx_d, 1)) || (st = tmp.get(&red_tmp, rbytes))) return st;
  BRAS_HIP(hipcub::DeviceReduce::Max(red_tmp, rbytes, ucol, mx_d, (int)bnnz, s));
  BRAS_HIP(hipMemcpyAsync(out, mx_d, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  return BRAS_OK;
}

constexpr int64_t kLongBatch = (int64_t)1 << 27;   // candidates sorted at once (24 bytes each when filling)

// BRAS_SPGEMM_BATCH (a positive integer) replaces kLongBatch: less device
// memory per call, more sorts.
int64_t long_batch() {
  const char* e = std::getenv("BRAS_SPGEMM_BATCH");
  const long long v = e ? std::atoll(e) : 0;
  return v > 0 ? (int64_t)v : kLongBatch;
}

// The rows past kGemmCap, in row order, in batches of at most long_batch()
// candidates (a longer row alone): expand, stable segmented radix sort
// (one segment per row), runs.  *bad: a malformed row (or, when filling, an output
// row of the wrong length).
template <int FILL>
int long_rows(int64_t m, int64_t k, const int64_t* a_rp, const int32_t* a_col, const double* a_val,
              const int64_t* b_rp, const int32_t* b_col, const double* b_val, int32_t* cnt, const int64_t* c_rp,
              int32_t* c_col, double* c_val, int* flag_d, hipStream_t s, int lmax, uint32_t maxcol, int* bad) {
  DevBufs tmp;
  int64_t* len = nullptr;
  int st, hf = 0;
  if ((st = tmp.get(&len, (size_t)m))) return st;
  BRAS_HIP(hipMemsetAsync(flag_d, 0, sizeof(int), s));
  k_long_len<<<grid_of((m + 255) / 256, 8), 256, 0, s>>>(m, k, a_rp, a_col, b_rp, len, flag_d, lmax);
  BRAS_HIP(hipGetLastError());
  std::vector<int64_t> hl(m);
  BRAS_HIP(hipMemcpyAsync(hl.data(), len, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipMemcpyAsync(&hf, flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  if (hf) {
    *bad = 1;
    return BRAS_OK;
  }
  std::vector<std::vector<int32_t>> rows;
  std::vector<std::vector<int64_t>> offs;
  const int64_t batch = long_batch();
  for (int64_t i = 0; i < m; ++i) {
    if (hl[i] < 0) continue;
    if (rows.empty() || (!rows.back().empty() && offs.back().back() + hl[i] > batch)) {
      rows.emplace_back();
      offs.emplace_back(1, 0);
    }
    rows.back().push_back((int32_t)i);
    offs.back().push_back(offs.back().back() + hl[i]);
  }
  // key bits: the widest column of B (unsigned); one segment per row
  int cbits = 1;
  while (cbits < 32 && (maxcol >> cbits) != 0) ++cbits;
  int64_t cap = 1;
  size_t maxnb = 1, bytes = 0;
  for (size_t b = 0; b < rows.size(); ++b) {
    const int64_t L = offs[b].back();
    BRAS_CHECK(L < (1LL << 31), "a row of A selects %lld candidate products; at most 2^31 - 1 are supported",
               (long long)L);
    cap = L > cap ? L : cap;
    maxnb = rows[b].size() > maxnb ? rows[b].size() : maxnb;
    size_t need = 0;
    hipcub::DoubleBuffer<uint32_t> kq(nullptr, nullptr);
    hipcub::DoubleBuffer<double> vq(nullptr, nullptr);
    const int ns = (int)rows[b].size();
    if (FILL)
      BRAS_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, need, kq, vq, (int)L, ns, (const int*)nullptr,
                                                           (const int*)nullptr, 0, cbits, s));
    else
      BRAS_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, need, kq, (int)L, ns, (const int*)nullptr,
                                                          (const int*)nullptr, 0, cbits, s));
    bytes = need > bytes ? need : bytes;
  }
  int32_t* rows_d = nullptr;
  int64_t* off_d = nullptr;
  int* off32_d = nullptr;
  uint32_t *k0 = nullptr, *k1 = nullptr;
  double *v0 = nullptr, *v1 = nullptr;
  char* cub_tmp = nullptr;
  if ((st = tmp.get(&rows_d, maxnb)) || (st = tmp.get(&off_d, maxnb + 1)) || (st = tmp.get(&off32_d, maxnb + 1)) ||
      (st = tmp.get(&k0, (size_t)cap)) ||
      (st = tmp.get(&k1, (size_t)cap)) || (st = tmp.get(&v0, FILL ? (size_t)cap : 1)) ||
      (st = tmp.get(&v1, FILL ? (size_t)cap : 1)) || (st = tmp.get(&cub_tmp, bytes)))
    return st;
  for (size_t b = 0; b < rows.size(); ++b) {
    const int nb = (int)rows[b].size();
    const int64_t L = offs[b].back();
    BRAS_HIP(hipMemcpyAsync(rows_d, rows[b].data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
    BRAS_HIP(hipMemcpyAsync(off_d, offs[b].data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice, s));
    std::vector<int> o32(offs[b].begin(), offs[b].end());   // below 2^31 (checked above)
    BRAS_HIP(hipMemcpyAsync(off32_d, o32.data(), sizeof(int) * (nb + 1), hipMemcpyHostToDevice, s));
    hipcub::DoubleBuffer<uint32_t> kb(k0, k1);
    hipcub::DoubleBuffer<double> vb(v0, v1);
    if (L > 0) {
      k_long_expand<FILL><<<grid_of(nb, 16), 64, 0, s>>>(nb, rows_d, off_d, a_rp, a_col, a_val, b_rp, b_col, b_val,
                                                          k0, v0);
      BRAS_HIP(hipGetLastError());
      size_t have = bytes;
      if (FILL)
        BRAS_HIP(hipcub::DeviceSegmentedRadixSort::SortPairs(cub_tmp, have, kb, vb, (int)L, nb, off32_d, off32_d + 1,
                                                             0, cbits, s));
      else
        BRAS_HIP(hipcub::DeviceSegmentedRadixSort::SortKeys(cub_tmp, have, kb, (int)L, nb, off32_d, off32_d + 1, 0,
                                                            cbits, s));
    }
    k_long_runs<FILL><<<grid_of(nb, 16), 64, 0, s>>>(m, nb, rows_d, off_d, kb.Current(), FILL ? vb.Current() : nullptr,
                                                      cnt, c_rp, c_col, c_val, flag_d);
    BRAS_HIP(hipGetLastError());
    BRAS_HIP(hipStreamSynchronize(s));   // the next batch reuses the buffers and the host lists stay valid
  }
  BRAS_HIP(hipMemcpyAsync(&hf, flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  *bad = hf;
  return BRAS_OK;
}

}  // namespace
}  // namespace bras

using namespace bras;

extern "C" int bras_spgemm_rowptr(int64_t m, int64_t k, const int64_t* a_rowptr_d, const int32_t* a_col_d,
                                  const int64_t* b_rowptr_d, const int32_t* b_col_d, int64_t* c_rowptr_d,
                                  int64_t* nnz_h, void* stream) {
  clear_error();
  BRAS_CHECK(m >= 0 && k >= 0, "negative size");
  BRAS_CHECK(m < (1LL << 31) && k < (1LL << 31), "sizes must stay below 2^31");
  BRAS_CHECK(a_rowptr_d && a_col_d && b_rowptr_d && b_col_d && c_rowptr_d && nnz_h, "null argument");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> rp(m + 1, 0);
  if (m > 0) {
    DevBufs tmp;
    int32_t* cnt = nullptr;
    int* flag = nullptr;
    int st, hf = 0;
    if ((st = tmp.get(&cnt, (size_t)m)) || (st = tmp.get(&flag, 3))) return st;
    if ((st = spgemm_pass<0>(m, k, a_rowptr_d, a_col_d, nullptr, b_rowptr_d, b_col_d, nullptr, cnt, nullptr, nullptr,
                             nullptr, flag, s, &hf)))
      return st;
    std::vector<int32_t> hc(m);
    BRAS_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    BRAS_HIP(hipStreamSynchronize(s));
    BRAS_CHECK(!hf, "a row of A has a column outside [0, %lld), or row pointers of A or B are malformed",
               (long long)k);
    for (int64_t i = 0; i < m; ++i) rp[i + 1] = rp[i] + hc[i];
  }
  BRAS_CHECK(rp[m] < (1LL << 31), "the product has %lld entries; at most 2^31 - 1 are supported", (long long)rp[m]);
  BRAS_HIP(hipMemcpyAsync(c_rowptr_d, rp.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, s));
  BRAS_HIP(hipStreamSynchronize(s));
  *nnz_h = rp[m];
  return BRAS_OK;
}

extern "C" int bras_spgemm_fill(int64_t m, int64_t k, const int64_t* a_rowptr_d, const int32_t* a_col_d,
                                const double* a_val_d, const int64_t* b_rowptr_d, const int32_t* b_col_d,
                                const double* b_val_d, const int64_t* c_rowptr_d, int32_t* c_col_d, double* c_val_d,
                                void* stream) {
  clear_error();
  BRAS_CHECK(m >= 0 && k >= 0, "negative size");
  BRAS_CHECK(m < (1LL << 31) && k < (1LL << 31), "sizes must stay below 2^31");
  if (m == 0) return BRAS_OK;
  BRAS_CHECK(a_rowptr_d && a_col_d && a_val_d && b_rowptr_d && b_col_d && b_val_d && c_rowptr_d && c_col_d && c_val_d,
             "null argument");
  hipStream_t s = (hipStream_t)stream;
  DevBufs tmp;
  int* flag = nullptr;
  int st, hf = 0;
  if ((st = tmp.get(&flag, 3))) return st;
  if ((st = spgemm_pass<1>(m, k, a_rowptr_d, a_col_d, a_val_d, b_rowptr_d, b_col_d, b_val_d, nullptr, c_rowptr_d,
                           c_col_d, c_val_d, flag, s, &hf)))
    return st;
  BRAS_CHECK(!hf, "a row of A has a column outside [0, %lld), malformed row pointers, or C's row pointers do not match "
                  "the counts", (long long)k);
  return BRAS_OK;
}

extern "C" int bras_csr_transpose(int64_t m, int64_t n, const int64_t* rowptr_d, const int32_t* col_d,
                                  const double* val_d, int64_t* rowptr_t_d, int32_t* col_t_d, double* val_t_d,
                                  void* stream) {
  clear_error();
  BRAS_CHECK(m >= 0 && n >= 0, "negative size");
  BRAS_CHECK(m < (1LL << 31) && n < (1LL << 31), "sizes must stay below 2^31");
  BRAS_CHECK(rowptr_d && rowptr_t_d, "null argument");
  hipStream_t s = (hipStream_t)stream;
  int64_t ends[2] = {0, 0};
  BRAS_HIP(hipMemcpyAsync(ends, rowptr_d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipMemcpyAsync(ends + 1, rowptr_d + m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  BRAS_CHECK(ends[0] == 0 && ends[1] >= 0 && ends[1] < (1LL << 31), "row pointers must start at 0 and end below 2^31");
  const int64_t nnz = ends[1];
  DevBufs tmp;
  int st;
  if (nnz == 0) {
    std::vector<int64_t> z(n + 1, 0);
    BRAS_HIP(hipMemcpyAsync(rowptr_t_d, z.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    BRAS_HIP(hipStreamSynchronize(s));
    return BRAS_OK;
  }
  BRAS_CHECK(col_d && val_d && col_t_d && val_t_d, "null argument");
  int32_t *rowof = nullptr, *idx = nullptr, *key_out = nullptr, *idx_out = nullptr;
  int* flag = nullptr;
  if ((st = tmp.get(&rowof, (size_t)nnz)) || (st = tmp.get(&idx, (size_t)nnz)) ||
      (st = tmp.get(&key_out, (size_t)nnz)) || (st = tmp.get(&idx_out, (size_t)nnz)) || (st = tmp.get(&flag, 1)))
    return st;
  BRAS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  BRAS_HIP(hipMemsetAsync(rowof, 0, sizeof(int32_t) * nnz, s));
  if (m > 0) k_row_of<<<grid_of((m + 255) / 256, 8), 256, 0, s>>>(m, nnz, rowptr_d, rowof, flag);
  k_iota<<<grid_of((nnz + 255) / 256, 8), 256, 0, s>>>(nnz, idx);
  BRAS_HIP(hipGetLastError());
  size_t bytes = 0;
  BRAS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, col_d, key_out, idx, idx_out, (int)nnz, 0, 32, s));
  void* cub_tmp = nullptr;
  if ((st = tmp.get((char**)&cub_tmp, bytes))) return st;
  // stable: entries of one column keep their (row-major) order
  BRAS_HIP(hipcub::DeviceRadixSort::SortPairs(cub_tmp, bytes, col_d, key_out, idx, idx_out, (int)nnz, 0, 32, s));
  k_gather_t<<<grid_of((nnz + 255) / 256, 8), 256, 0, s>>>(nnz, idx_out, rowof, val_d, col_t_d, val_t_d);
  k_col_starts<<<grid_of((n + 256) / 256, 8), 256, 0, s>>>(n, key_out, nnz, rowptr_t_d);
  BRAS_HIP(hipGetLastError());
  // every column inside [0, n): the first start is 0 and the last is nnz
  int64_t tb[2] = {-1, -1};
  int hf = 0;
  BRAS_HIP(hipMemcpyAsync(tb, rowptr_t_d, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipMemcpyAsync(tb + 1, rowptr_t_d + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  BRAS_CHECK(!hf, "row pointers must be non-decreasing from 0 to nnz");
  BRAS_CHECK(tb[0] == 0 && tb[1] == nnz, "a column index lies outside [0, %lld)", (long long)n);
  return BRAS_OK;
}

extern "C" int bras_csr_add_rowptr(int64_t m, const int64_t* a_rowptr_d, const int32_t* a_col_d,
                                   const int64_t* b_rowptr_d, const int32_t* b_col_d, int64_t* c_rowptr_d,
                                   int64_t* nnz_h, void* stream) {
  clear_error();
  BRAS_CHECK(m >= 0 && m < (1LL << 31), "size outside [0, 2^31)");
  BRAS_CHECK(a_rowptr_d && a_col_d && b_rowptr_d && b_col_d && c_rowptr_d && nnz_h, "null argument");
  hipStream_t s = (hipStream_t)stream;
  std::vector<int64_t> rp(m + 1, 0);
  if (m > 0) {
    DevBufs tmp;
    int32_t* cnt = nullptr;
    int* flag = nullptr;
    int st, hf = 0;
    if ((st = tmp.get(&cnt, (size_t)m)) || (st = tmp.get(&flag, 1))) return st;
    BRAS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_csr_add<0><<<grid_of((m + 255) / 256, 8), 256, 0, s>>>(m, a_rowptr_d, a_col_d, nullptr, b_rowptr_d, b_col_d,
                                                            nullptr, cnt, nullptr, nullptr, nullptr, flag);
    BRAS_HIP(hipGetLastError());
    std::vector<int32_t> hc(m);
    BRAS_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * m, hipMemcpyDeviceToHost, s));
    BRAS_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    BRAS_HIP(hipStreamSynchronize(s));
    BRAS_CHECK(!hf, "malformed row pointers");
    for (int64_t i = 0; i < m; ++i) rp[i + 1] = rp[i] + hc[i];
  }
  BRAS_CHECK(rp[m] < (1LL << 31), "the sum has %lld entries; at most 2^31 - 1 are supported", (long long)rp[m]);
  BRAS_HIP(hipMemcpyAsync(c_rowptr_d, rp.data(), sizeof(int64_t) * (m + 1), hipMemcpyHostToDevice, s));
  BRAS_HIP(hipStreamSynchronize(s));
  *nnz_h = rp[m];
  return BRAS_OK;
}

extern "C" int bras_csr_add_fill(int64_t m, const int64_t* a_rowptr_d, const int32_t* a_col_d, const double* a_val_d,
                                 const int64_t* b_rowptr_d, const int32_t* b_col_d, const double* b_val_d,
                                 const int64_t* c_rowptr_d, int32_t* c_col_d, double* c_val_d, void* stream) {
  clear_error();
  BRAS_CHECK(m >= 0 && m < (1LL << 31), "size outside [0, 2^31)");
  if (m == 0) return BRAS_OK;
  BRAS_CHECK(a_rowptr_d && a_col_d && a_val_d && b_rowptr_d && b_col_d && b_val_d && c_rowptr_d && c_col_d && c_val_d,
             "null argument");
  hipStream_t s = (hipStream_t)stream;
  DevBufs tmp;
  int* flag = nullptr;
  int st, hf = 0;
  if ((st = tmp.get(&flag, 1))) return st;
  BRAS_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
  k_csr_add<1><<<grid_of((m + 255) / 256, 8), 256, 0, s>>>(m, a_rowptr_d, a_col_d, a_val_d, b_rowptr_d, b_col_d,
                                                          b_val_d, nullptr, c_rowptr_d, c_col_d, c_val_d, flag);
  BRAS_HIP(hipGetLastError());
  BRAS_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  BRAS_HIP(hipStreamSynchronize(s));
  BRAS_CHECK(!hf, "malformed row pointers, or output rows that do not match the counts");
  return BRAS_OK;
}
