// Element pass for per-element matrices with n_loc > kLaneMaxNL (too large
// for one lane's registers): one work-group (4 wavefronts) per element, the
// element's packed matrix (element-major, stored in T) unpacked into a full
// symmetric float64 tile in LDS, the gathered input W^T (32 columns at a
// time) beside it, and Z = M W on the FP64 matrix cores
// (v_mfma_f64_16x16x4_f64).  Used for the conforming mass pass (M_K, eq.
// M_PMbrP) and for stored BRAS inverses D_K^-1 M_K^-1 D_K^-1 in FP64 or FP32
// (eq. mass_and_bras_element_sums); the products are formed in float64.
//
// MFMA operand layout (16x16x4, one double per lane):
//   A[i][k]: lane l holds i = l%16, k = l/16
//   B[k][j]: lane l holds j = l%16, k = l/16
//   D[i][j]: lane l, reg r holds j = l%16, i = l/16 + 4*r
#include <cmath>

#include "internal.h"
#include "cg_common.h"

namespace bras {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kMB = 256;   // 4 wavefronts

// Persistent: work-group g handles elements g, g + G, ... (G = grid size).
// While the matrix cores work on element K, the registers already hold the
// loads of element K + G (its matrix and its first 32 gathered columns) and
// the map of element K + 2G, so memory latency overlaps the products.
template <int NL, typename T, typename ZT>
__global__ void __launch_bounds__(kMB) k_elem_mfma(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                                   const T* __restrict__ mat, ZT* __restrict__ zb) {
  constexpr int MT = (NL + 15) / 16;       // 16-row tiles
  constexpr int KP = 4 * ((NL + 3) / 4);   // contraction length padded to the MFMA depth
  constexpr int LD = KP + 1;               // LDS row stride (odd: spreads banks)
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr int MPT = (NPK + kMB - 1) / kMB;      // matrix entries per thread
  constexpr int GPT = (32 * NL + kMB - 1) / kMB;  // gathered (k, column) pairs per thread
  __shared__ double sA[MT * 16 * LD];      // M (symmetric, zero padded)
  __shared__ double sW[32 * LD];           // W^T [column][k], zero padded
  __shared__ int32_t gidx[NL];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  __shared__ double red_s[kMB];
  if (in.apart) {
    alpha_prologue(in.apart, in.anb, R, in.sc, in.ic, coef_s, act_s, red_s);
    for (int c = threadIdx.x; c < R; c += kMB) coef_s[c] *= in.sign;
    __syncthreads();
  } else {
    for (int c = threadIdx.x; c < R; c += kMB) {
      act_s[c] = in.active ? in.active[c] : 1;
      coef_s[c] = in.cvec ? in.sign * in.cvec[c] : 0.0;
    }
    __syncthreads();
  }
  {
    bool any = false;
    for (int c = 0; c < R; ++c) any = any || act_s[c];
    if (!any) return;   // uniform across the grid
  }
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t G = gridDim.x;
  const int rc0 = R < 32 ? R : 32;
  // zero padding (never overwritten): rows NL.. of A, columns NL..LD-1 of
  // the other rows of A and of W^T
  constexpr int PC = LD - NL;
  for (int t = NL * LD + tid; t < MT * 16 * LD; t += kMB) sA[t] = 0.0;
  for (int t = tid; t < NL * PC; t += kMB) sA[(t / PC) * LD + NL + t % PC] = 0.0;
  for (int t = tid; t < 32 * PC; t += kMB) sW[(t / PC) * LD + NL + t % PC] = 0.0;
  // this thread's matrix entries q = tid + 256 u and their two LDS places
  int pa[MPT], pb[MPT];
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int q = tid + u * kMB;
    int i = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    while (i * (i + 1) / 2 > q) --i;
    const int j = q - i * (i + 1) / 2;
    pa[u] = q < NPK ? i * LD + j : -1;
    pb[u] = j * LD + i;
  }
  // this thread's gathered pairs: k = (tid + 256 u) / 32, column r = tid % 32
  const int r0 = tid & 31;
  T mreg[MPT];
  double xa[GPT], xb[GPT];
  int32_t gcur[GPT], gnxt[GPT];
  auto load_map = [&](int64_t Kx, int32_t* gm) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kMB) >> 5;
      gm[u] = (Kx < E && k < NL) ? l2g[Kx * NL + k] : 0;
    }
  };
  auto load_elem = [&](int64_t Kx, const int32_t* gm) {
    const bool ok = Kx < E;
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int q = tid + u * kMB;
      // read once per apply: the non-temporal hint keeps the vectors and the
      // broken values, not this stream, in the caches
      mreg[u] = (ok && q < NPK) ? __builtin_nontemporal_load(&mat[Kx * NPK + q]) : (T)0;
    }
    const bool cok = ok && r0 < rc0 && act_s[r0];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kMB) >> 5;
      const bool v = cok && k < NL;
      const int64_t gi = (int64_t)gm[u] * R + r0;
      xa[u] = v ? in.x[gi] : 0.0;
      xb[u] = (v && in.x2) ? in.x2[gi] : 0.0;
    }
  };
  auto tiles = [&](int64_t K, int c0, int rc) {
    const int nt_count = rc > 16 ? 2 : 1;
    for (int ti = wv; ti < MT * nt_count; ti += 4) {
      const int mt = ti / nt_count, nt = ti - mt * nt_count;
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      const double* arow = sA + (16 * mt + (lane & 15)) * LD + (lane >> 4);
      const double* brow = sW + (16 * nt + (lane & 15)) * LD + (lane >> 4);
#pragma unroll
      for (int s = 0; s < KP / 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(arow[4 * s], brow[4 * s], acc, 0, 0, 0);
      const int j = 16 * nt + (lane & 15);
      if (j < rc && act_s[c0 + j]) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * mt + (lane >> 4) + 4 * r;
          if (i < NL) zb[((int64_t)i * E + K) * R + c0 + j] = (ZT)acc[r];
        }
      }
    }
  };
  int64_t K = blockIdx.x;
  load_map(K, gcur);
  load_elem(K, gcur);
  load_map(K + G, gnxt);
  const double cf0 = r0 < R ? coef_s[r0] : 0.0;
  for (; K < E; K += G) {
    __syncthreads();   // the previous element's products are done with sA, sW
#pragma unroll
    for (int u = 0; u < MPT; ++u)
      if (pa[u] >= 0) {
        const double v = (double)mreg[u];
        sA[pa[u]] = v;
        sA[pb[u]] = v;
      }
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kMB) >> 5;
      if (k < NL) {
        sW[r0 * LD + k] = fma(cf0, xb[u], xa[u]);
        if (r0 == 0) gidx[k] = gcur[u];
      }
    }
    __syncthreads();
    // next element's loads go out before this element's products
#pragma unroll
    for (int u = 0; u < GPT; ++u) gcur[u] = gnxt[u];
    load_elem(K + G, gcur);
    load_map(K + 2 * G, gnxt);
    tiles(K, 0, rc0);
    // further blocks of 32 columns (more than 32 right-hand sides): gathered directly
    for (int c0 = 32; c0 < R; c0 += 32) {
      const int rc = (R - c0) < 32 ? (R - c0) : 32;
      __syncthreads();
      for (int q = tid; q < 32 * NL; q += kMB) {
        const int k = q >> 5, r = q & 31;
        double v = 0.0;
        if (r < rc && act_s[c0 + r]) {
          const int64_t gi = (int64_t)gidx[k] * R + c0 + r;
          v = in.x[gi];
          if (in.x2) v = fma(coef_s[c0 + r], in.x2[gi], v);
        }
        sW[r * LD + k] = v;
      }
      __syncthreads();
      tiles(K, c0, rc);
    }
  }
}

#define MFMA_CASES(X) X(42) X(45) X(56) X(60) X(70) X(72) X(84) X(105)

template <int NL, typename T, typename ZT>
static int mfma_launch(Ctx* c, int R, const InArgs& in, const T* mat, ZT* zb, hipStream_t s) {
  static int per_cu = 0;   // resident work-groups per compute unit (LDS bound)
  if (per_cu == 0) {
    int v = 0;
    BRAS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_elem_mfma<NL, T, ZT>, kMB, 0));
    per_cu = v > 0 ? v : 1;
  }
  const int64_t want = (int64_t)per_cu * c->ncu;
  const unsigned nb = (unsigned)(c->E < want ? c->E : want);
  k_elem_mfma<NL, T, ZT><<<nb, kMB, 0, s>>>(c->E, R, c->l2g, in, mat, zb);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

template <typename T, typename ZT>
static int mfma_dispatch(Ctx* c, int R, const InArgs& in, const T* mat, ZT* zb, hipStream_t s) {
#define CASE(N) \
  case N: return mfma_launch<N, T, ZT>(c, R, in, mat, zb, s);
  switch (c->nl) {
    MFMA_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no per-element matrix-core kernel", c->nl);
  }
#undef CASE
}

int mfma_elem_f64(Ctx* c, int R, const InArgs& in, const double* mat, double* zb, hipStream_t s) {
  return mfma_dispatch<double, double>(c, R, in, mat, zb, s);
}

int mfma_elem_f32(Ctx* c, int R, const InArgs& in, const float* mat, float* zb, hipStream_t s) {
  return mfma_dispatch<float, float>(c, R, in, mat, zb, s);
}

}  // namespace bras
