// Multi-right-hand-side BRAS element pass with the element inverses in BF16
// Gram-factor form, on MFMA (gfx950 v_mfma_f32_32x32x16_bf16, FP32
// accumulation).
//
// Setup stores, per element, Gtil = L_K^-1 D_K^-1 (M_K = L_K L_K^T, packed
// lower, BF16), so D_K^-1 M_K^-1 D_K^-1 = Gtil^T Gtil.  The element pass
// computes, for 32 columns at a time,
//     U = Gtil W          (W = gathered input, BF16)
//     Z = Gtil^T bf16(U)  (FP32)
// so that r^T z = ||Gtil r||^2 up to the BF16 rounding of the intermediate
// U: the preconditioner stays positive, which a BF16-rounded full inverse
// would not guarantee for ill-conditioned element matrices.
//
// One work-group (4 wavefronts) per element: Gtil and Gtil^T are unpacked
// into zero-padded LDS tiles [MP][KP] (MP = 32 * ceil(n_loc/32) rows, KP = 16 *
// ceil(n_loc/16) columns), W^T and U^T are [32][KP].  Wave t computes the
// 32-row output tile t of each product.  MFMA operand layout (32x32x16):
//   A[i][k]: lane l holds i = l%32, k = 8*(l/32) + e, e = 0..7
//   B[k][j]: lane l holds j = l%32, k = 8*(l/32) + e
//   D[i][j]: lane l, reg r holds j = l%32, i = 8*(r/4) + 4*(l/32) + r%4
// The broken output (FP32) goes to zb[l][K][R] like the other element passes.
#include <cmath>

#include "internal.h"
#include "cg_common.h"

namespace bras {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kB16 = 256;


// Persistent: work-group g handles elements g, g + G, ...; while the matrix
// cores work on element K the registers hold the loads of element K + G (its
// factor and first 32 gathered columns) and the map of element K + 2G.
template <int NL>
__global__ void __launch_bounds__(kB16) k_bras_bf16(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                                    const __bf16* __restrict__ G, float* __restrict__ zb) {
  constexpr int MT = (NL + 31) / 32;
  constexpr int KS = (NL + 15) / 16;
  constexpr int KP = 16 * KS;
  constexpr int MP = 32 * MT;
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr int MPT = (NPK + kB16 - 1) / kB16;      // factor entries per thread
  constexpr int GPT = (32 * NL + kB16 - 1) / kB16;  // gathered (k, column) pairs per thread
  __shared__ __attribute__((aligned(16))) __bf16 sG[MP * KP];
  __shared__ __attribute__((aligned(16))) __bf16 sGT[MP * KP];
  __shared__ __attribute__((aligned(16))) __bf16 sW[32 * KP];
  __shared__ __attribute__((aligned(16))) __bf16 sU[32 * KP];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  __shared__ double red_s[kB16];
  __shared__ int32_t gidx[KP];

  if (in.apart) {
    alpha_prologue(in.apart, in.anb, R, in.sc, in.ic, coef_s, act_s, red_s);
    for (int c = threadIdx.x; c < R; c += kB16) coef_s[c] *= in.sign;
    __syncthreads();
  } else {
    for (int c = threadIdx.x; c < R; c += kB16) {
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
  const int64_t GS = gridDim.x;
  const int rc0 = R < 32 ? R : 32;

  // zero the tiles once: only lower-triangle entries are written later, and
  // W^T / U^T only for k < NL (U rows < KP are all written)
  const __bf16 zero = (__bf16)0.0f;
  for (int q = tid; q < MP * KP; q += kB16) {
    sG[q] = zero;
    sGT[q] = zero;
  }
  for (int q = tid; q < 32 * KP; q += kB16) {
    sW[q] = zero;
    sU[q] = zero;
  }
  int pa[MPT], pb[MPT];
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int q = tid + u * kB16;
    int i = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    while (i * (i + 1) / 2 > q) --i;
    const int j = q - i * (i + 1) / 2;
    pa[u] = q < NPK ? i * KP + j : -1;
    pb[u] = j * KP + i;
  }
  const int r0 = tid & 31;
  __bf16 greg[MPT];
  double xa[GPT], xb[GPT];
  int32_t gcur[GPT], gnxt[GPT];
  auto load_map = [&](int64_t Kx, int32_t* gm) {
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kB16) >> 5;
      gm[u] = (Kx < E && k < NL) ? l2g[Kx * NL + k] : 0;
    }
  };
  auto load_elem = [&](int64_t Kx, const int32_t* gm) {
    const bool ok = Kx < E;
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int q = tid + u * kB16;
      // non-temporal: the factors are read once per apply
      greg[u] = (ok && q < NPK)
                    ? __builtin_bit_cast(__bf16, __builtin_nontemporal_load(
                                                     reinterpret_cast<const unsigned short*>(G) + Kx * NPK + q))
                    : zero;
    }
    const bool cok = ok && r0 < rc0 && act_s[r0];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kB16) >> 5;
      const bool v = cok && k < NL;
      const int64_t gi = (int64_t)gm[u] * R + r0;
      xa[u] = v ? in.x[gi] : 0.0;
      xb[u] = (v && in.x2) ? in.x2[gi] : 0.0;
    }
  };
  // Z = Gtil^T bf16(Gtil W) for the 32 columns c0.. in sW
  auto products = [&](int64_t K, int c0, int rc) {
    // U = Gtil W: wave t owns rows 32t..32t+31; Gtil row i has entries k <= i only
    if (wv < MT) {
      const int t = wv;
      f32x16 acc = {};
      const int kmax = (32 * t + 32) < NL ? (32 * t + 32) : NL;
      const int ssteps = (kmax + 15) / 16;
      const int i = 32 * t + (lane & 31);
      const int kh = 8 * (lane >> 5);
      for (int st = 0; st < ssteps; ++st) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sG[i * KP + 16 * st + kh]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sW[(lane & 31) * KP + 16 * st + kh]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < KP) sU[(lane & 31) * KP + row] = (__bf16)acc[r];
      }
    }
    __syncthreads();
    // Z = Gtil^T U: output row j needs k = i >= j, so tile t starts at k-step 2t
    if (wv < MT) {
      const int t = wv;
      f32x16 acc = {};
      const int j = 32 * t + (lane & 31);
      const int kh = 8 * (lane >> 5);
      for (int st = 2 * t; st < KS; ++st) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sGT[j * KP + 16 * st + kh]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sU[(lane & 31) * KP + 16 * st + kh]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
      const int col = lane & 31;
      if (col < rc && act_s[c0 + col]) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          if (row < NL) zb[((int64_t)row * E + K) * R + c0 + col] = acc[r];
        }
      }
    }
  };
  int64_t K = blockIdx.x;
  load_map(K, gcur);
  load_elem(K, gcur);
  load_map(K + GS, gnxt);
  const double cf0 = r0 < R ? coef_s[r0] : 0.0;
  for (; K < E; K += GS) {
    __syncthreads();   // the previous element's products are done with the tiles
#pragma unroll
    for (int u = 0; u < MPT; ++u)
      if (pa[u] >= 0) {
        sG[pa[u]] = greg[u];
        sGT[pb[u]] = greg[u];
      }
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kB16) >> 5;
      if (k < NL) {
        sW[r0 * KP + k] = (__bf16)(float)fma(cf0, xb[u], xa[u]);
        if (r0 == 0) gidx[k] = gcur[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GPT; ++u) gcur[u] = gnxt[u];
    load_elem(K + GS, gcur);
    load_map(K + 2 * GS, gnxt);
    products(K, 0, rc0);
    for (int c0 = 32; c0 < R; c0 += 32) {
      const int rc = (R - c0) < 32 ? (R - c0) : 32;
      __syncthreads();
      for (int q = tid; q < 32 * NL; q += kB16) {
        const int k = q >> 5, r = q & 31;
        double v = 0.0;
        if (r < rc && act_s[c0 + r]) {
          const int64_t gi = (int64_t)gidx[k] * R + c0 + r;
          v = in.x[gi];
          if (in.x2) v = fma(coef_s[c0 + r], in.x2[gi], v);
        }
        sW[r * KP + k] = (__bf16)(float)v;
      }
      __syncthreads();
      products(K, c0, rc);
    }
  }
}

#define BF16_CASES(X) X(3) X(4) X(6) X(8) X(10) X(15) X(20) X(24) X(35) X(36) X(45) X(56) X(70) X(84)

template <int NL>
static int bf16_launch(Ctx* c, const InArgs& in, int R, hipStream_t s, float* zb) {
  static int per_cu = 0;   // resident work-groups per compute unit
  if (per_cu == 0) {
    int v = 0;
    BRAS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_bras_bf16<NL>, kB16, 0));
    per_cu = v > 0 ? v : 1;
  }
  const int64_t want = (int64_t)per_cu * c->ncu;
  const unsigned nb = (unsigned)(c->E < want ? c->E : want);
  k_bras_bf16<NL><<<nb, kB16, 0, s>>>(c->E, R, c->l2g, in, (const __bf16*)c->ainv, zb);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int bf16_elem(Ctx* c, const InArgs& in, int R, hipStream_t s, float* zb) {
#define CASE(N) \
  case N: return bf16_launch<N>(c, in, R, s, zb);
  switch (c->nl) {
    BF16_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no BF16 element kernel", c->nl);
  }
#undef CASE
}

int bf16_elem_pass(Ctx* c, const InArgs& in, int R, hipStream_t s) { return bf16_elem(c, in, R, s, (float*)c->zb); }

int launch_bras_bf16(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                     const int* active, void* zb) {
  InArgs in;
  in.x = x;
  in.active = active;
  int st = bf16_elem(c, in, R, s, (float*)zb);
  if (st) return st;
  return reduce_float_plain(c, (const float*)zb, y, R, s, dotv, dotpart);
}

int cg_bras_bf16_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  InArgs in = precond_input(cg, R);
  int st = bf16_elem(c, in, R, s, (float*)c->zb);
  if (st) return st;
  return reduce_float_cg(c, (const float*)c->zb, R, s, cg);
}

}  // namespace bras
