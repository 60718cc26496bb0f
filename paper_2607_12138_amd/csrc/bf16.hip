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

__device__ __forceinline__ void unpack_tri(int q, int& i, int& j) {
  int r = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
  while ((r + 1) * (r + 2) / 2 <= q) ++r;
  while (r * (r + 1) / 2 > q) --r;
  i = r;
  j = q - r * (r + 1) / 2;
}

template <int NL>
__global__ void __launch_bounds__(kB16) k_bras_bf16(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                                    const __bf16* __restrict__ G, float* __restrict__ zb) {
  constexpr int MT = (NL + 31) / 32;
  constexpr int KS = (NL + 15) / 16;
  constexpr int KP = 16 * KS;
  constexpr int MP = 32 * MT;
  constexpr int NPK = NL * (NL + 1) / 2;
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
  const int64_t K = blockIdx.x;

  // unpack Gtil (zero padding first)
  const __bf16 zero = (__bf16)0.0f;
  for (int q = tid; q < MP * KP; q += kB16) {
    sG[q] = zero;
    sGT[q] = zero;
  }
  for (int q = tid; q < KP; q += kB16) gidx[q] = q < NL ? l2g[K * NL + q] : 0;
  __syncthreads();
  for (int q = tid; q < NPK; q += kB16) {
    int i, j;
    unpack_tri(q, i, j);
    const __bf16 v = G[K * NPK + q];
    sG[i * KP + j] = v;
    sGT[j * KP + i] = v;
  }

  for (int c0 = 0; c0 < R; c0 += 32) {
    const int rc = (R - c0) < 32 ? (R - c0) : 32;
    // gather W^T[r][k] = input[pi_k, c0 + r]
    for (int q = tid; q < 32 * KP; q += kB16) {
      const int k = q >> 5, r = q & 31;
      double v = 0.0;
      if (k < NL && r < rc && act_s[c0 + r]) {
        const int64_t gi = gidx[k];
        v = in.x[gi * R + c0 + r];
        if (in.x2) v = fma(coef_s[c0 + r], in.x2[gi * R + c0 + r], v);
      }
      sW[r * KP + k] = (__bf16)(float)v;
    }
    __syncthreads();
    // U = Gtil W: wave t owns rows 32t..32t+31; Gtil row i has entries k <= i only
    if (wv < MT) {
      const int t = wv;
      f32x16 acc = {};
      const int kmax = (32 * t + 32) < NL ? (32 * t + 32) : NL;
      const int ssteps = (kmax + 15) / 16;
      const int i = 32 * t + (lane & 31);
      const int kh = 8 * (lane >> 5);
      for (int s = 0; s < ssteps; ++s) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sG[i * KP + 16 * s + kh]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sW[(lane & 31) * KP + 16 * s + kh]);
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
      for (int s = 2 * t; s < KS; ++s) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sGT[j * KP + 16 * s + kh]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sU[(lane & 31) * KP + 16 * s + kh]);
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
    __syncthreads();
  }
}

#define BF16_CASES(X) X(3) X(4) X(6) X(8) X(10) X(15) X(20) X(24) X(35) X(36) X(45) X(56) X(70) X(84)

static int bf16_elem(Ctx* c, const InArgs& in, int R, hipStream_t s) {
  const unsigned nb = (unsigned)c->E;
#define CASE(N)                                                                                        \
  case N:                                                                                              \
    k_bras_bf16<N><<<nb, kB16, 0, s>>>(c->E, R, c->l2g, in, (const __bf16*)c->ainv, (float*)c->zb);    \
    break;
  switch (c->nl) {
    BF16_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no BF16 element kernel", c->nl);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

int launch_bras_bf16(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                     const int* active) {
  InArgs in;
  in.x = x;
  in.active = active;
  int st = bf16_elem(c, in, R, s);
  if (st) return st;
  return reduce_float_plain(c, (const float*)c->zb, y, R, s, dotv, dotpart);
}

int cg_bras_bf16_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  InArgs in = precond_input(cg, R);
  int st = bf16_elem(c, in, R, s);
  if (st) return st;
  return reduce_float_cg(c, (const float*)c->zb, R, s, cg);
}

}  // namespace bras
