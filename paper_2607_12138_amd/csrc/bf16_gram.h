// The two element-local Gram products of the BF16 BRAS element pass
// (bf16.hip), shared with the LDS-resident microbenchmark (microbench.hip):
//     U = Gtil W,   Z = Gtil^T bf16(U)
// for one element and 32 right-hand-side columns, on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation).  Tiles in LDS:
//   sG [MP][LD]  Gtil, lower triangle, zero elsewhere (rows padded to LD)
//   sW [32][LD]  W^T (column c of the block in row c)
//   sU [32][LD]  U^T, written by gram_u
// MFMA operand layout (32x32x16):
//   A[i][k]: lane l holds i = l%32, k = 8*(l/32) + e, e = 0..7
//   B[k][j]: lane l holds j = l%32, k = 8*(l/32) + e
//   D[i][j]: lane l, reg r holds j = l%32, i = 8*(r/4) + 4*(l/32) + r%4
#pragma once

#include <hip/hip_runtime.h>

namespace bras {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kB16 = 256;   // work-group of the BF16 element pass: 4 wavefronts

template <int NL>
struct Bf16Shape {
  static constexpr int MT = (NL + 31) / 32;   // 32-row tiles (one wavefront each)
  static constexpr int KS = (NL + 15) / 16;   // 16-deep k steps
  static constexpr int KP = 16 * KS;          // used columns
  static constexpr int MP = 32 * MT;          // rows
  static constexpr int LD = KP + 8;           // row stride: 16-byte reads of 8 consecutive rows hit distinct banks
  static_assert(MP >= KP, "the transposed reads of gram_z stay inside the tile");
};

// Issued MFMA instructions of one element and 32 columns (both products).
template <int NL>
constexpr int gram_mfma_count() {
  int n = 0;
  for (int t = 0; t < Bf16Shape<NL>::MT; ++t) {
    const int kmax = (32 * t + 32) < NL ? (32 * t + 32) : NL;
    n += (kmax + 15) / 16 + (Bf16Shape<NL>::KS - 2 * t);
  }
  return n;
}

// U = Gtil W for the 32-row tile t (wavefront t < MT): Gtil row i has entries
// k <= i only.  U is rounded to BF16 and stored transposed; registers 4m ..
// 4m+3 hold rows row0 .. row0+3 of one column: one 8-byte store.
template <int NL>
__device__ __forceinline__ void gram_u(const __bf16* sG, const __bf16* sW, __bf16* sU, int t, int lane) {
  constexpr int KP = Bf16Shape<NL>::KP, LD = Bf16Shape<NL>::LD;
  f32x16 acc = {};
  const int kmax = (32 * t + 32) < NL ? (32 * t + 32) : NL;
  const int ssteps = (kmax + 15) / 16;
  const int i = 32 * t + (lane & 31);
  const int kh = 8 * (lane >> 5);
  for (int st = 0; st < ssteps; ++st) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(&sG[i * LD + 16 * st + kh]);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sW[(lane & 31) * LD + 16 * st + kh]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    const int row0 = 32 * t + 8 * m + 4 * (lane >> 5);
    if (row0 < KP) {
      const bf16x4 v = {(__bf16)acc[4 * m], (__bf16)acc[4 * m + 1], (__bf16)acc[4 * m + 2], (__bf16)acc[4 * m + 3]};
      *reinterpret_cast<bf16x4*>(&sU[(lane & 31) * LD + row0]) = v;
    }
  }
}

// Z = Gtil^T U for the 32-row tile t: output row j needs k = i >= j, so the
// tile starts at k-step 2t; A[j][k] = Gtil[k][j] is read down column j of
// sG, one 2-byte element per k (for j >= n_loc the reads fall on other rows'
// entries: those outputs are never used).
template <int NL>
__device__ __forceinline__ f32x16 gram_z(const __bf16* sG, const __bf16* sU, int t, int lane) {
  constexpr int KS = Bf16Shape<NL>::KS, LD = Bf16Shape<NL>::LD;
  f32x16 acc = {};
  const int j = 32 * t + (lane & 31);
  const int kh = 8 * (lane >> 5);
  for (int st = 2 * t; st < KS; ++st) {
    const int k0 = 16 * st + kh;
    bf16x8 a;
#pragma unroll
    for (int e = 0; e < 8; ++e) a[e] = sG[(k0 + e) * LD + j];
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(&sU[(lane & 31) * LD + k0]);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  return acc;
}

}  // namespace bras
