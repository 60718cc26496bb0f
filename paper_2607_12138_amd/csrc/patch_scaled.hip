// Patch-form operator passes (patch_kern.h) for the scaled H1 form on the
// FP64 matrix cores.
//
// With affine H1 elements M_K = c_K Mhat (eq. h1_mass_pullback; c_K = rho_K
// |det J_K|), so one patch's element products are a single GEMM with the
// shared reference matrix:
//     Z = A W,   W [n_loc][elements] the patch's inputs,   z_K = s_K Z[:, K]
// A = Mhat (mass, s_K = c_K) or Mhat^-1 (BRAS, s_K = 1/c_K, inputs and
// outputs times D^-1).  A sits in LDS, zero padded to 16-row tiles and
// 4-deep k steps; each wavefront takes 16-element column tiles and runs
// v_mfma_f64_16x16x4_f64 with B read straight from the patch DOF values
// through the copy codes, then scales its columns.  The sums: DOF j's copies
// are counted (LDS integer adds), the counts scanned into segment starts, and
// the copy of rank r stored at start[j] + r; each DOF then adds its segment
// in order, the same additions as the rank-by-rank adds of the per-lane
// passes, with three barriers instead of one per rank (vertex DOFs of P4
// patches have up to 24 copies).
//
// MFMA operand layout (16x16x4, one double per lane):
//   A[i][k]: lane l holds i = l%16, k = l/16
//   B[k][j]: lane l holds j = l%16, k = l/16
//   D[i][j]: lane l, reg r holds j = l%16, i = l/16 + 4*r
#include "patch_kern.h"

namespace bras {

typedef double f64x4 __attribute__((ext_vector_type(4)));

// TPW: 16-element column tiles per wavefront (patches of up to 64 TPW elements).
template <int NL, int OUT, bool DS, int TPW>
__global__ void __launch_bounds__(kPatchBlock) k_patch_mfma(PatchArgs pa, InArgs in, const double* __restrict__ A,
                                                            const double* __restrict__ coefK,
                                                            const double* __restrict__ dscale, double* __restrict__ y,
                                                            const double* __restrict__ dotv,
                                                            double* __restrict__ dotpart, CgArgs cg,
                                                            double* __restrict__ spart) {
  constexpr int MT = (NL + 15) / 16;   // 16-row tiles
  constexpr int KS = (NL + 3) / 4;     // 4-deep k steps
  constexpr int LDA = 4 * KS + 1;      // LDS row stride of A (odd: spreads banks)
  extern __shared__ double wsh[];      // inputs, then sums, then dot partials
  __shared__ double sA[MT * 16 * LDA];
  __shared__ double zs[64 * TPW * NL];   // the patch's element outputs, segment by segment
  __shared__ int scan_s[kPatchBlock / 64];
  __shared__ double coef_s[1];
  __shared__ int act_s[1];
  const int tid = threadIdx.x;
  if (in.apart) {
    alpha_prologue(in.apart, in.anb, 1, in.sc, in.ic, coef_s, act_s, wsh);
  } else {
    if (tid == 0) {
      act_s[0] = in.active ? in.active[0] : 1;
      coef_s[0] = in.cvec ? in.cvec[0] : 0.0;
    }
    __syncthreads();
  }
  if (!act_s[0]) return;   // uniform across the grid
  const double cf = coef_s[0];
  const double c2 = in.x2 ? in.sign * cf : 0.0;
  const int64_t p = pa.xcd_per > 0 ? (int64_t)(blockIdx.x % 8) * pa.xcd_per + blockIdx.x / 8 : (int64_t)blockIdx.x;
  if (p >= pa.npatch) return;   // uniform across the work-group
  const int32_t e0 = pa.pe[p], ne = pa.pe[p + 1] - e0;
  const int32_t d0 = pa.pd[p], nd = pa.pd[p + 1] - d0, nloc = pa.pnl[p];
  __syncthreads();   // the prologue's use of wsh is over
  // 1. patch DOF values, and A (zero padded)
  const int32_t lbase = pa.ip ? d0 - pa.sbase[p] : -1;
  patch_gather<DS>(pa.pdof, d0, nd, nloc, lbase, in, c2, dscale, wsh, nullptr);
  for (int t = tid; t < MT * 16 * LDA; t += kPatchBlock) {
    const int i = t / LDA, k = t - i * LDA;
    sA[t] = (i < NL && k < NL) ? A[i * NL + k] : 0.0;
  }
  __syncthreads();
  // 2. products: wavefront wv takes column tiles wv, wv + 4, ...
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int col = lane & 15, kq = lane >> 4;
  const uint32_t lmask = (1u << pa.lbits) - 1u;
  const uint16_t* cbase = pa.code + (int64_t)e0 * NL;
  f64x4 acc[TPW][MT];
  uint32_t oc[TPW][MT][2];   // codes of the four outputs of each tile, two to a register
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int e = 16 * (wv + 4 * t) + col;
    const bool eon = e < ne;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[t][mt] = f64x4{0.0, 0.0, 0.0, 0.0};
    if (16 * (wv + 4 * t) < ne) {   // uniform across the wavefront
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + kq;
        const double b = (eon && k < NL) ? wsh[cbase[(int64_t)k * ne + e] & lmask] : 0.0;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
          const double a = sA[(16 * mt + col) * LDA + 4 * ks + kq];
          acc[t][mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t][mt], 0, 0, 0);
        }
      }
    }
    const double ck = eon ? coefK[e0 + e] : 0.0;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      uint32_t c4[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        acc[t][mt][r] *= ck;
        const int i = 16 * mt + kq + 4 * r;
        c4[r] = (eon && i < NL) ? (uint32_t)cbase[(int64_t)i * ne + e] : 0xFFFFu;   // 0xFFFF: no output
      }
      oc[t][mt][0] = c4[0] | (c4[1] << 16);
      oc[t][mt][1] = c4[2] | (c4[3] << 16);
    }
  }
  __syncthreads();   // every input read: wsh now holds the copy counts, then the segment starts
  int* I = reinterpret_cast<int*>(wsh);   // nd + 1 ints fit in the nd >= 1 doubles of wsh
  for (int j = tid; j <= nd; j += kPatchBlock) I[j] = 0;
  __syncthreads();
  const int lb = pa.lbits;
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t cl = (oc[t][mt][q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
        if (cl != 0xFFFFu) atomicAdd(&I[cl & lmask], 1);
      }
  __syncthreads();
  patch_count_scan(I, nd, scan_s);
  // each copy's value at start[j] + rank: every DOF's copies in rank (= element) order
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t cl = (oc[t][mt][q >> 1] >> (16 * (q & 1))) & 0xFFFFu;
        if (cl != 0xFFFFu) zs[I[cl & lmask] + (int)(cl >> lb)] = acc[t][mt][q];
      }
  __syncthreads();
  // 3. DOFs of the patch
  const double ep1 = OUT == OUT_STAT ? cg.sc[S_ALPHA] : cf;
  const double ep2 = OUT == OUT_STAT ? cg.sc[S_BETA] : 0.0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  patch_finish<OUT, DS, false>(pa.pdof, d0, nd, nloc, lbase, nullptr, SegmentSums{I, zs}, nullptr, dscale, ep1, ep2, cg, y, dotv, spart,
                        pa.sbase[p], a0, a1, a2);
  __syncthreads();   // wsh is free again
  patch_dots<OUT>(a0, a1, a2, p, OUT == OUT_PLAIN ? dotpart : cg.part0, cg, wsh);
}

template <int NL, int OUT, bool DS>
static int mfma_launch(Ctx* c, const PatchCall& pc, const double* A, const double* coefK, const double* dscale,
                       hipStream_t s) {
  const PatchDev& pt = c->pt;
  const bool ip = c->ip_mode != 0;
  const int xcd_per = c->patch_xcd ? (int)((pt.npatch + 7) / 8) : 0;
  PatchArgs pa{pt.pe, pt.pd, pt.pnl, ip ? pt.pidx : pt.pdof, pt.code, pt.sbase, c->E, pt.lbits, pt.maxrank,
               pt.npatch, xcd_per, ip ? 1 : 0, pt.maxdofs};
  if (ip && dscale) dscale = pt.invd_ip;
  const int words = pt.maxdofs > 3 * kPatchBlock ? pt.maxdofs : 3 * kPatchBlock;
  const unsigned grid = xcd_per > 0 ? (unsigned)(8 * xcd_per) : (unsigned)pt.npatch;
  if (pt.maxelems <= 64)
    k_patch_mfma<NL, OUT, DS, 1><<<grid, kPatchBlock, sizeof(double) * words, s>>>(pa, pc.in, A, coefK, dscale, pc.y,
                                                                                 pc.dotv, pc.dotpart, pc.cg,
                                                                                 pc.spart);
  else if (pt.maxelems <= 128)
    k_patch_mfma<NL, OUT, DS, 2><<<grid, kPatchBlock, sizeof(double) * words, s>>>(pa, pc.in, A, coefK, dscale, pc.y,
                                                                                 pc.dotv, pc.dotpart, pc.cg,
                                                                                 pc.spart);
  else
    k_patch_mfma<NL, OUT, DS, 4><<<grid, kPatchBlock, sizeof(double) * words, s>>>(pa, pc.in, A, coefK, dscale, pc.y,
                                                                                 pc.dotv, pc.dotpart, pc.cg,
                                                                                 pc.spart);
  BRAS_HIP(hipGetLastError());
  if (pt.ns > 0) {
    k_patch_shared<OUT, DS><<<(unsigned)pt.nb2, kPatchBlock, 0, s>>>(
        pt.ns, pt.srp, pt.spos, ip ? nullptr : pt.sdof, pt.nloc_total, pc.spart, dscale, pc.y, pc.dotv, pc.dotpart,
        pt.npatch, pc.in.active, pc.cg);
    BRAS_HIP(hipGetLastError());
  }
  return BRAS_OK;
}

template <int NL, int OUT>
static int bras_k(Ctx* c, const PatchCall& pc, hipStream_t s) {
  return mfma_launch<NL, OUT, true>(c, pc, c->refinv, c->icoef, c->invd, s);
}

template <int NL, int OUT>
static int mass_k(Ctx* c, const PatchCall& pc, hipStream_t s) {
  return mfma_launch<NL, OUT, false>(c, pc, c->ref, c->coef, nullptr, s);
}

template <int NL>
static int by_out(Ctx* c, const PatchCall& pc, hipStream_t s) {
  if (pc.op == 1) {
    switch (pc.out) {
      case OUT_PLAIN: return bras_k<NL, OUT_PLAIN>(c, pc, s);
      case OUT_BRAS_CG: return bras_k<NL, OUT_BRAS_CG>(c, pc, s);
      case OUT_STAT: return bras_k<NL, OUT_STAT>(c, pc, s);
      default: break;
    }
  }
  if (pc.op == 0) {
    switch (pc.out) {
      case OUT_PLAIN: return mass_k<NL, OUT_PLAIN>(c, pc, s);
      case OUT_MASS_CG: return mass_k<NL, OUT_MASS_CG>(c, pc, s);
      case OUT_RES: return mass_k<NL, OUT_RES>(c, pc, s);
      default: break;
    }
  }
  return fail(BRAS_EINVAL, "patch pass: operator %d has no epilogue %d in this form", pc.op, pc.out);
}

int patch_scaled(Ctx* c, const PatchCall& pc, hipStream_t s) {
#define CASE(N) \
  case N: return by_out<N>(c, pc, s);
  switch (c->nl) {
    PATCH_SCALED_NL(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no patch kernel", c->nl);
  }
#undef CASE
}

}  // namespace bras
