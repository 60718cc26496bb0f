// Patch form of the BRAS and mass operators (eqs. mhatinvbras_def,
// mass_and_bras_element_sums, M_PMbrP): one work-group per patch of up to 256
// elements (patch_setup.cpp); gather, element products and most of the
// scatter-sum in one kernel, without the broken vector in device memory.
//
//   1. the patch's DOF values w_j = x[g_j] (or an axpy of two vectors, times
//      D^-1 for the scaled H1 form) go to LDS, one float64 per DOF, read in
//      increasing DOF order;
//   2. each lane takes one element, reads its n_loc inputs from LDS through
//      the copy codes and forms z = M_K w (the per-lane product of
//      elem_lane.h: packed matrices, metric pair tables, or the shared
//      reference matrix times the element's coefficient); the LDS array then
//      collects the sums: the copies of rank 0 are added, then those of rank
//      1, ... (a barrier between ranks), so every DOF's copies are summed in
//      element order and no two lanes add to one entry at once (no atomics);
//   3. each DOF whose copies all lie in the patch gets its final value (times
//      D^-1 for the scaled H1 form) and the CG / stationary epilogue; each
//      shared DOF writes its patch's partial sum.
// A second kernel sums each shared DOF's partials in patch order and runs the
// same epilogue.  Dot-product partials: one per work-group of either kernel,
// patches first, summed in that fixed order by the consumer.
//
// One column only (R = 1); several columns use the element / reduce passes.
#pragma once

#include "internal.h"
#include "cg_common.h"
#include "elem_lane.h"
#include "patch.h"

namespace bras {

struct PatchArgs {
  const int32_t* pe;
  const int32_t* pd;
  const int32_t* pnl;
  const int32_t* pdof;
  const uint16_t* code;
  const int32_t* sbase;
  int64_t E;
  int lbits, maxrank;
  int64_t npatch;
  int xcd_per;   // > 0: work-group b takes patch (b % 8) * xcd_per + b / 8 (each XCD a contiguous run)
  int ip;        // vectors in the internal numbering: patch p's local DOFs are pd[p] - sbase[p] + j, j < pnl[p]
  int wstride;   // doubles of the gathered inputs in dynamic LDS (the sums follow them where both are kept)
};

// One call of the patch form of an operator (op 0 mass, 1 BRAS).
struct PatchCall {
  int op = 0;
  int out = 0;
  InArgs in;
  double* y = nullptr;
  const double* dotv = nullptr;
  double* dotpart = nullptr;
  CgArgs cg;
  double* spart = nullptr;   // partial sums of shared DOFs
};

// The CG / stationary epilogue of entry g in two halves: the vectors it reads
// (loaded early, beside other loads), then the update from them.
template <int OUT>
__device__ __forceinline__ void patch_epilogue_load(bool ok, int32_t g, const CgArgs& cg, const double* dotv,
                                                    double* v) {
  v[0] = v[1] = v[2] = v[3] = v[4] = 0.0;
  if (!ok) return;
  if (OUT == OUT_PLAIN) {
    v[0] = dotv ? dotv[g] : 0.0;
  } else if (OUT == OUT_MASS_CG) {
    v[0] = cg.p[g];
    v[1] = cg.z[g];
  } else if (OUT == OUT_BRAS_CG) {
    v[0] = cg.q[g];
    v[1] = cg.r[g];
    v[2] = cg.x[g];
    v[3] = cg.p[g];
    v[4] = cg.flexible ? cg.z[g] : 0.0;
  } else if (OUT == OUT_RES) {
    v[0] = cg.b[g];
  } else {
    v[0] = cg.p[g];
    v[1] = cg.x[g];
  }
}

template <int OUT>
__device__ __forceinline__ void patch_epilogue_pre(int32_t g, double acc, double coef, double coef2, const CgArgs& cg,
                                                   double* y, bool has_dotv, const double* v, double& d0, double& d1,
                                                   double& d2) {
  if (OUT == OUT_PLAIN) {
    y[g] = acc;
    if (has_dotv) d0 = fma(acc, v[0], d0);
  } else if (OUT == OUT_MASS_CG) {
    const double pn = fma(coef, v[0], v[1]);
    cg.p[g] = pn;
    cg.q[g] = acc;
    d0 = fma(pn, acc, d0);
  } else if (OUT == OUT_BRAS_CG) {
    const double rn = fma(-coef, v[0], v[1]);
    cg.x[g] = fma(coef, v[3], v[2]);
    if (cg.flexible) d2 = fma(rn, v[4], d2);
    cg.z[g] = acc;
    cg.r[g] = rn;
    d0 = fma(rn, rn, d0);
    d1 = fma(rn, acc, d1);
  } else if (OUT == OUT_RES) {
    const double rv = v[0] - acc;
    cg.r[g] = rv;
    d0 = fma(rv, rv, d0);
  } else {
    const double dn = fma(coef, v[0], coef2 * acc);
    cg.p[g] = dn;
    cg.x[g] = v[1] + dn;
  }
}

// Work-group sums of the epilogue's dot-product terms (fixed tree order) into
// slot b of the partial arrays; sh: 3 * kPatchBlock doubles of LDS, free.
template <int OUT>
__device__ __forceinline__ void patch_dots(double d0, double d1, double d2, int64_t b, double* out0,
                                           const CgArgs& cg, double* sh) {
  if (OUT == OUT_STAT) return;
  if (OUT == OUT_PLAIN && !out0) return;
  double* sh0 = sh;
  double* sh1 = sh + kPatchBlock;
  double* sh2 = sh + 2 * kPatchBlock;
  const int tid = threadIdx.x;
  sh0[tid] = d0;
  if (OUT == OUT_BRAS_CG) {
    sh1[tid] = d1;
    sh2[tid] = d2;
  }
  __syncthreads();
  for (int off = kPatchBlock / 2; off > 0; off >>= 1) {
    if (tid < off) {
      sh0[tid] += sh0[tid + off];
      if (OUT == OUT_BRAS_CG) {
        sh1[tid] += sh1[tid + off];
        sh2[tid] += sh2[tid + off];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    out0[b] = sh0[0];
    if (OUT == OUT_BRAS_CG) {
      cg.part1[b] = sh1[0];
      if (cg.flexible) cg.part2[b] = sh2[0];
    }
  }
}

// DOF number of patch DOF j: from the list, or (lbase >= 0: internal
// numbering) lbase + j for the patch's local DOFs, j < nloc.
__device__ __forceinline__ int32_t patch_dof(const int32_t* __restrict__ pdof, int32_t d0, int j, int nloc,
                                             int32_t lbase) {
  return (lbase >= 0 && j < nloc) ? lbase + j : pdof[d0 + j];
}

// Phase 1 of a patch pass: wsh[j] = input value of patch DOF j, the loads of
// U DOFs per thread issued together (out-of-range slots read DOF 0 of the
// patch and store nothing); gsh (if not null) keeps the DOF numbers for the
// last phase.
template <bool DS, int U = 4>
__device__ __forceinline__ void patch_gather(const int32_t* __restrict__ pdof, int32_t d0, int nd, int nloc,
                                             int32_t lbase, const InArgs& in, double c2,
                                             const double* __restrict__ dscale, double* wsh, int32_t* gsh) {
  for (int j0 = threadIdx.x; j0 < nd; j0 += U * kPatchBlock) {
    int32_t g[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * kPatchBlock;
      g[u] = patch_dof(pdof, d0, j < nd ? j : 0, nloc, lbase);
    }
    double v[U], v2[U], ds[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = in.x[g[u]];
      v2[u] = in.x2 ? in.x2[g[u]] : 0.0;
      ds[u] = DS ? dscale[g[u]] : 1.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * kPatchBlock;
      double t = in.x2 ? fma(c2, v2[u], v[u]) : v[u];
      if (DS) t *= ds[u];
      if (j < nd) {
        wsh[j] = t;
        if (gsh) gsh[j] = g[u];
      }
    }
  }
}

// Phase 3 of a patch pass: the final values of the patch's local DOFs with
// the epilogue, and the partial sums of its shared DOFs; the loads of U DOFs
// per thread are issued before any of their stores.
// Sum of patch DOF j's copies as collected in LDS by the rank-ordered adds.
struct LdsSums {
  const double* w;
  __device__ double operator()(int j) const { return w[j]; }
};

// Sum of patch DOF j's copies from their values stored in rank order at
// zs[start[j] .. start[j+1]) (the same additions, in the same order, as the
// rank-ordered adds).
struct SegmentSums {
  const int* start;
  const double* zs;
  __device__ double operator()(int j) const {
    double a = 0.0;
    for (int q = start[j]; q < start[j + 1]; ++q) a += zs[q];
    return a;
  }
};

// Exclusive scan, in place, of the copy counts I[0..nd) of a patch's DOFs
// into segment starts, with I[nd] = the total (work-group wide; ps: 4 ints of
// LDS).  Ends with a barrier.
__device__ __forceinline__ void patch_count_scan(int* I, int nd, int* ps) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int per = (nd + kPatchBlock - 1) / kPatchBlock;
  const int b0 = tid * per < nd ? tid * per : nd;
  const int b1 = b0 + per < nd ? b0 + per : nd;
  int s = 0;
  for (int j = b0; j < b1; ++j) s += I[j];
  int incl = s;   // inclusive prefix within the wavefront
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) ps[wv] = incl;
  __syncthreads();
  int off = incl - s;
  for (int w = 0; w < wv; ++w) off += ps[w];
  for (int j = b0; j < b1; ++j) {
    const int c = I[j];
    I[j] = off;
    off += c;
  }
  if (tid == kPatchBlock - 1) I[nd] = off;   // b1 = nd for the last thread
  __syncthreads();
}

// gdof (if not null): the DOF numbers kept by the gather phase.
// REUSE (CG epilogues without D^-1): win[j] holds the pass's gathered input
// of patch DOF j, which is the epilogue's new p (mass: z + beta p) or new r
// (BRAS: r - alpha q), computed in the same arithmetic; the epilogue takes it
// instead of reading the two vectors again.  Only local DOFs read epilogue
// vectors (boundary DOFs write their partial sums).
template <int OUT, bool DS, bool REUSE, typename VAL, int U = 4>
__device__ __forceinline__ void patch_finish(const int32_t* __restrict__ pdof, int32_t d0, int nd, int nloc,
                                             int32_t lbase, const int32_t* gdof, VAL val, const double* win,
                                             const double* __restrict__ dscale, double ep1,
                                             double ep2, const CgArgs& cg, double* __restrict__ y,
                                             const double* __restrict__ dotv, double* __restrict__ spart,
                                             int32_t sb, double& a0, double& a1, double& a2) {
  for (int j0 = threadIdx.x; j0 < nd; j0 += U * kPatchBlock) {
    int32_t g[U];
    double acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * kPatchBlock;
      const bool in_range = j < nd;
      g[u] = gdof ? gdof[in_range ? j : 0] : patch_dof(pdof, d0, in_range ? j : 0, nloc, lbase);
      acc[u] = in_range ? val(j) : 0.0;
    }
    // vectors the epilogue reads, for the U DOFs at once (local DOFs only)
    double v0[U], v1[U], v2[U], v3[U], v4[U], ds[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * kPatchBlock;
      const bool loc = j < nd && j < nloc;
      const int32_t gg = g[u];
      ds[u] = (DS && loc) ? dscale[gg] : 1.0;
      v0[u] = v1[u] = v2[u] = v3[u] = v4[u] = 0.0;
      if (!loc) continue;
      if (OUT == OUT_PLAIN) {
        v0[u] = dotv ? dotv[gg] : 0.0;
      } else if (OUT == OUT_MASS_CG) {
        if (REUSE) {
          v0[u] = win[j];
        } else {
          v0[u] = cg.p[gg];
          v1[u] = cg.z[gg];
        }
      } else if (OUT == OUT_BRAS_CG) {
        if (REUSE) {
          v0[u] = win[j];
        } else {
          v0[u] = cg.q[gg];
          v1[u] = cg.r[gg];
        }
        v2[u] = cg.x[gg];
        v3[u] = cg.p[gg];
        v4[u] = cg.flexible ? cg.z[gg] : 0.0;
      } else if (OUT == OUT_RES) {
        v0[u] = cg.b[gg];
      } else {
        v0[u] = cg.p[gg];
        v1[u] = cg.x[gg];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = j0 + u * kPatchBlock;
      if (j >= nd) continue;
      if (j >= nloc) {
        spart[sb + (j - nloc)] = acc[u];
        continue;
      }
      const int32_t gg = g[u];
      double t = acc[u];
      if (DS) t *= ds[u];
      if (OUT == OUT_PLAIN) {
        y[gg] = t;
        if (dotv) a0 = fma(t, v0[u], a0);
      } else if (OUT == OUT_MASS_CG) {
        const double pn = REUSE ? v0[u] : fma(ep1, v0[u], v1[u]);
        cg.p[gg] = pn;
        cg.q[gg] = t;
        a0 = fma(pn, t, a0);
      } else if (OUT == OUT_BRAS_CG) {
        const double rn = REUSE ? v0[u] : fma(-ep1, v0[u], v1[u]);
        cg.x[gg] = fma(ep1, v3[u], v2[u]);
        if (cg.flexible) a2 = fma(rn, v4[u], a2);
        cg.z[gg] = t;
        cg.r[gg] = rn;
        a0 = fma(rn, rn, a0);
        a1 = fma(rn, t, a1);
      } else if (OUT == OUT_RES) {
        const double rv = v0[u] - t;
        cg.r[gg] = rv;
        a0 = fma(rv, rv, a0);
      } else {
        const double dn = fma(ep1, v0[u], ep2 * t);
        cg.p[gg] = dn;
        cg.x[gg] = v1[u] + dn;
      }
    }
  }
}

// Waves per SIMD the register allocator is asked for: 4 (at most 128 VGPRs)
// where a lane's element fits without spilling (float64 data re-read their
// copy codes after the product instead of keeping them through it), else its
// natural count.
template <int NL, int FORM, typename T>
constexpr int kPatchWaves() {
  return sizeof(T) == 4 ? (NL <= 20 ? 4 : 1) : ((NL <= 12 || (FORM == FORM_METRIC && NL <= 20)) ? 4 : 1);
}

// FORM_PACKED: M_K (or the folded inverse) from ap; FORM_METRIC with NSYM > 1:
// pair tables symtab [q][NSYM] and coefficients coefK [nsym][E]; FORM_METRIC
// with NSYM = 1: the scaled H1 form, symtab = the shared reference matrix as
// a packed lower triangle, coefK [E] the element's factor.  Dynamic LDS (at
// least 3 * kPatchBlock doubles): maxdofs doubles of inputs, then maxdofs
// doubles of sums where the epilogue reuses the inputs, else maxdofs ints of
// DOF numbers (the sums overwrite the inputs).
template <int NL, int FORM, int NSYM, typename T, int OUT, bool DS, int VAR>
__global__ void __launch_bounds__(kPatchBlock) __attribute__((amdgpu_waves_per_eu(kPatchWaves<NL, FORM, T>())))
k_patch(PatchArgs pa, InArgs in, const T* __restrict__ ap,
                                                       const double* __restrict__ symtab,
                                                       const double* __restrict__ coefK, int nsym,
                                                       const double* __restrict__ dscale, double* __restrict__ y,
                                                       const double* __restrict__ dotv, double* __restrict__ dotpart,
                                                       CgArgs cg, double* __restrict__ spart) {
  extern __shared__ double wsh[];   // inputs, then sums, then dot partials
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
  const double cf = coef_s[0];                    // alpha (BRAS_CG) or beta (MASS_CG)
  const double c2 = in.x2 ? in.sign * cf : 0.0;   // weight of the second input vector
  const int64_t p = pa.xcd_per > 0 ? (int64_t)(blockIdx.x % 8) * pa.xcd_per + blockIdx.x / 8 : (int64_t)blockIdx.x;
  if (p >= pa.npatch) return;   // uniform across the work-group
  const int32_t e0 = pa.pe[p], ne = pa.pe[p + 1] - e0;
  const int32_t d0 = pa.pd[p], nd = pa.pd[p + 1] - d0, nloc = pa.pnl[p];
  __syncthreads();   // the prologue's use of wsh is over
  // 1. patch DOF values
  // wavefront priority: raised in the latency-bound phases (gather, sums,
  // last phase), normal while the element data stream in, so that a
  // work-group between two barriers is not kept waiting for issue slots by the
  // streaming wavefronts of the others on its SIMDs
  __builtin_amdgcn_s_setprio(2);
  const int32_t lbase = pa.ip ? d0 - pa.sbase[p] : -1;
  // the sums: after the inputs where the epilogue reuses them, else in their
  // place; otherwise the DOF numbers follow them for the last phase
  constexpr bool REUSE = !DS && (OUT == OUT_MASS_CG || OUT == OUT_BRAS_CG);
  double* wsum = REUSE ? wsh + pa.wstride : wsh;
  int32_t* gsh = REUSE ? nullptr : reinterpret_cast<int32_t*>(wsh + pa.wstride);
  // DOFs per thread whose loads go out together in the first and last phase
  // (fewer where the CG epilogue's vectors take the registers)
  constexpr int UD = REUSE ? 4 : 8;
  // the element data that do not depend on the gather (copy codes, metric
  // coefficients) are requested before it, so that they arrive during it
  // (idle lanes repeat element 0 and add nothing)
  const bool on = tid < ne;
  const int e = on ? tid : 0;
  const uint32_t lmask = (1u << pa.lbits) - 1u;
  const uint16_t* cdp = pa.code + (int64_t)e0 * NL + e;
  // codes two to a register (they stay live through the product)
  constexpr int NC2 = (NL + 1) / 2;
  uint32_t cd2[NC2];
#pragma unroll
  for (int h = 0; h < NC2; ++h) {
    const uint32_t lo = cdp[(int64_t)(2 * h) * ne];
    const uint32_t hi = 2 * h + 1 < NL ? (uint32_t)cdp[(int64_t)(2 * h + 1) * ne] : 0u;
    cd2[h] = lo | (hi << 16);
  }
  double g[NSYM > 0 ? NSYM : 1];
  if (FORM == FORM_METRIC) {
#pragma unroll
    for (int q = 0; q < NSYM; ++q)
      g[q] = q < nsym ? __builtin_nontemporal_load(&coefK[(int64_t)q * pa.E + e0 + e]) : 0.0;
  }
  patch_gather<DS, UD>(pa.pdof, d0, nd, nloc, lbase, in, c2, dscale, wsh, gsh);
  __syncthreads();
  // 2. one element per lane
  auto code = [&](int l) -> uint32_t { return (cd2[l >> 1] >> (16 * (l & 1))) & 0xFFFFu; };
  T wr[NL], z[NL];
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    wr[l] = (T)wsh[code(l) & lmask];
    z[l] = (T)0;
  }
  __syncthreads();   // every input read: the array now collects the sums
  __builtin_amdgcn_s_setprio(0);
  lane_product<NL, FORM, NSYM, T, VAR>(wr, z, e0, e, pa.E, ap, symtab, g);
  __builtin_amdgcn_s_setprio(2);
  // float64 element data: the codes again (an L2 or Infinity Cache read), so that they take no
  // registers during the product
  if (sizeof(T) == 8) {
    const uint16_t* cdq = cdp + pin_v(0, z[0]);
#pragma unroll
    for (int h = 0; h < NC2; ++h) {
      const uint32_t lo = cdq[(int64_t)(2 * h) * ne];
      const uint32_t hi = 2 * h + 1 < NL ? (uint32_t)cdq[(int64_t)(2 * h + 1) * ne] : 0u;
      cd2[h] = lo | (hi << 16);
    }
  }
  __syncthreads();
  const int lb = pa.lbits;
  // every patch DOF has a copy of rank 0, which starts its sum (0 + z, as an add to a zeroed sum)
  if (on) {
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const uint32_t cl = code(l);
      if ((cl >> lb) == 0) wsum[cl & lmask] = 0.0 + (double)z[l];
    }
  }
  __syncthreads();
  for (int r = 1; r <= pa.maxrank; ++r) {
    if (on) {
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const uint32_t cl = code(l);
        if ((int)(cl >> lb) == r) wsum[cl & lmask] += (double)z[l];
      }
    }
    __syncthreads();
  }
  // 3. DOFs of the patch
  const double ep1 = OUT == OUT_STAT ? cg.sc[S_ALPHA] : cf;
  const double ep2 = OUT == OUT_STAT ? cg.sc[S_BETA] : 0.0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  patch_finish<OUT, DS, REUSE, LdsSums, UD>(pa.pdof, d0, nd, nloc, lbase, gsh, LdsSums{wsum}, wsh, dscale, ep1, ep2, cg, y, dotv, spart, pa.sbase[p], a0,
                        a1, a2);
  __syncthreads();   // wsh is free again
  patch_dots<OUT>(a0, a1, a2, p, OUT == OUT_PLAIN ? dotpart : cg.part0, cg, wsh);
}

// Shared DOFs: the patch partials summed in patch order, then the epilogue.
// DOF of shared DOF s: sdof[s], or (internal numbering, sdof null) sbase + s.
// The partials of shared DOF s are spart[spos[k]], k = srp[s] .. srp[s+1]-1.
template <int OUT, bool DS>
__global__ void __launch_bounds__(kPatchBlock) k_patch_shared(int64_t ns, const int32_t* __restrict__ srp,
                                                              const int32_t* __restrict__ spos,
                                                              const int32_t* __restrict__ sdof, int64_t sbase,
                                                              const double* __restrict__ spart,
                                                              const double* __restrict__ dscale,
                                                              double* __restrict__ y, const double* __restrict__ dotv,
                                                              double* __restrict__ dotpart, int64_t pbase,
                                                              const int* __restrict__ active, CgArgs cg) {
  __shared__ double sh[3 * kPatchBlock];
  if (OUT != OUT_PLAIN && !cg.ic[I_ACTIVE]) return;   // uniform across the grid
  if (OUT == OUT_PLAIN && active && !active[0]) return;
  const double c1 = OUT == OUT_MASS_CG ? cg.sc[S_BETA]
                    : ((OUT == OUT_BRAS_CG || OUT == OUT_STAT) ? cg.sc[S_ALPHA] : 0.0);
  const double c2 = OUT == OUT_STAT ? cg.sc[S_BETA] : 0.0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  constexpr int U = kPatchSharedPerThread;
  for (int64_t s0 = (int64_t)blockIdx.x * kPatchSharedPerBlock + threadIdx.x; s0 < ns;
       s0 += (int64_t)gridDim.x * kPatchSharedPerBlock) {
    // U shared DOFs per thread, their loads issued together
    int32_t k0[U], k1[U], gd[U];
    double acc[U], ev[U][5], ds[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = s0 + (int64_t)u * kPatchBlock;
      const bool ok = s < ns;
      k0[u] = ok ? srp[s] : 0;
      k1[u] = ok ? srp[s + 1] : 0;
      gd[u] = ok ? (sdof ? sdof[s] : (int32_t)(sbase + s)) : 0;
    }
    // the vectors the epilogue reads, loaded beside the partials
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool ok = s0 + (int64_t)u * kPatchBlock < ns;
      ds[u] = (DS && ok) ? dscale[gd[u]] : 1.0;
      patch_epilogue_load<OUT>(ok, gd[u], cg, dotv, ev[u]);
    }
    // runs are short (the patches of one DOF): the first two partials of
    // every DOF are loaded together
    int32_t i0[U], i1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      i0[u] = k0[u] < k1[u] ? spos[k0[u]] : 0;
      i1[u] = k0[u] + 1 < k1[u] ? spos[k0[u] + 1] : 0;
    }
    double v0[U], v1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v0[u] = k0[u] < k1[u] ? spart[i0[u]] : 0.0;
      v1[u] = k0[u] + 1 < k1[u] ? spart[i1[u]] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double t = v0[u];
      if (k0[u] + 1 < k1[u]) t += v1[u];
      for (int32_t k = k0[u] + 2; k < k1[u]; ++k) t += spart[spos[k]];
      acc[u] = t;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t s = s0 + (int64_t)u * kPatchBlock;
      if (s >= ns) continue;
      double v = acc[u];
      if (DS) v *= ds[u];
      patch_epilogue_pre<OUT>(gd[u], v, c1, c2, cg, y, dotv != nullptr, ev[u], a0, a1, a2);
    }
  }
  patch_dots<OUT>(a0, a1, a2, pbase + blockIdx.x, OUT == OUT_PLAIN ? dotpart : cg.part0, cg, sh);
}

// Both kernels of one patch-form operator pass.
template <int NL, int FORM, int NSYM, typename T, int OUT, bool DS, int VAR>
int patch_launch(Ctx* c, const PatchCall& pc, const T* ap, const double* symtab, const double* coefK, int nsym,
                 const double* dscale, hipStream_t s) {
  // dscale: D^-1 (scaled H1 BRAS) in the caller's numbering; replaced below in internal mode
  const PatchDev& pt = c->pt;
  const bool ip = c->ip_mode != 0;   // vectors in the internal DOF numbering
  const int xcd_per = c->patch_xcd ? (int)((pt.npatch + 7) / 8) : 0;
  constexpr bool REUSE = !DS && (OUT == OUT_MASS_CG || OUT == OUT_BRAS_CG);
  PatchArgs pa{pt.pe, pt.pd, pt.pnl, ip ? pt.pidx : pt.pdof, pt.code, pt.sbase, c->E, pt.lbits, pt.maxrank,
               pt.npatch, xcd_per, ip ? 1 : 0, pt.maxdofs};
  if (ip && dscale) dscale = pt.invd_ip;
  // inputs and sums, or inputs (then sums) and the DOF numbers
  const int need = REUSE ? 2 * pt.maxdofs : pt.maxdofs + (pt.maxdofs + 1) / 2;
  const int words = need > 3 * kPatchBlock ? need : 3 * kPatchBlock;
  const unsigned grid = xcd_per > 0 ? (unsigned)(8 * xcd_per) : (unsigned)pt.npatch;
  k_patch<NL, FORM, NSYM, T, OUT, DS, VAR><<<grid, kPatchBlock, sizeof(double) * words, s>>>(
      pa, pc.in, ap, symtab, coefK, nsym, dscale, pc.y, pc.dotv, pc.dotpart, pc.cg, pc.spart);
  BRAS_HIP(hipGetLastError());
  if (pt.ns > 0) {
    k_patch_shared<OUT, DS><<<(unsigned)pt.nb2, kPatchBlock, 0, s>>>(
        pt.ns, pt.srp, pt.spos, ip ? nullptr : pt.sdof, pt.nloc_total, pc.spart, dscale, pc.y, pc.dotv, pc.dotpart,
        pt.npatch, pc.in.active, pc.cg);
    BRAS_HIP(hipGetLastError());
  }
  return BRAS_OK;
}

// n_loc of the per-lane forms: scaled H1 (Lagrange / Bernstein degree 1-4),
// the vector families up to n_loc 36
#define PATCH_SCALED_NL(X) X(3) X(4) X(6) X(10) X(15) X(20) X(35)
#define PATCH_VECTOR_NL(X) X(3) X(4) X(6) X(8) X(12) X(15) X(20) X(24) X(30) X(36)

// Per-form dispatchers (one translation unit each, patch_*.hip).
int patch_scaled(Ctx* c, const PatchCall& pc, hipStream_t s);
int patch_packed_f32(Ctx* c, const PatchCall& pc, hipStream_t s);
int patch_packed_f64(Ctx* c, const PatchCall& pc, hipStream_t s);
int patch_metric3(Ctx* c, const PatchCall& pc, hipStream_t s);
int patch_metric6(Ctx* c, const PatchCall& pc, hipStream_t s);

}  // namespace bras
