// Operator application: the BRAS inverse D^-1 P^T M_br^-1 P D^-1 (eqs.
// mhatinvbras_def, mass_and_bras_element_sums), the conforming mass
// M = P^T M_br P (eq. M_PMbrP), diag(M)^-1, and the density gradient.
//
// Every operator is two passes over device memory:
//   element pass  gathers each element's inputs (optionally an axpy of two
//                 vectors, times D^-1 for the H1 scaled form), multiplies by
//                 M_K or the folded inverse and writes the products to the
//                 broken vector zb[l][K][column] (local-index-major, so the 64
//                 lanes of a wavefront, one element each, store contiguously).
//                 Kernels: k_elem below (H1 scaled form), k_elem_lane
//                 (elem_lane.h: per-element matrices, n_loc <= 36),
//                 k_elem_mfma (elem_mfma.hip: n_loc > 36, FP64 matrix cores),
//                 k_bras_bf16 (bf16.hip: BF16 Gram factors on matrix cores);
//   reduce pass   sums each conforming DOF's broken copies in the fixed order
//                 of the transpose map (scaled by D^-1 for the H1 form) and
//                 either stores the result or runs the CG / stationary update
//                 that consumes it, writing per-block dot-product partials
//                 that a later kernel sums in block order (no floating-point
//                 atomics anywhere).
// Vectors with several columns are [n][R] (column fastest).
#include <cmath>

#include "internal.h"
#include "block_reduce.h"
#include "cg_common.h"
#include "elem_lane.h"

namespace bras {

constexpr int kBS = 256;                  // reduce / vector pass block size
constexpr int kEB = 256;                  // element pass block size
constexpr int kMaxVectorBlocks = 512;


// ---------------------------------------------------------------------------
// element pass, affine H1 (a shared reference matrix times one coefficient per
// element; eq. piola_mass_pullbacks).  Per-element matrices use the per-lane
// pass (elem_lane.h) or, for large n_loc, the matrix-core pass (elem_mfma.hip).
// ---------------------------------------------------------------------------
// A work-group owns 64 consecutive elements, one per lane.  Gather phase: all
// 256 threads read the 64 elements' map entries (contiguous) and the gathered
// input values into LDS, w[j][e] (row stride 65 to spread banks).  Product
// phase: wave v computes rows v, v+4, v+8, ... of all 64 elements, so every
// table entry it reads for a row is the same in all lanes (wave-uniform scalar
// loads) and every store of a row is 64 consecutive elements of the
// local-index-major broken vector zb[l][K] (column fastest).
//   z_l = coefK[K] sum_j A[l][j] w_j    (A shared; BRAS: A = Mhat^-1, coefK = 1/c_K,
//                                        and the input is scaled by dscale = D^-1)
constexpr int kEPB = 64;        // elements per work-group (one per lane)
constexpr int kWS = kEPB + 1;   // LDS row stride

// Up to n_loc 36 the register allocator is asked for 4 waves per SIMD (at
// most 128 VGPRs), which it meets without spilling (n_loc 35: 131 -> 123
// VGPRs, 3 -> 4 waves); larger n_loc keep their natural allocation.
template <int NL, bool DS>
__global__ void __launch_bounds__(kEB) __attribute__((amdgpu_waves_per_eu(NL <= 36 ? 4 : 1))) k_elem(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                              const double* __restrict__ dscale, const double* __restrict__ A,
                                              const double* __restrict__ coefK, double* __restrict__ zb) {
  typedef double T;
  constexpr int RPW = (NL + 3) / 4;   // rows per wave
  __shared__ T w[NL * kWS];
  __shared__ double coef_s[256];      // per-column coefficient of x2 (alpha or beta)
  __shared__ int act_s[256];          // per-column activity
  __shared__ double red_s[kEB];
  if (in.apart) {
    alpha_prologue(in.apart, in.anb, R, in.sc, in.ic, coef_s, act_s, red_s);
    for (int c = threadIdx.x; c < R; c += kEB) coef_s[c] *= in.sign;
    __syncthreads();
  } else {
    for (int c = threadIdx.x; c < R; c += kEB) {
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
  const int64_t K0 = (int64_t)blockIdx.x * kEPB;
  const int ne = (int)((E - K0) < kEPB ? (E - K0) : kEPB);
  const int64_t K = K0 + lane;
  const bool on = lane < ne;
  const double ck = on ? coefK[K] : 1.0;
  for (int col = 0; col < R; ++col) {
    if (!act_s[col]) continue;   // uniform
    const double cf = coef_s[col];
    {
      // all of this thread's map entries, then all gathers, then the LDS
      // stores; entries past the last element repeat its last map entry, so
      // no load needs a branch.  Without a second vector the first one is
      // read twice with weight 0.
      constexpr int GPT = (NL * kEPB + kEB - 1) / kEB;
      const int qmax = ne * NL - 1;
      int32_t gi[GPT];
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        const int q = tid + u * kEB;
        gi[u] = l2g[K0 * NL + (q < qmax ? q : qmax)];
      }
      const double* x2 = in.x2 ? in.x2 : in.x;
      const double c2 = in.x2 ? cf : 0.0;
      double v[GPT];
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        const int64_t g = (int64_t)gi[u] * R + col;
        double t = fma(c2, x2[g], in.x[g]);
        if (DS) t *= dscale[gi[u]];
        v[u] = t;
      }
#pragma unroll
      for (int u = 0; u < GPT; ++u) {
        const int q = tid + u * kEB;
        if (q < NL * kEPB) {   // only the last batch can pass the end (NL * 64 not a multiple of 256)
          const int e = q / NL, j = q - e * NL;
          w[j * kWS + e] = (T)v[u];
        }
      }
    }
    __syncthreads();
    if (on) {
      // rows past n_loc (last wave, n_loc not a multiple of 4) read row n_loc-1
      // and are not stored, so the product loops carry no branches
      int row[RPW];
#pragma unroll
      for (int k = 0; k < RPW; ++k) row[k] = (wv + 4 * k) < NL ? (wv + 4 * k) : NL - 1;
      T acc[RPW];
#pragma unroll
      for (int k = 0; k < RPW; ++k) acc[k] = (T)0;
#pragma unroll
      for (int j = 0; j < NL; ++j) {
        const T wj = w[j * kWS + lane];
#pragma unroll
        for (int k = 0; k < RPW; ++k) acc[k] = fma((T)A[row[k] * NL + j], wj, acc[k]);
      }
#pragma unroll
      for (int k = 0; k < RPW; ++k) {
        const int i = wv + 4 * k;
        if (i < NL) {
          T v = acc[k];
          v *= (T)ck;
          zb[((int64_t)i * E + K) * R + col] = v;
        }
      }
    }
    __syncthreads();
  }
}

// The same element pass on the FP64 matrix cores: per group of 64 elements
// Z = A W (W [n_loc][64] the gathered inputs in LDS, A the shared matrix,
// zero padded in LDS to 16-row tiles and 4-deep k steps), one 16-element
// column tile per wavefront on v_mfma_f64_16x16x4_f64, each column scaled by
// its element's coefficient on the way out.  Persistent: a work-group loads
// A once and strides over the element groups.
//   A[i][k]: lane l holds i = l%16, k = l/16;  B[k][j]: lane l holds j = l%16,
//   k = l/16;  D[i][j]: lane l, reg r holds j = l%16, i = l/16 + 4 r.
typedef double h1f64x4 __attribute__((ext_vector_type(4)));
template <int NL, bool DS>
__global__ void __launch_bounds__(kEB) k_elem_h1_mfma(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                                     const double* __restrict__ dscale,
                                                     const double* __restrict__ A,
                                                     const double* __restrict__ coefK, double* __restrict__ zb) {
  constexpr int MT = (NL + 15) / 16;
  constexpr int KS = (NL + 3) / 4;
  constexpr int LDA = 4 * KS + 1;
  __shared__ double sA[MT * 16 * LDA];
  __shared__ double w[NL * kWS];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  __shared__ double red_s[kEB];
  if (in.apart) {
    alpha_prologue(in.apart, in.anb, R, in.sc, in.ic, coef_s, act_s, red_s);
    for (int c = threadIdx.x; c < R; c += kEB) coef_s[c] *= in.sign;
    __syncthreads();
  } else {
    for (int c = threadIdx.x; c < R; c += kEB) {
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
  for (int t = tid; t < MT * 16 * LDA; t += kEB) {
    const int i = t / LDA, k = t - i * LDA;
    sA[t] = (i < NL && k < NL) ? A[i * NL + k] : 0.0;
  }
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int colq = lane & 15, kq = lane >> 4;
  const int64_t ngroups = (E + kEPB - 1) / kEPB;
  for (int64_t grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int64_t K0 = grp * kEPB;
    const int ne = (int)((E - K0) < kEPB ? (E - K0) : kEPB);
    const int e = 16 * wv + colq;
    const bool on = e < ne;
    const double ck = on ? coefK[K0 + e] : 0.0;
    for (int col = 0; col < R; ++col) {
      if (!act_s[col]) continue;   // uniform
      const double cf = coef_s[col];
      {
        // gather as in k_elem: map entries past the last element repeat its last entry
        constexpr int GPT = (NL * kEPB + kEB - 1) / kEB;
        const int qmax = ne * NL - 1;
        int32_t gi[GPT];
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const int q = tid + u * kEB;
          gi[u] = l2g[K0 * NL + (q < qmax ? q : qmax)];
        }
        const double* x2 = in.x2 ? in.x2 : in.x;
        const double c2 = in.x2 ? cf : 0.0;
        double v[GPT];
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const int64_t g = (int64_t)gi[u] * R + col;
          double t = fma(c2, x2[g], in.x[g]);
          if (DS) t *= dscale[gi[u]];
          v[u] = t;
        }
#pragma unroll
        for (int u = 0; u < GPT; ++u) {
          const int q = tid + u * kEB;
          if (q < NL * kEPB) {
            const int ee = q / NL, j = q - ee * NL;
            w[j * kWS + ee] = v[u];
          }
        }
      }
      __syncthreads();   // w (and, the first time, sA) complete
      h1f64x4 acc[MT];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = h1f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + kq;
        const double b = k < NL ? w[k * kWS + e] : 0.0;   // columns past ne hold stale values, never stored
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
          acc[mt] = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[(16 * mt + colq) * LDA + 4 * ks + kq], b, acc[mt], 0, 0, 0);
      }
      if (on) {
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * mt + kq + 4 * r;
            if (i < NL) zb[((int64_t)i * E + K0 + e) * R + col] = acc[mt][r] * ck;
          }
      }
      __syncthreads();   // before w is overwritten
    }
  }
}

// ---------------------------------------------------------------------------
// reduce pass, optionally fused with a CG update
// ---------------------------------------------------------------------------
// y_i = scale_i * sum of DOF i's broken copies, in the fixed order of the
// transpose map.  Work is cut into row chunks of at most kChunkRows
// consecutive conforming DOFs and kChunkCap copies; a grid of at most
// kMaxReduceBlocks work-groups strides over the chunks, so the per-block dot
// product partials stay few.  The fused epilogues:
//   OUT_MASS_CG  p_new = z + beta p (the element pass used the same p_new),
//                q = M p_new, partial p_new.q
//   OUT_BRAS_CG  r_new = r - alpha q, x += alpha p, z = C r_new, partials
//                r_new.r_new, r_new.z and (flexible) r_new.z_old
//   OUT_RES      r = b - M x, partial r.r           (stationary iterations)
//   OUT_STAT     d = a d + c C r, x += d            (a = sc[S_ALPHA], c = sc[S_BETA])
constexpr int kChunkRows = 512;
constexpr int kChunkCap = 2048;
constexpr int kRowsPerThread = kChunkRows / kBS;
constexpr int kMaxReduceBlocks = 2048;    // several columns
constexpr int kMaxReduceBlocks1 = 16384;  // one column

// CG epilogue of one output entry t (column col, sum acc); accumulates dots
template <int OUT>
__device__ __forceinline__ void reduce_epilogue(int64_t t, double acc, double coef, double coef2, const CgArgs& cg,
                                                double* y, const double* dotv, double& d0, double& d1,
                                                double& d2) {
  if (OUT == OUT_RES) {
    const double rv = cg.b[t] - acc;
    cg.r[t] = rv;
    d0 = fma(rv, rv, d0);
  } else if (OUT == OUT_STAT) {
    const double dn = fma(coef, cg.p[t], coef2 * acc);
    cg.p[t] = dn;
    cg.x[t] += dn;
  } else if (OUT == OUT_PLAIN) {
    y[t] = acc;
    if (dotv) d0 = fma(acc, dotv[t], d0);
  } else if (OUT == OUT_MASS_CG) {
    const double pn = fma(coef, cg.p[t], cg.z[t]);
    cg.p[t] = pn;
    cg.q[t] = acc;
    d0 = fma(pn, acc, d0);
  } else {
    const double rn = fma(-coef, cg.q[t], cg.r[t]);
    cg.x[t] = fma(coef, cg.p[t], cg.x[t]);
    if (cg.flexible) d2 = fma(rn, cg.z[t], d2);
    cg.z[t] = acc;
    cg.r[t] = rn;
    d0 = fma(rn, rn, d0);
    d1 = fma(rn, acc, d1);
  }
}

// One column: all threads load a chunk's broken values into LDS (independent
// loads, so long rows do not serialise), then each thread sums its rows.  The
// row bounds and the vectors the epilogue reads are loaded together with the
// chunk's slots, so a chunk costs two dependent memory round trips.
// skip1: rows with a single broken copy are left to the element pass (which
// then ran their epilogue itself).
template <typename ZT, int OUT>
__global__ void __launch_bounds__(kBS) k_reduce(int nchunk, const int32_t* __restrict__ chunk,
                                                const int32_t* __restrict__ rowptr,
                                                const int32_t* __restrict__ slot, const ZT* __restrict__ zb,
                                                const double* __restrict__ scale, double* __restrict__ y,
                                                const double* __restrict__ dotv, double* __restrict__ partial,
                                                CgArgs cg, int skip1) {
  __shared__ double vals[kChunkCap];
  __shared__ double sh0[kBS], sh1[kBS], sh2[kBS];
  if (OUT != OUT_PLAIN && !cg.ic[I_ACTIVE]) return;   // uniform across the grid
  const double coef = OUT == OUT_MASS_CG ? cg.sc[S_BETA]
                      : ((OUT == OUT_BRAS_CG || OUT == OUT_STAT) ? cg.sc[S_ALPHA] : 0.0);
  const double coef2 = OUT == OUT_STAT ? cg.sc[S_BETA] : 0.0;
  const int tid = threadIdx.x;
  constexpr int LPT = kChunkCap / kBS;   // copies per thread
  constexpr int NV = (OUT == OUT_PLAIN || OUT == OUT_MASS_CG) ? 2 : (OUT == OUT_RES ? 1 : (OUT == OUT_STAT ? 3 : 6));
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int32_t i0 = chunk[ch], i1 = chunk[ch + 1];
    const int32_t p0 = rowptr[i0];
    const int cnt = rowptr[i1] - p0;
    const bool big = cnt > kChunkCap;   // a single row longer than the chunk capacity
    int32_t sv[LPT];
    if (!big) {
#pragma unroll
      for (int u = 0; u < LPT; ++u) {
        const int t = tid + u * kBS;
        sv[u] = t < cnt ? __builtin_nontemporal_load(&slot[p0 + t]) : 0;   // streamed once per pass
      }
    }
    int32_t ra[kRowsPerThread], rb[kRowsPerThread];
    double pre[kRowsPerThread][NV];
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const int32_t i = i0 + tid + k * kBS;
      const bool own = i < i1;
      const int32_t ic = own ? i : i0;
      ra[k] = own ? rowptr[ic] - p0 : 0;
      rb[k] = own ? rowptr[ic + 1] - p0 : 0;
      if (OUT == OUT_RES) {
        pre[k][0] = cg.b[ic];
      } else if (OUT == OUT_STAT) {
        pre[k][0] = scale ? scale[ic] : 1.0;
        pre[k][1] = cg.p[ic];
        pre[k][2] = cg.x[ic];
      } else if (OUT == OUT_PLAIN) {
        pre[k][0] = scale ? scale[ic] : 1.0;
        pre[k][1] = dotv ? dotv[ic] : 0.0;
      } else if (OUT == OUT_MASS_CG) {
        pre[k][0] = cg.z[ic];
        pre[k][1] = cg.p[ic];
      } else {
        // q, r, x and the old z are not read again before this pass rewrites
        // them: non-temporal, so p, z and the new r stay in the caches
        pre[k][0] = scale ? scale[ic] : 1.0;
        pre[k][1] = __builtin_nontemporal_load(&cg.q[ic]);
        pre[k][2] = __builtin_nontemporal_load(&cg.r[ic]);
        pre[k][3] = __builtin_nontemporal_load(&cg.x[ic]);
        pre[k][4] = cg.p[ic];
        pre[k][5] = cg.flexible ? __builtin_nontemporal_load(&cg.z[ic]) : 0.0;
      }
    }
    if (!big) {
      double vv[LPT];
#pragma unroll
      for (int u = 0; u < LPT; ++u) {
        const int t = tid + u * kBS;
        vv[u] = t < cnt ? (double)zb[sv[u]] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < LPT; ++u) {
        const int t = tid + u * kBS;
        if (t < cnt) vals[t] = vv[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRowsPerThread; ++k) {
      const int32_t i = i0 + tid + k * kBS;
      if (i >= i1) continue;
      if (skip1 && rb[k] - ra[k] == 1) continue;
      double acc = 0.0;
      if (!big)
        for (int32_t q = ra[k]; q < rb[k]; ++q) acc += vals[q];
      else
        for (int32_t q = ra[k]; q < rb[k]; ++q) acc += (double)zb[slot[p0 + q]];
      if (OUT == OUT_RES) {
        const double rv = pre[k][0] - acc;
        cg.r[i] = rv;
        d0 = fma(rv, rv, d0);
      } else if (OUT == OUT_STAT) {
        acc *= pre[k][0];
        const double dn = fma(coef, pre[k][1], coef2 * acc);
        cg.p[i] = dn;
        cg.x[i] = pre[k][2] + dn;
      } else if (OUT == OUT_PLAIN) {
        acc *= pre[k][0];
        y[i] = acc;
        d0 = fma(acc, pre[k][1], d0);
      } else if (OUT == OUT_MASS_CG) {
        const double pn = fma(coef, pre[k][1], pre[k][0]);
        cg.p[i] = pn;
        cg.q[i] = acc;
        d0 = fma(pn, acc, d0);
      } else {
        acc *= pre[k][0];
        const double rn = fma(-coef, pre[k][1], pre[k][2]);
        __builtin_nontemporal_store(fma(coef, pre[k][4], pre[k][3]), &cg.x[i]);
        d2 = fma(rn, pre[k][5], d2);
        cg.z[i] = acc;
        cg.r[i] = rn;
        d0 = fma(rn, rn, d0);
        d1 = fma(rn, acc, d1);
      }
    }
    __syncthreads();
  }
  // partials of this block (fixed tree order)
  double* out0 = OUT == OUT_PLAIN ? partial : cg.part0;
  if (OUT == OUT_STAT) return;
  if (OUT == OUT_PLAIN && !(dotv && partial)) return;
  sh0[tid] = d0;
  if (OUT == OUT_BRAS_CG) {
    sh1[tid] = d1;
    sh2[tid] = d2;
  }
  __syncthreads();
  for (int off = kBS / 2; off > 0; off >>= 1) {
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
    out0[blockIdx.x] = sh0[0];
    if (OUT == OUT_BRAS_CG) {
      cg.part1[blockIdx.x] = sh1[0];
      if (cg.flexible) cg.part2[blockIdx.x] = sh2[0];
    }
  }
}

// Several columns (R >= 2): thread t owns column t % R of rows t / R,
// t / R + 256 / R, ... of each chunk, so consecutive threads read the
// consecutive columns of one broken copy; a row's copies are summed in
// transpose-map order as in the one-column pass.
template <typename ZT, int OUT>
__global__ void __launch_bounds__(kBS) k_reduce_mc(int R, int nchunk, const int32_t* __restrict__ chunk,
                                                   const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ slot, const ZT* __restrict__ zb,
                                                   const double* __restrict__ scale, double* __restrict__ y,
                                                   const double* __restrict__ dotv, double* __restrict__ partial,
                                                   CgArgs cg, int skip1) {
  __shared__ int32_t sl[kChunkCap];
  __shared__ int32_t rp[kChunkRows + 1];
  __shared__ double sh[kBS];
  __shared__ double coef_s[256], coef2_s[256];
  __shared__ int act_s[256];
  const int tid = threadIdx.x;
  for (int c = tid; c < R; c += kBS) {
    act_s[c] = OUT == OUT_PLAIN ? 1 : cg.ic[I_ACTIVE * R + c];
    coef_s[c] = OUT == OUT_MASS_CG ? cg.sc[S_BETA * R + c]
                : ((OUT == OUT_BRAS_CG || OUT == OUT_STAT) ? cg.sc[S_ALPHA * R + c] : 0.0);
    coef2_s[c] = OUT == OUT_STAT ? cg.sc[S_BETA * R + c] : 0.0;
  }
  __syncthreads();
  {
    bool any = false;
    for (int c = 0; c < R; ++c) any = any || act_s[c];
    if (!any) return;   // uniform across the grid
  }
  const int G = kBS / R;          // rows per pass (R <= 256)
  const bool mine = tid < G * R;
  const int col = mine ? tid % R : 0, g = tid / R;
  const bool act = mine && act_s[col];
  const double coef = coef_s[col], coef2 = coef2_s[col];
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  for (int ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int32_t i0 = chunk[ch], i1 = chunk[ch + 1];
    const int nr = i1 - i0;
    const int32_t p0 = rowptr[i0];
    const int cnt = rowptr[i1] - p0;
    const bool big = cnt > kChunkCap;
    if (!big)
      for (int t = tid; t < cnt; t += kBS) sl[t] = __builtin_nontemporal_load(&slot[p0 + t]);
    for (int t = tid; t <= nr; t += kBS) rp[t] = rowptr[i0 + t] - p0;
    __syncthreads();
    if (act) {
      for (int r = g; r < nr; r += G) {
        const int a = rp[r], b = rp[r + 1];
        if (skip1 && b - a == 1) continue;
        double acc = 0.0;
        int q = a;
        for (; q + 4 <= b; q += 4) {
          double v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int64_t s = big ? slot[p0 + q + u] : sl[q + u];
            v[u] = (double)zb[s * R + col];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc += v[u];
        }
        for (; q < b; ++q) {
          const int64_t s = big ? slot[p0 + q] : sl[q];
          acc += (double)zb[s * R + col];
        }
        const int64_t i = i0 + r;
        if (scale) acc *= scale[i];
        reduce_epilogue<OUT>(i * R + col, acc, coef, coef2, cg, y, dotv, d0, d1, d2);
      }
    }
    __syncthreads();
  }
  // per-column partials: thread c adds the row groups' sums in order
  double* out0 = OUT == OUT_PLAIN ? partial : cg.part0;
  if (OUT == OUT_STAT) return;
  if (OUT == OUT_PLAIN && !(dotv && partial)) return;
  double* outs[3] = {out0, cg.part1, cg.part2};
  const double ds[3] = {d0, d1, d2};
  const int nd = OUT == OUT_BRAS_CG ? (cg.flexible ? 3 : 2) : 1;
  for (int k = 0; k < nd; ++k) {
    sh[tid] = ds[k];
    __syncthreads();
    if (tid < R) {
      double v = 0.0;
      for (int gg = 0; gg < G; ++gg) v += sh[gg * R + tid];
      outs[k][(int64_t)blockIdx.x * R + tid] = v;
    }
    __syncthreads();
  }
}

// Diagonal (or identity) preconditioner fused with the CG update:
// alpha from the p.q partials, r_new = r - alpha q, x += alpha p,
// z = s .* r_new (s = diag(M)^-1, or 1), partials of r.r, r.z (and r.z_old).
__global__ void __launch_bounds__(kBS) k_diag_cg(int64_t n, int R, const double* __restrict__ s, CgArgs cg) {
  __shared__ double sh0[kBS], sh1[kBS], sh2[kBS];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  if (cg.apart) {
    alpha_prologue(cg.apart, cg.anb, R, cg.sc, cg.ic, coef_s, act_s, sh0);
  } else {
    for (int c = threadIdx.x; c < R; c += kBS) {
      act_s[c] = cg.ic[I_ACTIVE * R + c];
      coef_s[c] = cg.sc[S_ALPHA * R + c];
    }
    __syncthreads();
  }
  {
    bool any = false;
    for (int c = 0; c < R; ++c) any = any || act_s[c];
    if (!any) return;
  }
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;   // a multiple of R
  const int col = (int)(t0 % R);
  double d0 = 0.0, d1 = 0.0, d2 = 0.0;
  if (act_s[col]) {
    const double alpha = coef_s[col];
    for (int64_t t = t0; t < n * R; t += stride) {
      const int64_t i = R == 1 ? t : t / R;
      const double rn = fma(-alpha, cg.q[t], cg.r[t]);
      cg.x[t] = fma(alpha, cg.p[t], cg.x[t]);
      const double zv = s ? rn * s[i] : rn;
      if (cg.flexible) d2 = fma(rn, cg.z[t], d2);
      cg.z[t] = zv;
      cg.r[t] = rn;
      d0 = fma(rn, rn, d0);
      d1 = fma(rn, zv, d1);
    }
  }
  sh0[threadIdx.x] = d0;
  block_partials(sh0, R, cg.part0);
  sh1[threadIdx.x] = d1;
  block_partials(sh1, R, cg.part1);
  if (cg.flexible) {
    sh2[threadIdx.x] = d2;
    block_partials(sh2, R, cg.part2);
  }
}

// Stationary update with the diagonal preconditioner: d = a d + c (r ./ diag),
// x += d, for running columns (a = sc[S_ALPHA], c = sc[S_BETA]).
__global__ void __launch_bounds__(kBS) k_diag_st(int64_t n, int R, const double* __restrict__ s, CgArgs cg) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;   // a multiple of R
  const int col = (int)(t0 % R);
  if (!cg.ic[I_ACTIVE * R + col]) return;
  const double a = cg.sc[S_ALPHA * R + col], c = cg.sc[S_BETA * R + col];
  for (int64_t t = t0; t < n * R; t += stride) {
    const int64_t i = R == 1 ? t : t / R;
    const double dn = fma(a, cg.p[t], c * (cg.r[t] * s[i]));
    cg.p[t] = dn;
    cg.x[t] += dn;
  }
}

// y = s .* x with optional fused dot product y . dotv (plain Jacobi apply)
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
      const double v = x[t] * s[R == 1 ? t : t / R];
      y[t] = v;
      if (dotv) dot = fma(v, dotv[t], dot);
    }
  }
  if (!partial) return;
  sh[threadIdx.x] = dot;
  block_partials(sh, R, partial);
}

// g_K = -dcoef_K sum_r lam_K,r^T Mhat x_K,r  (density gradient, affine H1),
// one thread per element row, row sums reduced in LDS per element.
template <int NL>
__global__ void __launch_bounds__(kEB) k_rho_grad(int64_t E, int R, const int32_t* __restrict__ l2g,
                                                  const double* __restrict__ x, const double* __restrict__ lam,
                                                  const double* __restrict__ Mhat, const double* __restrict__ dcoef,
                                                  const int32_t* __restrict__ perm, double* __restrict__ g) {
  constexpr int EPB = kEB / NL;
  __shared__ double w[kEB];
  __shared__ double part[kEB];
  const int tid = threadIdx.x;
  const int e = tid / NL, l = tid - e * NL;
  const bool lane = e < EPB;
  double a[NL];
  if (lane) {
#pragma unroll
    for (int j = 0; j < NL; ++j) a[j] = Mhat[l * NL + j];
  }
  for (int64_t K0 = (int64_t)blockIdx.x * EPB; K0 < E; K0 += (int64_t)gridDim.x * EPB) {
    const int64_t K = K0 + e;
    const bool on = lane && K < E;
    const int32_t gi = on ? l2g[K * NL + l] : 0;
    double tot = 0.0;
    for (int r = 0; r < R; ++r) {
      if (on) w[tid] = x[(int64_t)gi * R + r];
      __syncthreads();
      if (on) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NL; ++j) acc = fma(a[j], w[e * NL + j], acc);
        tot = fma(lam[(int64_t)gi * R + r], acc, tot);
      }
      __syncthreads();
    }
    part[tid] = on ? tot : 0.0;
    __syncthreads();
    if (on && l == 0) {
      double s = 0.0;
      for (int j = 0; j < NL; ++j) s += part[e * NL + j];
      const int64_t Ku = perm ? perm[K] : K;   // the caller's element number
      g[Ku] = -dcoef[Ku] * s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int vector_blocks(Ctx* c, int R) {
  int64_t want = (c->n * R + kBS - 1) / kBS;
  int64_t nb = want < kMaxVectorBlocks ? want : kMaxVectorBlocks;
  if (nb < 1) nb = 1;
  // grid * kBS must be a multiple of R so that each thread keeps one column
  while (((int64_t)nb * kBS) % R) ++nb;
  return (int)nb;
}

#define NL_CASES(X) X(3) X(4) X(6) X(8) X(10) X(15) X(20) X(21) X(24) X(28) X(35) X(36) X(45) X(56) X(70) X(84)

// Scaled H1 element pass: variant 0 on the FP64 matrix cores (persistent,
// a few work-groups per compute unit), variant 1 the per-row FMA pass.
int scaled_variant(const Ctx* c) { return (c->variant == 0 || c->variant == 1) ? c->variant : 0; }

template <int NL>
static int elem_launch(Ctx* c, int R, const InArgs& in, const double* dscale, const double* A, const double* coefK,
                       double* zb, hipStream_t s) {
  const unsigned nb = (unsigned)((c->E + kEPB - 1) / kEPB);
  if (scaled_variant(c) == 0) {
    static int per_cu = 0;   // resident work-groups per compute unit (one grid of them strides over the groups)
    if (per_cu == 0) {
      int v = 0;
      BRAS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, k_elem_h1_mfma<NL, true>, kEB, 0));
      per_cu = v > 0 ? v : 1;
    }
    const unsigned cap = (unsigned)(c->ncu * per_cu);
    const unsigned g = nb < cap ? nb : cap;
    if (dscale)
      k_elem_h1_mfma<NL, true><<<g, kEB, 0, s>>>(c->E, R, c->l2g, in, dscale, A, coefK, zb);
    else
      k_elem_h1_mfma<NL, false><<<g, kEB, 0, s>>>(c->E, R, c->l2g, in, dscale, A, coefK, zb);
    BRAS_HIP(hipGetLastError());
    return BRAS_OK;
  }
  if (dscale)
    k_elem<NL, true><<<nb, kEB, 0, s>>>(c->E, R, c->l2g, in, dscale, A, coefK, zb);
  else
    k_elem<NL, false><<<nb, kEB, 0, s>>>(c->E, R, c->l2g, in, dscale, A, coefK, zb);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int scaled_dispatch(Ctx* c, int R, const InArgs& in, const double* dscale, const double* A,
                           const double* coefK, double* zb, hipStream_t s) {
#define CASE(N) \
  case N: return elem_launch<N>(c, R, in, dscale, A, coefK, zb, s);
  switch (c->nl) {
    NL_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no element kernel", c->nl);
  }
#undef CASE
}

// Scheduling variant of the 3D metric-form mass pass: the one set by the
// autotuner or an option, else diagonal order for n_loc 20 (fastest when timed
// on the 48^3 N1curl2 map) and row order otherwise.
int metric_variant(const Ctx* c) {
  if (c->variant >= 0 && c->variant < kMetricVariants) return c->variant;
  return c->nl == 20 ? 2 : 0;
}

// element pass of the mass operator (float64)
static int mass_elem(Ctx* c, const InArgs& in, int R, hipStream_t s) {
  double* zb = (double*)c->zb;
  if (c->form == BRAS_ELEM_SCALED_REF)
    return scaled_dispatch(c, R, in, nullptr, c->ref, c->coef, zb, s);
  if (c->mpack) {
    if (c->nl <= kLaneMaxNL) return lane_packed_f64(c, R, in, c->mpack, zb, s);
    return mfma_elem_f64(c, R, in, c->mpack, zb, s);
  }
  // metric tables (setup keeps them only for n_loc <= kLaneMaxNL)
  if (c->nsym <= 3) return lane_metric3(c, R, in, zb, s);
  switch (metric_variant(c)) {
    case 1: return lane_metric6_v1(c, R, in, zb, s);
    case 2: return lane_metric6_v2(c, R, in, zb, s);
    default: return lane_metric6_v0(c, R, in, zb, s);
  }
}

// element pass of the BRAS operator into the broken vector zb (the handle's
// own, or a caller-provided workspace of the same size); reports whether the
// broken vector is float32
static int bras_elem(Ctx* c, const InArgs& in, int R, hipStream_t s, bool* zb_float, void* zb) {
  *zb_float = false;
  if (c->form == BRAS_ELEM_SCALED_REF)
    return scaled_dispatch(c, R, in, c->invd, c->refinv, c->icoef, (double*)zb, s);
  const bool lane = c->nl <= kLaneMaxNL;
  if (c->prec == BRAS_FP64) {
    if (lane) return lane_packed_f64(c, R, in, (const double*)c->ainv, (double*)zb, s);
    return mfma_elem_f64(c, R, in, (const double*)c->ainv, (double*)zb, s);
  }
  *zb_float = true;
  if (lane) return lane_packed_f32(c, R, in, (const float*)c->ainv, (float*)zb, s);
  return mfma_elem_f32(c, R, in, (const float*)c->ainv, (float*)zb, s);
}

template <typename ZT, int OUT>
static int reduce_launch(Ctx* c, const ZT* zb, const double* scale, double* y, int R, hipStream_t s,
                         const double* dotv, double* partial, const CgArgs& cg, int skip1 = 0) {
  const unsigned nb = (unsigned)reduce_chunk_blocks(c, R);
  if (R == 1)
    k_reduce<ZT, OUT><<<nb, kBS, 0, s>>>((int)c->nchunk, c->chunk, c->rowptr, c->slot, zb, scale, y, dotv, partial,
                                         cg, skip1);
  else
    k_reduce_mc<ZT, OUT><<<nb, kBS, 0, s>>>(R, (int)c->nchunk, c->chunk, c->rowptr, c->slot, zb, scale, y, dotv,
                                            partial, cg, skip1);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// Work-groups of the transpose-map reduce: one column: one per chunk up to a
// large cap (latency hiding); several columns: fewer, longer-lived work-groups
// and fewer partials.
int reduce_chunk_blocks(const Ctx* c, int R) {
  const int64_t cap = R == 1 ? kMaxReduceBlocks1 : kMaxReduceBlocks;
  return (int)(c->nchunk < cap ? c->nchunk : cap);
}

int reduce_blocks(Ctx* c, int R) {
  if (patch_active(c, R)) return patch_blocks(c);   // patch pass: one partial per work-group of its two kernels
  return reduce_chunk_blocks(c, R);
}

int reduce_float_plain(Ctx* c, const float* zb, double* y, int R, hipStream_t s, const double* dotv,
                       double* dotpart, int skip1) {
  return reduce_launch<float, OUT_PLAIN>(c, zb, nullptr, y, R, s, dotv, dotpart, CgArgs(), skip1);
}

int reduce_float_cg(Ctx* c, const float* zb, int R, hipStream_t s, const CgArgs& cg) {
  return reduce_launch<float, OUT_BRAS_CG>(c, zb, nullptr, nullptr, R, s, nullptr, nullptr, cg);
}

int reduce_float_stat(Ctx* c, const float* zb, int R, hipStream_t s, const CgArgs& cg) {
  return reduce_launch<float, OUT_STAT>(c, zb, nullptr, nullptr, R, s, nullptr, nullptr, cg);
}

int launch_mass(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                const int* active) {
  InArgs in;
  in.x = x;
  in.active = active;
  if (patch_active(c, R)) return patch_pass(c, 0, OUT_PLAIN, in, y, dotv, dotpart, CgArgs(), s);
  int st = mass_elem(c, in, R, s);
  if (st) return st;
  return reduce_launch<double, OUT_PLAIN>(c, (const double*)c->zb, nullptr, y, R, s, dotv, dotpart, CgArgs());
}

size_t broken_bytes(const Ctx* c, int R) {
  if (patch_active(c, R)) return patch_workspace_bytes(c);
  const size_t esz = (c->form != BRAS_ELEM_SCALED_REF && c->prec != BRAS_FP64) ? sizeof(float) : sizeof(double);
  return esz * (size_t)c->nbr * (size_t)R;
}

int launch_bras(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                const int* active, void* ws) {
  void* zb = ws ? ws : c->zb;
  if (c->prec == BRAS_BF16) return launch_bras_bf16(c, x, y, R, s, dotv, dotpart, active, zb);
  InArgs in;
  in.x = x;
  in.active = active;
  if (patch_active(c, R)) return patch_pass(c, 1, OUT_PLAIN, in, y, dotv, dotpart, CgArgs(), s, (double*)ws);
  bool zf;
  int st = bras_elem(c, in, R, s, &zf, zb);
  if (st) return st;
  const double* scale = c->form == BRAS_ELEM_SCALED_REF ? c->invd : nullptr;
  if (zf) return reduce_launch<float, OUT_PLAIN>(c, (const float*)zb, scale, y, R, s, dotv, dotpart, CgArgs());
  return reduce_launch<double, OUT_PLAIN>(c, (const double*)zb, scale, y, R, s, dotv, dotpart, CgArgs());
}

int launch_jacobi(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                  const int* active) {
  k_diag_scale<<<vector_blocks(c, R), kBS, 0, s>>>(c->n, R, c->ip_mode ? c->pt.invdiag_ip : c->invdiag, x, y, dotv,
                                                   dotpart, active);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// Element-pass input r - alpha q of the preconditioner step: alpha either
// from the p.q partials in the pass's own prologue (cg.apart set) or as
// already stored in sc by a one-block kernel.
InArgs precond_input(const CgArgs& cg, int R) {
  InArgs in;
  in.x = cg.r;
  in.x2 = cg.q;
  in.sign = -1.0;
  if (cg.apart) {
    in.apart = cg.apart;
    in.anb = cg.anb;
    in.sc = cg.sc;
    in.ic = cg.ic;
  } else {
    in.cvec = cg.sc + S_ALPHA * R;
    in.active = cg.ic + I_ACTIVE * R;
  }
  return in;
}

// Work-groups of the pass that consumes alpha (each one would sum the p.q
// partials in its prologue).
int precond_consumer_blocks(Ctx* c, int pc, int R) {
  if (pc == BRAS_PC_BRAS && patch_active(c, R)) return (int)c->pt.npatch;
  if (pc == BRAS_PC_BRAS) return c->prec == BRAS_BF16 ? c->bf16_grid_x2 : (int)((c->E + kEPB - 1) / kEPB);
  return vector_blocks(c, R);
}

// q = M (z + beta p), p <- z + beta p, alpha = rho / p.q
int cg_mass_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  InArgs in;
  in.x = cg.z;
  in.x2 = cg.p;
  in.cvec = cg.sc + S_BETA * R;
  in.sign = 1.0;
  in.active = cg.ic + I_ACTIVE * R;
  if (patch_active(c, R)) return patch_pass(c, 0, OUT_MASS_CG, in, nullptr, nullptr, nullptr, cg, s);
  int st = mass_elem(c, in, R, s);
  if (st) return st;
  return reduce_launch<double, OUT_MASS_CG>(c, (const double*)c->zb, nullptr, nullptr, R, s, nullptr, nullptr, cg);
}

// r <- r - alpha q, x <- x + alpha p, z = C r, dot products, convergence, beta
int cg_precond_step(Ctx* c, int pc, const CgArgs& cg, int R, hipStream_t s) {
  if (pc == BRAS_PC_BRAS && c->prec != BRAS_BF16) {
    InArgs in = precond_input(cg, R);
    if (patch_active(c, R)) return patch_pass(c, 1, OUT_BRAS_CG, in, nullptr, nullptr, nullptr, cg, s);
    bool zf;
    int st = bras_elem(c, in, R, s, &zf, c->zb);
    if (st) return st;
    const double* scale = c->form == BRAS_ELEM_SCALED_REF ? c->invd : nullptr;
    if (zf)
      return reduce_launch<float, OUT_BRAS_CG>(c, (const float*)c->zb, scale, nullptr, R, s, nullptr, nullptr, cg);
    return reduce_launch<double, OUT_BRAS_CG>(c, (const double*)c->zb, scale, nullptr, R, s, nullptr, nullptr, cg);
  }
  if (pc == BRAS_PC_BRAS) return cg_bras_bf16_step(c, cg, R, s);
  const double* invdiag = c->ip_mode ? c->pt.invdiag_ip : c->invdiag;
  k_diag_cg<<<vector_blocks(c, R), kBS, 0, s>>>(c->n, R, pc == BRAS_PC_JACOBI ? invdiag : nullptr, cg);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

// Stationary iterations: r = b - M x with partial r.r
int st_mass_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  InArgs in;
  in.x = cg.x;
  in.active = cg.ic + I_ACTIVE * R;
  if (patch_active(c, R)) return patch_pass(c, 0, OUT_RES, in, nullptr, nullptr, nullptr, cg, s);
  int st = mass_elem(c, in, R, s);
  if (st) return st;
  return reduce_launch<double, OUT_RES>(c, (const double*)c->zb, nullptr, nullptr, R, s, nullptr, nullptr, cg);
}

// Stationary iterations: d = a d + c C r, x += d (pc: BRAS_PC_BRAS or BRAS_PC_JACOBI)
int st_precond_step(Ctx* c, int pc, const CgArgs& cg, int R, hipStream_t s) {
  if (pc == BRAS_PC_JACOBI) {
    k_diag_st<<<vector_blocks(c, R), kBS, 0, s>>>(c->n, R, c->ip_mode ? c->pt.invdiag_ip : c->invdiag, cg);
    BRAS_HIP(hipGetLastError());
    return BRAS_OK;
  }
  InArgs in;
  in.x = cg.r;
  in.active = cg.ic + I_ACTIVE * R;
  if (c->prec == BRAS_BF16) return bf16_stat_step(c, cg, in, R, s);
  if (patch_active(c, R)) return patch_pass(c, 1, OUT_STAT, in, nullptr, nullptr, nullptr, cg, s);
  bool zf;
  int st = bras_elem(c, in, R, s, &zf, c->zb);
  if (st) return st;
  const double* scale = c->form == BRAS_ELEM_SCALED_REF ? c->invd : nullptr;
  if (zf) return reduce_launch<float, OUT_STAT>(c, (const float*)c->zb, scale, nullptr, R, s, nullptr, nullptr, cg);
  return reduce_launch<double, OUT_STAT>(c, (const double*)c->zb, scale, nullptr, R, s, nullptr, nullptr, cg);
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
#define CASE(N)                                                                                          \
  case N: {                                                                                              \
    constexpr int EPB = kEB / N;                                                                         \
    const int64_t groups = (c->E + EPB - 1) / EPB;                                                      \
    const unsigned nb = (unsigned)(groups < 65536 ? groups : 65536);                                     \
    k_rho_grad<N><<<nb, kEB, 0, s>>>(c->E, nrhs, c->l2g, x_d, lam_d, c->ref, dcoef_d, c->pt.perm, g_d); \
    break;                                                                                               \
  }
  switch (c->nl) {
    NL_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no gradient kernel", c->nl);
  }
#undef CASE
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}
