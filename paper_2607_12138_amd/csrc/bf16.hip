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
// One work-group (4 wavefronts) per element at a time: Gtil is unpacked into
// a zero-padded LDS tile [MP][LD] (MP = 32 * ceil(n_loc/32) rows, KP = 16 *
// ceil(n_loc/16) used columns, LD = KP + 8), W^T and U^T are [32][LD].  Wave
// t computes the 32-row output tile t of each product.  MFMA operand layout
// (32x32x16):
//   A[i][k]: lane l holds i = l%32, k = 8*(l/32) + e, e = 0..7
//   B[k][j]: lane l holds j = l%32, k = 8*(l/32) + e
//   D[i][j]: lane l, reg r holds j = l%32, i = 8*(r/4) + 4*(l/32) + r%4
// The broken output (FP32) goes to zb[l][K][R] like the other element passes.
#include <cmath>
#include <cstdlib>

#include "internal.h"
#include "cg_common.h"
#include "bf16_gram.h"

namespace bras {



// Persistent: the grid (a multiple of 8) splits the elements into 8
// contiguous ranges, one per XCD (work-group g runs on XCD g % 8), so that
// neighbouring elements, which share face DOFs, are gathered through the
// same L2; work-group g takes elements Kbeg + g/8, Kbeg + g/8 + G/8, ... of
// its range.  While the matrix cores work on element K the registers hold the
// loads of the next element (its factor and first 32 gathered columns) and
// the map of the one after.
// One LDS tile holds Gtil (rows padded to LD = KP + 8 bf16, so that 16-byte
// row reads of 8 consecutive rows hit distinct banks); the second product
// reads it transposed, one 2-byte element per lane and k.
// DIRECT (plain applies of at most 32 columns): map holds the DOF numbers
// with bit 31 set where the DOF has a single broken copy (e.g. the
// cell-interior DOFs of H(div) elements); those rows skip the broken vector
// and are written to y here, and the reduce then skips them.
template <int NL, bool DIRECT, bool X2>
__global__ void __launch_bounds__(kB16) __attribute__((amdgpu_waves_per_eu(NL <= 36 ? 3 : (NL <= 70 ? 2 : 1))))
k_bras_bf16(int64_t E, int R, const int32_t* __restrict__ map, InArgs in, const __bf16* __restrict__ G,
            float* __restrict__ zb, double* __restrict__ y) {
  constexpr int MT = Bf16Shape<NL>::MT;
  constexpr int KP = Bf16Shape<NL>::KP;
  constexpr int MP = Bf16Shape<NL>::MP;
  constexpr int LD = Bf16Shape<NL>::LD;
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr int MPT = (NPK + kB16 - 1) / kB16;      // factor entries per thread
  constexpr int GPT = (32 * NL + kB16 - 1) / kB16;  // gathered (k, column) pairs per thread
  __shared__ __attribute__((aligned(16))) __bf16 sG[MP * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sW[32 * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sU[32 * LD];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  __shared__ double red_s[kB16];
  __shared__ int32_t gidx[KP];   // map of the current element (DIRECT: bit 31 = single copy)

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
  const int64_t GS = gridDim.x / 8;
  const int64_t chunk = (E + 7) / 8;
  const int64_t Kbeg = (int64_t)(blockIdx.x % 8) * chunk;
  const int64_t Kend = Kbeg + chunk < E ? Kbeg + chunk : E;
  const int rc0 = R < 32 ? R : 32;

  // zero the tiles once: only lower-triangle entries are written later, and
  // W^T / U^T only for k < NL (U rows < KP are all written)
  const __bf16 zero = (__bf16)0.0f;
  for (int q = tid; q < MP * LD; q += kB16) sG[q] = zero;
  for (int q = tid; q < 32 * LD; q += kB16) {
    sW[q] = zero;
    sU[q] = zero;
  }
  int pa[MPT];
#pragma unroll
  for (int u = 0; u < MPT; ++u) {
    const int q = tid + u * kB16;
    int i = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
    while ((i + 1) * (i + 2) / 2 <= q) ++i;
    while (i * (i + 1) / 2 > q) --i;
    const int j = q - i * (i + 1) / 2;
    pa[u] = q < NPK ? i * LD + j : -1;
  }
  const int r0 = tid & 31;
  __bf16 greg[MPT];
  double xa[GPT], xb[X2 ? GPT : 1];
  int32_t gcur[GPT], gnxt[GPT];
  // Loads below are issued unconditionally from clamped (valid) addresses and
  // their raw values kept: entries past the element range, past n_loc or in
  // columns that are inactive or past R are never staged, or only reach
  // outputs that are not stored.  Without branches or selects after them the
  // compiler can count the loads, so waiting for one element's loads does not
  // wait for the later map loads and stores.
  auto load_map = [&](int64_t Kx, int32_t* gm) {
    const int64_t Kc = Kx < E ? Kx : E - 1;
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kB16) >> 5;
      gm[u] = map[Kc * NL + (k < NL ? k : NL - 1)];
    }
  };
  auto load_elem = [&](int64_t Kx, const int32_t* gm) {
    const int64_t Kc = Kx < E ? Kx : E - 1;
#pragma unroll
    for (int u = 0; u < MPT; ++u) {
      const int q = tid + u * kB16;
      // non-temporal: the factors are read once per apply
      greg[u] = __builtin_bit_cast(__bf16, __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(G) +
                                                                      Kc * NPK + (q < NPK ? q : NPK - 1)));
    }
    const int rcl = r0 < R ? r0 : R - 1;
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int64_t gi = (int64_t)(gm[u] & 0x7fffffff) * R + rcl;
      xa[u] = in.x[gi];
      if (X2) xb[u] = in.x2[gi];
    }
  };
  // Z = Gtil^T bf16(Gtil W) for the 32 columns c0.. in sW
  auto products = [&](int64_t K, int c0, int rc) {
    if (wv < MT) gram_u<NL>(sG, sW, sU, wv, lane);
    __syncthreads();
    if (wv < MT) {
      const int t = wv;
      const f32x16 acc = gram_z<NL>(sG, sU, t, lane);
      const int col = lane & 31;
      if (col < rc && act_s[c0 + col]) {
        // the 16 rows' map entries read together, then the stores
        int32_t gr[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          gr[r] = (DIRECT && row < NL) ? gidx[row] : 0;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * t + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          if (row >= NL) continue;
          if (DIRECT && gr[r] < 0) {
            y[(int64_t)(gr[r] & 0x7fffffff) * R + c0 + col] = (double)acc[r];
          } else {
            zb[((int64_t)row * E + K) * R + c0 + col] = acc[r];
          }
        }
      }
    }
  };
  int64_t K = Kbeg + blockIdx.x / 8;
  load_map(K, gcur);
  load_elem(K, gcur);
  load_map(K + GS, gnxt);
  const double cf0 = r0 < R ? coef_s[r0] : 0.0;
  for (; K < Kend; K += GS) {
    __syncthreads();   // the previous element's products are done with the tiles
#pragma unroll
    for (int u = 0; u < MPT; ++u)
      if (pa[u] >= 0) sG[pa[u]] = greg[u];
#pragma unroll
    for (int u = 0; u < GPT; ++u) {
      const int k = (tid + u * kB16) >> 5;
      if (k < NL) {
        sW[r0 * LD + k] = (__bf16)(float)(X2 ? fma(cf0, xb[u], xa[u]) : xa[u]);
        if (r0 == 0) {
          gidx[k] = gcur[u];
        }
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
          const int64_t gi = (int64_t)(gidx[k] & 0x7fffffff) * R + c0 + r;
          v = in.x[gi];
          if (X2) v = fma(coef_s[c0 + r], in.x2[gi], v);
        }
        sW[r * LD + k] = (__bf16)(float)v;
      }
      __syncthreads();
      products(K, c0, rc);
    }
  }
}

#define BF16_CASES(X) X(3) X(4) X(6) X(8) X(10) X(15) X(20) X(24) X(35) X(36) X(45) X(56) X(70) X(84)

// One BF16 element pass: the broken vector zb, and (direct) y of the
// single-copy DOFs.
template <int NL>
static int bf16_launch(Ctx* c, const InArgs& in, int R, float* zb, double* y, bool direct, hipStream_t s) {
  const __bf16* G = (const __bf16*)c->ainv;
  if (direct)
    k_bras_bf16<NL, true, false><<<(unsigned)c->bf16_grid, kB16, 0, s>>>(c->E, R, c->l2g_dir, in, G, zb, y);
  else if (in.x2)
    k_bras_bf16<NL, false, true><<<(unsigned)c->bf16_grid_x2, kB16, 0, s>>>(c->E, R, c->l2g, in, G, zb, nullptr);
  else
    k_bras_bf16<NL, false, false><<<(unsigned)c->bf16_grid_plain, kB16, 0, s>>>(c->E, R, c->l2g, in, G, zb, nullptr);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

static int bf16_elem(Ctx* c, const InArgs& in, int R, float* zb, double* y, bool direct, hipStream_t s) {
#define CASE(N) \
  case N: return bf16_launch<N>(c, in, R, zb, y, direct, s);
  switch (c->nl) {
    BF16_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no BF16 element kernel", c->nl);
  }
#undef CASE
}

template <typename KF>
static int resident(const Ctx* c, KF kern, int* grid) {
  int v = 0;
  BRAS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, kB16, 0));
  const int64_t want = (int64_t)(v > 0 ? v : 1) * c->ncu;
  const int64_t g = c->E < want ? c->E : want;
  *grid = (int)(8 * ((g + 7) / 8));   // the kernel splits the elements over 8 XCDs
  return BRAS_OK;
}

template <int NL>
static int grids(Ctx* c) {
  int st = resident(c, k_bras_bf16<NL, false, false>, &c->bf16_grid_plain);
  if (st == BRAS_OK) st = resident(c, k_bras_bf16<NL, false, true>, &c->bf16_grid_x2);
  if (st == BRAS_OK) st = resident(c, k_bras_bf16<NL, true, false>, &c->bf16_grid);
  return st;
}

__global__ void k_flag_single(int64_t cnt, const int32_t* __restrict__ l2g, const int32_t* __restrict__ mult,
                              int32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) {
    const int32_t g = l2g[t];
    out[t] = mult[g] == 1 ? (int32_t)((uint32_t)g | 0x80000000u) : g;
  }
}

// Persistent grids of the BF16 element pass and (unless BRAS_BF16_DIRECT=0)
// the flagged map of its single-copy variant; once per handle.
int bf16_setup(Ctx* c, hipStream_t s) {
  if (const char* e = getenv("BRAS_BF16_DIRECT")) c->bf16_direct = atoi(e) != 0;
  int st;
#define CASE(N) \
  case N: st = grids<N>(c); break;
  switch (c->nl) {
    BF16_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no BF16 element kernel", c->nl);
  }
#undef CASE
  if (st || !c->bf16_direct) return st;
  const int64_t cnt = c->E * (int64_t)c->nl;
  if (hipMalloc((void**)&c->l2g_dir, sizeof(int32_t) * (size_t)cnt) != hipSuccess) {
    c->l2g_dir = nullptr;
    return fail(BRAS_ENOMEM, "flagged element map allocation failed");
  }
  k_flag_single<<<(unsigned)((cnt + 255) / 256), 256, 0, s>>>(cnt, c->l2g, c->mult, c->l2g_dir);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

int launch_bras_bf16(Ctx* c, const double* x, double* y, int R, hipStream_t s, const double* dotv, double* dotpart,
                     const int* active, void* zb) {
  InArgs in;
  in.x = x;
  in.active = active;
  // plain applies: single-copy DOFs go straight to y (with dot products the reduce writes them all)
  const bool direct = bf16_bypass(c, R) && !(dotv && dotpart);
  int st = bf16_elem(c, in, R, (float*)zb, y, direct, s);
  if (st) return st;
  return reduce_float_plain(c, (const float*)zb, y, R, s, dotv, dotpart, direct ? 1 : 0);
}

int cg_bras_bf16_step(Ctx* c, const CgArgs& cg, int R, hipStream_t s) {
  int st = bf16_elem(c, precond_input(cg, R), R, (float*)c->zb, nullptr, false, s);
  if (st) return st;
  return reduce_float_cg(c, (const float*)c->zb, R, s, cg);
}

int bf16_stat_step(Ctx* c, const CgArgs& cg, const InArgs& in, int R, hipStream_t s) {
  int st = bf16_elem(c, in, R, (float*)c->zb, nullptr, false, s);
  if (st) return st;
  return reduce_float_stat(c, (const float*)c->zb, R, s, cg);
}

}  // namespace bras
