// Per-lane element pass (one element per lane, all rows), included by apply.hip.
#pragma once

#include <type_traits>
#include <utility>

#include "cg_common.h"
#include "internal.h"

namespace bras {

enum { FORM_SCALED = 0, FORM_PACKED = 1, FORM_METRIC = 2 };

// Element pass for per-element matrices, one lane per element computing all
// n_loc rows (n_loc <= kLaneMaxNL): a single wavefront owns 64 consecutive
// elements, gathers their inputs into LDS w[j][e], and each lane then walks the
// lower triangle of its element's symmetric matrix once, every entry m_ij
// (i > j) feeding both z_i += m_ij w_j and z_j += m_ij w_i, so each stored
// entry is read exactly once.
//   FORM_PACKED  m_ij = P_K[q], q = i(i+1)/2 + j, stored in 16-byte groups of
//                V = 16 / sizeof(T) consecutive q: P[(q / V) * E + K][q % V],
//                so one lane reads V entries per load and a wavefront's load
//                is 1 KiB contiguous; loads go in batches, the next batch in
//                flight while the current one is used
//   FORM_METRIC  m_ij = sum_p G_p,K S_p[q]           (S packed [q][NSYM], G [p][E];
//                                                    pairs p >= nsym are zero;
//                                                    S read as scalar loads)
// The metric form rebuilds M_K entry by entry from the shared pair tables
// (eq. piola_mass_pullbacks), 6 multiply-adds per entry in 3D.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}
constexpr int tri_row(int q) {
  int i = 0;
  while ((i + 1) * (i + 2) / 2 <= q) ++i;
  return i;
}
// t-th entry in diagonal order (d = 0, 1, ..., entries (i, i - d)) as a
// row-order packed index q = i(i+1)/2 + j
template <int NL>
constexpr int diag_q(int t) {
  int d = 0;
  while (t >= NL - d) {
    t -= NL - d;
    ++d;
  }
  const int i = d + t, j = t;
  return i * (i + 1) / 2 + j;
}
// Return i unchanged, but only once dep has been computed: loads indexed by
// the result cannot be issued before the arithmetic that produced dep, which
// bounds how many loads of the unrolled product are in flight (otherwise the
// scheduler hoists all of them and runs out of registers).  pin_s keeps a
// wave-uniform index in scalar registers, pin_v a per-lane one.
template <typename I, typename D>
__device__ __forceinline__ I pin_s(I i, D dep) {
  __asm__ volatile("" : "+s"(i) : "v"(dep));
  return i;
}
template <typename I, typename D>
__device__ __forceinline__ I pin_v(I i, D dep) {
  __asm__ volatile("" : "+v"(i) : "v"(dep));
  return i;
}
// Marks every accumulator as used here: volatile asm statements keep their
// order, so all arithmetic feeding z so far happens before the next pin.
template <int N, typename T>
__device__ __forceinline__ void touch_all(T (&z)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) __asm__ volatile("" : "+v"(z[i]));
}

// Product z = M_K w of one element in one lane, over the stored lower
// triangle (each entry used for both z_i and z_j): FORM_PACKED reads the
// element's packed matrix from ap (16-byte groups, layout of packed_at with
// element index K0 + lt), FORM_METRIC rebuilds each entry from the pair
// tables symtab [q][NSYM] and the element's coefficients g.  z must be zero
// on entry.  VAR: scheduling variant (see k_elem_lane).
template <int NL, int FORM, int NSYM, typename T, int VAR>
__device__ __forceinline__ void lane_product(const T (&wr)[NL], T (&z)[NL], int64_t K0, int lt, int64_t E,
                                             const T* __restrict__ ap, const double* __restrict__ symtab,
                                             const double (&g)[NSYM > 0 ? NSYM : 1]) {
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr int V = 16 / (int)sizeof(T);
  typedef T vec_t __attribute__((ext_vector_type(V)));
  // one stored entry q = i(i+1)/2 + j applied symmetrically
  auto use = [&](auto qc, T m) {
    constexpr int q = decltype(qc)::value;
    constexpr int i = tri_row(q), j = q - i * (i + 1) / 2;
    z[i] = fma(m, wr[j], z[i]);
    if constexpr (j < i) z[j] = fma(m, wr[i], z[j]);
  };
  if constexpr (FORM == FORM_METRIC) {
    // table entries are wave-uniform scalar loads (SGPR operands, no LDS
    // traffic), in batches of CQ entries, the next batch in flight.
    // Visiting order: row by row, or diagonal by diagonal (entries (i, i-d)
    // for i = d..NL-1), where consecutive entries update different
    // accumulators.
    constexpr int CQS = (VAR >> 2) & 3;
    constexpr int CQ = (VAR & 64) ? ((VAR & 128) ? 16 : 12) : (CQS == 0 ? 2 : (CQS == 1 ? 4 : (CQS == 2 ? 1 : 8)));
    constexpr bool DIAG = (VAR & 1) != 0;
    constexpr bool PIN_M = (VAR & 2) != 0;
    constexpr int NBQ = (NPK + CQ - 1) / CQ;
    double tb[2][CQ * NSYM];
    double mlast = wr[0];
    auto tload = [&](auto bc, int64_t o) {
      constexpr int b = decltype(bc)::value;
      const double* src = symtab + o;
      static_for<CQ>([&](auto ec) {
        constexpr int t = b * CQ + decltype(ec)::value;
        if constexpr (t < NPK) {
          constexpr int q = DIAG ? diag_q<NL>(t) : t;
#pragma unroll
          for (int p = 0; p < NSYM; ++p) tb[b & 1][decltype(ec)::value * NSYM + p] = src[q * NSYM + p];
        }
      });
    };
    tload(std::integral_constant<int, 0>{}, pin_s((int64_t)0, wr[0]));
    static_for<NBQ>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      if constexpr (b + 1 < NBQ) tload(std::integral_constant<int, b + 1>{}, pin_s((int64_t)0, mlast));
      static_for<CQ>([&](auto ec) {
        constexpr int e = decltype(ec)::value;
        constexpr int t = b * CQ + e;
        if constexpr (t < NPK) {
          constexpr int q = DIAG ? diag_q<NL>(t) : t;
          double acc = 0.0;
#pragma unroll
          for (int p = 0; p < NSYM; ++p) acc = fma(g[p], tb[b & 1][e * NSYM + p], acc);
          use(std::integral_constant<int, q>{}, (T)acc);
          if (PIN_M) mlast = acc;
        }
      });
      if constexpr (!PIN_M) touch_all(z);
    });
  } else {
    constexpr int NQ = (NPK + V - 1) / V;   // 16-byte groups
    constexpr int CV = ((VAR >> 4) & 3) == 0 ? 6 : (((VAR >> 4) & 3) == 1 ? 3 : (((VAR >> 4) & 3) == 2 ? 10 : 14));
    constexpr int NB = (NQ + CV - 1) / CV;
    // uniform base + per-lane offset (lanes past the last element read its data)
    const vec_t* sbase = reinterpret_cast<const vec_t*>(ap) + K0;
    vec_t buf[2][CV];
    auto load = [&](auto bc, int64_t boff) {
      constexpr int b = decltype(bc)::value;
      const vec_t* src = sbase + boff;
#pragma unroll
      for (int v = 0; v < CV; ++v)
        if (b * CV + v < NQ) {
          // VAR bit 8: the matrix stream is read with the non-temporal hint
          if constexpr ((VAR & 256) != 0)
            buf[b & 1][v] = __builtin_nontemporal_load(&src[(int64_t)v * E + lt]);
          else
            buf[b & 1][v] = src[(int64_t)v * E + lt];
        }
    };
    load(std::integral_constant<int, 0>{}, pin_s((int64_t)0, wr[0]));
    static_for<NB>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      // batch b+1 goes out once batch b-1 has been used: two batches in flight
      if constexpr (b + 1 < NB) load(std::integral_constant<int, b + 1>{}, pin_s((int64_t)((b + 1) * CV) * E, wr[0]));
      static_for<CV * V>([&](auto ec) {
        constexpr int q = b * CV * V + decltype(ec)::value;
        if constexpr (q < NPK) use(std::integral_constant<int, q>{}, buf[b & 1][(q / V) % CV][q % V]);
      });
      touch_all(z);
    });
  }
}

// VAR selects scheduling variants: metric form bit 0 diagonal order, bit 1
// pinning on the entry values, bits 2-3 and 6-7 the batch size; packed form
// bits 4-5 the batch size, bit 8 non-temporal loads of the matrix stream
// (read once per apply, it then does not evict the vectors and the broken
// values the next pass reads).  The metric variants the library offers to
// its autotuner are kMetricVar[] below.  The per-element metric
// coefficients are read non-temporally for the same reason.
template <int NL, int FORM, int NSYM, typename T, typename ZT, int EPB, int VAR = 0>
__global__ void __launch_bounds__(EPB) k_elem_lane(int64_t E, int R, const int32_t* __restrict__ l2g, InArgs in,
                                                   const double* __restrict__ symtab,
                                                   const double* __restrict__ coefK, int nsym,
                                                   const T* __restrict__ ap, ZT* __restrict__ zb) {
  constexpr int NPK = NL * (NL + 1) / 2;
  constexpr int V = 16 / (int)sizeof(T);
  constexpr int WSL = EPB + 1;   // LDS row stride
  typedef T vec_t __attribute__((ext_vector_type(V)));
  __shared__ T w[NL * WSL];
  __shared__ double coef_s[256];
  __shared__ int act_s[256];
  __shared__ double red_s[EPB];
  if (in.apart) {
    alpha_prologue(in.apart, in.anb, R, in.sc, in.ic, coef_s, act_s, red_s);
    for (int c = threadIdx.x; c < R; c += EPB) coef_s[c] *= in.sign;
    __syncthreads();
  } else {
    for (int c = threadIdx.x; c < R; c += EPB) {
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
  const int64_t K0 = (int64_t)blockIdx.x * EPB;
  const int ne = (int)((E - K0) < EPB ? (E - K0) : EPB);
  const bool on = tid < ne;
  const int64_t K = on ? K0 + tid : K0;   // idle lanes read element K0's data and store nothing
  double g[NSYM > 0 ? NSYM : 1];
  if (FORM == FORM_METRIC) {
#pragma unroll
    for (int p = 0; p < NSYM; ++p) g[p] = p < nsym ? __builtin_nontemporal_load(&coefK[(int64_t)p * E + K]) : 0.0;
  }
  for (int col = 0; col < R; ++col) {
    if (!act_s[col]) continue;   // uniform
    const double cf = coef_s[col];
    {
      // map entries past the last element repeat its last entry, so every
      // load is valid and none needs a branch (those lanes store nothing)
      // (indices pinned inside the column loop so that nothing of the gather
      // is hoisted out of it and kept live through the product)
      const int qmax = ne * NL - 1;
      const int tq = pin_v(tid, col);
      const int32_t* mp = l2g + pin_s(K0 * NL, col);
      int32_t gi[NL];
#pragma unroll
      for (int u = 0; u < NL; ++u) {
        const int q = tq + u * EPB;
        gi[u] = mp[q < qmax ? q : qmax];
      }
      // gathers in chunks of G entries, two chunks in flight; 32-bit byte
      // offsets from a uniform base (setup guarantees n * nrhs * 8 < 4 GiB).
      // Without a second vector the first one is read twice with weight 0.
      const char* xb = reinterpret_cast<const char*>(in.x + col);
      const char* x2b = in.x2 ? reinterpret_cast<const char*>(in.x2 + col) : xb;
      const double c2 = in.x2 ? cf : 0.0;
      const uint32_t rb = 8u * (uint32_t)R;
      constexpr int G = 8;
      constexpr int NC = (NL + G - 1) / G;
      double v[NL];
      auto gload = [&](auto cc) {
        constexpr int c = decltype(cc)::value;
        const uint32_t rbp = pin_s(rb, tq);
#pragma unroll
        for (int u = c * G; u < (c + 1) * G && u < NL; ++u) {
          const uint32_t o = (uint32_t)gi[u] * rbp;
          v[u] = fma(c2, *reinterpret_cast<const double*>(x2b + o), *reinterpret_cast<const double*>(xb + o));
        }
      };
      gload(std::integral_constant<int, 0>{});
      static_for<NC>([&](auto cc) {
        constexpr int c = decltype(cc)::value;
        if constexpr (c + 1 < NC) gload(std::integral_constant<int, c + 1>{});
#pragma unroll
        for (int u = c * G; u < (c + 1) * G && u < NL; ++u) {
          const int q = tq + u * EPB;   // < EPB * NL: always inside w
          const int e = q / NL, j = q - e * NL;
          w[j * WSL + e] = (T)v[u];
        }
        __asm__ volatile("" ::: "memory");   // chunk c stored before chunk c+2 is loaded
      });
    }
    __syncthreads();
    T wr[NL], z[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      wr[j] = w[j * WSL + tid];
      z[j] = (T)0;
    }
    lane_product<NL, FORM, NSYM, T, VAR>(wr, z, K0, on ? tid : 0, E, ap, symtab, g);
    if (on) {
#pragma unroll
      for (int i = 0; i < NL; ++i) zb[((int64_t)i * E + K) * R + col] = (ZT)z[i];
    }
    __syncthreads();
  }
}

#define LANE_CASES(X) X(3) X(4) X(6) X(8) X(10) X(12) X(15) X(20) X(21) X(24) X(28) X(30) X(35) X(36)

template <int NL, int FORM, int NSYM, typename T, typename ZT, int VAR>
static int lane_launch(Ctx* c, int R, const InArgs& in, const T* ap, ZT* zb, hipStream_t s) {
  constexpr int EPB = 64;   // one wavefront per work-group
  const unsigned nb = (unsigned)((c->E + EPB - 1) / EPB);
  k_elem_lane<NL, FORM, NSYM, T, ZT, EPB, VAR><<<nb, EPB, 0, s>>>(c->E, R, c->l2g, in, c->symtab, c->coef, c->nsym,
                                                                   ap, zb);
  BRAS_HIP(hipGetLastError());
  return BRAS_OK;
}

template <int FORM, int NSYM, typename T, typename ZT, int VAR = 0>
static int lane_dispatch(Ctx* c, int R, const InArgs& in, const T* ap, ZT* zb, hipStream_t s) {
#define CASE(N) \
  case N: return lane_launch<N, FORM, NSYM, T, ZT, VAR>(c, R, in, ap, zb, s);
  switch (c->nl) {
    LANE_CASES(CASE)
    default: return fail(BRAS_EINVAL, "n_loc %d has no per-lane element kernel", c->nl);
  }
#undef CASE
}

// One translation unit each (lane_*.hip), so they compile in parallel.
int lane_packed_f64(Ctx* c, int R, const InArgs& in, const double* ap, double* zb, hipStream_t s);
int lane_packed_f32(Ctx* c, int R, const InArgs& in, const float* ap, float* zb, hipStream_t s);
int lane_metric3(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s);
// 3D metric form: kMetricVariants (internal.h) scheduling variants (row
// order in batches of 2 and 4 entries, diagonal order in batches of 8), one
// translation unit each.
int lane_metric6_v0(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s);
int lane_metric6_v1(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s);
int lane_metric6_v2(Ctx* c, int R, const InArgs& in, double* zb, hipStream_t s);
// Per-element matrix-core pass for n_loc > kLaneMaxNL (elem_mfma.hip).
int mfma_elem_f64(Ctx* c, int R, const InArgs& in, const double* mat, double* zb, hipStream_t s);
int mfma_elem_f32(Ctx* c, int R, const InArgs& in, const float* mat, float* zb, hipStream_t s);

}  // namespace bras
