// Microbenchmark (not part of the operator passes): the element-local Gram
// products of the BF16 element pass (bf16_gram.h) on LDS-resident tiles, with
// no HBM traffic, to measure the matrix-core rate those products reach by
// themselves.  Each work-group fills one Gtil / W tile pair with fixed small
// values and runs `iters` rounds of U = Gtil W, Z = Gtil^T bf16(U), with the
// element pass's barrier between the products and after them.
#include "internal.h"
#include "bf16_gram.h"

namespace bras {

template <int NL>
__global__ void __launch_bounds__(kB16) __attribute__((amdgpu_waves_per_eu(2)))
k_local_gram_bench(int iters, float* __restrict__ out) {
  constexpr int MT = Bf16Shape<NL>::MT, MP = Bf16Shape<NL>::MP, LD = Bf16Shape<NL>::LD;
  __shared__ __attribute__((aligned(16))) __bf16 sG[MP * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sW[32 * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sU[32 * LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int q = tid; q < MP * LD; q += kB16) {
    const int i = q / LD, k = q - i * LD;
    sG[q] = (__bf16)((i < NL && k <= i) ? (float)((i * 7 + k * 3 + blockIdx.x) % 17 - 8) * 0.0625f : 0.0f);
  }
  for (int q = tid; q < 32 * LD; q += kB16) {
    const int c = q / LD, k = q - c * LD;
    sW[q] = (__bf16)(k < NL ? (float)((k * 5 + c) % 13 - 6) * 0.125f : 0.0f);
    sU[q] = (__bf16)0.0f;
  }
  __syncthreads();
  float sum = 0.0f;
  for (int it = 0; it < iters; ++it) {
    if (wv < MT) gram_u<NL>(sG, sW, sU, wv, lane);
    __syncthreads();
    if (wv < MT) {
      const f32x16 z = gram_z<NL>(sG, sU, wv, lane);
      sum += z[it & 15];
    }
    __syncthreads();
  }
  out[(int64_t)blockIdx.x * kB16 + tid] = sum;
}

template <int NL>
static int bench_launch(int iters, int blocks, float* out, hipStream_t s, int* mfma) {
  *mfma = gram_mfma_count<NL>();
  if (blocks > 0) {
    k_local_gram_bench<NL><<<(unsigned)blocks, kB16, 0, s>>>(iters, out);
    BRAS_HIP(hipGetLastError());
  }
  return BRAS_OK;
}

}  // namespace bras

using namespace bras;

extern "C" int bras_bench_bf16_local_gemm(int n_loc, int iters, int blocks, float* out_d, long long* flops_h,
                                          void* stream) {
  clear_error();
  BRAS_CHECK(iters >= 0 && blocks >= 0, "iters and blocks must be >= 0");
  BRAS_CHECK(blocks == 0 || out_d, "null output");
  int mfma = 0, st;
  hipStream_t s = (hipStream_t)stream;
  switch (n_loc) {
#define CASE(N) \
  case N: st = bench_launch<N>(iters, blocks, out_d, s, &mfma); break;
    CASE(20) CASE(36) CASE(70) CASE(84)
#undef CASE
    default: return fail(BRAS_EINVAL, "n_loc %d: the microbenchmark covers 20, 36, 70 and 84", n_loc);
  }
  if (st) return st;
  // 32x32x16 MFMA: 2 * 32 * 32 * 16 flop; blocks = 0: one round of one work-group
  const long long rounds = blocks > 0 ? (long long)iters * blocks : 1;
  if (flops_h) *flops_h = (long long)mfma * 32768LL * rounds;
  return BRAS_OK;
}
