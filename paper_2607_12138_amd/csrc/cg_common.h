// Device-side CG state shared by the operator passes and the CG driver.
//
// Scalars of every column live in device memory (sc: float64 [S_NSC][R],
// ic: int [I_NIC][R]).  Every dot product is written as per-block partials
// [blocks][R] by the pass that produces its terms and summed in block order
// by the next kernel (a kernel boundary separates writers and readers), so
// results are bitwise reproducible and no atomics are involved.
#pragma once

#include <hip/hip_runtime.h>

namespace bras {

enum { S_RZ = 0, S_R0, S_TARGET, S_ALPHA, S_BETA, S_RZOLD, S_RELRES, S_RR, S_NSC };
enum { I_ACTIVE = 0, I_ITERS, I_STATUS, I_NIC };
enum { ST_RUN = 0, ST_OK = 1, ST_NOCONV = 2, ST_BREAK = 3 };

// What a reduce (or patch) pass does with each conforming sum acc_i:
//   OUT_PLAIN    y_i = acc_i (optional partials of y . dotv)
//   OUT_MASS_CG  p_new = z + beta p, q = acc, partials p_new . q
//   OUT_BRAS_CG  r_new = r - alpha q, x += alpha p, z = acc, partials r_new . r_new,
//                r_new . z and (flexible) r_new . z_old
//   OUT_RES      r = b - acc, partials r . r             (stationary iterations)
//   OUT_STAT     d = a d + c acc, x += d                 (a = sc[S_ALPHA], c = sc[S_BETA])
enum { OUT_PLAIN = 0, OUT_MASS_CG = 1, OUT_BRAS_CG = 2, OUT_RES = 3, OUT_STAT = 4 };

// Input of an element pass: w = x + sign * c_r * x2 (x2 optional), where c_r
// is cvec[r], or, when apart is set, alpha_r = rho_r / (sum of the p.q
// partials apart[anb][R]) computed in the pass's own prologue (block 0 stores
// alpha and any breakdown in sc / ic for the kernels that follow).
struct InArgs {
  const double* x = nullptr;
  const double* x2 = nullptr;
  const double* cvec = nullptr;
  double sign = 0.0;
  const int* active = nullptr;   // per-column flags (nullptr: all columns)
  const double* apart = nullptr;
  int anb = 0;
  double* sc = nullptr;
  int* ic = nullptr;
};

// Buffers and scalars of a fused CG pass.
struct CgArgs {
  double *x = nullptr, *r = nullptr, *p = nullptr, *z = nullptr, *q = nullptr;
  const double* b = nullptr;      // right-hand side (stationary iterations)
  double* sc = nullptr;
  int* ic = nullptr;
  double *part0 = nullptr, *part1 = nullptr, *part2 = nullptr;
  const double* apart = nullptr;  // p.q partials for the alpha prologue
  int anb = 0;
  int flexible = 0;
  int maxit = 0;
};

// Fixed-order sum of partial[b*R + col], b < nb, by one block.
__device__ inline double block_sum(const double* partial, int nb, int R, int col, double* sh) {
  // loads in batches of 8 per thread (independent), summed in index order
  double s = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 8 * (int)blockDim.x) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int b = b0 + (int)threadIdx.x + u * (int)blockDim.x;
      v[u] = b < nb ? partial[(int64_t)b * R + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  const double v = sh[0];
  __syncthreads();
  return v;
}

// Fixed-order sums of part[b*R + c], b < nb, for every column c, by one
// block; out (shared memory, R entries) receives them.  sh holds blockDim.x
// doubles.  With one column (or more columns than threads) each column is
// summed by block_sum; otherwise thread t takes column t % R and every
// (blockDim/R)-th partial, and thread c then adds the per-thread sums of
// column c in thread order.
__device__ inline void block_sums_all(const double* part, int nb, int R, double* out, double* sh) {
  const int bs = blockDim.x, t = threadIdx.x;
  if (R == 1 || R > bs) {
    for (int col = 0; col < R; ++col) {
      const double v = block_sum(part, nb, R, col, sh);
      if (t == 0) out[col] = v;
    }
    __syncthreads();
    return;
  }
  const int G = bs / R;
  double s = 0.0;
  if (t < G * R) {
    const int col = t % R, g = t / R;
    for (int b0 = g; b0 < nb; b0 += 8 * G) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int b = b0 + u * G;
        v[u] = b < nb ? part[(int64_t)b * R + col] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
  }
  sh[t] = s;
  __syncthreads();
  if (t < R) {
    double v = 0.0;
    for (int g = 0; g < G; ++g) v += sh[g * R + t];
    out[t] = v;
  }
  __syncthreads();
}

// alpha_r = rho_r / p.q for every column, into coef[R] (0 for stopped
// columns) and act[R]; block 0 records alpha and breakdowns.  Every block
// derives the same values from the same partials.
__device__ inline void alpha_prologue(const double* apart, int anb, int R, double* sc, int* ic, double* coef,
                                      int* act, double* sh) {
  block_sums_all(apart, anb, R, coef, sh);   // coef[c] = p.q for now
  for (int col = threadIdx.x; col < R; col += blockDim.x) {
    const double pq = coef[col];
    if (!ic[I_ACTIVE * R + col]) {
      coef[col] = 0.0;
      act[col] = 0;
    } else if (!(pq > 0.0) || !isfinite(pq)) {
      coef[col] = 0.0;
      act[col] = 0;
      if (blockIdx.x == 0) {
        ic[I_ACTIVE * R + col] = 0;
        ic[I_STATUS * R + col] = ST_BREAK;
      }
    } else {
      const double a = sc[S_RZ * R + col] / pq;
      coef[col] = a;
      act[col] = 1;
      if (blockIdx.x == 0) sc[S_ALPHA * R + col] = a;
    }
  }
  __syncthreads();
}

// Convergence test on the updated recursive residual, then beta and rho
// (one block, after the residual / preconditioner pass).  rr, rz, rzo: shared
// memory of R entries each; sh: blockDim.x doubles.
__device__ inline void finish_iteration(const double* part0, const double* part1, const double* part2, int nb,
                                        int R, double* sc, int* ic, int flexible, int maxit, double* sh, double* rr,
                                        double* rz, double* rzo) {
  block_sums_all(part0, nb, R, rr, sh);
  block_sums_all(part1, nb, R, rz, sh);
  if (flexible) block_sums_all(part2, nb, R, rzo, sh);
  for (int col = threadIdx.x; col < R; col += blockDim.x) {
    if (!ic[I_ACTIVE * R + col]) continue;
    const int it = ic[I_ITERS * R + col] + 1;
    ic[I_ITERS * R + col] = it;
    const double nrm = sqrt(rr[col]);
    sc[S_RR * R + col] = rr[col];
    sc[S_RELRES * R + col] = nrm / sc[S_R0 * R + col];
    const double old = sc[S_RZ * R + col];
    const double z = rz[col];
    if (!isfinite(nrm)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else if (nrm <= sc[S_TARGET * R + col]) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_OK;
    } else if (it >= maxit) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_NOCONV;
    } else if (!(z > 0.0) || !isfinite(z)) {
      ic[I_ACTIVE * R + col] = 0;
      ic[I_STATUS * R + col] = ST_BREAK;
    } else {
      sc[S_BETA * R + col] = flexible ? (z - rzo[col]) / old : z / old;
      sc[S_RZ * R + col] = z;
    }
  }
  __syncthreads();
}

}  // namespace bras
