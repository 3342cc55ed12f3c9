// rb_reconstruct.hpp -- pressure reconstruction from a combined velocity-pressure basis.
//
// With the second construction of a combined basis (Section 4.2, after eqn z_c), every
// reduced velocity function carries a pressure part built from the same snapshot
// coefficients, so the pressure of a solution is the same linear combination of those parts
// as its velocity: with Pc the pressure-basis coefficients of the pressure parts,
//   p = Pc u,   Pc [Np][N]  (one small matrix-vector product per request).
// The paper notes that this presumes a linear dependence of the pressure on the velocity
// (its remark on linearity); the a posteriori recovery of eqn sup-vvar does not.
#pragma once

#include "rb_common.hpp"

namespace rb {

// One 256-thread workgroup per group of requests: Pc^T staged in LDS once, then thread t
// computes p[b][i] for consecutive (b, i) pairs, so the iterate u[b][.] is read by the Np
// threads of a request from the same cache line and the writes of p are contiguous.
// LDS: N * Np doubles (at most 152 * 64 * 8 = 78 KB).
static __global__ __launch_bounds__(256) void reconstruct_kernel(
    const double* __restrict__ Pc, int ldpc, int N, int Np, int B, const double* __restrict__ u,
    int ldu, double* __restrict__ p, int ldp) {
  extern __shared__ double pct[];                 // [N][Np]
  for (int idx = threadIdx.x; idx < N * Np; idx += blockDim.x) {
    const int i = idx / N, j = idx - i * N;       // coalesced read of row i of Pc
    pct[j * Np + i] = Pc[(int64_t)i * ldpc + j];
  }
  __syncthreads();
  const int64_t total = (int64_t)B * ldp;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / ldp;
    const int i = (int)(idx - b * ldp);
    double s = 0.0;
    if (i < Np) {
      const double* ub = u + b * ldu;
      for (int j = 0; j < N; ++j) s = fma(pct[j * Np + i], ub[j], s);
    }
    p[idx] = s;
  }
}

}  // namespace rb
