// rb_tail.hpp -- the Newton iterations of a batch beyond the expected count, in one launch.
//
// A batch whose requests all converge within K Newton steps still has max_iter - K launch
// pairs in a fixed schedule, each of which finds every request done and exits (Section 3.5
// fixes no iteration count; the stopping test is per request). The host therefore issues K
// regular pairs, K learned from earlier calls, and then this kernel once: workgroup g owns the
// 64-request tile g and, for it = it0, it0 + 1, ... while some request of the tile iterates,
// forms the tile's Jacobian and partial sums of A(mu) u and then takes the Newton step of each
// of its requests. When every request has converged it reads the tile's flags and exits, so
// the whole tail costs one launch.
//
// The contraction visits the row splits, chunks, row blocks and k-steps in the order of
// contract_f64_kernel and accumulates each chunk on the matrix cores from zero exactly as it
// does (same operand tiles, same W values, same fold order into the LDS partial sums, J of a
// later chunk added to the stored one), and the Newton step is lu_f64_request itself, so a
// request's iterates are bitwise those of the regular launches whichever launch takes its
// step. It runs each step one row block at a time with the W values formed on the fly, far
// slower than the regular launches: it is meant for the few requests that need more steps
// than the batches before them.
#pragma once

#include "rb_kernels.hpp"

namespace rb {

// LDS: iterates [kTile][N], row sums [kTile][N], LU rows [kWaves][NP + 8].
__host__ __device__ inline int64_t tail_lds_bytes(int N, int NP) {
  return 8 * ((int64_t)kTile * 2 * N + kWaves * (NP + 8));
}

template <int NP>
__global__ __launch_bounds__(kThreads) void newton_tail_f64_kernel(ContractArgs g, NewtonF64Args a,
                                                                   int it0) {
  extern __shared__ double smem[];
  const int N = g.N;                       // solve operand: R = N
  double* ul = smem;                       // [kTile][N]
  double* pl = ul + kTile * N;             // [kTile][N]
  double* prow = pl + kTile * N + (threadIdx.x >> 6) * (NP + 8);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b0 = blockIdx.x * kTile;
  const int bl = 16 * wv + (lane & 15), bg = b0 + bl, k0 = lane >> 4;
  const int KC = (g.nks - g.kA) / g.nchunk;
  const double* ub = ul + bl * N;

  // theta^a_k of this lane's request; theta^c_q u_l for tensor row t = q*N + l (0 past Qc)
  auto wa = [&](int k) { return (bg < g.B && k < g.Q) ? g.ta[(int64_t)bg * g.Q + k] : 0.0; };
  auto tcq = [&](int q) { return (bg < g.B && q < g.Qc) ? g.tc[(int64_t)bg * g.Qc + q] : 0.0; };
  // wt * acc into the row sums, as the regular kernel's fold for one row block
  auto fold = [&](const f64x4& c, int rb, double wt) {
    const int m0 = rb * 16 + k0;
    const int j0 = m0 / N, i0 = m0 - j0 * N;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int i = i0 + 4 * v, j = j0;
      while (i >= N) { i -= N; ++j; }
      if (j < N) atomicAdd(&pl[bl * N + i], wt * c[v] * ul[bl * N + j]);
    }
  };

  for (int it = it0; it < a.maxit; ++it) {
    if (__syncthreads_and(tid < kTile ? a.s.done[b0 + tid] : 1)) return;
    for (int idx = tid; idx < kTile * N; idx += kThreads) {
      const int b = idx / N, l = idx - b * N, bb = b0 + b;
      ul[idx] = bb < g.B ? g.U[(int64_t)bb * g.ldU + l] : 0.0;
    }
    for (int sp = 0; sp < g.nsplit; ++sp) {
      for (int idx = tid; idx < kTile * N; idx += kThreads) pl[idx] = 0.0;
      __syncthreads();
      const int rb_lo = (int)((int64_t)sp * g.nrb / g.nsplit);
      const int rb_hi = (int)((int64_t)(sp + 1) * g.nrb / g.nsplit);
      for (int ch = 0; ch < g.naff + g.nchunk; ++ch) {
        const bool aff_chunk = ch < g.naff;
        const bool prefix = g.naff == 0 && ch == 0;   // kAmax affine k-steps, then tensor chunk 0
        const int tch = ch - g.naff;
        const int k_first = aff_chunk ? ch * KC : (prefix ? 0 : g.kA + tch * KC);
        const int nks_c = prefix ? kAmax + KC : KC;
        const double end_wt = aff_chunk ? 1.0 : 0.0;
        for (int rb = rb_lo; rb < rb_hi; ++rb) {
          const double* op = g.op + (int64_t)rb * g.nks * 64 + (int64_t)k_first * 64 + lane;
          f64x4 c = {0.0, 0.0, 0.0, 0.0};
          // tensor W walk of this chunk (as the regular kernel forms its register copy)
          int t = tch * KC * 4 + k0, q = 0;
          double th = 0.0;
          if (!aff_chunk) {
            while (t >= N && q < g.Qc) { t -= N; ++q; }
            th = tcq(q);
          }
          for (int k8 = 0; k8 < nks_c; k8 += 8) {
            double x[8];                   // operand tiles of 8 k-steps in flight
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = k8 + u < nks_c ? op[(int64_t)(k8 + u) * 64] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int ks = k8 + u;
              if (ks >= nks_c) break;
              double w;
              if (aff_chunk) {
                w = wa((ch * KC + ks) * 4 + k0);
              } else if (prefix && ks < kAmax) {
                w = wa(ks * 4 + k0);
              } else {
                w = q < g.Qc ? th * ub[t] : 0.0;
                t += 4;
                while (t >= N && q < g.Qc) {
                  t -= N;
                  ++q;
                  th = tcq(q);
                }
                if (q >= g.Qc) t = 0;
              }
              c = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], w, c, 0, 0, 0);
              if (prefix && ks == kAmax - 1) fold(c, rb, 1.0);   // A(mu) u
            }
          }
          if (end_wt != 0.0) fold(c, rb, end_wt);
          // J rows 16 rb + k0 + 4v of request bg (column-major per request)
          double* jp = g.J + (int64_t)bg * g.mp + rb * 16 + k0;
#pragma unroll
          for (int v = 0; v < 4; ++v) jp[4 * v] = c[v] + (ch > 0 ? jp[4 * v] : 0.0);
        }
      }
      __syncthreads();
      for (int idx = tid; idx < kTile * N; idx += kThreads) {
        const int b = idx / N, i = idx - b * N;
        g.part[((int64_t)sp * g.Bp + b0 + b) * g.ldp + i] = pl[idx];
      }
      __syncthreads();
    }
    // Newton steps of the tile's requests, wavefront wv taking 16wv .. 16wv + 15 in turn
    for (int r = 0; r < 16; ++r) {
      const int b = __builtin_amdgcn_readfirstlane(b0 + 16 * wv + r);
      if (b < a.B && !a.s.done[b]) lu_f64_request<NP, false>(a, it, b, prow);
    }
    __syncthreads();
  }
}

}  // namespace rb
