// rb_assemble.hpp -- offline assembly of the convection tensors on the device (eqn tensor,
// Section 3.5): for an affine expansion c_q(u, v, t) = int ((u . grad) v) . (M_q t),
//   out[q][i][j][k] = w sum_x sum_{b,c} M_q[b][c] ((phi_j . grad) phi_k)^b(x) t_i^c(x),
// with quadrature weight w over the points x. Every c_q is linear in its weight matrix, so the
// Qc tensors are combinations of four base tensors
//   T_bc[i][j][k] = w sum_x t_i^c(x) D_b[j][k](x),   D_b[j][k](x) = sum_a phi_j^a(x) d_a phi_k^b(x),
// each a contraction (test index) x (quadrature point) x (index pair): R x X x N^2, which runs
// on MFMA-F64 with the pair factor D_b formed in registers (never stored).
#pragma once

#include "rb_common.hpp"

namespace rb {

constexpr int kAsmTiles = 4;      // 16-row test tiles per wavefront
constexpr int kAsmWaves = 4;      // wavefronts per workgroup: four consecutive advecting j

struct AssembleArgs {
  int N, R, X;                    // velocity functions, test functions, quadrature points
  int nsx;                        // quadrature-point splits (partial sums of the base tensors)
  const double* phiT;             // [X][2][N]      phi_j^a(x)
  const double* dphiT;            // [X][2][2][N]   d_a phi_k^b(x)
  const double* testT;            // [X][2][R]      t_i^c(x)
  double* part;                   // [nsx][4][R][N][N] partial base tensors (bc = 2b + c)
};

// Workgroup (ig, jg, kt, sx): test rows 64*ig .. +63 (four 16-row tiles), advecting functions
// j = 4*jg + wave, advected k = 16*kt + lane%16, quadrature points of split sx. Per step of four
// points lane l takes point x0 + l/16: A operand t_i^c (row l%16 of each tile), B operand
// D_b[j][k](x) for its k; four MFMAs per tile (b, c) accumulate the base tensors.
__global__ __launch_bounds__(kWave * kAsmWaves) void assemble_conv_kernel(AssembleArgs g) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  const int nkt = (g.N + 15) / 16, njg = (g.N + kAsmWaves - 1) / kAsmWaves;
  int blk = blockIdx.x;
  const int kt = blk % nkt;
  blk /= nkt;
  const int jg = blk % njg;
  blk /= njg;
  const int ig = blk % ((g.R + 63) / 64);
  const int sx = blk / ((g.R + 63) / 64);
  const int j = jg * kAsmWaves + wv;
  const int k = kt * 16 + li;
  const int i0 = ig * 64;
  const int xs = (int)((int64_t)sx * g.X / g.nsx), xe = (int)((int64_t)(sx + 1) * g.X / g.nsx);
  f64x4 acc[kAsmTiles][4];
#pragma unroll
  for (int t = 0; t < kAsmTiles; ++t)
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) acc[t][bc] = f64x4{0.0, 0.0, 0.0, 0.0};
  const bool jk_ok = j < g.N && k < g.N;
  for (int x0 = xs; x0 < xe; x0 += 4) {
    const int x = x0 + lg;
    const bool x_ok = x < xe;
    double dv[2] = {0.0, 0.0};             // D_b[j][k](x), b = 0, 1
    if (x_ok && jk_ok) {
      const double p0 = g.phiT[((int64_t)x * 2 + 0) * g.N + j];
      const double p1 = g.phiT[((int64_t)x * 2 + 1) * g.N + j];
#pragma unroll
      for (int b = 0; b < 2; ++b)
        dv[b] = fma(p0, g.dphiT[(((int64_t)x * 2 + 0) * 2 + b) * g.N + k],
                    p1 * g.dphiT[(((int64_t)x * 2 + 1) * 2 + b) * g.N + k]);
    }
#pragma unroll
    for (int t = 0; t < kAsmTiles; ++t) {
      const int i = i0 + 16 * t + li;
      double tv[2] = {0.0, 0.0};
      if (x_ok && i < g.R) {
        tv[0] = g.testT[((int64_t)x * 2 + 0) * g.R + i];
        tv[1] = g.testT[((int64_t)x * 2 + 1) * g.R + i];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[t][2 * b + c] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(tv[c], dv[b], acc[t][2 * b + c], 0, 0, 0);
    }
  }
  // accumulator layout: lane l, element v = test row 16t + l/16 + 4v, advected k = 16kt + l%16
  if (j >= g.N || k >= g.N) return;
  const int64_t NN = (int64_t)g.N * g.N;
#pragma unroll
  for (int t = 0; t < kAsmTiles; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = i0 + 16 * t + lg + 4 * v;
      if (i >= g.R) continue;
#pragma unroll
      for (int bc = 0; bc < 4; ++bc)
        g.part[(((int64_t)sx * 4 + bc) * g.R + i) * NN + (int64_t)j * g.N + k] = acc[t][bc][v];
    }
}

// out[q][i][j][k] = w sum_bc M_q[b][c] sum_sx part[sx][bc][i][j][k].
__global__ __launch_bounds__(256) void assemble_combine_kernel(const double* __restrict__ part,
                                                               int nsx, int R, int N, int Qc,
                                                               const double* __restrict__ M,
                                                               double w, double* __restrict__ out) {
  const int64_t per = (int64_t)R * N * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < per;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double t[4];
#pragma unroll
    for (int bc = 0; bc < 4; ++bc) {
      double sum = 0.0;
      for (int sx = 0; sx < nsx; ++sx) sum += part[((int64_t)sx * 4 + bc) * per + idx];
      t[bc] = w * sum;
    }
    for (int q = 0; q < Qc; ++q) {
      const double* m = M + 4 * q;             // M_q[b][c] at m[2b + c]
      out[(int64_t)q * per + idx] = fma(m[0], t[0], fma(m[1], t[1], fma(m[2], t[2], m[3] * t[3])));
    }
  }
}

}  // namespace rb
