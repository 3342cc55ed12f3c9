// rb_kernels.hpp -- gfx950 kernels of the online reduced Navier-Stokes solver.
//
// Work decomposition (one workgroup = BT requests that share a basis size N):
//   * Jacobian + affine contraction on MFMA (paper Section 3.5 / 3.4): for the BT requests
//       J[(i,j), b] = sum_k Op[(i,j), k] W[k, b],  Op = [ S_flat | A_flat ],
//       S_q[i,j,l] = C_q[i,j,l] + C_q[i,l,j],  W = [ theta^c_q(b) u_l(b) ; theta^a_q(b) ],
//     i.e. one GEMM of shape (N^2) x (Qc N + Q) x BT per Newton step, with the operand
//     tiles pre-packed in MFMA order so every wave load is a contiguous 512-byte line.
//     W lives in LDS; Op streams from L2/HBM once per workgroup per step.
//   * Residual in the GEMM epilogue: after the S part the accumulator holds J_c = C(.,u) +
//     C(u,.), whose product with u is 2 C(u,u); the epilogue folds J_c[i,j] u_j into an LDS
//     vector w, so F(u) = J u - w/2 - f needs no second pass over the tensors.
//   * Pivoted LU in registers: one wavefront per system, one row per lane, pivot search by
//     a wavefront argmax, pivot-row broadcast by readlane; the update is applied and the
//     stopping test (norm given by the Gram matrix H) evaluated in the same wavefront.
//   * The whole Newton loop of the workgroup runs inside one launch; requests that have
//     converged drop out of the LU phase, and the workgroup exits when all have.
#pragma once

#include "rb_common.hpp"

namespace rb {

constexpr int kBT = 16;        // requests per workgroup = MFMA 16x16 output columns
constexpr int kWaves = 4;      // wavefronts per workgroup
constexpr int kThreads = kWave * kWaves;
constexpr int kMaxQ = 12, kMaxQc = 4, kMaxQf = 2, kMaxQb = 2;

// ------------------------------------------------------------------ packing -----------
// Packed operand layout for v_mfma_f64_16x16x4f64 (A operand: lane l holds row l%16,
// k-column l/16 of a 16x4 tile): tile (rb, ks) = 64 consecutive doubles at
// ((rb * nks + ks) * 64), element e <-> (row rb*16 + e%16, k = ks*4 + e/16).
//
// Solve operand rows: m = j*N + i (so J is written column-major per request); columns:
// k < Qc*N -> S_q[i,j,l] with q = k / N, l = k % N; ks0*4 <= k < ks0*4 + Q -> A_q[i,j].
__global__ void pack_solve_f64(const double* __restrict__ C, const double* __restrict__ A,
                               int Nm, int N, int Q, int Qc, int nrb, int nks, int ksA,
                               double* __restrict__ out) {
  const int64_t total = (int64_t)nrb * nks * 64;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = idx & 63;
    const int64_t tile = idx >> 6;
    const int rb = tile / nks, ks = tile % nks;
    const int m = rb * 16 + (e & 15), k = ks * 4 + (e >> 4);
    double v = 0.0;
    if (m < N * N) {
      const int j = m / N, i = m - j * N;
      if (k < Qc * N) {
        const int q = k / N, l = k - q * N;
        v = C[(((int64_t)q * Nm + i) * Nm + j) * Nm + l] + C[(((int64_t)q * Nm + i) * Nm + l) * Nm + j];
      } else if (k >= ksA * 4 && k < ksA * 4 + Q) {
        v = A[((int64_t)(k - ksA * 4) * Nm + i) * Nm + j];
      }
    }
    out[idx] = v;
  }
}

// Pressure operand rows: m = j*Np + i; columns as for the solve operand but with the
// unsymmetrised C_sv (the epilogue contracts with u_j, giving C_sv(u,u)) and A_sv.
__global__ void pack_pressure_f64(const double* __restrict__ Csv, const double* __restrict__ Asv,
                                  int Nm, int Npm, int N, int Np, int Q, int Qc, int nrb,
                                  int nks, int ksA, double* __restrict__ out) {
  const int64_t total = (int64_t)nrb * nks * 64;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = idx & 63;
    const int64_t tile = idx >> 6;
    const int rb = tile / nks, ks = tile % nks;
    const int m = rb * 16 + (e & 15), k = ks * 4 + (e >> 4);
    double v = 0.0;
    if (m < N * Np) {
      const int j = m / Np, i = m - j * Np;
      if (k < Qc * N) {
        const int q = k / N, l = k - q * N;
        v = Csv[(((int64_t)q * Npm + i) * Nm + j) * Nm + l];
      } else if (k >= ksA * 4 && k < ksA * 4 + Q) {
        v = Asv[((int64_t)(k - ksA * 4) * Npm + i) * Nm + j];
      }
    }
    out[idx] = v;
  }
}

// ------------------------------------------------------------------ theta(mu) ---------
__global__ void theta_kernel(const double* __restrict__ mu, int B, int Q, int Qc, int Qf,
                             int Qb, double* __restrict__ ta, double* __restrict__ tc,
                             double* __restrict__ tf, double* __restrict__ tb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double a = mu[2 * b], re = mu[2 * b + 1];
  const double ca = cos(a), sa = sin(a), h = sin(0.5 * a);
  const double la[kMaxQ] = {1.0 / re, ca, sa, a, a * a, a * a * a, cos(2.0 * a),
                            sin(2.0 * a), 2.0 * h * h, a * a * a * a, a * ca, a * sa};
  const double lc[kMaxQc] = {1.0, ca, sa, a};
  for (int q = 0; q < Q; ++q) ta[(int64_t)b * Q + q] = la[q];
  for (int q = 0; q < Qc; ++q) tc[(int64_t)b * Qc + q] = lc[q];
  if (tf) {
    if (Qf == 1) tf[b] = 1.0;
    else { tf[2 * (int64_t)b] = ca; tf[2 * (int64_t)b + 1] = sa; }
  }
  if (tb) {
    tb[(int64_t)b * Qb] = 1.0;
    if (Qb == 2) tb[(int64_t)b * Qb + 1] = a;
  }
}

// ------------------------------------------------------------------ Newton (FP64) -----
// Per-call device state of a batch solve (padded to whole 16-request tiles):
//   U [Bp][NP] current iterates, Fv [Bp][NP] right-hand sides f(mu), Wv [Bp][NP] = J_c u,
//   J [Bp][mp] Jacobians (column-major, mp >= N*N), done/iters/status [Bp].
struct NewtonState {
  double* U;
  double* Fv;
  double* Wv;
  double* J;
  int* done;
  int* iters;
  int* status;
  int64_t mp;
  int NP;
};

struct NewtonF64Args {
  const double* op;        // packed solve operand
  int nrb, nks_s, nks;     // row blocks, S-part k-steps, total k-steps (A part at nks_s)
  int N, Nm, Q, Qc, Qf, B, ldu, maxit;
  double tol;
  const double* ta;        // [B][Q]
  const double* tc;        // [B][Qc]
  const double* tf;        // [B][Qf] (used when fover == nullptr)
  const double* fover;     // [B][ldu] or nullptr
  const double* u0;        // [B][ldu] or nullptr
  const double* F;         // [Qf][Nm]
  const double* H;         // [Nm][Nm] or nullptr
  double* u;               // [B][ldu]
  int* iters;              // [B]
  int* status;             // [B]
  NewtonState s;
};

// Build W[k][b] (k-major, kBT columns) from the current iterates: rows k < Qc*N hold
// theta^c_q(b) u_l(b) (q = k/N, l = k%N), rows ksA*4 + q hold theta^a_q(b), the rest 0.
__device__ __forceinline__ void build_w(double* __restrict__ Wl, const double* __restrict__ ul,
                                        const double* __restrict__ tal,
                                        const double* __restrict__ tcl, int NP, int N, int Q,
                                        int Qc, int nks, int ksA) {
  const int K = nks * 4;
  for (int idx = threadIdx.x; idx < K * kBT; idx += blockDim.x) {
    const int k = idx / kBT, b = idx - k * kBT;
    double v = 0.0;
    if (k < Qc * N) {
      const int q = k / N, l = k - q * N;
      v = tcl[b * kMaxQc + q] * ul[b * NP + l];
    } else if (k >= ksA * 4 && k < ksA * 4 + Q) {
      v = tal[b * kMaxQ + (k - ksA * 4)];
    }
    Wl[idx] = v;
  }
}

// Start of a batch solve: iterates from u0 (or 0), f(mu) (or the override), flags.
__global__ void newton_init_kernel(NewtonF64Args a) {
  const int64_t Bp = (int64_t)(a.B + kBT - 1) / kBT * kBT;
  const int NP = a.s.NP, N = a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < Bp * NP;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / NP;
    const int i = idx - b * NP;
    double uv = 0.0, fv = 0.0;
    if (b < a.B && i < N) {
      if (a.u0) uv = a.u0[b * a.ldu + i];
      if (a.fover) {
        fv = a.fover[b * a.ldu + i];
      } else {
        for (int q = 0; q < a.Qf; ++q) fv += a.tf[b * a.Qf + q] * a.F[(int64_t)q * a.Nm + i];
      }
    }
    a.s.U[idx] = uv;
    a.s.Fv[idx] = fv;
    if (i == 0) {
      a.s.done[b] = (b >= a.B);
      a.s.iters[b] = 0;
      a.s.status[b] = 1;
    }
  }
}

// Jacobian + residual contraction for 16 requests per workgroup (see file header).
__global__ __launch_bounds__(kThreads) void jac_f64_kernel(NewtonF64Args a) {
  extern __shared__ double smem[];
  const int K = a.nks * 4;
  const int NP = a.s.NP;
  double* Wl = smem;                       // [K][kBT]
  double* ul = Wl + K * kBT;               // [kBT][NP]
  double* wl = ul + kBT * NP;              // [kBT][NP]
  double* tal = wl + kBT * NP;             // [kBT][kMaxQ]
  double* tcl = tal + kBT * kMaxQ;         // [kBT][kMaxQc]

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b0 = blockIdx.x * kBT;
  const int N = a.N, M = N * N;
  if (__syncthreads_and(tid < kBT ? a.s.done[b0 + tid] : 1)) return;

  for (int idx = tid; idx < kBT * NP; idx += kThreads) {
    ul[idx] = a.s.U[(int64_t)b0 * NP + idx];
    wl[idx] = 0.0;
  }
  for (int idx = tid; idx < kBT * kMaxQ; idx += kThreads) {
    const int b = idx / kMaxQ, q = idx - b * kMaxQ, bg = b0 + b;
    tal[idx] = (bg < a.B && q < a.Q) ? a.ta[(int64_t)bg * a.Q + q] : 0.0;
  }
  for (int idx = tid; idx < kBT * kMaxQc; idx += kThreads) {
    const int b = idx / kMaxQc, q = idx - b * kMaxQc, bg = b0 + b;
    tcl[idx] = (bg < a.B && q < a.Qc) ? a.tc[(int64_t)bg * a.Qc + q] : 0.0;
  }
  __syncthreads();
  build_w(Wl, ul, tal, tcl, NP, N, a.Q, a.Qc, a.nks, a.nks_s);
  __syncthreads();

  const int bcol = lane & 15;
  const double* wp = Wl + (lane >> 4) * kBT + bcol;
  double* jcol = a.s.J + (int64_t)(b0 + bcol) * a.s.mp;
  for (int rb = wv; rb < a.nrb; rb += kWaves) {
    const double* opp = a.op + (int64_t)rb * a.nks * 64 + lane;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    int ks = 0;
    for (; ks < a.nks_s; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opp[ks * 64], wp[ks * 4 * kBT], acc, 0, 0, 0);
    // epilogue: accumulate J_c[i,j] u_j into w_i. Accumulator layout of
    // v_mfma_f64_16x16x4f64: lane l, element v holds row l/16 + 4v, column l%16.
    const int m0 = rb * 16 + (lane >> 4);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + 4 * v;
      if (m < M) {
        const int j = m / N, i = m - j * N;
        atomicAdd(&wl[bcol * NP + i], acc[v] * ul[bcol * NP + j]);
      }
    }
    for (; ks < a.nks; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opp[ks * 64], wp[ks * 4 * kBT], acc, 0, 0, 0);
    jcol[m0 + 0] = acc[0];
    jcol[m0 + 4] = acc[1];
    jcol[m0 + 8] = acc[2];
    jcol[m0 + 12] = acc[3];
  }
  __syncthreads();
  for (int idx = tid; idx < kBT * NP; idx += kThreads) a.s.Wv[(int64_t)b0 * NP + idx] = wl[idx];
}

// One wavefront per request: residual F(u) = J u - w/2 - f, pivoted LU solve of
// J delta = -F(u), update, and the stopping test ||delta||_H <= tol ||u||_H.
template <int NP>
__global__ __launch_bounds__(kThreads) void lu_f64_kernel(NewtonF64Args a, int it) {
  __shared__ double prow[kWaves][NP + 8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = blockIdx.x * kWaves + wv;
  if (b >= a.B || a.s.done[b]) return;
  const int N = a.N;
  const double* jb = a.s.J + (int64_t)b * a.s.mp;
  const double* ub = a.s.U + (int64_t)b * NP;
  double r[NP];
  const int lc = lane < N ? lane : N - 1;
  double ju = 0.0;
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const double v = jb[(c < N ? c : N - 1) * N + lc];       // clamped: always in bounds
    r[c] = (c < N && lane < N) ? v : (c == lane ? 1.0 : 0.0);
    ju = fma(r[c], ub[c], ju);
    bad |= !finite_val(r[c]);
  }
  double rhs = 0.0;
  if (lane < N) rhs = -(ju - 0.5 * a.s.Wv[(int64_t)b * NP + lane] - a.s.Fv[(int64_t)b * NP + lane]);
  bad |= !finite_val(rhs);
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  double dx = 0.0;
  if (flag == 0) flag = lu_solve_rows<NP>(r, rhs, lane, &prow[wv][0], dx);
  if (flag == 0) {
    const double uo = lane < N ? ub[lane] : 0.0;
    const double un = uo + (lane < N ? dx : 0.0);
    double hd = dx, hu = un;
    if (a.H) {
      hd = 0.0;
      hu = 0.0;
      for (int c = 0; c < N; ++c) {
        const double h = a.H[(int64_t)c * a.Nm + lc];
        hd = fma(h, bcast(dx, c), hd);
        hu = fma(h, bcast(un, c), hu);
      }
    }
    if (lane >= N) { hd = 0.0; hu = 0.0; }
    const double nd2 = wave_sum(dx * hd), nu2 = wave_sum(un * hu);
    if (!finite_val(nd2) || !finite_val(nu2)) flag = 3;
    if (flag == 0) {
      if (lane < N) a.s.U[(int64_t)b * NP + lane] = un;
      if (lane == 0) {
        a.s.iters[b] = it + 1;
        if (sqrt(nd2) <= a.tol * sqrt(nu2)) {
          a.s.status[b] = 0;
          a.s.done[b] = 1;
        }
      }
    }
  }
  if (flag != 0 && lane == 0) {
    a.s.status[b] = flag;
    a.s.done[b] = 1;
  }
}

__global__ void newton_final_kernel(NewtonF64Args a) {
  const int NP = a.s.NP;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < (int64_t)a.B * a.ldu;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / a.ldu;
    const int i = idx - b * a.ldu;
    a.u[idx] = (i < a.N) ? a.s.U[b * NP + i] : 0.0;
    if (i == 0) {
      a.iters[b] = a.s.iters[b];
      a.status[b] = a.s.status[b];
    }
  }
}

__host__ __device__ inline int64_t jac_lds_bytes(int nks, int NP) {
  return 8 * ((int64_t)nks * 4 * kBT + 2 * (int64_t)kBT * NP + kBT * (kMaxQ + kMaxQc));
}

// ------------------------------------------------------------------ pressure (FP64) ---
struct PressureF64Args {
  const double* op;        // packed pressure operand (rows (i,j), m = j*Np + i)
  int nrb, nks_s, nks;
  int N, Np, Nm, Npm, Q, Qc, Qf, Qb, B, ldu, ldp;
  const double* ta;
  const double* tc;
  const double* tf;
  const double* tb;
  const double* u;         // [B][ldu]
  const double* BpT;       // [Qb][Npm][Npm] transposed: BpT[q][c][i] = B_q[i][c]
  const double* Fs;        // [Qf][Npm]
  double* p;               // [B][ldp]
  int* status;             // [B]
};

__host__ __device__ inline int64_t pressure_lds_bytes(int nks, int NPU, int NPP) {
  return 8 * ((int64_t)nks * 4 * kBT + (int64_t)kBT * NPU + (int64_t)kBT * NPP +
              kBT * (kMaxQ + kMaxQc) + kWaves * (NPP + 8));
}

template <int NPP>
__global__ __launch_bounds__(kThreads) void pressure_f64_kernel(PressureF64Args a, int NPU) {
  extern __shared__ double smem[];
  const int K = a.nks * 4;
  double* Wl = smem;                       // [K][kBT]
  double* ul = Wl + K * kBT;               // [kBT][NPU]
  double* rl = ul + kBT * NPU;             // [kBT][NPP] A_sv u + C_sv(u,u)
  double* tal = rl + kBT * NPP;
  double* tcl = tal + kBT * kMaxQ;
  double* prow = tcl + kBT * kMaxQc;       // [kWaves][NPP + 8]

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int b0 = blockIdx.x * kBT;
  const int N = a.N, Np = a.Np;
  const int M = N * Np;
  for (int idx = tid; idx < kBT * NPU; idx += kThreads) {
    const int b = idx / NPU, i = idx - b * NPU, bg = b0 + b;
    ul[idx] = (bg < a.B && i < N) ? a.u[(int64_t)bg * a.ldu + i] : 0.0;
  }
  for (int idx = tid; idx < kBT * NPP; idx += kThreads) rl[idx] = 0.0;
  for (int idx = tid; idx < kBT * kMaxQ; idx += kThreads) {
    const int b = idx / kMaxQ, q = idx - b * kMaxQ, bg = b0 + b;
    tal[idx] = (bg < a.B && q < a.Q) ? a.ta[(int64_t)bg * a.Q + q] : 0.0;
  }
  for (int idx = tid; idx < kBT * kMaxQc; idx += kThreads) {
    const int b = idx / kMaxQc, q = idx - b * kMaxQc, bg = b0 + b;
    tcl[idx] = (bg < a.B && q < a.Qc) ? a.tc[(int64_t)bg * a.Qc + q] : 0.0;
  }
  __syncthreads();
  build_w(Wl, ul, tal, tcl, NPU, N, a.Q, a.Qc, a.nks, a.nks_s);
  __syncthreads();

  const int bcol = lane & 15;
  const double* wp = Wl + (lane >> 4) * kBT + bcol;
  for (int rb = wv; rb < a.nrb; rb += kWaves) {
    const double* opp = a.op + (int64_t)rb * a.nks * 64 + lane;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int ks = 0; ks < a.nks; ++ks)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(opp[ks * 64], wp[ks * 4 * kBT], acc, 0, 0, 0);
    const int m0 = rb * 16 + (lane >> 4);      // lane l, element v: row l/16 + 4v
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + 4 * v;
      if (m < M) {
        const int j = m / Np, i = m - j * Np;
        atomicAdd(&rl[bcol * NPP + i], acc[v] * ul[bcol * NPU + j]);
      }
    }
  }
  __syncthreads();

  for (int b = wv; b < kBT; b += kWaves) {
    const int bg = b0 + b;
    if (bg >= a.B) continue;
    double r[NPP];
    double tbv[kMaxQb];
#pragma unroll
    for (int q = 0; q < kMaxQb; ++q) tbv[q] = q < a.Qb ? a.tb[(int64_t)bg * a.Qb + q] : 0.0;
#pragma unroll
    for (int c = 0; c < NPP; ++c) {
      double s = 0.0;
      if (c < Np && lane < Np) {
        for (int q = 0; q < a.Qb; ++q)
          s = fma(tbv[q], a.BpT[((int64_t)q * a.Npm + c) * a.Npm + lane], s);
      } else if (c == lane) {
        s = 1.0;
      }
      r[c] = s;
    }
    double rhs = 0.0;
    if (lane < Np) {
      for (int q = 0; q < a.Qf; ++q)
        rhs = fma(a.tf[(int64_t)bg * a.Qf + q], a.Fs[(int64_t)q * a.Npm + lane], rhs);
      rhs -= rl[b * NPP + lane];
    }
    bool bad = !finite_val(rhs);
#pragma unroll
    for (int c = 0; c < NPP; ++c) bad |= !finite_val(r[c]);
    int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
    double x = 0.0;
    if (flag == 0) flag = lu_solve_rows<NPP>(r, rhs, lane, prow + wv * (NPP + 8), x);
    if (flag == 0 && !finite_val(wave_sum(x))) flag = 3;
    for (int i = lane; i < a.ldp; i += kWave)
      a.p[(int64_t)bg * a.ldp + i] = (flag == 0 && i < Np) ? (i == lane ? x : 0.0) : 0.0;
    if (lane == 0) a.status[bg] = flag;
  }
}

}  // namespace rb
