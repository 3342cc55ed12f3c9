// rb_kernels.hpp -- gfx950 kernels of the online reduced Navier-Stokes solver (FP64 path).
//
// One Newton step of a batch of same-N requests is two launches (Sections 3.4, 3.5):
//   * contract_f64_kernel: the Jacobian and affine contraction on MFMA,
//       J[(j,i), b] = sum_k Op[(j,i), k] W[k, b],  Op = [ A_flat | S_flat ],
//       S_q[i,j,l] = C_q[i,j,l] + C_q[i,l,j],  W = [ theta^a_q(b) ; theta^c_q(b) u_l(b) ],
//     one GEMM of shape N^2 x (Q + Qc N) x B per step, the operand pre-packed in MFMA order
//     so that every wavefront load is one contiguous 512-byte line; its epilogue also folds
//     the affine accumulator with u into A(mu) u, from which the LU kernel forms the residual
//     F(u) = (J u + A(mu) u)/2 - f without a second pass over the tensors (J u = A u + 2
//     C(u,u) for the symmetrised tensor part). The same kernel, with other epilogues, gives
//     the FP64 residual of the mixed-precision refinement and the pressure right-hand side.
//   * lu_f64_kernel: one wavefront per request, one row per lane in registers, partial
//     pivoting (wavefront argmax), pivot-row broadcast by readlane, update of the FP64
//     iterate and the stopping test; lu_f64_mw_kernel spreads larger systems over a workgroup.
// Requests that have converged are skipped by both kernels through per-request flags.
#pragma once

#include <type_traits>

#include "rb_common.hpp"

namespace rb {

constexpr int kWaves = 4;      // wavefronts per workgroup
constexpr int kThreads = kWave * kWaves;
// Lengths of the trigonometric theta lists (longer expansions take the power families; the
// low-precision contraction holds these many theta values per request in registers).
constexpr int kMaxQ = 12, kMaxQc = 4, kMaxQf = 2, kMaxQb = 2;

// ------------------------------------------------------------------ packing -----------
// Packed operand layout for v_mfma_f64_16x16x4f64 (A operand: lane l holds row l%16,
// k-column l/16 of a 16x4 tile): tile (rb, ks) = 64 consecutive doubles at
// ((rb * nks + ks) * 64), element e <-> (row rb*16 + e%16, k = ks*4 + e/16).
// The k range of every row block is [ affine part: kA = ceil(Q/4) k-steps | tensor part:
// KT k-steps = ceil(Qc*N/4) rounded up to even, zero padded ].
// Solve operand rows: m = j*N + i (J is written column-major per request); columns:
// k < Q -> A_q[i,j] (q = k); k = 4*kA + q*N + l -> S_q[i,j,l] = C_q[i,j,l] + C_q[i,l,j].
// Pressure operand rows: m = j*Np + i; affine part A_sv, tensor part the unsymmetrised C_sv
// (the epilogue contracts with u_j, giving A_sv u + C_sv(u,u)).
template <bool kSolve>
__global__ void pack_f64(const double* __restrict__ T3, const double* __restrict__ T2,
                         int Nm, int Npm, int N, int R, int Q, int Qc, int kA, int nrb, int nks,
                         double* __restrict__ out) {
  const int64_t total = (int64_t)nrb * nks * 64;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int e = idx & 63;
    const int64_t tile = idx >> 6;
    const int rb = tile / nks, ks = tile % nks;
    const int m = rb * 16 + (e & 15), k = ks * 4 + (e >> 4);
    double v = 0.0;
    if (m < N * R) {
      const int j = m / R, i = m - j * R;
      const int Rm = kSolve ? Nm : Npm;        // stored row count of the test index
      if (k < 4 * kA) {
        if (k < Q) v = T2[((int64_t)k * Rm + i) * Nm + j];
      } else if (k - 4 * kA < Qc * N) {
        const int kk = k - 4 * kA, q = kk / N, l = kk - q * N;
        v = T3[(((int64_t)q * Rm + i) * Nm + j) * Nm + l];
        if (kSolve) v += T3[(((int64_t)q * Rm + i) * Nm + l) * Nm + j];
      }
    }
    out[idx] = v;
  }
}

// ------------------------------------------------------------------ theta(mu) ---------
static __global__ void theta_kernel(const double* __restrict__ mu, int B, int Q, int Qc, int Qf,
                             int Qb, double* __restrict__ ta, double* __restrict__ tc,
                             double* __restrict__ tf, double* __restrict__ tb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double a = mu[2 * b], re = mu[2 * b + 1];
  const double ca = cos(a), sa = sin(a), h = sin(0.5 * a);
  const double la[kMaxQ] = {1.0 / re, ca, sa, a, a * a, a * a * a, cos(2.0 * a),
                            sin(2.0 * a), 2.0 * h * h, a * a * a * a, a * ca, a * sa};
  const double lc[kMaxQc] = {1.0, ca, sa, a};
  // Longer expansions are the Piola-mapped forms' truncated power series in the angle
  // (Section 5): theta^a_q = a^q / Re (viscous), theta^c_q = a^q.
  double pw = 1.0 / re;
  for (int q = 0; q < Q; ++q) {
    ta[(int64_t)b * Q + q] = Q <= kMaxQ ? la[q] : pw;
    pw *= a;
  }
  pw = 1.0;
  for (int q = 0; q < Qc; ++q) {
    tc[(int64_t)b * Qc + q] = Qc <= kMaxQc ? lc[q] : pw;
    pw *= a;
  }
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
// Per-call device state of a batch solve (padded to whole 64-request tiles):
//   U [Bp][NP] current iterates, Fv [Bp][NP] right-hand sides f(mu), Wv partial A(mu) u,
//   J [Bp][mp] Jacobians (column-major, mp >= N*N), done/iters/status [Bp].
struct NewtonState {
  double* U;
  double* Fv;
  double* Wv;              // [nsplit][Bp][NP] partial sums of A(mu) u
  int64_t Bp;
  double* J;
  int* done;
  int* iters;
  int* status;
  double* dprev;           // previous update norm (stagnation test of the low-precision phase)
  int64_t mp;
  int NP;
  int nsplit;              // partial sums per request in Wv / the mixed-precision partials
};

struct NewtonF64Args {
  const double* op;        // packed solve operand
  int nrb, nks_s, nks;     // row blocks, affine k-steps, total k-steps
  int nchunk;              // tensor chunks
  int naff;                // affine chunks (long expansions; 0: affine part of kAmax k-steps)
  int N, Nm, Q, Qc, Qf, B, ldu, maxit;
  double tol;
  const double* ta;        // [B][Q]
  const double* tc;        // [B][Qc]
  const double* tf;        // [B][Qf] (used when fover == nullptr)
  const double* fover;     // [B][ldu] or nullptr
  const double* u0;        // [B][ldu] or nullptr
  const int* nreq;         // [B] basis size of each request (<= N, the leading block of the
                           // group's size-N system; the rest is held at zero), or nullptr
  const double* F;         // [Qf][Nm]
  const double* H;         // [Nm][Nm] or nullptr
  double* u;               // [B][ldu]
  int* iters;              // [B]
  int* status;             // [B]
  int* max_iters;          // largest iteration count of the batch (written by the final
                           // kernel into pinned host memory), or nullptr
  NewtonState s;
};

// First Newton step from u = 0 (no initial iterates given): the convection terms of the
// Jacobian J(u) = A(mu) + C(., u) + C(u, .) vanish (Section 3.5), so J = sum_q theta^a_q A_q
// is assembled from the Q affine operators alone instead of by the contraction over the
// whole tensor, and the partial sums of A(mu) u are zero; the step is the Stokes solve.
// The operators are read from the affine k-steps of the packed operand, where row m = j N + i
// of A_q sits at ((m/16) nks + q/4) 64 + (q%4) 16 + m%16 (16 consecutive rows per 128 bytes),
// and J is stored as the contraction stores it (J[b][m] = A(mu)[i][j]). Workgroup (x, y) takes
// requests 16x .. 16x + 15 and rows 256y .. 256y + 255: each thread reads its row of A_q once
// per q for 16 requests (theta^a uniform across the workgroup), the stores of a request are
// contiguous. Sums run over q in order from zero, so every request gets the same J.
constexpr int kStokesReq = 16;

template <typename T>
__device__ __forceinline__ void stokes_tile(const NewtonF64Args& a, T* J, int64_t mp, T* part,
                                            int64_t npart) {
  const int NN = a.N * a.N, Q = a.Q;
  const int m = blockIdx.y * 256 + threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * kStokesReq;
  if (m < NN) {
    const double* op = a.op + (int64_t)(m >> 4) * a.nks * 64 + (m & 15);
    double acc[kStokesReq];
#pragma unroll
    for (int r = 0; r < kStokesReq; ++r) acc[r] = 0.0;
    int q = 0;
    for (; q + 4 <= Q; q += 4) {           // one k-step (four operators) at a time
      double x[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) x[j] = op[(q >> 2) * 64 + 16 * j];
#pragma unroll
      for (int r = 0; r < kStokesReq; ++r) {
        const int64_t b = b0 + r < a.B ? b0 + r : a.B - 1;
        const double* t = a.ta + b * Q + q;
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[r] = fma(t[j], x[j], acc[r]);
      }
    }
    for (; q < Q; ++q) {
      const double x = op[(q >> 2) * 64 + ((q & 3) << 4)];
#pragma unroll
      for (int r = 0; r < kStokesReq; ++r) {
        const int64_t b = b0 + r < a.B ? b0 + r : a.B - 1;
        acc[r] = fma(a.ta[b * Q + q], x, acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < kStokesReq; ++r)
      if (b0 + r < a.B) J[(b0 + r) * mp + m] = static_cast<T>(acc[r]);
  }
  // zero partial sums of A(mu) u
  const int64_t nthr = (int64_t)gridDim.x * gridDim.y * blockDim.x;
  for (int64_t idx = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
       idx < npart; idx += nthr)
    part[idx] = T(0);
}

__host__ inline dim3 stokes_grid(int B, int N) {
  return dim3((unsigned)((B + kStokesReq - 1) / kStokesReq), (unsigned)((N * N + 255) / 256));
}

static __global__ __launch_bounds__(256) void stokes_jacobian_kernel(NewtonF64Args a) {
  stokes_tile<double>(a, a.s.J, a.s.mp, a.s.Wv, (int64_t)a.s.nsplit * a.s.Bp * a.s.NP);
}

// Start of a batch solve: iterates from u0 (or 0), f(mu) (or the override), flags.
static __global__ void newton_init_kernel(NewtonF64Args a) {
  const int64_t Bp = a.s.Bp;
  const int NP = a.s.NP, N = a.N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < Bp * NP;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / NP;
    const int i = idx - b * NP;
    double uv = 0.0, fv = 0.0;
    const int nb = (a.nreq && b < a.B) ? a.nreq[b] : N;
    if (b < a.B && i < nb) {
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

// ------------------------------------------------------------------ contraction ------
// One MFMA-F64 contraction kernel serves the Jacobian of a Newton step, the FP64 residual of
// the mixed-precision refinement and the pressure right-hand side. Workgroup g handles the
// 64-request tile g / nsplit and the row split g % nsplit (nsplit is a tuning knob, 8 by
// default); with round-robin dispatch over the 8 XCDs and nsplit = 8 every workgroup of one
// XCD reads the same eighth of the packed operand, which therefore stays in that XCD's L2.
// Wavefront w of the workgroup owns requests 16w..16w+15 of the tile and keeps its slice of
// W (the B operand: the affine k-steps and one chunk of at most kMaxKC tensor k-steps) in
// registers, so the main loop touches no LDS; the four wavefronts walk the same row blocks in
// the same order and share each A tile (one 512-byte line per k-step and row block) through
// L1. Row blocks go kGroup at a time; every k-step issues their A loads kDepth k-steps ahead
// and kGroup v_mfma_f64_16x16x4f64. The k loop is unrolled at its compile-time length, and the
// loads of the next group of row blocks are issued during the tail of the current one, so the
// pipeline does not drain between groups. The affine part is padded to kAmax = 3 k-steps
// (zero columns) so that every row block has the same static pipeline. Tensor parts longer
// than kMaxKC k-steps run as nchunk chunks, each walking the row blocks again with fresh
// accumulators; the Jacobian adds each later chunk to what the earlier ones stored (the lane
// that stores a J piece in one chunk is the one that reads and updates it in the next, and it
// loads the old piece at the start of the row group, so the read is off the critical path). Long
// affine expansions (Q > 12, the Piola-mapped forms of Section 5) go in naff chunks of their
// own in front of the tensor chunks, with the same chunk length, and the affine accumulator
// is folded at the end of those passes.
//
// Rows are m = j*R + i (R = N for the solve operand, R = Np for the pressure one). The
// epilogue folds acc[m, b] * u_j(b) into per-row sums p_i(b) in LDS:
//   Jacobian: the affine accumulator (A(mu) u; with J u the LU kernel forms
//             F(u) = (J u + A u)/2 - f); each 16x16 accumulator tile is transposed through
//             a small per-wavefront LDS stage so that J goes out column-major per request
//             (mp doubles per request) in 128-byte pieces;
//   residual: affine accumulator with weight 1, tensor accumulators with weight 1/2, so
//             p = A(mu) u + C(mu)(u,u)  (the tensor part applied to u is 2 C(u,u));
//   pressure: every accumulator with weight 1, p = A_sv u + C_sv(u,u).
// Each workgroup writes its split's partial sums; the solve kernels add the nsplit partials.
constexpr int kTile = 64;      // requests per workgroup tile (16 per wavefront)
constexpr int kSplit = 8;      // default row splits, one per XCD
constexpr int kMaxSplit = 64;  // largest split count (small batches split rows further)
constexpr int kGroup = 2;      // row blocks per wavefront pass
constexpr int kDepth = 6;      // k-steps of A operand in flight
constexpr int kMaxKC = 40;     // longest tensor chunk held in registers (no spills at 2 waves/SIMD)
constexpr int kAmax = 3;       // affine k-steps of every packed row block (Q <= 12)

struct ContractArgs {
  const double* op;        // packed operand [nrb][nks][64], nks = kA + nchunk*KC
  int nrb, nks, kA;        // row blocks, k-steps per row block, affine k-steps (kAmax, or
                           // naff*KC for long expansions)
  int nchunk;              // tensor chunks of KC k-steps
  int naff;                // affine chunks of KC k-steps (0: the kAmax affine k-steps ride
                           // in front of the first tensor chunk)
  int nsplit;              // row splits per tile (1..kMaxSplit)
  int R, N, M;             // rows m = j*R + i, M = R*N
  int Q, Qc, B;
  int64_t Bp;              // padded request count (multiple of kTile)
  const double* ta;        // [B][Q]
  const double* tc;        // [B][Qc]
  const double* U;         // iterates, row b at U + b*ldU (rows >= B are not read)
  int ldU;
  const int* done;         // Newton flags [Bp] or nullptr
  double* J;               // Jacobians [Bp][mp] (column-major per request), or nullptr
  int64_t mp;
  double* part;            // partial row sums [nsplit][Bp][ldp]
  int ldp;
};

// LDS: the tile's iterates [kTile][N], row sums [kTile][R] and, for the Jacobian, the
// transpose stage [kWaves][16][kStageLd].
constexpr int kStageLd = 20;   // padded row of the stage (16-byte aligned, spreads banks)
__host__ __device__ inline int64_t contract_lds_bytes(int N, int R, bool jac) {
  return 8 * ((int64_t)kTile * (N + R) + (jac ? kWaves * 16 * kStageLd : 0));
}

constexpr int kModeJac = 0, kModePressure = 1, kModeResid = 2;

template <int kMode, int KC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void contract_f64_kernel(ContractArgs a) {
  extern __shared__ double smem[];
  const int N = a.N, R = a.R;
  double* ul = smem;                       // [kTile][N]
  double* pl = ul + kTile * N;             // [kTile][R]

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int split = blockIdx.x % a.nsplit;
  const int b0 = (blockIdx.x / a.nsplit) * kTile;
  if (a.done && __syncthreads_and(tid < kTile ? a.done[b0 + tid] : 1)) return;

  for (int idx = tid; idx < kTile * N; idx += kThreads) {
    const int b = idx / N, l = idx - b * N, bg = b0 + b;
    ul[idx] = bg < a.B ? a.U[(int64_t)bg * a.ldU + l] : 0.0;
  }
  for (int idx = tid; idx < kTile * R; idx += kThreads) pl[idx] = 0.0;

  // This lane's B-operand column: request bl = 16*wv + lane%16, k = ks*4 + lane/16.
  // Affine rows k < 4*kAmax: theta^a_k (0 beyond Q); tensor row t = q*N + l: theta^c_q u_l.
  const int bl = 16 * wv + (lane & 15);
  const int bg = b0 + bl;
  const int k0 = lane >> 4;
  double wa[kAmax];
#pragma unroll
  for (int ks = 0; ks < kAmax; ++ks) {
    const int k = ks * 4 + k0;
    wa[ks] = (bg < a.B && k < a.Q) ? a.ta[(int64_t)bg * a.Q + k] : 0.0;
  }
  __syncthreads();

  const int rb_lo = (int)((int64_t)split * a.nrb / a.nsplit);
  const int rb_hi = (int)((int64_t)(split + 1) * a.nrb / a.nsplit);
  const int col = bl;                      // accumulator column (request) of this lane
  double* stg = pl + kTile * R + wv * 16 * kStageLd;   // this wavefront's stage

  // Accumulator layout of v_mfma_f64_16x16x4f64: lane l, element v = row l/16 + 4v,
  // column l%16 of the 16x16 tile. fold(): wt * acc[m] * u_j into p_i for m = j*R + i.
  auto fold = [&](const f64x4 (&c)[kGroup], int g0, double wt) {
    const int m0 = g0 * 16 + (lane >> 4);
    const int j0 = m0 / R, i0 = m0 - j0 * R;
#pragma unroll
    for (int r = 0; r < kGroup; ++r) {
      if (g0 + r < rb_hi) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          int i = i0 + 16 * r + 4 * v, j = j0;
          while (i >= R) { i -= R; ++j; }
          if (j < N) atomicAdd(&pl[col * R + i], wt * c[r][v] * ul[col * N + j]);
        }
      }
    }
  };

  // One pass over this split's row blocks for the k-steps [k_first, k_first + NKS) of every
  // packed row block, with W values w[0..NKS). end_wt: weight of the accumulator folded into
  // the row sums at the end of each row block (the Jacobian folds only the affine chunks of a
  // long expansion, and writes its slice of J either way).
  auto pass = [&](auto nks_c, const double* w, int k_first, int chunk, double end_wt) {
    constexpr int NKS = decltype(nks_c)::value;
    constexpr bool kAff = NKS == kAmax + KC;   // this pass starts with the affine k-steps
    if (rb_lo >= rb_hi) return;            // no row blocks in this split: load nothing
    auto row_ptr = [&](int rb) {
      return a.op + (int64_t)min(rb, rb_hi - 1) * a.nks * 64 + (int64_t)k_first * 64 + lane;
    };
    double x[NKS + kDepth][kGroup];
#pragma unroll
    for (int ks = 0; ks < kDepth; ++ks)
#pragma unroll
      for (int r = 0; r < kGroup; ++r) x[ks][r] = row_ptr(rb_lo + r)[ks * 64];
    for (int g0 = rb_lo; g0 < rb_hi; g0 += kGroup) {
      const double* cur[kGroup];
      const double* nxt[kGroup];
#pragma unroll
      for (int r = 0; r < kGroup; ++r) {
        cur[r] = row_ptr(g0 + r);
        nxt[r] = row_ptr(g0 + kGroup + r);
      }
      f64x4 c[kGroup];
#pragma unroll
      for (int r = 0; r < kGroup; ++r) c[r] = f64x4{0.0, 0.0, 0.0, 0.0};
      // Jacobian pieces of this group stored by the earlier chunks (this lane's own stores)
      f64x4* jp[kGroup];
      f64x4 jold[kGroup];
      if (kMode == kModeJac) {
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
          jp[r] = reinterpret_cast<f64x4*>(a.J + (int64_t)(b0 + 16 * wv + (lane >> 2)) * a.mp +
                                           (g0 + r) * 16 + 4 * (lane & 3));
          jold[r] = (chunk > 0 && g0 + r < rb_hi) ? *jp[r] : f64x4{0.0, 0.0, 0.0, 0.0};
        }
      }
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const int pf = ks + kDepth;
#pragma unroll
        for (int r = 0; r < kGroup; ++r)
          x[pf][r] = pf < NKS ? cur[r][pf * 64] : nxt[r][(pf - NKS) * 64];
#pragma unroll
        for (int r = 0; r < kGroup; ++r)
          c[r] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[ks][r], w[ks], c[r], 0, 0, 0);
        if (kAff && ks == kAmax - 1 && kMode != kModePressure) {
          fold(c, g0, 1.0);                // A(mu) u
          if (kMode == kModeResid) {
#pragma unroll
            for (int r = 0; r < kGroup; ++r) c[r] = f64x4{0.0, 0.0, 0.0, 0.0};
          }
        }
      }
#pragma unroll
      for (int t = 0; t < kDepth; ++t)
#pragma unroll
        for (int r = 0; r < kGroup; ++r) x[t][r] = x[NKS + t][r];
      if (kMode == kModeJac) {
        if (end_wt != 0.0) fold(c, g0, end_wt);
        // stage [request][row] -> lane l takes request l/4, rows 4*(l%4)..+3 of the block
        const int q2 = lane >> 2, e0 = 4 * (lane & 3);
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
#pragma unroll
          for (int v = 0; v < 4; ++v) stg[(lane & 15) * kStageLd + (lane >> 4) + 4 * v] = c[r][v];
          wave_lds_order();
          const f64x4 val = *reinterpret_cast<const f64x4*>(&stg[q2 * kStageLd + e0]);
          wave_lds_order();
          if (g0 + r < rb_hi) *jp[r] = val + jold[r];   // cached: the LU kernel reads J next
        }
      } else {
        fold(c, g0, end_wt);
      }
    }
  };

  const double* ub = ul + bl * N;
  // theta^c_q of this lane's request (read when q changes along the k range)
  auto tcq = [&](int q) {
    return (bg < a.B && q < a.Qc) ? a.tc[(int64_t)bg * a.Qc + q] : 0.0;
  };
  const double tens_wt = kMode == kModeJac ? 0.0 : (kMode == kModeResid ? 0.5 : 1.0);
  for (int ch = 0; ch < a.naff + a.nchunk; ++ch) {
    double w[kAmax + KC];
    if (ch < a.naff) {                     // affine chunk of a long expansion: W = theta^a
#pragma unroll
      for (int ks = 0; ks < KC; ++ks) {
        const int k = (ch * KC + ks) * 4 + k0;
        w[kAmax + ks] = (bg < a.B && k < a.Q) ? a.ta[(int64_t)bg * a.Q + k] : 0.0;
      }
      pass(std::integral_constant<int, KC>{}, w + kAmax, ch * KC, ch, 1.0);
      continue;
    }
    const int tch = ch - a.naff;            // tensor chunk: W = theta^c_q u_l, t = q*N + l
    {
      int t = tch * KC * 4 + k0, q = 0;
      while (t >= N && q < a.Qc) { t -= N; ++q; }
      double th = tcq(q);
#pragma unroll
      for (int ks = 0; ks < KC; ++ks) {
        w[kAmax + ks] = q < a.Qc ? th * ub[t] : 0.0;   // padding k-steps: W = 0
        t += 4;
        while (t >= N && q < a.Qc) {
          t -= N;
          ++q;
          th = tcq(q);
        }
        if (q >= a.Qc) t = 0;
      }
    }
    if (a.naff == 0 && ch == 0) {
#pragma unroll
      for (int ks = 0; ks < kAmax; ++ks) w[ks] = wa[ks];
      pass(std::integral_constant<int, kAmax + KC>{}, w, 0, 0, tens_wt);
    } else {
      pass(std::integral_constant<int, KC>{}, w + kAmax, a.kA + tch * KC, ch, tens_wt);
    }
  }
  __syncthreads();
  for (int idx = tid; idx < kTile * R; idx += kThreads) {
    const int b = idx / R, i = idx - b * R;
    a.part[((int64_t)split * a.Bp + b0 + b) * a.ldp + i] = pl[idx];
  }
}

// One wavefront per request: residual F(u) = (J u + A u)/2 - f, pivoted LU solve of
// J delta = -F(u), update, and the stopping test ||delta||_H <= tol ||u||_H.
// The Newton step of request b (wave-uniform, b < B, not done) by the calling wavefront;
// prow: NP + 8 doubles of LDS owned by the wavefront.
template <int NP, bool kLdsBcast>
__device__ __forceinline__ void lu_f64_request(const NewtonF64Args& a, int it, int b,
                                               double* prow) {
  const int lane = threadIdx.x & 63;
  const int N = a.N;
  const int nb = a.nreq ? a.nreq[b] : N;   // this request's size; rows/columns beyond: identity
  const double* jb = a.s.J + (int64_t)b * a.s.mp;
  const double* ub = a.s.U + (int64_t)b * NP;
  double r[NP];
  const int lc = lane < N ? lane : N - 1;
  double ju = 0.0;
  bool bad = false;
  // J row of this lane, padded to identity beyond the request's size; loads clamped in bounds.
#pragma unroll
  for (int c0 = 0; c0 < NP; c0 += 8) {
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      if (c0 + t < NP) v[t] = jb[(c0 + t < N ? c0 + t : N - 1) * N + lc];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int c = c0 + t;
      if (c < NP) r[c] = (c < nb && lane < nb) ? v[t] : (c == lane ? 1.0 : 0.0);
    }
  }
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    ju = fma(r[c], ub[c], ju);
    bad |= !finite_val(r[c]);
  }
  double rhs = 0.0;
  if (lane < nb) {
    double w = 0.0;
#pragma unroll
    for (int sp = 0; sp < a.s.nsplit; ++sp) w += a.s.Wv[((int64_t)sp * a.s.Bp + b) * NP + lane];
    rhs = -(0.5 * (ju + w) - a.s.Fv[(int64_t)b * NP + lane]);   // F(u) = (J u + A u)/2 - f
  }
  bad |= !finite_val(rhs);
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  double dx = 0.0;
  if (flag == 0) flag = lu_solve_rows<NP, kLdsBcast>(r, rhs, lane, prow, dx);
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

template <int NP, bool kLdsBcast>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(!kLdsBcast && NP <= 56 ? 4 : 1)))
void lu_f64_kernel(NewtonF64Args a, int it) {
  __shared__ double prow[kWaves][NP + 8];
  const int wv = threadIdx.x >> 6;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);   // wave-uniform
  if (b >= a.B || a.s.done[b]) return;
  lu_f64_request<NP, kLdsBcast>(a, it, b, &prow[wv][0]);
}

// NP > 64: one request per workgroup of W wavefronts (Gauss-Jordan over the workgroup).
template <int NP, int W>
__global__ __launch_bounds__(kWave * W) void lu_f64_mw_kernel(NewtonF64Args a, int it) {
  __shared__ GjShared<NP, W, double> sh;
  const int b = blockIdx.x;
  if (a.s.done[b]) return;
  const int N = a.N;
  const double* jb = a.s.J + (int64_t)b * a.s.mp;
  auto jload = [&](int c, int row) { return jb[c * N + row]; };
  double* ub = a.s.U + (int64_t)b * NP;
  auto rhs_of = [&](int row, double ju) {
    double w = 0.0;
#pragma unroll
    for (int sp = 0; sp < a.s.nsplit; ++sp) w += a.s.Wv[((int64_t)sp * a.s.Bp + b) * NP + row];
    return -(0.5 * (ju + w) - a.s.Fv[(int64_t)b * NP + row]);
  };
  double nd2, nu2;
  const int nb = a.nreq ? a.nreq[b] : N;
  const int flag = mw_newton_update<double, NP, W>(jload, nb, a.Nm, ub, a.H, rhs_of,
                                                   sh, nd2, nu2);
  if (threadIdx.x != 0) return;
  if (flag != 0) {
    a.s.status[b] = flag;
    a.s.done[b] = 1;
    return;
  }
  a.s.iters[b] = it + 1;
  if (sqrt(nd2) <= a.tol * sqrt(nu2)) {
    a.s.status[b] = 0;
    a.s.done[b] = 1;
  }
}

// (launched with 256-thread blocks)
static __global__ void newton_final_kernel(NewtonF64Args a) {
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
  if (a.max_iters && blockIdx.x == 0) {    // the batch's largest count, by block 0 alone
    __shared__ uint32_t wmax[4];
    uint32_t most = 0;
    for (int b = threadIdx.x; b < a.B; b += blockDim.x) most = max(most, (uint32_t)a.s.iters[b]);
    most = wave_max_u32(most);
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = most;
    __syncthreads();
    if (threadIdx.x == 0) {                // pinned host word: made visible system-wide
      *a.max_iters = (int)max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
      __threadfence_system();
    }
  }
}

// ------------------------------------------------------------------ uneven batches ----
// Staging of an uneven batch: requests regrouped by basis size (perm[r] = source request of
// staging row r, -1 for padding rows, which get zero coefficients and so stop at once).
struct UnevenIo {
  int64_t Bs;              // staging rows (same-N groups, each padded to whole tiles)
  int nbad;                // requests with an invalid N, listed at perm[Bs..Bs+nbad)
  const int* perm;
  int Q, Qc, Qf, Nm, ldu;
  const double* ta;        // caller arrays [B][...]
  const double* tc;
  const double* tf;
  const double* fover;     // [B][ldu] or nullptr
  const double* u0;        // [B][ldu] or nullptr
  double* ta_s;            // staging [Bs][Q], [Bs][Qc], [Bs][Qf] or [Bs][Nm], [Bs][Nm]
  double* tc_s;
  double* f_s;
  double* u0_s;
  double* u_s;             // staging results [Bs][Nm], iters / status [Bs]
  int* it_s;
  int* st_s;
  double* u;               // caller results [B][ldu], [B], [B]
  int* iters;
  int* status;
  const double* tb;        // pressure coefficients theta^b [B][Qb] or nullptr
  double* tb_s;            // staging [Bs][Qb]
  int Qb;
};

static __global__ void uneven_gather_kernel(UnevenIo g) {
  const int wf = g.Q + g.Qc + (g.fover ? 0 : g.Qf);
  const int w = wf + (g.tb ? g.Qb : 0);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < g.Bs * w; idx += stride) {
    const int64_t r = idx / w;
    const int k = idx - r * w;
    const int b = g.perm[r];
    if (k < g.Q) g.ta_s[r * g.Q + k] = b >= 0 ? g.ta[(int64_t)b * g.Q + k] : 0.0;
    else if (k < g.Q + g.Qc) g.tc_s[r * g.Qc + k - g.Q] = b >= 0 ? g.tc[(int64_t)b * g.Qc + k - g.Q] : 0.0;
    else if (k < wf) g.f_s[r * g.Qf + k - g.Q - g.Qc] = b >= 0 ? g.tf[(int64_t)b * g.Qf + k - g.Q - g.Qc] : 0.0;
    else g.tb_s[r * g.Qb + k - wf] = b >= 0 ? g.tb[(int64_t)b * g.Qb + k - wf] : 0.0;
  }
  if (!g.fover && !g.u0) return;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < g.Bs * g.Nm; idx += stride) {
    const int64_t r = idx / g.Nm;
    const int i = idx - r * g.Nm;
    const int b = g.perm[r];
    if (g.fover) g.f_s[idx] = b >= 0 ? g.fover[(int64_t)b * g.ldu + i] : 0.0;
    if (g.u0) g.u0_s[idx] = b >= 0 ? g.u0[(int64_t)b * g.ldu + i] : 0.0;
  }
}

static __global__ void uneven_scatter_kernel(UnevenIo g) {
  const int64_t rows = g.Bs + g.nbad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < rows * g.ldu;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx / g.ldu;
    const int i = idx - r * g.ldu;
    const int b = g.perm[r];
    if (b < 0) continue;
    const bool ok = r < g.Bs;
    g.u[(int64_t)b * g.ldu + i] = (ok && i < g.Nm) ? g.u_s[r * g.Nm + i] : 0.0;
    if (i == 0) {
      g.iters[b] = ok ? g.it_s[r] : 0;
      g.status[b] = ok ? g.st_s[r] : 4;
    }
  }
}

// ------------------------------------------------------------------ pressure (FP64) ---
// One wavefront per request: rhs = f_s(mu) - (A_sv u + C_sv(u,u)) (the contraction kernel's
// partial sums), B(mu) = sum_q theta^b_q B_q, pivoted LU solve B(mu) p = rhs.
struct PressureF64Args {
  int Np, Npm, Qf, Qb, B, ldp;
  int64_t Bp;
  const double* tf;        // [B][Qf]
  const double* tb;        // [B][Qb]
  const double* BpT;       // [Qb][Npm][Npm] transposed: BpT[q][c][i] = B_q[i][c]
  const double* Fs;        // [Qf][Npm]
  const double* part;      // [nsplit][Bp][ldpart] partial sums of A_sv u + C_sv(u,u)
  int nsplit;
  int ldpart;              // row stride of the partial sums (the row bucket NPP)
  double* p;               // [B][ldp]
  int* status;             // [B]
};

template <int NPP, bool kLdsBcast>
__global__ __launch_bounds__(kThreads) void plu_f64_kernel(PressureF64Args a) {
  __shared__ double prow[kWaves][NPP + 8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);   // wave-uniform
  if (b >= a.B) return;
  const int Np = a.Np;
  const int lc = lane < Np ? lane : Np - 1;
  double tbv[kMaxQb];
#pragma unroll
  for (int q = 0; q < kMaxQb; ++q) tbv[q] = q < a.Qb ? a.tb[(int64_t)b * a.Qb + q] : 0.0;
  double r[NPP];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NPP; ++c) {
    const int cc = c < Np ? c : Np - 1;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxQb; ++q)
      if (q < a.Qb) s = fma(tbv[q], a.BpT[((int64_t)q * a.Npm + cc) * a.Npm + lc], s);
    r[c] = (c < Np && lane < Np) ? s : (c == lane ? 1.0 : 0.0);
    bad |= !finite_val(r[c]);
  }
  double rhs = 0.0;
  if (lane < Np) {
    for (int q = 0; q < a.Qf; ++q) rhs = fma(a.tf[(int64_t)b * a.Qf + q], a.Fs[(int64_t)q * a.Npm + lane], rhs);
#pragma unroll
    for (int sp = 0; sp < a.nsplit; ++sp) rhs -= a.part[((int64_t)sp * a.Bp + b) * NPP + lane];
  }
  bad |= !finite_val(rhs);
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  double x = 0.0;
  if (flag == 0) flag = lu_solve_rows<NPP, kLdsBcast>(r, rhs, lane, &prow[wv][0], x);
  if (flag == 0 && !finite_val(wave_sum(lane < Np ? x : 0.0))) flag = 3;
  for (int i = lane; i < a.ldp; i += kWave)
    a.p[(int64_t)b * a.ldp + i] = (flag == 0 && i < Np) ? x : 0.0;
  if (lane == 0) a.status[b] = flag;
}

}  // namespace rb
