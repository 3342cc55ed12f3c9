// rb_mfma_lu.hpp -- dense pivoted solve of one small FP64 system per wavefront with the
// trailing updates on the matrix cores (v_mfma_f64_16x16x4f64).
//
// The reduced Newton system J delta = -F(u) and the pressure system B(mu) p = rhs are dense,
// with at most a few dozen unknowns (Section 3.5). Solving them one row per lane costs, for
// every eliminated entry, an FMA plus a cross-lane broadcast of the pivot-row value; here the
// elimination is blocked by panels of four columns instead, so that all the broadcasting of
// a panel's update is done by one 16x16x4 MFMA per 16x16 tile.
//
// Layout. The system is padded to P = 16*NT rows and columns (identity rows beyond N, the
// right-hand side in column P-1) and held in registers as NT x NT tiles in the MFMA
// accumulator layout: lane l, element v of tile (a, b) is X[16a + l%16][16b + l/16 + 4v]
// (the accumulator of the transposed tile). Row r lives in the four lanes with l%16 = r%16,
// column c in the sixteen lanes with l/16 = c%4.
//
// Panel step (columns 4p .. 4p+3, Gauss-Jordan with partial pivoting):
//   1. the panel's four columns go through LDS to one row per lane;
//   2. four pivot steps on the panel rows, the pivot being the one partial pivoting picks (the
//      largest magnitude among the rows not yet pivoted, ties to the smallest position under
//      the row swaps), eliminating the column from every other row and scaling the pivot row
//      to 1. Each row tracks coefficients z[s] with which its new value is
//      X[r] + sum_s z[s] X[P_s], X[P_s] being the pivot rows at the start of the panel;
//   3. the z's go through LDS into the B operand, the four pivot rows into the A operand, and
//      one MFMA per tile right of the panel applies X[r] += sum_s z_r[s] X[P_s] to every row.
// No rows move between lanes. After the last panel the pivot row of column k holds x_k in
// column P-1. The pivots are those of partial pivoting on the same matrix (same candidates,
// same tie rule), so the result agrees with the oracle's GEPP to rounding.
#pragma once

#include "rb_kernels.hpp"

namespace rb {

// LDS exchange area of one wavefront.
template <int NT>
struct MluShared {
  static constexpr int P = 16 * NT;
  __attribute__((aligned(16))) double pan[P][4];      // panel rows; later the solution
  __attribute__((aligned(16))) double zc[P][4];       // update coefficients per row
  __attribute__((aligned(16))) double urow[4][NT][4][4];   // pivot rows [s][b][l/16][v]
  int slot[P];                                         // pivot index of each panel row
};

// Tiles per side for a system of N unknowns: column P-1 holds the right-hand side, so
// N <= 16*NT - 1 (N <= 63: one row per lane in the panel step).
__host__ __device__ constexpr int mlu_tiles(int n) { return n / 16 + 1; }

// Solve the system in R (see the layout above; R[a][b][v]) for its first N <= 16*NT - 1
// unknowns. On return lane c < N holds x_c in x (0 elsewhere). Returns 0, or 2 (RB_ST_SINGULAR)
// if a pivot was zero (x is then meaningless). Wave-uniform; every lane must call it.
template <int NT>
__device__ __forceinline__ int mfma_gj_solve(f64x4 (&R)[NT][NT], int N, MluShared<NT>& sh,
                                             double& x) {
  constexpr int P = 16 * NT, NPAN = (P - 1 + 3) / 4;   // most panels: N <= P - 1
  static_assert(P <= kWave, "one row per lane in the panel step");
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const bool row_ok = lane < P;
  int pos = lane;                      // position of row `lane` under the row swaps
  bool singular = false;
#pragma unroll
  for (int p = 0; p < NPAN; ++p) {
    if (4 * p >= N) break;             // uniform
    const int bp = p >> 2, vp = p & 3;
    const int T = min(4, N - 4 * p);   // columns to eliminate in this panel (uniform, >= 1)
    // 1. panel columns 4p..4p+3 of row 16a + l%16 sit in lane l (column l/16): to rows
#pragma unroll
    for (int a = 0; a < NT; ++a) sh.pan[16 * a + li][lg] = R[a][bp][vp];
    wave_lds_order();
    double xr[4];
    {
      const int rr = row_ok ? lane : 0;
      const f64x4 v = *reinterpret_cast<const f64x4*>(&sh.pan[rr][0]);
#pragma unroll
      for (int t = 0; t < 4; ++t) xr[t] = row_ok ? v[t] : 0.0;
    }
    // 2. pivot steps on the panel rows
    double z[4] = {0.0, 0.0, 0.0, 0.0};
    int myslot = -1;                   // the panel step at which row `lane` pivoted
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (t < T) {
        const int k = 4 * p + t;
        const bool cand = row_ok && pos >= k;
        const double av = absv(xr[t]);
        uint32_t key = cand ? pivot_key(av) : 0u;
        if (cand && !(av == av)) key = 0xffffffffu;   // a NaN pivot surfaces
        if (cand && key == 0u) key = 1u;              // zero candidates beat non-candidates
        const uint32_t kmax = wave_max_u32(key);
        const uint64_t tied = __ballot(key == kmax);
        int pv = __ffsll(static_cast<unsigned long long>(tied)) - 1;
        if (__popcll(tied) > 1) {                      // same key: exact value, then position
          double bv = bcast(av, pv);
          int best = bcast(pos, pv);
          for (uint64_t m = tied & (tied - 1); m; m &= m - 1) {
            const int l2 = __ffsll(static_cast<unsigned long long>(m)) - 1;
            const double v2 = bcast(av, l2);
            const int p2 = bcast(pos, l2);
            if (v2 > bv || (v2 == bv && p2 < best)) { bv = v2; best = p2; pv = l2; }
          }
        }
        const bool me = lane == pv;
        myslot = me ? t : myslot;
        const double piv = bcast(xr[t], pv);
        singular |= piv == 0.0;
        const double pinv = 1.0 / (piv == 0.0 ? 1.0 : piv);
        const int ppos = bcast(pos, pv);
        pos = (pos == k) ? ppos : pos;
        pos = me ? k : pos;
        // the pivot row scaled to 1 in column k, as coefficients on the panel's pivot rows
        double xp[4], zp[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          xp[u] = u > t ? bcast(xr[u], pv) * pinv : 0.0;
          zp[u] = u < t ? bcast(z[u], pv) * pinv : (u == t ? pinv - 1.0 : 0.0);
        }
        const double f = me ? 0.0 : xr[t];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (u > t) xr[u] = me ? xp[u] : fma(-f, xp[u], xr[u]);
          if (u < t) z[u] = me ? zp[u] : fma(-f, zp[u], z[u]);
        }
        z[t] = me ? zp[t] : -f * pinv;
        xr[t] = me ? 1.0 : 0.0;
      }
    }
    // 3a. B operand of row tile a: lane l takes z[l/16] of row 16a + l%16
    if (row_ok) {
      *reinterpret_cast<f64x4*>(&sh.zc[lane][0]) = f64x4{z[0], z[1], z[2], z[3]};
      sh.slot[lane] = myslot;
    }
    wave_lds_order();
    // 3b. A operand of column tile b: lane l takes the value of pivot row P_{l/16} at column
    //     16b + l%16. Every lane stores the tiles of those of its rows that pivoted, under
    //     their pivot index (the register tile is a compile-time index, the LDS slot a
    //     per-lane address); rows s >= T of the operand are zero.
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const int sa = sh.slot[16 * a + li];
      if (sa >= 0) {
#pragma unroll
        for (int b = bp; b < NT; ++b)
          *reinterpret_cast<f64x4*>(&sh.urow[sa][b][lg][0]) = R[a][b];
      }
    }
    if (T < 4 && li < 4 - T) {
      const int s0 = T + li;
#pragma unroll
      for (int b = bp; b < NT; ++b)
        *reinterpret_cast<f64x4*>(&sh.urow[s0][b][lg][0]) = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    wave_lds_order();
    double bop[NT], aop[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) bop[a] = sh.zc[16 * a + li][lg];
#pragma unroll
    for (int b = bp; b < NT; ++b) aop[b] = sh.urow[lg][b][li & 3][li >> 2];
    wave_lds_order();
    // 3c. X[r] += sum_s z_r[s] X[P_s] on every tile right of the panel's first column tile;
    //     the tile of the next panel first, so its columns are ready soonest
#pragma unroll
    for (int b = bp; b < NT; ++b)
#pragma unroll
      for (int a = 0; a < NT; ++a)
        R[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop[b], bop[a], R[a][b], 0, 0, 0);
  }
  // 4. x_k is column P-1 of the row that pivoted column k (its position k)
  if (lg == 3) {
#pragma unroll
    for (int a = 0; a < NT; ++a) sh.pan[16 * a + li][0] = R[a][NT - 1][3];
  }
  wave_lds_order();
  const double xv = row_ok ? sh.pan[lane][0] : 0.0;
  wave_lds_order();
  if (row_ok) sh.pan[pos][1] = xv;
  wave_lds_order();
  x = lane < N ? sh.pan[lane][1] : 0.0;
  wave_lds_order();
  return singular ? 2 : 0;
}

}  // namespace rb

namespace rb {

// Newton step of one request per wavefront with the matrix-core solve (N <= 63): residual
// F(u) = (J u + A u)/2 - f, J delta = -F(u) by mfma_gj_solve, update of the FP64 iterate and
// the stopping test ||delta||_H <= tol ||u||_H (same contract as lu_f64_kernel).
template <int NT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT >= 3 ? 2 : 4)))
void lu_mfma_f64_kernel(NewtonF64Args a, int it) {
  __shared__ MluShared<NT> sh[kWaves];
  constexpr int P = 16 * NT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);   // wave-uniform
  if (b >= a.B || a.s.done[b]) return;
  const int N = a.N;
  const int nb = a.nreq ? a.nreq[b] : N;   // this request's size; rows/columns beyond: identity
  const double* jb = a.s.J + (int64_t)b * a.s.mp;
  const double* ub = a.s.U + (int64_t)b * a.s.NP;
  f64x4 R[NT][NT];
  double ju[NT];
  bool bad = false;
#pragma unroll
  for (int r0 = 0; r0 < NT; ++r0) ju[r0] = 0.0;
  // J (column-major per request) into the tile layout, identity rows and columns beyond the
  // request's size; this lane's share of J u on the way. One column tile at a time: its loads
  // are issued together (offsets from the request's base, clamped in bounds).
  const int lc = li < N ? li : N - 1;
#pragma unroll
  for (int bt = 0; bt < NT; ++bt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * bt + lg + 4 * v, cc = c < N ? c : N - 1;
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        const int r = 16 * at + li, rr = r < N ? r : lc;
        R[at][bt][v] = jb[cc * N + rr];
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * bt + lg + 4 * v;
      const double uc = c < nb ? ub[c] : 0.0;
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        const int r = 16 * at + li;
        const double val = (r < nb && c < nb) ? R[at][bt][v]
                                              : ((r == c && c < P - 1) ? 1.0 : 0.0);
        bad |= !finite_val(val);
        ju[at] = fma(val, uc, ju[at]);
        R[at][bt][v] = val;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // right-hand side -F(u) of row 16a + l%16 into column P-1 (lanes l/16 = 3, element 3)
#pragma unroll
  for (int at = 0; at < NT; ++at) {
    double s = ju[at];
    s += __shfl_xor(s, 16);
    s += __shfl_xor(s, 32);
    const int r = 16 * at + li;
    double rhs = 0.0;
    if (r < nb) {
      double w = 0.0;
      for (int sp = 0; sp < a.s.nsplit; ++sp) w += a.s.Wv[((int64_t)sp * a.s.Bp + b) * a.s.NP + r];
      rhs = -(0.5 * (s + w) - a.s.Fv[(int64_t)b * a.s.NP + r]);   // F(u) = (J u + A u)/2 - f
    }
    bad |= !finite_val(rhs);
    if (lg == 3) R[at][NT - 1][3] = rhs;
  }
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  double dx = 0.0;
  if (flag == 0) flag = mfma_gj_solve<NT>(R, N, sh[wv], dx);
  if (flag == 0) {
    const int lc = lane < N ? lane : N - 1;
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
      if (lane < N) a.s.U[(int64_t)b * a.s.NP + lane] = un;
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

// Pressure solve B(mu) p = f_s - (A_sv u + C_sv(u,u)) of one request per wavefront with the
// matrix-core solve (Np <= 63); same contract as plu_f64_kernel.
template <int NT>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(NT >= 3 ? 2 : 4)))
void plu_mfma_f64_kernel(PressureF64Args a) {
  __shared__ MluShared<NT> sh[kWaves];
  constexpr int P = 16 * NT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, li = lane & 15, lg = lane >> 4;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);   // wave-uniform
  if (b >= a.B) return;
  const int Np = a.Np;
  double tbv[kMaxQb];
#pragma unroll
  for (int q = 0; q < kMaxQb; ++q) tbv[q] = q < a.Qb ? a.tb[(int64_t)b * a.Qb + q] : 0.0;
  f64x4 R[NT][NT];
  bool bad = false;
#pragma unroll
  for (int bt = 0; bt < NT; ++bt)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = 16 * bt + lg + 4 * v;
#pragma unroll
      for (int at = 0; at < NT; ++at) {
        const int r = 16 * at + li;
        double val = (r == c && c < P - 1) ? 1.0 : 0.0;
        if (r < Np && c < Np) {
          double s = 0.0;
#pragma unroll
          for (int q = 0; q < kMaxQb; ++q)
            if (q < a.Qb) s = fma(tbv[q], a.BpT[((int64_t)q * a.Npm + c) * a.Npm + r], s);
          val = s;
        }
        bad |= !finite_val(val);
        R[at][bt][v] = val;
      }
    }
#pragma unroll
  for (int at = 0; at < NT; ++at) {
    const int r = 16 * at + li;
    double rhs = 0.0;
    if (r < Np) {
      for (int q = 0; q < a.Qf; ++q)
        rhs = fma(a.tf[(int64_t)b * a.Qf + q], a.Fs[(int64_t)q * a.Npm + r], rhs);
      for (int sp = 0; sp < a.nsplit; ++sp)
        rhs -= a.part[((int64_t)sp * a.Bp + b) * a.ldpart + r];
    }
    bad |= !finite_val(rhs);
    if (lg == 3) R[at][NT - 1][3] = rhs;
  }
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  double x = 0.0;
  if (flag == 0) flag = mfma_gj_solve<NT>(R, Np, sh[wv], x);
  if (flag == 0 && !finite_val(wave_sum(lane < Np ? x : 0.0))) flag = 3;
  for (int i = lane; i < a.ldp; i += kWave)
    a.p[(int64_t)b * a.ldp + i] = (flag == 0 && i < Np) ? x : 0.0;
  if (lane == 0) a.status[b] = flag;
}

}  // namespace rb
