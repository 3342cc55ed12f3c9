// rb_lowprec.hpp -- mixed-precision Newton for gfx950: the Jacobian contraction from FP32 or
// BF16 copies of the tensors on MFMA with FP32 accumulation, an FP32 register LU, iterates
// and updates kept in FP64, and refinement steps whose residual F(u) = A(mu)u + C(mu)(u,u) - f
// is evaluated from the FP64 tensors (kModeResid of the FP64 contraction).
#pragma once

#include <type_traits>

#include "rb_kernels.hpp"

namespace rb {

typedef short bf16x8 __attribute__((ext_vector_type(8)));

// FP64 -> BF16, round to nearest even, in one step (no intermediate FP32 rounding). Values
// below the smallest normal BF16 flush to signed zero; overflow gives infinity.
__host__ __device__ inline uint16_t f64_to_bf16(double x) {
  uint64_t u;
  __builtin_memcpy(&u, &x, 8);
  const uint32_t sign = static_cast<uint32_t>(u >> 63) << 15;
  const int e = static_cast<int>((u >> 52) & 0x7ff);
  const uint64_t m = u & ((1ull << 52) - 1);
  if (e == 0x7ff) return static_cast<uint16_t>(sign | 0x7f80 | (m ? 0x40 : 0));
  int eb = e - 1023 + 127;
  if (eb >= 255) return static_cast<uint16_t>(sign | 0x7f80);
  if (eb <= 0) return static_cast<uint16_t>(sign);
  uint64_t keep = m >> 45;
  const uint64_t rest = m & ((1ull << 45) - 1), half = 1ull << 44;
  if (rest > half || (rest == half && (keep & 1))) {
    if (++keep == 128) {
      keep = 0;
      if (++eb >= 255) return static_cast<uint16_t>(sign | 0x7f80);
    }
  }
  return static_cast<uint16_t>(sign | (static_cast<uint32_t>(eb) << 7) | keep);
}

// Low-precision packed solve operand, same rows (m = j*N + i) and column order as the FP64
// one, in MFMA operand order:
//   FP32 (v_mfma_f32_16x16x4f32): tile (rb, ks) = 64 floats, element e <-> (row rb*16 + e%16,
//        k = ks*4 + e/16); affine part kA = ceil(Q/4) k-steps, tensor part KT k-steps.
//   BF16 (v_mfma_f32_16x16x32_bf16): tile (rb, ks) = 64 lanes x 8 bf16, lane e holds row
//        rb*16 + e%16, k = ks*32 + 8*(e/16) + t (t = 0..7); affine part 1 k-step (Q <= 32),
//        tensor part KT = ceil(Qc*N/32) k-steps.
//   BF16x3 (kSplit3): the BF16 layout twice, hi = bf16(v) then lo = bf16(v - hi) at out + total
//        (a 16-bit-mantissa representation of v as the sum of two BF16 numbers).
__host__ __device__ inline double bf16_to_f64(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return static_cast<double>(f);
}

template <bool kBF16, bool kSplit3 = false>
__global__ void pack_lp(const double* __restrict__ C, const double* __restrict__ A, int Nm, int N,
                        int Q, int Qc, int kA, int nrb, int nks, void* __restrict__ out) {
  constexpr int kK = kBF16 ? 32 : 4;        // k per k-step
  const int64_t total = (int64_t)nrb * nks * 64 * (kBF16 ? 8 : 1);
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int e, t;
    int64_t tile;
    if (kBF16) {
      t = idx & 7;
      e = (idx >> 3) & 63;
      tile = idx >> 9;
    } else {
      t = 0;
      e = idx & 63;
      tile = idx >> 6;
    }
    const int rb = tile / nks, ks = tile % nks;
    const int m = rb * 16 + (e & 15);
    const int k = kBF16 ? ks * kK + 8 * (e >> 4) + t : ks * kK + (e >> 4);
    double v = 0.0;
    if (m < N * N) {
      const int j = m / N, i = m - j * N;
      if (k < kK * kA) {
        if (k < Q) v = A[((int64_t)k * Nm + i) * Nm + j];
      } else if (k - kK * kA < Qc * N) {
        const int kk = k - kK * kA, q = kk / N, l = kk - q * N;
        v = C[(((int64_t)q * Nm + i) * Nm + j) * Nm + l] + C[(((int64_t)q * Nm + i) * Nm + l) * Nm + j];
      }
    }
    if (kBF16) {
      const uint16_t hi = f64_to_bf16(v);
      static_cast<uint16_t*>(out)[idx] = hi;
      if (kSplit3) static_cast<uint16_t*>(out)[total + idx] = f64_to_bf16(v - bf16_to_f64(hi));
    } else {
      static_cast<float*>(out)[idx] = static_cast<float>(v);
    }
  }
}

struct ContractLpArgs {
  const void* op;          // packed operand (float or bf16)
  const void* op_lo;       // BF16x3: the low parts (same layout), else nullptr
  int nrb, kA, nks;        // row blocks, affine k-steps, k-steps per row block
  int N, M, Q, Qc, B;
  int64_t Bp;
  const double* ta;
  const double* tc;
  const double* U;         // FP64 iterates [Bp][ldU]
  int ldU;
  const int* done;         // skip flags or nullptr
  float* J;                // FP32 Jacobians [Bp][mp], column-major per request
  int64_t mp;
  float* part;             // partial A(mu) u [nsplit][Bp][ldp]
  int nsplit;
  int ldp;
};

__host__ __device__ inline int64_t contract_lp_lds_bytes(int N) {
  return 4 * 2 * (int64_t)kTile * N;
}

// Same decomposition as contract_f64_kernel (64-request tile x row split per workgroup,
// 16 requests and their W slice per wavefront, four row blocks per pass, static prefetch),
// with FP32 (or BF16) operands and FP32 accumulators; the whole tensor part (KT k-steps) is
// one chunk. kS3 (BF16x3): operand and W are both split into hi + lo BF16 parts and every
// product is hi*hi + hi*lo + lo*hi (three MFMAs, about 16 mantissa bits). Accumulator layout
// of the 16x16 FP32 MFMAs: lane l, element v = row 4*(l/16) + v, column l%16.
// BF16x3 with KT <= 14 runs two waves per SIMD with a four-k-step prefetch (hi + lo W in
// registers, two BF16 values per register); two and six steps measured slower, and one wave
// per SIMD with a six-step prefetch 26 % slower.
template <bool kBF16, int KT, bool kS3 = false>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(kS3 && KT <= 14 ? 2 : 1)))
void contract_lp_kernel(ContractLpArgs a) {
  extern __shared__ float smemf[];
  typedef typename std::conditional<kBF16, bf16x8, float>::type opnd;
  constexpr int kK = kBF16 ? 32 : 4;
  constexpr int kAmax = kBF16 ? 1 : 3;
  const int N = a.N;
  float* ul = smemf;                       // [kTile][N]
  float* pl = ul + kTile * N;              // [kTile][N]

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int split = blockIdx.x % a.nsplit;
  const int b0 = (blockIdx.x / a.nsplit) * kTile;
  if (a.done && __syncthreads_and(tid < kTile ? a.done[b0 + tid] : 1)) return;

  for (int idx = tid; idx < kTile * N; idx += kThreads) {
    const int b = idx / N, l = idx - b * N, bg = b0 + b;
    ul[idx] = bg < a.B ? static_cast<float>(a.U[(int64_t)bg * a.ldU + l]) : 0.f;
    pl[idx] = 0.f;
  }
  // W column of this lane: request bl, k = ks*kK + (kBF16 ? 8*(lane/16) + t : lane/16).
  const int bl = 16 * wv + (lane & 15);
  const int bg = b0 + bl;
  float tav[kMaxQ], tcv[kMaxQc];
#pragma unroll
  for (int q = 0; q < kMaxQ; ++q)
    tav[q] = (bg < a.B && q < a.Q) ? static_cast<float>(a.ta[(int64_t)bg * a.Q + q]) : 0.f;
#pragma unroll
  for (int q = 0; q < kMaxQc; ++q)
    tcv[q] = (bg < a.B && q < a.Qc) ? static_cast<float>(a.tc[(int64_t)bg * a.Qc + q]) : 0.f;
  __syncthreads();

  auto wval = [&](int k) -> float {
    if (k < kK * a.kA) {
      float v = 0.f;
#pragma unroll
      for (int q = 0; q < kMaxQ; ++q) v = (k == q) ? tav[q] : v;
      return v;
    }
    int l = k - kK * a.kA, q = 0;
    while (l >= N && q < kMaxQc) { l -= N; ++q; }
    float tq = 0.f;
#pragma unroll
    for (int qq = 0; qq < kMaxQc; ++qq) tq = (q == qq) ? tcv[qq] : tq;
    return q < kMaxQc ? tq * ul[bl * N + l] : 0.f;
  };
  constexpr int kP = kS3 ? 2 : 1;           // hi (and lo) parts
  constexpr int kDep = (kS3 && KT <= 14) ? 4 : kDepth;   // k-steps loaded ahead
  opnd wA[kP][kAmax], wT[kP][KT];
  // hi (and lo) BF16 parts of the eight float W values of a k-step, two per register by the
  // hardware conversion (round to nearest even); v - hi is exact in float
  auto parts = [&](const float (&v)[8], opnd (&dst)[kP]) {
    if constexpr (kBF16) {
      typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
      typedef float f32x2 __attribute__((ext_vector_type(2)));
      typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
      u32x4 h, l;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        h[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){v[2 * i], v[2 * i + 1]}, bf16x2));
        if constexpr (kS3) {
          const float r0 = v[2 * i] - __uint_as_float(h[i] << 16);
          const float r1 = v[2 * i + 1] - __uint_as_float(h[i] & 0xffff0000u);
          l[i] = __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2){r0, r1}, bf16x2));
        }
      }
      dst[0] = __builtin_bit_cast(opnd, h);
      if constexpr (kS3) dst[kP - 1] = __builtin_bit_cast(opnd, l);
    }
  };
  auto make = [&](int ks, opnd (&dst)[kP]) {
    if constexpr (kBF16) {
      float v[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) v[t] = wval(ks * kK + 8 * (lane >> 4) + t);
      parts(v, dst);
    } else {
      dst[0] = wval(ks * kK + (lane >> 4));
    }
  };
  // BF16 tensor k-step ks: rows t = 32 ks + 8 (lane/16) + e, e = 0..7, walked as (q, l) with
  // t = q N + l instead of one division per value
  auto make_t = [&](int ks, opnd (&dst)[kP]) {
    int l = kK * ks + 8 * (lane >> 4), q = 0;
    while (l >= N && q < kMaxQc) { l -= N; ++q; }
    float v[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float tq = 0.f;
#pragma unroll
      for (int qq = 0; qq < kMaxQc; ++qq) tq = (q == qq) ? tcv[qq] : tq;
      v[e] = q < kMaxQc ? tq * ul[bl * N + l] : 0.f;
      if (++l == N) { l = 0; ++q; }
      if (q >= kMaxQc) l = 0;
    }
    parts(v, dst);
  };
#pragma unroll
  for (int ks = 0; ks < kAmax; ++ks) {
    opnd tmp[kP];
    make(ks, tmp);
#pragma unroll
    for (int pp = 0; pp < kP; ++pp) wA[pp][ks] = tmp[pp];
  }
#pragma unroll
  for (int ks = 0; ks < KT; ++ks) {
    opnd tmp[kP];
    if constexpr (kBF16) make_t(ks, tmp);
    else make(a.kA + ks, tmp);
#pragma unroll
    for (int pp = 0; pp < kP; ++pp) wT[pp][ks] = tmp[pp];
  }

  const int rb_lo = (int)((int64_t)split * a.nrb / a.nsplit);
  const int rb_hi = (int)((int64_t)(split + 1) * a.nrb / a.nsplit);
  const int col = bl;
  const opnd* opb[kP];
  opb[0] = static_cast<const opnd*>(a.op);
  if constexpr (kS3) opb[kP - 1] = static_cast<const opnd*>(a.op_lo);

  for (int g0 = rb_lo; g0 < rb_hi; g0 += kGroup) {
    const opnd* opg[kP][kGroup];
#pragma unroll
    for (int pp = 0; pp < kP; ++pp)
#pragma unroll
      for (int r = 0; r < kGroup; ++r)
        opg[pp][r] = opb[pp] + (int64_t)min(g0 + r, rb_hi - 1) * a.nks * 64 + lane;
    opnd xa[kP][kAmax][kGroup];
#pragma unroll
    for (int pp = 0; pp < kP; ++pp)
#pragma unroll
      for (int ks = 0; ks < kAmax; ++ks)
#pragma unroll
        for (int r = 0; r < kGroup; ++r) xa[pp][ks][r] = opg[pp][r][min(ks, a.kA - 1) * 64];
    opnd x[kP][KT][kGroup];
#pragma unroll
    for (int ks = 0; ks < kDep && ks < KT; ++ks)
#pragma unroll
      for (int pp = 0; pp < kP; ++pp)
#pragma unroll
        for (int r = 0; r < kGroup; ++r) x[pp][ks][r] = opg[pp][r][(a.kA + ks) * 64];

    auto mfma = [](opnd xx, opnd ww, f32x4 cc) -> f32x4 {
      if constexpr (kBF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(xx, ww, cc, 0, 0, 0);
      else
        return __builtin_amdgcn_mfma_f32_16x16x4f32(xx, ww, cc, 0, 0, 0);
    };
    f32x4 c[kGroup];
#pragma unroll
    for (int r = 0; r < kGroup; ++r) c[r] = f32x4{0.f, 0.f, 0.f, 0.f};
    // hi*hi (+ hi*lo + lo*hi for BF16x3)
    auto mac = [&](const opnd (&xx)[kP], const opnd (&ww)[kP], f32x4 cc) -> f32x4 {
      cc = mfma(xx[0], ww[0], cc);
      if constexpr (kS3) {
        cc = mfma(xx[0], ww[kP - 1], cc);
        cc = mfma(xx[kP - 1], ww[0], cc);
      }
      return cc;
    };
#pragma unroll
    for (int ks = 0; ks < kAmax; ++ks) {
      if (ks < a.kA) {
#pragma unroll
        for (int r = 0; r < kGroup; ++r) {
          opnd xx[kP], ww[kP];
#pragma unroll
          for (int pp = 0; pp < kP; ++pp) { xx[pp] = xa[pp][ks][r]; ww[pp] = wA[pp][ks]; }
          c[r] = mac(xx, ww, c[r]);
        }
      }
    }
    // fold A(mu) rows: acc[m] * u_j into p_i (m = j*N + i)
    {
      const int m0 = g0 * 16 + 4 * (lane >> 4);
      const int j0 = m0 / N, i0 = m0 - j0 * N;
#pragma unroll
      for (int r = 0; r < kGroup; ++r) {
        if (g0 + r < rb_hi) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int i = i0 + 16 * r + v, j = j0;
            while (i >= N) { i -= N; ++j; }
            if (j < N) atomicAdd(&pl[col * N + i], c[r][v] * ul[col * N + j]);
          }
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) {
      if (ks + kDep < KT) {
#pragma unroll
        for (int pp = 0; pp < kP; ++pp)
#pragma unroll
          for (int r = 0; r < kGroup; ++r)
            x[pp][ks + kDep][r] = opg[pp][r][(a.kA + ks + kDep) * 64];
      }
#pragma unroll
      for (int r = 0; r < kGroup; ++r) {
        opnd xx[kP], ww[kP];
#pragma unroll
        for (int pp = 0; pp < kP; ++pp) { xx[pp] = x[pp][ks][r]; ww[pp] = wT[pp][ks]; }
        c[r] = mac(xx, ww, c[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < kGroup; ++r) {
      if (g0 + r < rb_hi) {
        float* jp = a.J + (int64_t)(b0 + col) * a.mp + (g0 + r) * 16 + 4 * (lane >> 4);
        *reinterpret_cast<f32x4*>(jp) = c[r];
      }
    }
  }
  __syncthreads();
  for (int idx = tid; idx < kTile * N; idx += kThreads) {
    const int b = idx / N, i = idx - b * N;
    a.part[((int64_t)split * a.Bp + b0 + b) * a.ldp + i] = pl[idx];
  }
}

// First low-precision Newton step from u = 0 (as stokes_jacobian_kernel): J32 = A(mu),
// summed in FP64 from the packed FP64 operand and rounded once, and zero partial sums of
// A(mu) u.
static __global__ __launch_bounds__(256) void stokes_jacobian_lp_kernel(NewtonF64Args a,
                                                                      float* J32, int64_t mp,
                                                                      float* part32,
                                                                      int nsplit) {
  stokes_tile<float>(a, J32, mp, part32, (int64_t)nsplit * a.s.Bp * a.s.NP);
}

// Status of a request whose refinement steps ran out while each refinement update after the
// first was at most half the update before it (the refinement still contracting): its error is
// of the order of the last update times that contraction. RB_ST_MAXIT then marks stagnation or
// divergence.
constexpr int kStRefined = 6;

struct LpNewtonArgs {
  int N, Nm, B;
  double tol;              // stopping test ||delta||_H <= tol ||u||_H
  double stag;             // low-precision phase: stagnation counts below stag ||u||_H
  const double* H;         // [Nm][Nm] norm Gram or nullptr
  const float* J;          // [Bp][mp]
  int64_t mp;
  const float* part;       // [nsplit][Bp][NP] A(mu) u (low-precision phase)
  const double* partA;     // [nsplit][Bp][NP] A(mu) u + C(mu)(u,u) (FP64 refinement)
  const int* nreq;         // [B] per-request basis size (<= N) or nullptr
  NewtonState s;           // FP64 iterates, f, flags
};

// One wavefront per request. Low-precision phase (kRefine = false): F(u) ~ (J u + A u)/2 - f
// from the FP32 / BF16 contraction, a request stops when its update is below tol or has
// stagnated (below stag and no longer halving). Refinement (kRefine = true): F(u) =
// A(mu)u + C(mu)(u,u) - f from the FP64 residual contraction, with the Jacobian of the last
// low-precision step. Either way the correction solves J32 delta = -F(u) by the FP32 register LU and is
// added to the FP64 iterate.
template <int NP, bool kRefine>
__global__ __launch_bounds__(kThreads) void lu_lp_kernel(LpNewtonArgs a, int it) {
  __shared__ float prow[kWaves][NP + 8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int b = __builtin_amdgcn_readfirstlane(blockIdx.x * kWaves + wv);   // wave-uniform
  if (b >= a.B || a.s.done[b]) return;
  const int N = a.N;
  const int nb = a.nreq ? a.nreq[b] : N;   // this request's size; rows/columns beyond: identity
  const int64_t Bp = a.s.Bp;
  const float* jb = a.J + (int64_t)b * a.mp;
  const double* ub = a.s.U + (int64_t)b * NP;
  float r[NP];
  const int lc = lane < N ? lane : N - 1;
  bool bad = false;
  double rhs64 = 0.0;
  float ju = 0.f;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    const float v = jb[(c < N ? c : N - 1) * N + lc];
    r[c] = (c < nb && lane < nb) ? v : (c == lane ? 1.f : 0.f);
    ju = fmaf(r[c], static_cast<float>(ub[c]), ju);
    bad |= !finite_val(r[c]);
  }
  if (lane < nb) {
    if (kRefine) {
      double g = 0.0;
#pragma unroll
      for (int sp = 0; sp < a.s.nsplit; ++sp) g += a.partA[((int64_t)sp * Bp + b) * NP + lane];
      rhs64 = -(g - a.s.Fv[(int64_t)b * NP + lane]);
    } else {
      float au = 0.f;
#pragma unroll
      for (int sp = 0; sp < a.s.nsplit; ++sp) au += a.part[((int64_t)sp * Bp + b) * NP + lane];
      rhs64 = -(0.5 * (static_cast<double>(ju) + au) - a.s.Fv[(int64_t)b * NP + lane]);
    }
  }
  float rhs = static_cast<float>(rhs64);
  bad |= !finite_val(rhs);
  int flag = __builtin_amdgcn_readfirstlane(__any(bad) ? 3 : 0);
  float dxf = 0.f;
  if (flag == 0) flag = lu_solve_rows<NP, false>(r, rhs, lane, &prow[wv][0], dxf);
  if (flag == 0) {
    const double dx = lane < N ? static_cast<double>(dxf) : 0.0;
    const double un = (lane < N ? ub[lane] : 0.0) + dx;
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
        a.s.iters[b] = a.s.iters[b] + 1;
        const double nd = sqrt(nd2), nu = sqrt(nu2);
        if (nd <= a.tol * nu) {
          a.s.status[b] = 0;
          a.s.done[b] = 1;
        } else if (!kRefine && it > 0 && nd <= a.stag * nu && nd > 0.5 * a.s.dprev[b]) {
          a.s.done[b] = 1;                 // stagnated: status stays RB_ST_MAXIT
        } else if (kRefine) {              // still contracting: RB_ST_REFINED, else MAXIT
          a.s.status[b] = nd <= 0.5 * a.s.dprev[b] ? kStRefined : 1;
        }
        a.s.dprev[b] = nd;
      }
    }
  }
  if (flag != 0 && lane == 0) {
    a.s.status[b] = flag;
    a.s.done[b] = 1;
  }
}

// NP > 64: one request per workgroup of W wavefronts (Gauss-Jordan over the workgroup),
// same right-hand sides and stopping rules as lu_lp_kernel. Up to 72 unknowns the rows fit
// in 128 registers (four wavefronts per SIMD), up to 104 in 168 (three); the solve is bound
// by its per-step latency chain, so resident requests are what hides it.
template <int NP, int W>
__global__ __launch_bounds__(kWave * W) __attribute__((amdgpu_waves_per_eu(NP <= 72 ? 4 : (NP <= 104 ? 3 : 1))))
void lu_lp_mw_kernel(LpNewtonArgs a, int it, int refine) {
  __shared__ GjShared<NP, W, float> sh;
  const int b = blockIdx.x;
  if (a.s.done[b]) return;
  const int64_t Bp = a.s.Bp;
  const float* jb = a.J + (int64_t)b * a.mp;
  const int N = a.N;
  auto jload = [&](int c, int row) { return jb[c * N + row]; };
  double* ub = a.s.U + (int64_t)b * NP;
  auto rhs_of = [&](int row, float ju) {
    const double f = a.s.Fv[(int64_t)b * NP + row];
    if (refine) {
      double g = 0.0;
#pragma unroll
      for (int sp = 0; sp < a.s.nsplit; ++sp) g += a.partA[((int64_t)sp * Bp + b) * NP + row];
      return -(g - f);
    }
    float au = 0.f;
#pragma unroll
    for (int sp = 0; sp < a.s.nsplit; ++sp) au += a.part[((int64_t)sp * Bp + b) * NP + row];
    return -(0.5 * (static_cast<double>(ju) + au) - f);
  };
  double nd2, nu2;
  const int nb = a.nreq ? a.nreq[b] : N;
  const int flag = mw_newton_update<float, NP, W>(jload, nb, a.Nm, ub, a.H, rhs_of, sh, nd2,
                                                  nu2);
  if (threadIdx.x != 0) return;
  if (flag != 0) {
    a.s.status[b] = flag;
    a.s.done[b] = 1;
    return;
  }
  a.s.iters[b] = a.s.iters[b] + 1;
  const double nd = sqrt(nd2), nu = sqrt(nu2);
  if (nd <= a.tol * nu) {
    a.s.status[b] = 0;
    a.s.done[b] = 1;
  } else if (!refine && it > 0 && nd <= a.stag * nu && nd > 0.5 * a.s.dprev[b]) {
    a.s.done[b] = 1;
  } else if (refine) {
    a.s.status[b] = nd <= 0.5 * a.s.dprev[b] ? kStRefined : 1;
  }
  a.s.dprev[b] = nd;
}

// Between the phases: every request without a failure status is refined (status back to
// RB_ST_MAXIT until a refinement update meets the tolerance). The first refinement update has
// nothing to contract against (the last low-precision updates are at the noise level of the
// low precision, as large as the error the refinement removes); later ones are measured
// against the one before.
static __global__ void lp_refine_reset_kernel(int B, int64_t Bp, int* done, int* status,
                                              double* dprev) {
  for (int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; b < Bp;
       b += (int64_t)gridDim.x * blockDim.x) {
    if (b >= B) { done[b] = 1; continue; }
    const int s = status[b];
    done[b] = s >= 2;
    if (s < 2) dprev[b] = __builtin_huge_val();
    if (s < 2) status[b] = 1;
  }
}

}  // namespace rb
