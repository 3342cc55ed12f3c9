// rb_common.hpp -- wavefront helpers shared by the gfx950 kernels of the reduced
// Navier-Stokes online solver. Everything here assumes 64-wide wavefronts (CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rb {

constexpr int kWave = 64;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Broadcast lane `l` (wave-uniform) of a 64-bit value to every lane.
__device__ __forceinline__ double bcast(double x, int l) {
  const int64_t v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(v), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), l);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) |
                              static_cast<uint32_t>(lo));
}

__device__ __forceinline__ float bcast(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ int bcast(int x, int l) { return __builtin_amdgcn_readlane(x, l); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Lane holding the largest candidate value; ties go to the smallest `key`. Non-candidates
// pass v = -1. Every lane receives the same answer.
template <typename T>
__device__ __forceinline__ int wave_argmax(T v, int key, int lane) {
  T bv = v;
  int bk = key, bl = lane;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const T ov = __shfl_xor(bv, off);
    const int ok = __shfl_xor(bk, off);
    const int ol = __shfl_xor(bl, off);
    const bool take = (ov > bv) || (ov == bv && ok < bk);
    bv = take ? ov : bv;
    bk = take ? ok : bk;
    bl = take ? ol : bl;
  }
  return __builtin_amdgcn_readfirstlane(bl);
}

__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }

template <typename T>
__device__ __forceinline__ bool finite_val(T x) {
  return x - x == T(0);   // false for NaN and +-Inf
}

// 64-bit DPP move of a double (both halves with the same control). Lanes whose source is
// out of range read 0 (bound_ctrl); lanes outside row_mask keep their own value.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double x) {
  const int64_t v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(v), static_cast<int>(v), CTRL,
                                             ROW_MASK, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(v >> 32),
                                             static_cast<int>(v >> 32), CTRL, ROW_MASK, 0xf,
                                             true);
  return __longlong_as_double((static_cast<int64_t>(hi) << 32) | static_cast<uint32_t>(lo));
}

template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ float dpp_f32(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x),
                                                    CTRL, ROW_MASK, 0xf, true));
}

// Wave-wide maximum of max(v, 0): row_shr 1,2,4,8 inside each 16-lane row, then
// row_bcast15 / row_bcast31 across rows; lane 63 ends with the maximum.
__device__ __forceinline__ double wave_max_pos(double v) {
  v = fmax(v, dpp_f64<0x111>(v));
  v = fmax(v, dpp_f64<0x112>(v));
  v = fmax(v, dpp_f64<0x114>(v));
  v = fmax(v, dpp_f64<0x118>(v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v));
  return bcast(v, 63);
}

__device__ __forceinline__ float wave_max_pos(float v) {
  v = fmaxf(v, dpp_f32<0x111>(v));
  v = fmaxf(v, dpp_f32<0x112>(v));
  v = fmaxf(v, dpp_f32<0x114>(v));
  v = fmaxf(v, dpp_f32<0x118>(v));
  v = fmaxf(v, dpp_f32<0x142, 0xa>(v));
  v = fmaxf(v, dpp_f32<0x143, 0xc>(v));
  return bcast(v, 63);
}

__device__ __forceinline__ void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Dense solve of one N x N system held one row per lane (row i in lane i, NP >= N columns
// in registers), by Gaussian elimination with partial pivoting. The caller pads the system
// to NP x NP with identity rows/columns (lanes N..NP-1) and a zero right-hand side there;
// the padded rows never win a pivot search in the first N columns and pivot on themselves
// afterwards, so every step runs unconditionally (no data-dependent control flow around the
// register-resident rows). Rows are not moved between lanes: `pos` tracks each row's current
// position so that the pivot choice (largest magnitude, ties to the smallest current row
// index) is the one row-swapping elimination makes. The pivot row reaches the other lanes
// either through `prow` (this wavefront's LDS row, >= NP + 1 entries; kLdsBcast) or lane by
// lane through scalar registers (readlane); the right-hand side rides along as an extra
// column. On return lane c < NP holds x_c in `x`. Returns 0, or RB_ST_SINGULAR (2)
// if a pivot was zero (the values returned are then meaningless).
template <int NP, bool kLdsBcast, typename T>
__device__ __forceinline__ int lu_solve_rows(T (&a)[NP], T rhs, int lane, T* prow, T& x) {
  int pos = lane;
  bool singular = false;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    T v = (pos >= k && lane < NP) ? absv(a[k]) : T(-1);
    if (!(v == v)) v = static_cast<T>(__builtin_huge_val());  // a NaN pivot surfaces
    const T vmax = wave_max_pos(v);
    const uint64_t tied = __ballot(v == vmax);
    int pv = __ffsll(static_cast<unsigned long long>(tied)) - 1;
    if (__popcll(tied) > 1) {            // exact tie (rare): smallest current position wins
      int best = bcast(pos, pv);
      for (uint64_t m = tied & (tied - 1); m; m &= m - 1) {
        const int l2 = __ffsll(static_cast<unsigned long long>(m)) - 1;
        const int p2 = bcast(pos, l2);
        if (p2 < best) { best = p2; pv = l2; }
      }
    }
    T piv = bcast(a[k], pv);
    singular |= (piv == T(0));
    piv = (piv == T(0)) ? T(1) : piv;
    const int ppos = bcast(pos, pv);
    pos = (pos == k) ? ppos : pos;
    pos = (lane == pv) ? k : pos;
    const T l = (pos > k) ? a[k] / piv : T(0);
    if (kLdsBcast) {
      if (lane == pv) {
#pragma unroll
        for (int j = k + 1; j < NP; ++j) prow[j] = a[j];
        prow[NP] = rhs;
      }
      wave_lds_order();
#pragma unroll
      for (int j0 = k + 1; j0 < NP; j0 += 8) {
        T pj[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) pj[t] = prow[j0 + t];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) a[j0 + t] = fma(-l, pj[t], a[j0 + t]);
        __builtin_amdgcn_sched_barrier(0);
      }
      rhs = fma(-l, prow[NP], rhs);
      wave_lds_order();
    } else {
      // Pivot-row entries go lane -> SGPR (readlane) and feed the FMA as its scalar operand,
      // in chunks of 8 so the scalar registers in flight stay bounded.
#pragma unroll
      for (int j0 = k + 1; j0 < NP; j0 += 8) {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) a[j0 + t] = fma(-l, bcast(a[j0 + t], pv), a[j0 + t]);
        __builtin_amdgcn_sched_barrier(0);
      }
      rhs = fma(-l, bcast(rhs, pv), rhs);
    }
  }
  // Back substitution: the row that pivoted at step k (pos == k) holds U[k][k..] and the
  // eliminated right-hand side; x_k = rhs / U[k][k], then every earlier pivot row drops its
  // x_k term.
  x = T(0);
#pragma unroll
  for (int k = NP - 1; k >= 0; --k) {
    const int p = __ffsll(static_cast<unsigned long long>(__ballot(pos == k))) - 1;
    T d = bcast(a[k], p);
    d = (d == T(0)) ? T(1) : d;
    const T xk = bcast(rhs, p) / d;
    rhs = (pos < k) ? fma(-a[k], xk, rhs) : rhs;
    x = (lane == k) ? xk : x;
  }
  return singular ? 2 : 0;
}

}  // namespace rb
