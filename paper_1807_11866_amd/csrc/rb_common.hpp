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

// Search key of a pivot candidate: the high 32 bits of |a| (monotonic in |a| for doubles,
// the whole value for floats), so the wavefront maximum is a 32-bit DPP reduction.
__device__ __forceinline__ uint32_t pivot_key(double av) {
  return static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(av)) >> 32);
}
__device__ __forceinline__ uint32_t pivot_key(float av) { return __float_as_uint(av); }

// Wavefront maximum of an unsigned key (row_shr 1,2,4,8, row_bcast 15/31), in every lane.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x111, 0xf, 0xf, true)));
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x112, 0xf, 0xf, true)));
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x114, 0xf, 0xf, true)));
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x118, 0xf, 0xf, true)));
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x142, 0xa, 0xf, true)));
  v = max(v, static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x143, 0xc, 0xf, true)));
  return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), 63));
}

// Dense solve of one N x N system held one row per lane (row i in lane i, NP >= N columns
// in registers), by Gauss-Jordan elimination with partial pivoting: at step k column k is
// eliminated from every row but the pivot row, so no back substitution is needed. The caller
// pads the system to NP x NP with identity rows/columns (lanes N..NP-1) and a zero
// right-hand side there; the padded rows never win a pivot search in the first N columns and
// pivot on themselves afterwards, so every step runs unconditionally. Rows are not moved
// between lanes: `pos` tracks each row's position under row swaps, and the pivot is the one
// partial pivoting picks: the largest magnitude among the rows at positions >= k, ties to
// the smallest position (the wavefront maximum of pivot_key, then an exact comparison among
// the lanes sharing the maximal key). The pivot row reaches the other lanes either through
// `prow` (this wavefront's LDS row, >= NP + 1 entries; kLdsBcast) or lane by lane through
// scalar registers (readlane); the right-hand side rides along as an extra column. Finally
// the row at position k holds x_k * pivot_k; `prow` serves to put x back in lane order. On
// return lane c < NP holds x_c in `x`. Returns 0, or RB_ST_SINGULAR (2) if a pivot was zero
// (the values returned are then meaningless).
template <int NP, bool kLdsBcast, typename T>
__device__ __forceinline__ int lu_solve_rows(T (&a)[NP], T rhs, int lane, T* prow, T& x) {
  int pos = lane;
  T mypiv = T(1);                          // this row's pivot, once it has been the pivot row
  // Pivot search of column k over the rows at positions >= k: the wavefront maximum of the
  // key, the first lane holding it (`tied`: every lane holding it), and, assuming that lane
  // is the pivot, the pivot value and this row's multiplier. Branch-free, so that the search
  // of column k+1 is scheduled among the trailing updates of step k.
  uint64_t tied;
  int pv;
  T piv, l;
  auto search = [&](int k) {
    const bool cand = pos >= k && lane < NP;
    const T av = absv(a[k]);
    uint32_t key = cand ? pivot_key(av) : 0u;
    if (cand && !(av == av)) key = 0xffffffffu;    // a NaN pivot surfaces
    if (cand && key == 0u) key = 1u;               // zero candidates still beat non-candidates
    const uint32_t kmax = wave_max_u32(key);
    tied = __ballot(key == kmax);
    pv = __ffsll(static_cast<unsigned long long>(tied)) - 1;
    piv = bcast(a[k], pv);
    l = lane == pv ? T(0) : a[k] / (piv == T(0) ? T(1) : piv);
  };
  search(0);
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    if (__popcll(tied) > 1) {        // same key: exact magnitude, then smallest position
      const T av = absv(a[k]);
      T bv = bcast(av, pv);
      int best = bcast(pos, pv);
      for (uint64_t m = tied & (tied - 1); m; m &= m - 1) {
        const int l2 = __ffsll(static_cast<unsigned long long>(m)) - 1;
        const T v2 = bcast(av, l2);
        const int p2 = bcast(pos, l2);
        if (v2 > bv || (v2 == bv && p2 < best)) { bv = v2; best = p2; pv = l2; }
      }
      piv = bcast(a[k], pv);
      l = lane == pv ? T(0) : a[k] / (piv == T(0) ? T(1) : piv);
    }
    const int pk = pv;
    const T lk = l;
    const int ppos = bcast(pos, pk);
    const bool me = lane == pk;
    pos = (pos == k) ? ppos : pos;
    pos = me ? k : pos;
    mypiv = me ? piv : mypiv;
    if (kLdsBcast) {
      if (me) {
#pragma unroll
        for (int j = k + 1; j < NP; ++j) prow[j] = a[j];
        prow[NP] = rhs;
      }
      wave_lds_order();
    }
    // Update of columns j > k in chunks of 8; the pivot row's entries come from `prow` or,
    // lane -> SGPR (readlane), as the FMA's scalar operand. The search of column k+1 follows
    // the first chunk (which finishes column k+1) and overlaps the next two.
    auto chunk = [&](int j0) {
      if (kLdsBcast) {
        T pj[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) pj[t] = prow[j0 + t];
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) a[j0 + t] = fma(-lk, pj[t], a[j0 + t]);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t)
          if (j0 + t < NP) a[j0 + t] = fma(-lk, bcast(a[j0 + t], pk), a[j0 + t]);
      }
    };
    chunk(k + 1);
    __builtin_amdgcn_sched_barrier(0);
    if (k + 1 < NP) search(k + 1);
#pragma unroll
    for (int j0 = k + 9; j0 < NP; j0 += 8) {
      chunk(j0);
      if (j0 >= k + 17) __builtin_amdgcn_sched_barrier(0);
    }
    rhs = fma(-lk, kLdsBcast ? prow[NP] : bcast(rhs, pk), rhs);
    if (kLdsBcast) wave_lds_order();
  }
  // Every row is the pivot row of exactly one step, so a zero pivot shows in its row's mypiv
  // (tested here rather than per step, which would keep every step's pivot live).
  const bool zero = lane < NP && mypiv == T(0);
  if (lane < NP) prow[pos] = rhs / (zero ? T(1) : mypiv);
  wave_lds_order();
  x = lane < NP ? prow[lane] : T(0);
  wave_lds_order();
  return __any(zero) ? 2 : 0;
}

}  // namespace rb

namespace rb {

// LDS scratch of gj_solve_mw for one system: candidate rows (double-buffered by step
// parity), candidate values and positions, and the solution vector.
template <int NP, int W, typename T>
struct GjShared {
  static constexpr int kVec = 16 / sizeof(T);      // elements per 16-byte LDS access
  static constexpr int kRow = (NP + 1 + kVec - 1) / kVec * kVec;   // pivot row + rhs, padded
  __attribute__((aligned(16))) T rows[2][W][kRow];
  T cv[2][W];
  int cp[2][W];
  T xs[NP];
  double red[W][2];
};

// Dense solve of one NP x NP system spread over the W wavefronts of a workgroup, one row
// per lane (row = 64*wave + lane; rows >= NP hold nothing), by Gauss-Jordan elimination
// with partial pivoting: column k is eliminated from every row but the pivot row, so no
// back substitution (and no further pass of barriers) is needed. The caller pads the system
// to NP x NP with identity rows and columns and a zero right-hand side there (see
// lu_solve_rows). Rows stay in their lanes; `pos` tracks the position each row would have
// after row swaps, so the pivot is the one partial pivoting picks (largest magnitude, ties to
// the smallest current position). Each step: every wavefront offers its best row (value,
// position, and the row itself in LDS), one barrier, then every lane takes the best of the W
// offers and applies the elimination from the LDS copy (broadcast reads). On return every
// thread of the workgroup can read x from sh.xs (x_c at index c < NP); the return value is 0,
// or 2 if a pivot was zero. Must be called by all threads of the workgroup.
template <int NP, int W, typename T>
__device__ __forceinline__ int gj_solve_mw(T (&a)[NP], T rhs, int row, int lane, int wv,
                                           GjShared<NP, W, T>& sh) {
  constexpr int kRow = GjShared<NP, W, T>::kRow;
  constexpr int kVec = GjShared<NP, W, T>::kVec;
  typedef T vec_t __attribute__((ext_vector_type(kVec)));
  int pos = row;
  T mypiv = T(1);                          // this row's pivot, once it has been the pivot row
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const int buf = k & 1;
    const bool cand = pos >= k && row < NP;
    const T av = absv(a[k]);
    uint32_t key = cand ? pivot_key(av) : 0u;
    if (cand && !(av == av)) key = 0xffffffffu;    // a NaN pivot surfaces
    if (cand && key == 0u) key = 1u;               // zero candidates still beat non-candidates
    const uint32_t kmax = wave_max_u32(key);
    const uint64_t tied = kmax ? __ballot(key == kmax) : 0ull;   // none: no candidate here
    int pl = tied ? __ffsll(static_cast<unsigned long long>(tied)) - 1 : -1;
    T vmax = pl >= 0 ? bcast(av, pl) : T(-1);
    if (pl >= 0 && __popcll(tied) > 1) {  // same key: exact magnitude, then smallest position
      int best = bcast(pos, pl);
      for (uint64_t m = tied & (tied - 1); m; m &= m - 1) {
        const int l2 = __ffsll(static_cast<unsigned long long>(m)) - 1;
        const T v2 = bcast(av, l2);
        const int p2 = bcast(pos, l2);
        if (v2 > vmax || (v2 == vmax && p2 < best)) { vmax = v2; best = p2; pl = l2; }
      }
    }
    if (pl >= 0 && !(vmax == vmax)) vmax = static_cast<T>(__builtin_huge_val());
    if (lane == pl) {                     // 16-byte stores of a[k..NP) and the rhs
#pragma unroll
      for (int j0 = k & ~(kVec - 1); j0 < kRow; j0 += kVec) {
        vec_t v;
#pragma unroll
        for (int t = 0; t < kVec; ++t)
          v[t] = j0 + t < NP ? a[j0 + t < NP ? j0 + t : 0] : (j0 + t == NP ? rhs : T(0));
        *reinterpret_cast<vec_t*>(&sh.rows[buf][wv][j0]) = v;
      }
    }
    const int ppos_w = pl >= 0 ? bcast(pos, pl) : 0x7fffffff;
    if (lane == 0) {
      sh.cv[buf][wv] = pl >= 0 ? vmax : T(-1);
      sh.cp[buf][wv] = ppos_w;
    }
    __syncthreads();
    int ws = 0;
    T bv = sh.cv[buf][0];
    int bp = sh.cp[buf][0];
#pragma unroll
    for (int w = 1; w < W; ++w) {
      const T v2 = sh.cv[buf][w];
      const int p2 = sh.cp[buf][w];
      const bool take = (v2 > bv) || (v2 == bv && p2 < bp);
      ws = take ? w : ws;
      bv = take ? v2 : bv;
      bp = take ? p2 : bp;
    }
    const T* pr = &sh.rows[buf][ws][0];
    const T piv = pr[k];
    const bool me = (wv == ws) && (lane == pl);
    pos = (pos == k) ? bp : pos;
    pos = me ? k : pos;
    mypiv = me ? piv : mypiv;
    const T l = me ? T(0) : a[k] / (piv == T(0) ? T(1) : piv);
#pragma unroll
    for (int j0 = (k + 1) & ~(kVec - 1); j0 < kRow; j0 += 2 * kVec) {
      vec_t pj[2];
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2)
        if (j0 + h2 * kVec < kRow) pj[h2] = *reinterpret_cast<const vec_t*>(&pr[j0 + h2 * kVec]);
#pragma unroll
      for (int h2 = 0; h2 < 2; ++h2) {
#pragma unroll
        for (int t = 0; t < kVec; ++t) {
          const int j = j0 + h2 * kVec + t;
          if (j > k && j < NP) a[j] = fma(-l, pj[h2][t], a[j]);
          else if (j == NP) rhs = fma(-l, pj[h2][t], rhs);
        }
      }
      // pin the chunk's updates here: otherwise they sink to their next use, past the next
      // step's pivot search, and every value read from the pivot row stays live until then
      // (beyond 104 unknowns the pins make the compile take tens of minutes, so not there)
      if constexpr (NP <= 104) {
#pragma unroll
        for (int j = j0; j < j0 + 2 * kVec; ++j) {
          if (j > k && j < NP) asm volatile("" : "+v"(a[j]));
          else if (j == NP) asm volatile("" : "+v"(rhs));
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // a zero pivot shows in its row's mypiv (every row is the pivot row of exactly one step)
  const bool zero = row < NP && mypiv == T(0);
  if (row < NP) sh.xs[pos] = rhs / (zero ? T(1) : mypiv);
  return __syncthreads_or(zero) ? 2 : 0;
}

// Sum of a per-thread double over the workgroup (W wavefronts), two values at once.
template <int W>
__device__ __forceinline__ void block_sum2(double& s0, double& s1, int lane, int wv,
                                           double (&red)[W][2]) {
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) { red[wv][0] = s0; red[wv][1] = s1; }
  __syncthreads();
  s0 = 0.0;
  s1 = 0.0;
#pragma unroll
  for (int w = 0; w < W; ++w) { s0 += red[w][0]; s1 += red[w][1]; }
}

}  // namespace rb

namespace rb {

// One Newton update of one request whose system is spread over the W wavefronts of the
// workgroup (NP > 64). Loads J row by row into the lanes (J[i][c] = jload(c, i)), forms the
// right-hand side -F(u) via rhs_of(row, J_row . u), solves by gj_solve_mw, and adds the
// correction to the FP64 iterate. Returns the status flag (0 ok, 2 singular, 3 non-finite)
// and the squared H-norms of the update and of the new iterate. Uniform over the workgroup;
// every thread must call it.
template <typename T, int NP, int W, typename JLoad, typename RhsOf>
__device__ __forceinline__ int mw_newton_update(JLoad jload, int N, int Nm,
                                                double* __restrict__ ub,
                                                const double* __restrict__ H, RhsOf rhs_of,
                                                GjShared<NP, W, T>& sh, double& nd2,
                                                double& nu2) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, row = wv * 64 + lane;
  const int rc = row < N ? row : N - 1;
  T r[NP];
  T ju = T(0);
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NP; ++c) r[c] = jload(c < N ? c : N - 1, rc);
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    r[c] = (c < N && row < N) ? r[c] : (c == row ? T(1) : T(0));
    ju = fma(r[c], static_cast<T>(ub[c]), ju);
    bad |= !finite_val(r[c]);
  }
  double rhs64 = row < N ? rhs_of(row, ju) : 0.0;
  const T rhs = static_cast<T>(rhs64);
  bad |= !finite_val(rhs);
  int flag = __syncthreads_or(bad) ? 3 : 0;
  if (flag == 0) flag = gj_solve_mw<NP, W, T>(r, rhs, row, lane, wv, sh);
  if (flag != 0) return flag;
  const double dx = row < N ? static_cast<double>(sh.xs[row]) : 0.0;
  const double un = (row < N ? ub[row] : 0.0) + dx;
  double hd = dx, hu = un;
  if (H) {
    hd = 0.0;
    hu = 0.0;
    for (int c = 0; c < N; ++c) {
      const double h = H[(int64_t)c * Nm + rc];
      const double xc = static_cast<double>(sh.xs[c]);
      hd = fma(h, xc, hd);
      hu = fma(h, ub[c] + xc, hu);
    }
  }
  if (row >= N) { hd = 0.0; hu = 0.0; }
  nd2 = dx * hd;
  nu2 = un * hu;
  __syncthreads();                        // every lane has read ub before it is overwritten
  block_sum2<W>(nd2, nu2, lane, wv, sh.red);
  if (!finite_val(nd2) || !finite_val(nu2)) return 3;
  if (row < N) ub[row] = un;
  return 0;
}

}  // namespace rb
