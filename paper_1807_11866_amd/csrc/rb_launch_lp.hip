// Instantiations of the mixed-precision kernels: FP32 / BF16 contraction per tensor length
// and the FP32 LU (iteration and refinement) per size bucket.
#include "rb_launch.hpp"

namespace rb {
namespace launch {

template <bool kBF16, int KT>
static int go_c(const ContractLpArgs& g, hipStream_t st) {
  const size_t lds = (size_t)contract_lp_lds_bytes(g.N);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)contract_lp_kernel<kBF16, KT>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -3;
  const int grid = (int)(g.Bp / kTile) * kSplit;
  hipLaunchKernelGGL((contract_lp_kernel<kBF16, KT>), dim3(grid), dim3(kThreads), lds, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int contract_lp(bool bf16, int KT, const ContractLpArgs& g, hipStream_t st) {
  if (bf16) {
    switch (KT) {
#define RB_KT(n) case n: return go_c<true, n>(g, st);
      RB_KT(1) RB_KT(2) RB_KT(3) RB_KT(4) RB_KT(5) RB_KT(6) RB_KT(7) RB_KT(8)
#undef RB_KT
    }
    return -5;
  }
  switch (KT) {
#define RB_KT(n) case n: return go_c<false, n>(g, st);
    RB_KT(2) RB_KT(4) RB_KT(6) RB_KT(8) RB_KT(10) RB_KT(12) RB_KT(14) RB_KT(16) RB_KT(18)
    RB_KT(20) RB_KT(22) RB_KT(24) RB_KT(26) RB_KT(28) RB_KT(30) RB_KT(32) RB_KT(34) RB_KT(36)
    RB_KT(38) RB_KT(40) RB_KT(42) RB_KT(44) RB_KT(46) RB_KT(48) RB_KT(50) RB_KT(52) RB_KT(54)
    RB_KT(56) RB_KT(58) RB_KT(60) RB_KT(62) RB_KT(64)
#undef RB_KT
  }
  return -5;
}

template <int NP>
static int go_lu(bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  const dim3 grid((a.B + kWaves - 1) / kWaves);
  if (refine)
    hipLaunchKernelGGL((lu_lp_kernel<NP, true>), grid, dim3(kThreads), 0, st, a, it);
  else
    hipLaunchKernelGGL((lu_lp_kernel<NP, false>), grid, dim3(kThreads), 0, st, a, it);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int lu_lp(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  switch (NP) {
#define RB_C(n) case n: return go_lu<n>(refine, a, it, st);
    RB_C(4) RB_C(8) RB_C(12) RB_C(16) RB_C(20) RB_C(24) RB_C(28) RB_C(32) RB_C(36) RB_C(40)
    RB_C(44) RB_C(48) RB_C(52) RB_C(56) RB_C(60) RB_C(64)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
