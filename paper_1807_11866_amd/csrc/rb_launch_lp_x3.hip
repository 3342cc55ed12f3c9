// Instantiations of the BF16x3 (hi/lo split) mixed-precision contraction for tensor lengths
// KT = 1..20 k-steps of 32, i.e. Qc*N up to 640.
#include "rb_launch.hpp"

namespace rb {
namespace launch {

template <int KT>
static int go_c(const ContractLpArgs& g, hipStream_t st) {
  if (!g.op_lo) return -5;
  const size_t lds = (size_t)contract_lp_lds_bytes(g.N);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)contract_lp_kernel<true, KT, true>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -3;
  const int grid = (int)(g.Bp / kTile) * g.nsplit;
  hipLaunchKernelGGL((contract_lp_kernel<true, KT, true>), dim3(grid), dim3(kThreads), lds, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int contract_lp_bf16x3(int KT, const ContractLpArgs& g, hipStream_t st) {
  switch (KT) {
#define RB_KT(n) case n: return go_c<n>(g, st);
    RB_KT(1) RB_KT(2) RB_KT(3) RB_KT(4) RB_KT(5) RB_KT(6) RB_KT(7) RB_KT(8) RB_KT(9) RB_KT(10)
    RB_KT(11) RB_KT(12) RB_KT(13) RB_KT(14) RB_KT(15) RB_KT(16) RB_KT(17) RB_KT(18) RB_KT(19)
    RB_KT(20)
#undef RB_KT
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
