// Instantiations of the FP32 mixed-precision contraction for tensor lengths KT = 68..152
// (multiples of 4), i.e. Qc*N up to 608.
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
  const int grid = (int)(g.Bp / kTile) * g.nsplit;
  hipLaunchKernelGGL((contract_lp_kernel<kBF16, KT>), dim3(grid), dim3(kThreads), lds, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int contract_lp_f32_wide(int KT, const ContractLpArgs& g, hipStream_t st) {
  switch (KT) {
#define RB_KT(n) case n: return go_c<false, n>(g, st);
    RB_KT(68) RB_KT(72) RB_KT(76) RB_KT(80) RB_KT(84) RB_KT(88) RB_KT(92) RB_KT(96) RB_KT(100)
    RB_KT(104) RB_KT(108) RB_KT(112) RB_KT(116) RB_KT(120) RB_KT(124) RB_KT(128) RB_KT(132)
    RB_KT(136) RB_KT(140) RB_KT(144) RB_KT(148) RB_KT(152)
#undef RB_KT
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
