// Instantiations of contract_f64_kernel<kModeResid, KT> for every even tensor chunk length KC <= kMaxKC (40).
#include "rb_launch.hpp"

namespace rb {
namespace launch {

template <int KT>
static int go(const ContractArgs& g, hipStream_t st) {
  const size_t lds = (size_t)contract_lds_bytes(g.N, g.R, false);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)contract_f64_kernel<kModeResid, KT>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -3;
  const int grid = (int)(g.Bp / kTile) * g.nsplit;
  hipLaunchKernelGGL((contract_f64_kernel<kModeResid, KT>), dim3(grid), dim3(kThreads), lds, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int contract_f64_resid(const ContractArgs& g, hipStream_t st) {
  if (g.nchunk < 1 || (g.nks - g.kA) % g.nchunk) return -5;
  switch ((g.nks - g.kA) / g.nchunk) {
#define RB_KT(n) case n: return go<n>(g, st);
    RB_KT(2) RB_KT(4) RB_KT(6) RB_KT(8) RB_KT(10) RB_KT(12) RB_KT(14) RB_KT(16) RB_KT(18)
    RB_KT(20) RB_KT(22) RB_KT(24) RB_KT(26) RB_KT(28) RB_KT(30) RB_KT(32) RB_KT(34) RB_KT(36)
    RB_KT(38) RB_KT(40)
#undef RB_KT
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
