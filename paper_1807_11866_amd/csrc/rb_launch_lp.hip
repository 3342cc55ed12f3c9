// Instantiations of the mixed-precision contraction: BF16 per tensor length KT <= 20, FP32 per
// even KT <= 64 (longer FP32 tensor parts: rb_launch_lp_wide.hip; BF16x3: rb_launch_lp_x3.hip).
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

int contract_lp(int prec, int KT, const ContractLpArgs& g, hipStream_t st) {
  if (prec == RB_PREC_BF16X3) return contract_lp_bf16x3(KT, g, st);
  if (prec == RB_PREC_BF16) {
    switch (KT) {
#define RB_KT(n) case n: return go_c<true, n>(g, st);
      RB_KT(1) RB_KT(2) RB_KT(3) RB_KT(4) RB_KT(5) RB_KT(6) RB_KT(7) RB_KT(8) RB_KT(9) RB_KT(10)
      RB_KT(11) RB_KT(12) RB_KT(13) RB_KT(14) RB_KT(15) RB_KT(16) RB_KT(17) RB_KT(18) RB_KT(19)
      RB_KT(20)
#undef RB_KT
    }
    return -5;
  }
  if (KT > 64) return contract_lp_f32_wide(KT, g, st);
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

}  // namespace launch
}  // namespace rb
