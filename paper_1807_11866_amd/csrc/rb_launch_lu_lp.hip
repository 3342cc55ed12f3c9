// Instantiations of the FP32 LU of the mixed-precision Newton (iteration and refinement) per
// size bucket NP in 2..64 (even); larger systems go to rb_launch_lu_mw.hip.
#include "rb_launch.hpp"

namespace rb {
namespace launch {

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
  if (NP > 64) return lu_lp_mw(NP, refine, a, it, st);
  switch (NP) {
#define RB_C(n) case n: return go_lu<n>(refine, a, it, st);
    RB_C(2) RB_C(4) RB_C(6) RB_C(8) RB_C(10) RB_C(12) RB_C(14) RB_C(16) RB_C(18) RB_C(20)
    RB_C(22) RB_C(24) RB_C(26) RB_C(28) RB_C(30) RB_C(32) RB_C(34) RB_C(36) RB_C(38) RB_C(40)
    RB_C(42) RB_C(44) RB_C(46) RB_C(48) RB_C(50) RB_C(52) RB_C(54) RB_C(56) RB_C(58) RB_C(60)
    RB_C(62) RB_C(64)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
