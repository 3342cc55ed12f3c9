// Instantiations of the multi-wavefront FP32 LU kernel for NP = 112 and 120, and the
// dispatcher over NP = 112..152 (multiples of 8; 128..152 in rb_launch_lu_mw_wide2.hip and
// rb_launch_lu_mw_wide3.hip, so that the sizes compile in parallel).
#include "rb_launch.hpp"

namespace rb {
namespace launch {

template <int NP>
static int go_lp(bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  constexpr int W = (NP + kWave - 1) / kWave;
  hipLaunchKernelGGL((lu_lp_mw_kernel<NP, W>), dim3(a.B), dim3(kWave * W), 0, st, a, it,
                     refine ? 1 : 0);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int lu_lp_mw_wide(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  if (NP == 128 || NP == 136) return lu_lp_mw_wide2(NP, refine, a, it, st);
  if (NP == 144 || NP == 152) return lu_lp_mw_wide3(NP, refine, a, it, st);
  switch (NP) {
#define RB_C(n) case n: return go_lp<n>(refine, a, it, st);
    RB_C(112) RB_C(120)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
