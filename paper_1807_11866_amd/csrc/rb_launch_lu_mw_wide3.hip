// Instantiations of the multi-wavefront FP32 LU kernel for NP = 144 and 152.
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

int lu_lp_mw_wide3(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  switch (NP) {
#define RB_C(n) case n: return go_lp<n>(refine, a, it, st);
    RB_C(144) RB_C(152)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
