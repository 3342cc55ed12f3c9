// Instantiations of the multi-wavefront (Gauss-Jordan) FP32 mixed-precision LU kernel for
// NP = 72..104 (multiples of 8; larger systems: rb_launch_lu_mw_wide*.hip, FP64 Newton
// systems: rb_launch_lu_mw_f64.hip); W = ceil(NP/64) wavefronts per system. The sizes are
// spread over several translation units so that they compile in parallel.
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

int lu_lp_mw(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st) {
  if (NP > 104) return lu_lp_mw_wide(NP, refine, a, it, st);
  switch (NP) {
#define RB_C(n) case n: return go_lp<n>(refine, a, it, st);
    RB_C(72) RB_C(80) RB_C(88) RB_C(96) RB_C(104)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
