// Instantiations of the multi-wavefront (Gauss-Jordan) FP64 Newton LU kernel for NP = 72..96
// (multiples of 8); W = ceil(NP/64) wavefronts per system.
#include "rb_launch.hpp"

namespace rb {
namespace launch {

template <int NP>
static int go_f64(const NewtonF64Args& a, int it, hipStream_t st) {
  constexpr int W = (NP + kWave - 1) / kWave;
  hipLaunchKernelGGL((lu_f64_mw_kernel<NP, W>), dim3(a.B), dim3(kWave * W), 0, st, a, it);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int lu_f64_mw(int NP, const NewtonF64Args& a, int it, hipStream_t st) {
  switch (NP) {
#define RB_C(n) case n: return go_f64<n>(a, it, st);
    RB_C(72) RB_C(80) RB_C(88) RB_C(96)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
