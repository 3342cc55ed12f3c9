// Instantiations of the matrix-core FP64 solves (Newton step and pressure) per tile count
// NT = 1..4 (systems of up to 16*NT - 1 unknowns).
#include "rb_launch.hpp"
#include "rb_mfma_lu.hpp"

namespace rb {
namespace launch {

int lu_f64_mfma(const NewtonF64Args& a, int it, hipStream_t st) {
  const dim3 grid((a.B + kWaves - 1) / kWaves);
  switch (mlu_tiles(a.N)) {
#define RB_C(nt) case nt: hipLaunchKernelGGL((lu_mfma_f64_kernel<nt>), grid, dim3(kThreads), 0, st, a, it); break;
    RB_C(1) RB_C(2) RB_C(3) RB_C(4)
#undef RB_C
    default: return -5;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int plu_f64_mfma(const PressureF64Args& a, hipStream_t st) {
  const dim3 grid((a.B + kWaves - 1) / kWaves);
  switch (mlu_tiles(a.Np)) {
#define RB_C(nt) case nt: hipLaunchKernelGGL((plu_mfma_f64_kernel<nt>), grid, dim3(kThreads), 0, st, a); break;
    RB_C(1) RB_C(2) RB_C(3) RB_C(4)
#undef RB_C
    default: return -5;
  }
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace launch
}  // namespace rb
