// Instantiations of the FP64 LU kernels (Newton step and pressure solve) per size bucket
// NP in 2..64 (even), and the dispatcher over the mode-specific contraction TUs.
#include "rb_launch.hpp"

namespace rb {
namespace launch {

int contract_f64(int mode, const ContractArgs& g, hipStream_t st) {
  if (mode == kModeJac) return contract_f64_jac(g, st);
  if (mode == kModePressure) return contract_f64_press(g, st);
  return contract_f64_resid(g, st);
}

template <int NP>
static int go_lu(const NewtonF64Args& a, int it, bool lds, hipStream_t st) {
  const dim3 grid((a.B + kWaves - 1) / kWaves);
  if (lds)
    hipLaunchKernelGGL((lu_f64_kernel<NP, true>), grid, dim3(kThreads), 0, st, a, it);
  else
    hipLaunchKernelGGL((lu_f64_kernel<NP, false>), grid, dim3(kThreads), 0, st, a, it);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

template <int NPP>
static int go_plu(const PressureF64Args& a, bool lds, hipStream_t st) {
  const dim3 grid((a.B + kWaves - 1) / kWaves);
  if (lds)
    hipLaunchKernelGGL((plu_f64_kernel<NPP, true>), grid, dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((plu_f64_kernel<NPP, false>), grid, dim3(kThreads), 0, st, a);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

#define RB_NP_CASES(X) X(4) X(8) X(12) X(16) X(20) X(24) X(28) X(32) X(36) X(40) X(44) X(48) \
  X(52) X(56) X(60) X(64)
#define RB_NP_ODD2(X) X(2) X(6) X(10) X(14) X(18) X(22) X(26) X(30) X(34) X(38) X(42) X(46) \
  X(50) X(54) X(58) X(62)

int lu_f64_variant(int NP, int N, int variant) {
  if (NP > 64) return -1;
  if (variant == RB_LU_AUTO) variant = N <= RB_LU_AUTO_MFMA_N ? RB_LU_MFMA : RB_LU_READLANE;
  if (variant == RB_LU_MFMA && N > RB_LU_MFMA_MAX_N) variant = RB_LU_READLANE;
  return variant;
}

int lu_f64(int NP, const NewtonF64Args& a, int it, int variant, hipStream_t st) {
  variant = lu_f64_variant(NP, a.N, variant);
  if (variant < 0) return lu_f64_mw(NP, a, it, st);
  if (variant == RB_LU_MFMA) return lu_f64_mfma(a, it, st);
  const bool lds = variant == RB_LU_LDS;
  switch (NP) {
#define RB_C(n) case n: return go_lu<n>(a, it, lds, st);
    RB_NP_CASES(RB_C)
    RB_NP_ODD2(RB_C)
#undef RB_C
  }
  return -5;
}

int plu_f64(int NPP, const PressureF64Args& a, int variant, hipStream_t st) {
  if (variant == RB_LU_AUTO) variant = a.Np <= RB_LU_AUTO_MFMA_N ? RB_LU_MFMA : RB_LU_READLANE;
  if (variant == RB_LU_MFMA && a.Np <= RB_LU_MFMA_MAX_N) return plu_f64_mfma(a, st);
  const bool lds = variant == RB_LU_LDS;
  switch (NPP) {
#define RB_C(n) case n: return go_plu<n>(a, lds, st);
    RB_NP_CASES(RB_C)
    RB_NP_ODD2(RB_C)
#undef RB_C
  }
  return -5;
}

}  // namespace launch
}  // namespace rb
