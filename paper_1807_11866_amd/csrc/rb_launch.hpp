// rb_launch.hpp -- host-side launchers of the templated kernels. Each kernel family is
// instantiated (per size bucket) in its own translation unit so the library builds in
// parallel; the API layer calls these entry points. Return value: 0, RB_E_UNSUPPORTED when
// no instantiation covers the requested size, or RB_E_DEVICE on a launch error.
#pragma once

#include <hip/hip_runtime.h>

#include "rb_lowprec.hpp"

namespace rb {
namespace launch {

int contract_f64(int mode, const ContractArgs& g, hipStream_t st);
int lu_f64(int NP, const NewtonF64Args& a, int it, bool lds_bcast, hipStream_t st);
int plu_f64(int NPP, const PressureF64Args& a, bool lds_bcast, hipStream_t st);
int contract_lp(bool bf16, int KT, const ContractLpArgs& g, hipStream_t st);
int lu_lp(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);

}  // namespace launch
}  // namespace rb
