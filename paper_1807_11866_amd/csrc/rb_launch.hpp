// rb_launch.hpp -- host-side launchers of the templated kernels. Each kernel family is
// instantiated (per size bucket) in its own translation unit so the library builds in
// parallel; the API layer calls these entry points. Return value: 0, RB_E_UNSUPPORTED when
// no instantiation covers the requested size, or RB_E_DEVICE on a launch error.
#pragma once

#include <hip/hip_runtime.h>

#include "rb_lowprec.hpp"
#include "rbns.h"

namespace rb {
namespace launch {

// FP64 contraction (chunk length (g.nks - g.kA) / g.nchunk: even, <= kMaxKC).
int contract_f64(int mode, const ContractArgs& g, hipStream_t st);
// FP64 Newton LU: NP <= 64 one wavefront per system, NP > 64 (multiple of 8, <= 96) one
// workgroup per system.
// `variant` is one of RB_LU_*; RB_LU_MFMA beyond RB_LU_MFMA_MAX_N falls back to readlane.
int lu_f64(int NP, const NewtonF64Args& a, int it, int variant, hipStream_t st);
// The RB_LU_* variant that lu_f64 runs for this NP, N and requested variant (RB_LU_AUTO
// resolved; -1 for the workgroup LU of NP > 64).
int lu_f64_variant(int NP, int N, int variant);
// The Newton iterations it0 .. maxit-1 of the batch in one launch (rb_tail.hpp): for batches
// whose regular launches use the readlane LU (NP <= 64).
int newton_tail_f64(int NP, const ContractArgs& g, const NewtonF64Args& a, int it0,
                    hipStream_t st);
int plu_f64(int NPP, const PressureF64Args& a, int variant, hipStream_t st);
// Low-precision contraction, prec = RB_PREC_F32 (KT even <= 64 or a multiple of 4 <= 152),
// RB_PREC_BF16 (KT <= 20) or RB_PREC_BF16X3 (KT <= 20).
int contract_lp(int prec, int KT, const ContractLpArgs& g, hipStream_t st);
// FP32 LU of the mixed-precision Newton: NP <= 64 or a multiple of 8 <= 152.
int lu_lp(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);

// per-TU pieces behind the dispatchers above
int contract_f64_jac(const ContractArgs& g, hipStream_t st);
int contract_f64_press(const ContractArgs& g, hipStream_t st);
int contract_f64_resid(const ContractArgs& g, hipStream_t st);
int lu_f64_mw(int NP, const NewtonF64Args& a, int it, hipStream_t st);
int lu_f64_mfma(const NewtonF64Args& a, int it, hipStream_t st);
int plu_f64_mfma(const PressureF64Args& a, hipStream_t st);
int lu_lp_mw(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);
int lu_lp_mw_wide(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);
int lu_lp_mw_wide2(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);
int lu_lp_mw_wide3(int NP, bool refine, const LpNewtonArgs& a, int it, hipStream_t st);
int contract_lp_f32_wide(int KT, const ContractLpArgs& g, hipStream_t st);
int contract_lp_bf16x3(int KT, const ContractLpArgs& g, hipStream_t st);

}  // namespace launch
}  // namespace rb
