// Instantiations of newton_tail_f64_kernel<NP> for the one-wavefront LU sizes NP in 2..64.
#include "rb_launch.hpp"
#include "rb_tail.hpp"

namespace rb {
namespace launch {

template <int NP>
static int go_tail(const ContractArgs& g, const NewtonF64Args& a, int it0, hipStream_t st) {
  const size_t lds = (size_t)tail_lds_bytes(g.N, NP);
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)newton_tail_f64_kernel<NP>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return -3;
  hipLaunchKernelGGL((newton_tail_f64_kernel<NP>), dim3((unsigned)(g.Bp / kTile)),
                     dim3(kThreads), lds, st, g, a, it0);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int newton_tail_f64(int NP, const ContractArgs& g, const NewtonF64Args& a, int it0,
                    hipStream_t st) {
  if (g.nchunk < 1 || (g.nks - g.kA) % g.nchunk || g.R != g.N) return -5;
  switch (NP) {
#define RB_C(n) case n: return go_tail<n>(g, a, it0, st);
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
