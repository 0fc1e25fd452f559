// Batched one-dimensional pressure operators: launches for 257 to 512
// unknowns (built with the compiler's default MFMA register forms, like the
// large viscous systems, since these instantiations spill).
#include "visc1d_kernel.hpp"

namespace vd {

template <int OP>
static hipError_t pres1d_large_dispatch(const Visc1dArgs& a, hipStream_t st) {
  switch (visc1d_tpw(a.ni)) {
    case 5: return launch_tpw<5, OP>(a, st);
    case 6: return launch_tpw<6, OP>(a, st);
    case 7: return launch_tpw<7, OP>(a, st);
    case 8: return launch_tpw<8, OP>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t pres1d_launch_large(const Visc1dArgs& a, hipStream_t st) {
  if (a.op == OP1D_PRES_L) return pres1d_large_dispatch<OP1D_PRES_L>(a, st);
  if (a.op == OP1D_PRES_K) return pres1d_large_dispatch<OP1D_PRES_K>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace vd
