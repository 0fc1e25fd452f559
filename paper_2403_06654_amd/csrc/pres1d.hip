// Batched one-dimensional Chebyshev-collocation pressure operators (Sec. 3.2:
// L_rho and K_rho with Neumann walls): the launches for up to 256 unknowns.
// The kernel is the batched solver of visc1d_kernel.hpp with the pressure
// operator family; it is built apart so that the viscous instantiations stay
// as they are.
#include "visc1d_kernel.hpp"

namespace vd {

template <int OP>
static hipError_t pres1d_dispatch(const Visc1dArgs& a, hipStream_t st) {
  switch (visc1d_tpw(a.ni)) {
    case 1: return launch_tpw<1, OP>(a, st);
    case 2: return launch_tpw<2, OP>(a, st);
    case 3: return launch_tpw<3, OP>(a, st);
    case 4: return launch_tpw<4, OP>(a, st);
    default: return pres1d_launch_large(a, st);
  }
}

hipError_t pres1d_launch(const Visc1dArgs& a, hipStream_t st) {
  if (a.op == OP1D_PRES_L) return pres1d_dispatch<OP1D_PRES_L>(a, st);
  if (a.op == OP1D_PRES_K) return pres1d_dispatch<OP1D_PRES_K>(a, st);
  return hipErrorInvalidValue;
}

}  // namespace vd
