// Batched one-dimensional implicit viscous solver: launches for 257 to 512
// unknowns.  These instantiations keep more vectors live than the register
// file holds and spill; they are built apart from visc1d.hip because the
// VGPR-form MFMA selection used there does not handle spilling kernels.
#include "visc1d_kernel.hpp"

namespace vd {

hipError_t visc1d_launch_large(const Visc1dArgs& a, hipStream_t st) {
  switch (visc1d_tpw(a.ni)) {
    case 5: return launch_tpw<5, OP1D_VISC>(a, st);
    case 6: return launch_tpw<6, OP1D_VISC>(a, st);
    case 7: return launch_tpw<7, OP1D_VISC>(a, st);
    case 8: return launch_tpw<8, OP1D_VISC>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vd
