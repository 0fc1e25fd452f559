// Batched one-dimensional implicit viscous solver: workspace sizes and the
// launches of the viscous operator for up to 256 unknowns (the kernel is in visc1d_kernel.hpp; larger
// systems are launched from visc1d_large.hip, built with the compiler's
// default MFMA register forms).
#include "visc1d_kernel.hpp"

namespace vd {

size_t visc1d_work_doubles(int tpw, int mode, int solver, int restart) {
  const size_t V = (size_t)visc1d_rows(tpw) * kG;
  size_t n = 5 * V;
  if (mode == VISC1D_SOLVE && solver == VISC1D_CG) n += V;  // the search direction
  if (mode == VISC1D_SOLVE && solver == VISC1D_GMRES) {
    const size_t m = (size_t)restart;
    n += (m + 1) * V + ((m + 1) * m + 2 * m + (m + 1)) * kG;
  }
  return n;
}

hipError_t visc1d_launch(const Visc1dArgs& a, hipStream_t st) {
  if (a.op != OP1D_VISC) return pres1d_launch(a, st);
  switch (visc1d_tpw(a.ni)) {
    case 1: return launch_tpw<1, OP1D_VISC>(a, st);
    case 2: return launch_tpw<2, OP1D_VISC>(a, st);
    case 3: return launch_tpw<3, OP1D_VISC>(a, st);
    case 4: return launch_tpw<4, OP1D_VISC>(a, st);
    default: return visc1d_launch_large(a, st);
  }
}

}  // namespace vd
