// Host set-up of the Chebyshev wall-normal direction (x periodic, z on the
// Chebyshev-Gauss-Lobatto points of [-1, 1], Neumann walls).
//
// The pressure operator is the Galerkin weak form of div(a grad p) = f on the
// nodal polynomial space of the CGL points, with z integrals taken by
// Legendre-Gauss-Lobatto quadrature after interpolation I from the CGL nodes:
//     A p = I^T D_x^T (W a_L D_x I p) + G^T (W a_L G p),   G = I D_z,
//     b   = -I^T W I f,   W = h_x diag(w_LGL),   a_L = 1 / (I rho),
// symmetric positive semi-definite with nullspace {1, (-1)^i} x {1}.  Its
// constant-density inverse per x wavenumber is (h_x / rho0)^-1 times the
// inverse of k'^2 M_z + S_z, M_z = I^T diag(w) I, S_z = G^T diag(w) G.  With
// the generalised eigenvectors S_z V = M_z V Lambda, V^T M_z V = 1 the
// inverse is V diag(1 / (k'^2 + lambda_j)) V^T for every kx: two dense
// contractions with kx-independent matrices (the one place where the
// operator is a dense product, done with MFMA).
#pragma once

#include <vector>

namespace vd {

struct ChebSetup {
  int nz = 0;                  // CGL points (M + 1)
  std::vector<double> zc;      // CGL nodes, descending
  std::vector<double> zl, wl;  // LGL nodes (descending) and weights
  std::vector<double> D;       // CGL first-derivative matrix [nz][nz]
  std::vector<double> I;       // interpolation CGL -> LGL [nz][nz]
  std::vector<double> G;       // I D
  std::vector<double> V;       // generalised eigenvectors, column j = v_j [nz][nz]
  std::vector<double> lam;     // eigenvalues, ascending (lam[0] ~ 0: constants)
};

// Builds every matrix above for nz = M + 1 nodes.  Returns false if the
// eigen-solver did not converge.
bool cheb_setup(int nz, ChebSetup* out);

}  // namespace vd
