"""One-dimensional Chebyshev-collocation pressure operators with Neumann
walls, and their constant-density preconditioner.  Oracle; test
infrastructure only.

Sec. 3.2 studies the pressure operators on a 1D test discretised with
Chebyshev collocation matrices, with the top-hat density of eq.
VDINSE.rho.hat and wall conditions d(rho)/dn = d(phi)/dn = 0 (so that
d(Phi)/dn = 0 too):

    L_rho phi = d/dx (rho^-1 dphi/dx)                      (eq. VDINSE.Lrho)
    K_rho Phi = d2Phi/dx2 + c Phi,
        c = rho'' / (2 rho) - (3/4) rho'^2 / rho^2         (eq. VDINSE.Krho)

preconditioned by the inverse of the discrete Laplacian, the inverse of
K_rho at constant density.  The paper does not spell out the discrete form;
the readings taken here:

* Points: the n Chebyshev-Gauss-Lobatto points x_j = cos(pi j / m),
  m = n - 1 (descending); D1 the collocation first-derivative matrix,
  D2 = D1 D1.
* Neumann walls by elimination: the two wall values are the ones that make
  the collocation derivative vanish at both walls,
      D1[w, w] u_w + D1[w, i] u_i = 0   =>   u_w = E u_i,
  so a field is its n - 2 interior values u_i, extended to every point by
  P = [E_0; I; E_m].  The equations are the interior collocation rows, and
  the discrete operators act on the interior values:  D1N = D1[i, :] P,
  D2N = D2[i, :] P.
* L_rho in its expanded form (1/rho) D2N - (rho'/rho^2) D1N, with
  rho' = D1 rho over every point (the same way eq. VDINSE.Vrho forms the
  density derivatives of the viscous operator).
* K_rho = D2N + diag(c).  c is evaluated as -D2N psi / psi with
  psi = rho^-1/2 on the interior points: by the chain rule
  c = -psi'' / psi for psi = rho^-1/2, and in this form psi is an exact null
  vector of the discrete K_rho (continuum: phi constant <=> Phi ~ psi).
  The printed expression with rho' = D1 rho, rho'' = D2 rho is kept as
  `k_coefficient_literal`; the two agree to the discretisation error.
* Preconditioner: the Moore-Penrose pseudo-inverse of D2N, which is singular
  with the constants as its null vectors (Sec. 4.2 removes the constant
  mode the same way).  L_rho also annihilates the constants, so L_rho and
  K_rho are singular; right-hand sides must lie in their range (a component
  outside it cannot be reduced by any iteration).

The condition numbers of Figs. 5-6 are computed by a singular value
decomposition (as Sec. 3.1 says for the viscous operators) on the range:
the smallest singular value is dropped for each factor that is singular.
"""
import numpy as np

from . import grids


def tophat(x, s, x0=0.4, d=0.1):
    """rho = 1 + (s-1)/2 [tanh((x + x0)/d) - tanh((x - x0)/d)] (eq.
    VDINSE.rho.hat) with x0 one fifth of the domain length 2 and d = 0.1."""
    return 1.0 + 0.5 * (s - 1.0) * (np.tanh((x + x0) / d) - np.tanh((x - x0) / d))


def points(n):
    """The n Chebyshev-Gauss-Lobatto points of [-1, 1], descending."""
    return grids.cheb_points(n - 1)


def neumann_extension(n):
    """P ((n) x (n-2)): every point's value from the interior values, the wall
    values chosen so that the collocation derivative vanishes at both walls."""
    m = n - 1
    d1 = grids.cheb_diff_matrix(m)
    walls, inner = [0, m], slice(1, m)
    E = -np.linalg.solve(d1[np.ix_(walls, walls)], d1[walls, inner])
    P = np.zeros((n, n - 2))
    P[inner] = np.eye(n - 2)
    P[walls] = E
    return P


def matrices(n):
    """(x, D1, D2, D1N, D2N, P): the full collocation matrices and the
    Neumann-eliminated ones on the interior values."""
    m = n - 1
    x = points(n)
    d1 = grids.cheb_diff_matrix(m)
    d2 = d1 @ d1
    P = neumann_extension(n)
    inner = slice(1, m)
    return x, d1, d2, d1[inner] @ P, d2[inner] @ P, P


def operator_L(rho):
    """Dense L_rho on the interior values (expanded form, Neumann walls)."""
    n = rho.size
    _, d1, _, d1n, d2n, _ = matrices(n)
    rp = (d1 @ rho)[1:-1]
    ri = rho[1:-1]
    return (1.0 / ri)[:, None] * d2n - (rp / ri ** 2)[:, None] * d1n


def k_coefficient(rho):
    """c of eq. VDINSE.Krho as -D2N psi / psi, psi = rho^-1/2 (interior)."""
    _, _, _, _, d2n, _ = matrices(rho.size)
    psi = rho[1:-1] ** -0.5
    return -(d2n @ psi) / psi


def k_coefficient_literal(rho):
    """c as printed in eq. VDINSE.Krho, rho' = D1 rho and rho'' = D2 rho."""
    _, d1, d2, _, _, _ = matrices(rho.size)
    rp, rpp = d1 @ rho, d2 @ rho
    c = rpp / (2.0 * rho) - 0.75 * rp ** 2 / rho ** 2
    return c[1:-1]


def operator_K(rho, literal=False):
    """Dense K_rho = D2N + diag(c) on the interior values."""
    _, _, _, _, d2n, _ = matrices(rho.size)
    c = k_coefficient_literal(rho) if literal else k_coefficient(rho)
    return d2n + np.diag(c)


def laplacian(n):
    """D2N: the Neumann Laplacian on the interior values."""
    return matrices(n)[4]


def laplacian_pinv(n):
    """The preconditioner: Moore-Penrose pseudo-inverse of D2N (SVD)."""
    return np.linalg.pinv(laplacian(n), rcond=1e-13)


def kappa(A, nnull=0):
    """sigma_max / sigma_min of A on its range: the nnull smallest singular
    values (those of the null vectors) are dropped."""
    sv = np.linalg.svd(A, compute_uv=False)
    return float(sv[0] / sv[-1 - nnull])


def left_null_vector(A):
    """Unit vector w with w^T A = 0 (the last left singular vector)."""
    U, _, _ = np.linalg.svd(A)
    return U[:, -1]


def range_part(A, f):
    """f minus its component along the left null vector of a singular A:
    the compatible right-hand side nearest to f."""
    w = left_null_vector(A)
    return f - (w @ f) * w


def extend(u_interior):
    """Every point's values from interior ones (the Neumann walls)."""
    return neumann_extension(u_interior.size + 2) @ u_interior
