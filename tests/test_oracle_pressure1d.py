"""Pins for oracle.pressure1d: the one-dimensional Chebyshev-collocation
pressure operators with Neumann walls of Sec. 3.2 (eqs. VDINSE.Lrho and
VDINSE.Krho) and the pseudo-inverse of the Neumann Laplacian that
preconditions them.

Closed forms: for polynomial densities and fields that satisfy the Neumann
condition the collocation operators are exact at the nodes (D1 and D2 are
exact on polynomials of degree <= m), so they must reproduce the calculus
formulas; psi = rho^-1/2 polynomial gives the K_rho coefficient in closed
form.  Invariants: nullspaces, the Moore-Penrose conditions, one iteration
at constant density, dense solves.  Then the paper's statements about
these operators (Figs. 5-7): which of them the discretisation reproduces."""
import numpy as np
import pytest

from oracle import krylov, pressure1d as p1


def _poly(n):
    """x, rho = 2 + x^2, phi = x^2 - x^4/2 (phi'(+-1) = 0) and their
    derivatives at the n Chebyshev-Gauss-Lobatto points."""
    x = p1.points(n)
    rho, rp, rpp = 2 + x ** 2, 2 * x, 2 + 0 * x
    phi, dphi, d2phi = x ** 2 - x ** 4 / 2, 2 * x - 2 * x ** 3, 2 - 6 * x ** 2
    return x, rho, rp, rpp, phi, dphi, d2phi


@pytest.mark.parametrize("n", [9, 17, 33, 65])
def test_neumann_extension(n):
    x, d1, _, _, _, P = p1.matrices(n)
    scale = np.abs(d1).max()
    # the extended field has zero collocation derivative at both walls
    assert np.abs((d1 @ P)[[0, n - 1]]).max() < 1e-13 * scale * n
    # constants extend to constants; a Neumann polynomial to itself
    np.testing.assert_allclose(P @ np.ones(n - 2), np.ones(n), atol=1e-12)
    _, _, _, _, phi, _, _ = _poly(n)
    np.testing.assert_allclose(P @ phi[1:-1], phi, atol=1e-12)
    np.testing.assert_allclose(p1.extend(phi[1:-1]), phi, atol=1e-12)


@pytest.mark.parametrize("n", [9, 17, 33, 65])
def test_L_closed_form(n):
    """L_rho phi = phi''/rho - rho' phi'/rho^2 at the interior nodes."""
    x, rho, rp, rpp, phi, dphi, d2phi = _poly(n)
    exact = (d2phi / rho - rp * dphi / rho ** 2)[1:-1]
    got = p1.operator_L(rho) @ phi[1:-1]
    assert np.abs(got - exact).max() < 1e-13 * n ** 4 * np.abs(exact).max()
    # the divergence form gives the same values: d/dx(phi'/rho)
    div = (d2phi * rho - dphi * rp) / rho ** 2
    np.testing.assert_allclose(div[1:-1], exact, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", [9, 17, 33, 65])
def test_K_literal_closed_form(n):
    """K_rho phi = phi'' + (rho''/(2 rho) - 3/4 rho'^2/rho^2) phi (the
    printed coefficient, exact here because rho is a polynomial)."""
    x, rho, rp, rpp, phi, dphi, d2phi = _poly(n)
    c = rpp / (2 * rho) - 0.75 * rp ** 2 / rho ** 2
    exact = (d2phi + c * phi)[1:-1]
    got = p1.operator_K(rho, literal=True) @ phi[1:-1]
    assert np.abs(got - exact).max() < 1e-13 * n ** 4 * np.abs(exact).max()
    np.testing.assert_allclose(p1.k_coefficient_literal(rho), c[1:-1], atol=1e-15 * n ** 4)


@pytest.mark.parametrize("n", [9, 17, 33, 65])
def test_K_psi_form_closed_form_and_null_vector(n):
    """psi = 2 + x^2 - x^4/2 (psi'(+-1) = 0), rho = psi^-2: the coefficient
    -D2 psi / psi equals -psi''/psi exactly, psi is a null vector of K_rho,
    and the printed coefficient (rho no longer a polynomial) converges to
    the same function spectrally."""
    x = p1.points(n)
    psi = 2 + x ** 2 - x ** 4 / 2
    d2psi = 2 - 6 * x ** 2
    rho = psi ** -2
    c = p1.k_coefficient(rho)
    np.testing.assert_allclose(c, (-d2psi / psi)[1:-1], rtol=1e-13 * n ** 2, atol=1e-13 * n ** 2)
    K = p1.operator_K(rho)
    assert np.linalg.norm(K @ psi[1:-1]) < 1e-12 * n ** 4 * np.linalg.norm(psi)
    lit = p1.k_coefficient_literal(rho)
    err = np.abs(lit - c).max() / np.abs(c).max()
    if n >= 33:
        assert err < 1e-8
    else:
        assert err < 0.2


def test_literal_coefficient_converges_spectrally():
    errs = []
    for n in (17, 33, 65):
        x = p1.points(n)
        psi = 2 + x ** 2 - x ** 4 / 2
        rho = psi ** -2
        errs.append(np.abs(p1.k_coefficient_literal(rho) - p1.k_coefficient(rho)).max())
    # spectral convergence down to the rounding floor of D2 (~ eps n^4)
    assert errs[1] < 1e-3 * errs[0] and errs[2] < 2e-15 * 65 ** 4


@pytest.mark.parametrize("n", [17, 65])
def test_nullspaces(n):
    x = p1.points(n)
    rho = p1.tophat(x, 3.0)
    one = np.ones(n - 2)
    D2N = p1.laplacian(n)
    scale = np.abs(D2N).max()
    assert np.abs(D2N @ one).max() < 1e-12 * scale
    assert np.abs(p1.operator_L(rho) @ one).max() < 1e-12 * scale
    psi = rho[1:-1] ** -0.5
    assert np.abs(p1.operator_K(rho) @ psi).max() < 1e-12 * scale
    # exactly one null direction each (the next singular value is O(1))
    for A in (D2N, p1.operator_L(rho), p1.operator_K(rho)):
        sv = np.linalg.svd(A, compute_uv=False)
        assert sv[-1] < 1e-10 * sv[0] and sv[-2] > 1e-3


@pytest.mark.parametrize("n", [17, 65, 257])
def test_preconditioner_is_the_moore_penrose_inverse(n):
    A = p1.laplacian(n)
    X = p1.laplacian_pinv(n)
    s = np.abs(A).max() * np.abs(X).max()
    assert np.abs(A @ X @ A - A).max() < 1e-12 * s * np.abs(A).max()
    assert np.abs(X @ A @ X - X).max() < 1e-12 * s * np.abs(X).max()
    AX, XA = A @ X, X @ A
    assert np.abs(AX - AX.T).max() < 1e-11 * s and np.abs(XA - XA.T).max() < 1e-11 * s
    # XA is the orthogonal projector onto the zero-mean vectors
    one = np.ones(n - 2) / np.sqrt(n - 2)
    np.testing.assert_allclose(XA, np.eye(n - 2) - np.outer(one, one), atol=1e-10)


@pytest.mark.parametrize("form", ["L", "K"])
@pytest.mark.parametrize("solver", ["gmres", "rmr", "pcg"])
def test_constant_density_converges_in_one_iteration(form, solver):
    """At constant density both operators are multiples of the Neumann
    Laplacian (c = 0), so the preconditioned system is the identity on the
    range and every method converges in one iteration."""
    n = 33
    rho = np.full(n, 1.7)
    A = p1.operator_L(rho) if form == "L" else p1.operator_K(rho)
    if form == "K":
        assert np.abs(p1.k_coefficient(rho)).max() < 1e-10
    X = p1.laplacian_pinv(n)
    b = p1.range_part(A, np.random.default_rng(1).standard_normal(n - 2))
    res = getattr(krylov, solver)(lambda u: A @ u, b, lambda r: X @ r, rtol=1e-11)
    assert res["status"] == "converged" and res["iterations"] == 1


@pytest.mark.parametrize("form", ["L", "K"])
@pytest.mark.parametrize("solver", ["gmres", "rmr"])
def test_solves_match_dense(form, solver):
    """Krylov solutions equal the dense least-squares solution modulo the
    null vector (constants for L_rho, psi for K_rho)."""
    n, s = 33, 2.0
    rho = p1.tophat(p1.points(n), s)
    A = p1.operator_L(rho) if form == "L" else p1.operator_K(rho)
    null = np.ones(n - 2) if form == "L" else rho[1:-1] ** -0.5
    null = null / np.linalg.norm(null)
    b = p1.range_part(A, np.random.default_rng(2).standard_normal(n - 2))
    ref = np.linalg.lstsq(A, b, rcond=1e-12)[0]
    res = getattr(krylov, solver)(lambda u: A @ u, b, lambda r: p1.laplacian_pinv(n) @ r,
                                  rtol=1e-11, max_iter=400)
    assert res["status"] == "converged"
    d = res["x"] - ref
    d -= (null @ d) * null
    assert np.linalg.norm(d) <= 1e-8 * np.linalg.norm(ref)


# ------------------------------------------------------ the paper's statements

def _forms(n, s):
    rho = p1.tophat(p1.points(n), s)
    return p1.operator_L(rho), p1.operator_K(rho), p1.laplacian_pinv(n)


def test_both_operators_ill_conditioned_and_growing_with_n():
    """Sec. 3.2: L_rho and K_rho are both ill-conditioned (like V_rho, whose
    condition numbers Sec. 3.1 places at 1e4-1e8)."""
    prev = None
    for n in (65, 129, 257):
        L, K, _ = _forms(n, 2.0)
        kl, kk = p1.kappa(L, 1), p1.kappa(K, 1)
        assert kl > 1e5 and kk > 1e5
        if prev:
            assert kl > 10 * prev[0] and kk > 10 * prev[1]
        prev = (kl, kk)
    assert prev[0] > 1e7 and prev[1] > 1e7


@pytest.mark.parametrize("s", [0.1, 0.5, 2.0, 10.0, 100.0])
def test_preconditioned_K_better_than_preconditioned_L(s):
    """Sec. 3.2 (Fig. 6): kappa(Lap^-1 K_rho) < kappa(Lap^-1 L_rho) for
    0.1 <= s <= 100, at N = 256."""
    L, K, X = _forms(257, s)
    assert p1.kappa(X @ K, 1) < p1.kappa(X @ L, 1)


def test_preconditioned_K_independent_of_n():
    """Sec. 3.2 (Fig. 5): the preconditioned K_rho has a condition number
    independent of N, left and right, and O(1)-O(10^2) for moderate s."""
    for s in (0.5, 2.0, 10.0):
        left, right = [], []
        for n in (65, 129, 257):
            _, K, X = _forms(n, s)
            left.append(p1.kappa(X @ K, 1))
            right.append(p1.kappa(K @ X, 1))
        for v in (left, right):
            assert max(v) / min(v) < 1.03
        assert max(left + right) < (30 if s <= 2 else 400)


def test_left_preconditioned_L_grows_with_n():
    """Not the paper's picture: on this discretisation kappa(Lap^-1 L_rho)
    grows roughly like N^2 (27, 105, 426 at s = 2), although the right-
    preconditioned L_rho Lap^-1 stays at 2.6.  Reported, not hidden."""
    vals = []
    for n in (65, 129, 257):
        L, _, X = _forms(n, 2.0)
        vals.append((p1.kappa(X @ L, 1), p1.kappa(L @ X, 1)))
    assert vals[1][0] > 3 * vals[0][0] and vals[2][0] > 3 * vals[1][0]
    assert max(v[1] for v in vals) < 3.0


def _histories(s, n=257):
    L, K, X = _forms(n, s)
    b = p1.range_part(K, np.random.default_rng(0).standard_normal(n - 2))
    A = lambda u: K @ u
    M = lambda r: X @ r
    out = {}
    for name, fn, kw in (("gmres", krylov.gmres, dict(restart=30, max_iter=80)),
                         ("rmr", krylov.rmr, dict(max_iter=300)),
                         ("cg", krylov.pcg, dict(max_iter=150))):
        out[name] = np.array(fn(A, b, M, rtol=1e-12, **kw)["history"])
    return out


def _first_below(h, t):
    i = np.nonzero(h <= t)[0]
    return int(i[0]) if i.size else None


def test_convergence_histories_of_K():
    """Sec. 3.2 (Fig. 7 and App. B), K_rho at N = 256, compatible
    right-hand side.  What holds: GMRES has the fastest convergence and its
    residual falls by 12 decades in every case (the paper: in about 10
    iterations; here 16-57, growing with s); RMR is slower than GMRES at
    s = 2 and does not converge for the higher density ratios; CG stalls at
    O(1) for s = 100.  What does not: CG at s <= 2 does reach 1e-9 here
    (the paper sees a plateau near 0.5 for every case)."""
    h2, h10, h100 = _histories(2.0), _histories(10.0), _histories(100.0)
    for h, cap in ((h2, 30), (h10, 60), (h100, 70)):
        assert _first_below(h["gmres"], 1e-12) is not None and _first_below(h["gmres"], 1e-12) <= cap
    # RMR at s = 2: converges, more slowly than GMRES
    g9, r9 = _first_below(h2["gmres"], 1e-9), _first_below(h2["rmr"], 1e-9)
    assert r9 is not None and r9 >= 2 * g9
    # RMR fails for s >= 10
    assert h10["rmr"].min() > 1e-2 and h100["rmr"].min() > 1e-2
    # CG: plateau at O(1) for s = 100, no convergence for s = 10
    assert h100["cg"].min() > 0.3
    assert h10["cg"].min() > 1e-7
    # not reproduced: CG at s = 2 reaches 1e-9
    assert h2["cg"].min() < 1e-9
