"""GPU parity of the batched 1D implicit viscous solver (Sec. 3.1, eq.
VDINSE.Vrho, preconditioner eq. VDINSE.V) against the oracle.

Tolerances: applications are dense FP64 matrix products whose rounding grows
with the matrix norms (D2 ~ N^4 on Chebyshev points), so the operator is
compared at 1e-13 ||D2|| ||u|| / ||V_rho u|| and V^-1 at 1e-14 kappa(V); solves
must have an oracle-evaluated relative residual <= 1e-10 and match a dense LU
solution to 1e-10 kappa(V^-1 V_rho)."""
import numpy as np
import pytest

from oracle import krylov, viscous
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(basis, n, s_list, a, seed=0):
    """Batch of densities (top-hat, one ratio per system) on the grid."""
    if basis == "cheb":
        x, _, _ = viscous.cheb_matrices(n - 1)
        rho = np.stack([viscous.tophat(x, s, 0.4) for s in s_list])
        systems = [viscous.cheb_system(r, a) for r in rho]
    else:
        x, _, _ = viscous.fourier_matrices(n)
        rho = np.stack([viscous.tophat(x - np.pi, s, 2 * np.pi / 5) for s in s_list])
        systems = [viscous.fourier_system(r, a) for r in rho]
    return x, rho, systems


def _inner(basis, v):
    return v[..., 1:-1] if basis == "cheb" else v


@pytest.mark.parametrize("basis,n", [("cheb", 17), ("cheb", 65), ("cheb", 257), ("cheb", 512),
                                     ("fourier", 16), ("fourier", 64), ("fourier", 256), ("fourier", 512)])
def test_apply_parity(basis, n):
    from paper_2403_06654_amd.api import Visc1d
    print(f"case visc1d apply {basis} n={n}", flush=True)
    a = 1e-2
    x, rho, systems = _case(basis, n, [2.0, 10.0, 1000.0], a)
    u = np.random.default_rng(3).standard_normal(rho.shape)
    if basis == "cheb":
        u[:, 0] = u[:, -1] = 0.0
    h = Visc1d(basis, n, a)
    y = to_host(h.apply(to_dev(rho), to_dev(u)))
    z = to_host(h.apply(to_dev(rho), to_dev(u), precond=True))
    _, _, d2 = viscous.cheb_matrices(n - 1) if basis == "cheb" else viscous.fourier_matrices(n)
    for k, (A, V) in enumerate(systems):
        ui = _inner(basis, u[k])
        ref = A @ ui
        tol = 1e-13 * np.linalg.norm(d2, 2) * np.linalg.norm(ui) / np.linalg.norm(ref)
        assert rel2(_inner(basis, y[k]), ref) <= max(tol, 1e-14), (k, rel2(_inner(basis, y[k]), ref), tol)
        zr = np.linalg.solve(V, ui)
        assert rel2(_inner(basis, z[k]), zr) <= 1e-14 * np.linalg.cond(V) + 1e-14
        if basis == "cheb":
            assert y[k, 0] == 0.0 and y[k, -1] == 0.0
    h.close()


@pytest.mark.parametrize("basis,n", [("cheb", 129), ("cheb", 257), ("fourier", 128), ("fourier", 256)])
@pytest.mark.parametrize("solver", ["gmres", "rmr"])
def test_solve_parity(basis, n, solver):
    from paper_2403_06654_amd.api import Visc1d
    print(f"case visc1d solve {basis} n={n} {solver}", flush=True)
    a = 1e-3
    ratios = [1.5, 2.0, 5.0, 10.0]
    x, rho, systems = _case(basis, n, ratios, a)
    b = np.random.default_rng(4).standard_normal(rho.shape)
    h = Visc1d(basis, n, a)
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver=solver, restart=128, max_iter=2000)
    u = to_host(u)
    print(it, rr, info, flush=True)
    assert info["status"] == 0
    for k, (A, V) in enumerate(systems):
        bi, ui = _inner(basis, b[k]), _inner(basis, u[k])
        assert rel2(A @ ui, bi) <= 1.01e-10, (k, rel2(A @ ui, bi))
        ref = np.linalg.solve(A, bi)
        kap = np.linalg.cond(np.linalg.solve(V, A))
        assert rel2(ui, ref) <= 1e-10 * kap, (k, rel2(ui, ref), kap)
        # the same count as the oracle's method, up to rounding (GMRES: MGS there, CGS2 here)
        orc = getattr(krylov, solver)(lambda v: A @ v, bi, lambda r: np.linalg.solve(V, r),
                                      rtol=1e-10, max_iter=2000, **({"restart": 128} if solver == "gmres" else {}))
        assert abs(int(it[k]) - orc["iterations"]) <= 2, (k, it[k], orc["iterations"])
    h.close()


def test_rmr_fails_where_the_paper_says_and_gmres_converges():
    """a = 1e-2, s = 100 on 257 Chebyshev points (Sec. 3.1)."""
    from paper_2403_06654_amd.api import Visc1d, VD_NOT_CONVERGED
    x, rho, systems = _case("cheb", 257, [100.0], 1e-2)
    b = np.random.default_rng(5).standard_normal(rho.shape)
    h = Visc1d("cheb", 257, 1e-2)
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver="rmr", max_iter=500)
    assert info["status"] == VD_NOT_CONVERGED and it[0] == 500 and rr[0] > 1e-10
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver="gmres", restart=128, max_iter=2000)
    assert info["status"] == 0 and rr[0] <= 1e-10
    A, _ = systems[0]
    assert rel2(A @ to_host(u)[0, 1:-1], b[0, 1:-1]) <= 1.01e-10
    h.close()


def test_edge_cases():
    from paper_2403_06654_amd.api import Visc1d, VdError
    n, a = 65, 1e-2
    x, _, _ = viscous.cheb_matrices(n - 1)
    h = Visc1d("cheb", n, a)
    rho = np.stack([np.ones(n), viscous.tophat(x, 3.0, 0.4)])
    # rho = 1: the operator is V, one iteration for both methods
    b = np.random.default_rng(6).standard_normal((2, n))
    for solver in ("gmres", "rmr"):
        u, it, rr, info = h.solve(to_dev(rho[:1]), to_dev(b[:1]), solver=solver)
        assert it[0] == 1 and info["status"] == 0
    # zero right-hand side: zero solution, no iterations
    u, it, rr, info = h.solve(to_dev(rho), to_dev(np.zeros((2, n))))
    assert (it == 0).all() and float(to_host(u).__abs__().max()) == 0.0
    # warm start from the solution needs no iteration; a system alone and in
    # a batch gives the same bits (one workgroup per system)
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), restart=64)
    u1, it1, _, _ = h.solve(to_dev(rho[1:]), to_dev(b[1:]), restart=64)
    assert np.array_equal(to_host(u)[1], to_host(u1)[0]) and it1[0] == it[1]
    u2, it2, _, _ = h.solve(to_dev(rho), to_dev(b), u=u.clone(), restart=64, use_x0=True)
    assert (it2 == 0).all()
    # a non-positive density is rejected
    bad = rho.copy()
    bad[1, 7] = 0.0
    with pytest.raises(VdError):
        h.solve(to_dev(bad), to_dev(b))
    with pytest.raises(VdError):
        h.apply(to_dev(bad), to_dev(b))
    h.close()


def test_ragged_groups_restarts_and_mixed_outcomes():
    """Batches that end inside a group of 16, GMRES cycles shorter than the
    solve (restart 16), and a group whose systems stop at different
    iterations or fail: every system gives the bits it gives alone and the
    iteration count of the oracle's method."""
    from paper_2403_06654_amd.api import Visc1d, VD_NOT_CONVERGED
    n, a = 129, 1e-2
    ratios = [1.5, 2.0, 3.0, 5.0, 8.0, 10.0] * 3   # 18 systems: groups of 16 and 2
    _, rho, systems = _case("cheb", n, ratios, a)
    b = np.random.default_rng(7).standard_normal(rho.shape)
    h = Visc1d("cheb", n, a)
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver="gmres", restart=16, max_iter=3000)
    assert info["status"] == 0
    u = to_host(u)
    for k in (0, 5, 16, 17):
        A, V = systems[k]
        assert rel2(A @ u[k, 1:-1], b[k, 1:-1]) <= 1.01e-10
        orc = krylov.gmres(lambda v: A @ v, b[k, 1:-1], lambda r: np.linalg.solve(V, r), rtol=1e-10,
                           restart=16, max_iter=3000)
        assert abs(int(it[k]) - orc["iterations"]) <= 2, (k, it[k], orc["iterations"])
        u1, it1, _, _ = h.solve(to_dev(rho[k:k + 1]), to_dev(b[k:k + 1]), solver="gmres", restart=16, max_iter=3000)
        assert np.array_equal(to_host(u1)[0], u[k]) and it1[0] == it[k]
    # RMR: s = 100 fails at a = 1e-2 (Sec. 3.1) next to systems that converge
    _, rho2, _ = _case("cheb", n, [2.0, 100.0, 5.0], a)
    b2 = b[:3]
    u2, it2, rr2, info2 = h.solve(to_dev(rho2), to_dev(b2), solver="rmr", max_iter=300)
    assert info2["status"] == VD_NOT_CONVERGED
    assert rr2[0] <= 1e-10 and rr2[2] <= 1e-10 and rr2[1] > 1e-10 and it2[1] == 300
    u3, it3, _, _ = h.solve(to_dev(rho2[2:]), to_dev(b2[2:]), solver="rmr", max_iter=300)
    assert np.array_equal(to_host(u3)[0], to_host(u2)[2]) and it3[0] == it2[2]
    h.close()


def test_results_of_batches_beyond_one_readback_chunk():
    """More systems than the host staging buffer holds (16384): the per-system
    iteration counts, residuals and fields of both chunks are those of the
    same systems solved in small batches of their own."""
    from paper_2403_06654_amd.api import Visc1d
    n, a, nb = 33, 1e-2, 16384 + 100
    ratios = [1.5, 3.0, 10.0, 2.0, 6.0, 8.0, 4.0]
    _, base, _ = _case("cheb", n, ratios, a)
    rho = base[np.arange(nb) % len(ratios)]
    b = np.random.default_rng(17).standard_normal((nb, n))
    h = Visc1d("cheb", n, a)
    u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver="rmr", max_iter=2000)
    print(info, sorted(set(int(v) for v in it[:len(ratios)])), flush=True)
    assert info["status"] == 0 and len(set(int(v) for v in it[:len(ratios)])) > 2
    u = to_host(u)
    for lo in (0, 16384 - 50, nb - 100):          # the first chunk, across the boundary, the second chunk
        hi = min(lo + 100, nb)
        u1, it1, rr1, _ = h.solve(to_dev(rho[lo:hi]), to_dev(b[lo:hi]), solver="rmr", max_iter=2000)
        assert np.array_equal(to_host(u1), u[lo:hi]), lo
        assert np.array_equal(it1, it[lo:hi]) and np.array_equal(rr1, rr[lo:hi]), lo
    h.close()


@pytest.mark.parametrize("basis,n", [("cheb", 512), ("fourier", 512)])
def test_largest_systems_solve(basis, n):
    """512 points (the kernel instantiations built apart, which spill)."""
    from paper_2403_06654_amd.api import Visc1d
    print(f"case visc1d solve largest {basis} n={n}", flush=True)
    a = 1e-3
    _, rho, systems = _case(basis, n, [2.0, 10.0], a)
    b = np.random.default_rng(8).standard_normal(rho.shape)
    h = Visc1d(basis, n, a)
    for solver in ("gmres", "rmr"):
        u, it, rr, info = h.solve(to_dev(rho), to_dev(b), solver=solver, restart=64, max_iter=3000)
        assert info["status"] == 0, (solver, info)
        u = to_host(u)
        for k, (A, V) in enumerate(systems):
            uk, bk = _inner(basis, u[k]), _inner(basis, b[k])
            # 1e-10 plus the rounding of evaluating A u in a different order
            # (n eps |A| |u|, relative to ||b||); ||D2|| ~ N^4 at 512 points
            slack = n * np.finfo(float).eps * np.linalg.norm(np.abs(A) @ np.abs(uk)) / np.linalg.norm(bk)
            assert rel2(A @ uk, bk) <= 1e-10 + slack, (solver, k, rel2(A @ uk, bk), slack)
    h.close()


def test_bench_configuration_sampled():
    """The launch the bench times (8192 systems, 257 Chebyshev points,
    s = 1000, a = 1e-3, exactly 40 RMR or GMRES(40) iterations): sampled
    systems from both ends of the batch against the oracle's same 40
    iterations.  The recurrences agree to rounding: 40 steps of a
    kappa ~ 1e3 preconditioned operator leave ~1e-11, bound 1e-9."""
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Visc1d
    n, a, big = 257, 1e-3, 8192
    inp = workloads.visc1d_inputs(big, n=n, s=1000.0, seed=0)
    h = Visc1d("cheb", n, a)
    for solver, kw in (("rmr", {}), ("gmres", {"restart": 40})):
        print(f"case visc1d bench config {solver}", flush=True)
        u, it, rr, info = h.solve(to_dev(inp["rho"]), to_dev(inp["b"]), solver=solver, rtol=1e-300, max_iter=40, **kw)
        assert (it == 40).all()
        u = to_host(u)
        for k in (0, 1, 4095, 4096, 8190, 8191):
            A, V = viscous.cheb_system(inp["rho"][k], a)
            orc = getattr(krylov, solver)(lambda v: A @ v, inp["b"][k, 1:-1], lambda r: np.linalg.solve(V, r),
                                          rtol=1e-300, max_iter=40, **kw)
            assert orc["iterations"] == 40
            assert rel2(u[k, 1:-1], orc["x"]) < 1e-9, (solver, k, rel2(u[k, 1:-1], orc["x"]))
            assert abs(rr[k] / orc["rel_residual"] - 1.0) < 1e-6, (solver, k, rr[k], orc["rel_residual"])
    h.close()
