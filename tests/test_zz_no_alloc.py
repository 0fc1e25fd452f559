"""The allocation-free batched 1D solve (vd_visc1d_solve_noalloc, for callers
that cannot allocate device memory) against the allocating entry point
vd_visc1d_solve, both called through the C ABI: the same solutions,
iteration counts, residuals and histories, bit for bit (the same kernel runs
on the library's static scratch instead of the handle's buffers), on two
calls in a row with the second smaller, in both solvers.  A call larger than
the scratch array is refused and writes nothing."""
import numpy as np
import pytest

from paper_2403_06654_amd import api, workloads
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

N, A = 257, 1e-3


def _both(h, inp, solver, cap):
    rho, b = to_dev(inp["rho"]), to_dev(inp["b"])
    ref = h.solve(rho, b, solver=solver, restart=30, max_iter=400, history=cap)
    # the output starts from garbage: the solve must overwrite every entry
    u0 = to_dev(np.full(inp["b"].shape, 7.0))
    got = h.solve_noalloc(rho, b, u=u0, solver=solver, restart=30, max_iter=400, history=cap)
    return ref, got


@pytest.mark.parametrize("solver", ["gmres", "rmr"])
def test_noalloc_matches_allocating_solve(solver):
    h = api.Visc1d("cheb", N, A)
    for call, (batch, seed) in enumerate([(200, 3), (37, 4)]):   # second call smaller (ragged group)
        print(f"case noalloc {solver} call {call} batch {batch}", flush=True)
        inp = workloads.visc1d_inputs(batch, n=N, s=1000.0, seed=seed)
        (u1, it1, rr1, d1), (u2, it2, rr2, d2) = _both(h, inp, solver, cap=64)
        assert d1["status"] in (0, 1) and d2["status"] == d1["status"]
        assert np.array_equal(to_host(u1), to_host(u2))
        assert np.array_equal(it1, it2) and np.array_equal(rr1, rr2)
        assert np.array_equal(d1["history"], d2["history"])
        assert d1["iterations"] == d2["iterations"] and d1["history_len"] == d2["history_len"]
        assert (it2 > 0).all()
    h.close()


def test_noalloc_refuses_a_call_beyond_its_scratch():
    h = api.Visc1d("cheb", N, A)
    batch = 2048                              # GMRES(30) at 255 unknowns fits 816 systems
    inp = workloads.visc1d_inputs(batch, n=N, s=2.0, seed=5)
    rho, b = to_dev(inp["rho"]), to_dev(inp["b"])
    u = to_dev(np.full(inp["b"].shape, 7.0))
    print("case noalloc over the limit", flush=True)
    with pytest.raises(api.VdError) as e:
        h.solve_noalloc(rho, b, u=u, solver="gmres", restart=30)
    assert e.value.status == -6               # VD_ETOOBIG
    assert float(u.min()) == 7.0 and float(u.max()) == 7.0
    # the same batch fits with RMR (smaller workspace) and matches the allocating solve
    (u1, it1, rr1, d1), (u2, it2, rr2, d2) = _both(h, inp, "rmr", cap=0)
    assert np.array_equal(to_host(u1), to_host(u2)) and np.array_equal(it1, it2)
    h.close()


def test_noalloc_pressure_handle_and_cg():
    """The same for a 1D pressure handle (K_rho, Neumann walls) with CG and
    GMRES: the wall values of the Neumann extension come out the same too."""
    from oracle import pressure1d as p1
    h = api.Visc1d.pressure(65, "K")
    x = p1.points(65)
    for call, batch in enumerate((48, 5)):
        rng = np.random.default_rng(10 + call)
        rho = np.stack([p1.tophat(x, s) for s in rng.uniform(0.5, 3.0, batch)])
        b = np.zeros_like(rho)
        for k in range(batch):
            b[k, 1:-1] = p1.operator_K(rho[k]) @ rng.standard_normal(63)
        for solver in ("cg", "gmres"):
            print(f"case noalloc pressure {solver} call {call} batch {batch}", flush=True)
            inp = {"rho": rho, "b": b}
            (u1, it1, rr1, d1), (u2, it2, rr2, d2) = _both(h, inp, solver, cap=16)
            assert np.array_equal(to_host(u1), to_host(u2))
            assert np.array_equal(it1, it2) and np.array_equal(rr1, rr2)
            assert np.array_equal(d1["history"], d2["history"])
    h.close()
