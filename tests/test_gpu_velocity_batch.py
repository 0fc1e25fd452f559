"""The components of a velocity solve rho u - dt nu Lap u = g (Sec. 3.1,
solved with GMRES on a Fourier grid) run together: one launch per operator
pass and per Gram-Schmidt kernel serves up to three systems, each with its
own basis, device state and stopping test.  Every component's result must
be bit for bit the one of a solve of that component alone (same kernels,
same reduction order), including its iteration count and residual history,
whatever the other components do (converge earlier, need no iteration,
stop on the iteration budget).  The oracle's residual checks of the same
solves are in test_gpu_solve (test_helmholtz_solve, test_c3_full_size_velocity)."""
import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import smooth_density, to_dev, to_host

pytestmark = pytest.mark.gpu

NU = 1e-3


def _fields(shape, ncomp, seed):
    """Right-hand sides of different difficulty: a broad band, a narrow one,
    zero (no iteration), a scaled copy of the first."""
    out = []
    for c in range(ncomp):
        kind = c % 4
        if kind == 0:
            out.append(workloads.band_limited(shape, min(shape) // 4, seed=seed, keep_mean=True))
        elif kind == 1:
            out.append(workloads.band_limited(shape, 2, seed=seed + 1, keep_mean=True))
        elif kind == 2:
            out.append(np.zeros(shape))
        else:
            out.append(1e3 * out[0])
    return np.stack(out)


def _alone(g, gfield, **opts):
    us, its, refs, hists = [], [], [], []
    for c in range(gfield.shape[0]):
        h = np.zeros(200) if "history" in opts else None
        o = dict(opts)
        if h is not None:
            o["history"] = h
        u0 = opts.get("u0")
        o.pop("u0", None)
        u = to_dev(u0[c]) if u0 is not None else None
        u, info = g.solve_helmholtz(to_dev(gfield[c]), NU, u=u, **o)
        us.append(to_host(u))
        its.append(info["iterations"])
        refs.append(info["refinements"])
        hists.append(h[:info["history_len"]].copy() if h is not None else None)
    return np.stack(us), its, refs, hists


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("shape,ncomp", [((32, 32, 32), 3), ((64, 128), 2), ((16, 32, 64), 4)])
def test_components_together_equal_alone(shape, ncomp, precision):
    from paper_2403_06654_amd.api import Grid
    print(f"case velocity batch shape={shape} ncomp={ncomp} {precision}", flush=True)
    rho = smooth_density(shape, 21, 0.5, 5.0)
    gfield = _fields(shape, ncomp, seed=3)
    g = Grid(shape)
    g.set_density(to_dev(rho))
    hist = np.zeros(200)
    u, info = g.solve_helmholtz(to_dev(gfield), NU, precision=precision, history=hist)
    u = to_host(u)
    ua, its, refs, hists = _alone(g, gfield, precision=precision, history=True)
    print(info, its, refs, flush=True)
    assert info["status"] == 0
    for c in range(ncomp):
        assert np.array_equal(u[c], ua[c]), c
    assert info["iterations"] == sum(its) and info["refinements"] == sum(refs)
    assert np.array_equal(hist[:info["history_len"]], hists[0])
    if ncomp >= 3:          # the zero right-hand side: zero field, no iteration, the others go on
        assert not u[2].any() and its[2] == 0 and min(its[:2]) > 0
    g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_initial_guess_and_budget(precision):
    """A nonzero initial guess (true residual of each system at the start)
    and an iteration budget that stops every component early."""
    from paper_2403_06654_amd.api import Grid
    shape = (32, 32, 32)
    rho = smooth_density(shape, 5, 0.2, 8.0)
    gfield = _fields(shape, 3, seed=7)
    u0 = np.stack([workloads.band_limited(shape, 4, seed=30 + c, keep_mean=True) for c in range(3)])
    g = Grid(shape)
    g.set_density(to_dev(rho))
    for opts in (dict(use_x0=True), dict(max_iter=4, restart=3)):
        u = to_dev(u0.copy()) if opts.get("use_x0") else None
        ub, info = g.solve_helmholtz(to_dev(gfield), NU, u=u, precision=precision, **opts)
        ub = to_host(ub)
        ua, its, refs, _ = _alone(g, gfield, precision=precision, u0=u0 if opts.get("use_x0") else None,
                                  **opts)
        print(opts, info, its, flush=True)
        for c in range(3):
            assert np.array_equal(ub[c], ua[c]), (opts, c)
        assert info["iterations"] == sum(its)
        if "max_iter" in opts:
            assert info["status"] == 1
    g.close()


def test_oracle_residuals_of_the_batch():
    """Each component of a batched FP64 solve meets the tolerance by the
    oracle's own operator."""
    from paper_2403_06654_amd.api import Grid
    shape = (32, 32, 32)
    rho = smooth_density(shape, 9, 0.5, 5.0)
    gfield = _fields(shape, 3, seed=11)
    g = Grid(shape)
    g.set_density(to_dev(rho))
    u, info = g.solve_helmholtz(to_dev(gfield), NU, rtol=1e-10)
    u = to_host(u)
    for c in (0, 1):
        r = gfield[c] - operators.apply_helmholtz(u[c], rho, NU)
        assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(gfield[c]), c
    assert not u[2].any()
    g.close()
