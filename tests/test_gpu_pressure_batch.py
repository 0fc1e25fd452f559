"""Pressure solves L_rho p = f (Sec. 3.2) of several grids of one shape
solved together (vd_solve_pressure_batch): every grid's field, iteration
count, residual and history must be bit for bit those of its solve alone,
whatever the other grids do (a zero right-hand side, an earlier stop, the
iteration budget), and every result passes the oracle's residual check.
Cases that cannot share launches (CG, the modified form, 1D and
Fourier-Chebyshev grids) run one grid after another, with the same
guarantee.  The server batches queued requests of one shape through the
same call: served results equal the alone ones."""
import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, smooth_density, to_dev, to_host

pytestmark = pytest.mark.gpu


def _problem(shape, k):
    """Grid k's density (its own ratio) and right-hand side; k = 2: zero."""
    rho = smooth_density(shape, 40 + k, 0.5, [3.0, 8.0, 5.0][k % 3])
    if k % 3 == 2:
        return rho, np.zeros(shape)
    return rho, workloads.band_limited(shape, max(2, min(shape) // (4 + 4 * k)), seed=50 + k)


def _grids(shape, n, cheb=False):
    from paper_2403_06654_amd.api import Grid
    gs, fs, rhos = [], [], []
    for k in range(n):
        rho, f = _problem(shape, k)
        g = Grid(shape, cheb=cheb) if cheb else Grid(shape)
        g.set_density(to_dev(rho))
        gs.append(g)
        fs.append(f)
        rhos.append(rho)
    return gs, fs, rhos


def _alone(gs, fs, **opts):
    out, infos = [], []
    for g, f in zip(gs, fs):
        h = np.zeros(300) if "history" in opts else None
        o = dict(opts)
        if h is not None:
            o["history"] = h
        x0 = o.pop("x0", None)
        p = to_dev(x0) if x0 is not None else None
        p, info = g.solve_pressure(to_dev(f), p=p, **o)
        out.append(to_host(p))
        infos.append(info)
    return out, infos


def _check_equal(pb, ib, pa, ia):
    for k in range(len(pa)):
        assert np.array_equal(pb[k], pa[k]), k
        for key in ("status", "iterations", "refinements", "gs_second_passes"):
            assert ib[k][key] == ia[k][key], (k, key, ib[k][key], ia[k][key])
        assert ib[k]["rel_residual"] == ia[k]["rel_residual"] or (
            np.isnan(ib[k]["rel_residual"]) and np.isnan(ia[k]["rel_residual"]))
        assert ib[k]["rhs_null_norm"] == ia[k]["rhs_null_norm"]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("shape,n", [((128, 128), 3), ((256, 256), 2), ((32, 32, 32), 3), ((16, 32, 64), 3)])
def test_batch_equals_alone(shape, n, precision):
    from paper_2403_06654_amd.api import Grid
    print(f"case pressure batch shape={shape} n={n} {precision}", flush=True)
    gs, fs, rhos = _grids(shape, n)
    hist = np.zeros(300)
    pb, ib = Grid.solve_pressure_batch(gs, [to_dev(f) for f in fs], precision=precision, history=hist)
    pb = [to_host(p) for p in pb]
    pa, ia = _alone(gs, fs, precision=precision, history=True)
    print([i["iterations"] for i in ib], flush=True)
    _check_equal(pb, ib, pa, ia)
    assert np.array_equal(hist[:ib[0]["history_len"]], ia[0]["history"])
    for k in range(n):
        assert ib[k]["status"] == 0
        if not fs[k].any():
            assert ib[k]["iterations"] == 0 and not pb[k].any()
            continue
        b, _ = operators.project_range(-fs[k], operators.nullspace_basis(shape))
        rr = rel2(operators.apply_pressure(pb[k], rhos[k]), b)
        assert rr <= 1.01e-10, (k, rr)
    for g in gs:
        g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_batch_initial_guess_and_budget(precision):
    from paper_2403_06654_amd.api import Grid
    shape = (64, 128)
    gs, fs, _ = _grids(shape, 3)
    x0 = [workloads.band_limited(shape, 6, seed=70 + k) for k in range(3)]
    for opts in (dict(use_x0=True), dict(max_iter=5, restart=4)):
        ps = [to_dev(x) for x in x0] if opts.get("use_x0") else None
        pb, ib = Grid.solve_pressure_batch(gs, [to_dev(f) for f in fs], ps, precision=precision, **opts)
        pb = [to_host(p) for p in pb]
        pa, ia = [], []
        for k, (g, f) in enumerate(zip(gs, fs)):
            p = to_dev(x0[k]) if opts.get("use_x0") else None
            p, info = g.solve_pressure(to_dev(f), p=p, precision=precision, **opts)
            pa.append(to_host(p))
            ia.append(info)
        print(opts, [i["iterations"] for i in ib], flush=True)
        _check_equal(pb, ib, pa, ia)
        if "max_iter" in opts:
            assert ib[0]["status"] == 1
    for g in gs:
        g.close()


@pytest.mark.parametrize("case", ["cg", "kform", "1d", "cheb", "one"])
def test_unbatchable_cases_run_one_by_one(case):
    from paper_2403_06654_amd.api import Grid
    print(f"case pressure batch fallback {case}", flush=True)
    shape = {"1d": (256,), "cheb": (65, 64)}.get(case, (64, 64))
    n = 1 if case == "one" else 2
    if case == "cheb":
        gs, fs = [], []
        for k in range(n):
            x = np.linspace(0, 2 * np.pi, 64, endpoint=False)
            z = np.cos(np.pi * np.arange(65) / 64)
            rho = 1.5 + 0.5 * np.tanh((z[:, None] - 0.2 * np.sin(x[None, :] + k)) / 0.1)
            f = np.cos(2 * x[None, :]) * (1 + z[:, None] ** 2)
            g = Grid(shape, cheb=True)
            g.set_density(to_dev(rho))
            gs.append(g)
            fs.append(f)
    else:
        gs, fs, _ = _grids(shape, n)
    opts = {"cg": dict(solver="cg"), "kform": dict(formulation="K")}.get(case, {})
    pb, ib = Grid.solve_pressure_batch(gs, [to_dev(f) for f in fs], **opts)
    pa, ia = _alone(gs, fs, **opts)
    _check_equal([to_host(p) for p in pb], ib, pa, ia)
    for g in gs:
        g.close()


def test_invalid_batches():
    from paper_2403_06654_amd.api import Grid, VdError
    gs, fs, _ = _grids((32, 32), 2)
    with pytest.raises(VdError) as e:                  # one grid twice
        Grid.solve_pressure_batch([gs[0], gs[0]], [to_dev(fs[0]), to_dev(fs[1])])
    assert e.value.status == -1
    with pytest.raises(VdError):                       # more than three
        Grid.solve_pressure_batch(gs * 2, [to_dev(f) for f in fs] * 2)
    with pytest.raises(ValueError):
        Grid.solve_pressure_batch(gs, [to_dev(fs[0])])
    for g in gs:
        g.close()


def test_rejected_solves_report_their_status():
    """Arguments rejected before any work still set every info's status:
    through the batch entry, whose grids then run one by one, and through
    the single-grid solves (the server reads each request's status there)."""
    import ctypes
    from paper_2403_06654_amd.api import lib, make_opts, vd_solve_info, _P
    gs, fs, _ = _grids((32, 32), 2)
    fd = [to_dev(f) for f in fs]
    ps = [to_dev(np.zeros_like(f)) for f in fs]
    o = make_opts(rho0=-1.0)
    infos = (vd_solve_info * 2)()
    for k in range(2):
        infos[k].status, infos[k].iterations = 99, 77     # junk that must be overwritten
    hs = (_P * 2)(*[g._h.value for g in gs])
    fp = (_P * 2)(*[f.data_ptr() for f in fd])
    pp = (_P * 2)(*[p.data_ptr() for p in ps])
    st = lib().vd_solve_pressure_batch(hs, 2, fp, pp, ctypes.byref(o), infos)
    assert st == -1
    assert [infos[k].status for k in range(2)] == [-1, -1]
    assert [infos[k].iterations for k in range(2)] == [0, 0]
    one = vd_solve_info()
    one.status = 99
    st = lib().vd_solve_pressure(gs[0]._h, _P(fd[0].data_ptr()), _P(ps[0].data_ptr()), ctypes.byref(o),
                                 ctypes.byref(one))
    assert st == -1 and one.status == -1
    one.status = 99
    st = lib().vd_solve_helmholtz(gs[0]._h, ctypes.c_double(-1.0), 1, _P(fd[0].data_ptr()),
                                  _P(ps[0].data_ptr()), None, ctypes.byref(one))
    assert st == -1 and one.status == -1
    for g in gs:
        g.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_breakdown_of_one_grid_leaves_the_others_alone(precision):
    """A non-finite right-hand side on one grid of a batch ends that grid's
    solve with VD_EBREAKDOWN; the other grids share the same launches and
    still return exactly their solves alone."""
    import ctypes
    from paper_2403_06654_amd.api import lib, make_opts, vd_solve_info, _P
    shape = (64, 64)
    gs, fs, _ = _grids(shape, 3)
    bad = fs[1].copy()
    bad[5, 7] = np.nan
    fd = [to_dev(fs[0]), to_dev(bad), to_dev(workloads.band_limited(shape, 8, seed=81))]
    ps = [to_dev(np.zeros(shape)) for _ in range(3)]
    o = make_opts(precision=precision)
    infos = (vd_solve_info * 3)()
    hs = (_P * 3)(*[g._h.value for g in gs])
    fp = (_P * 3)(*[f.data_ptr() for f in fd])
    pp = (_P * 3)(*[p.data_ptr() for p in ps])
    st = lib().vd_solve_pressure_batch(hs, 3, fp, pp, ctypes.byref(o), infos)
    print(precision, st, [infos[k].status for k in range(3)], [infos[k].iterations for k in range(3)], flush=True)
    assert st == -4 and infos[1].status == -4                  # VD_EBREAKDOWN
    for k in (0, 2):
        assert infos[k].status == 0 and infos[k].iterations > 0
        pa, ia = gs[k].solve_pressure(fd[k], precision=precision)
        assert np.array_equal(to_host(ps[k]), to_host(pa)), k
        assert ia["iterations"] == infos[k].iterations and ia["rel_residual"] == infos[k].rel_residual
    for g in gs:
        g.close()


def test_server_batches_queued_requests():
    """Nine requests of one shape queued at once on one slot are served in
    batches; each result equals its solve alone (one slot, no batching)."""
    from paper_2403_06654_amd.api import Server
    import torch
    shape = (128, 128)
    probs = [_problem(shape, k % 2) for k in range(9)]
    dev = [(to_dev(r), to_dev(f)) for r, f in probs]

    def serve(batch):
        srv = Server(hbm_budget=4 << 30, max_slots=1, batch=batch)
        xs = [torch.zeros_like(fd) for _, fd in dev]
        torch.cuda.synchronize()
        for i, (rd, fd) in enumerate(dev):
            srv.submit(shape, rho=rd, f=fd, x=xs[i], precision="fp32_refine", user_tag=i)
        got = {}
        while len(got) < len(dev):
            for r in srv.wait(timeout=60.0):
                got[r["user_tag"]] = r
        srv.close()
        return [to_host(x) for x in xs], got

    xa, ra = serve(1)
    xb, rb = serve(3)
    starts = {rb[i]["t_start"] for i in rb}
    print(f"  {len(starts)} slot runs for 9 requests", flush=True)
    assert len(starts) < 9                              # batches formed
    for i in range(9):
        assert rb[i]["status"] == 0 and ra[i]["iterations"] == rb[i]["iterations"]
        assert np.array_equal(xa[i], xb[i]), i
