"""The solve server on the GPU: every result is bitwise the same whether the
request ran alone or concurrently with others (fixed launch configurations
and reduction orders), and every served result, at every grid size of the
serving stream (128^2 to 1024^2) and in both precisions, passes the
oracle's residual check."""
import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = (128, 256, 512, 1024)


def _requests():
    """Every size in both precisions (solvers cycling), then a few more
    draws of the serving stream; density ratios from the stream."""
    draws = workloads.serving_requests(count=64, master_seed=7, sizes=SIZES)
    pool = workloads.serving_pool(sizes=SIZES, pool=2, seed=11)
    plan = [(n, prec) for n in SIZES for prec in ("fp64", "fp32_refine")]
    plan += [(d["n"], "fp32_refine") for d in draws[:6]]
    out = []
    for i, (n, prec) in enumerate(plan):
        d = draws[i]
        S, f = pool[n][d["seed"] % 2]
        rho = workloads.serving_density(S, d["r"])
        solver = ["gmres", "cg", "rmr"][i % 3]
        out.append((n, rho, f, prec, solver))
    return out


def _run(reqs, slots):
    from paper_2403_06654_amd.api import Server
    import torch
    srv = Server(hbm_budget=8 << 30, max_slots=slots)
    infos = {}
    dev = [(to_dev(rho), to_dev(f)) for (_, rho, f, _, _) in reqs]
    # outputs are allocated and zeroed before the synchronize: the server
    # writes them on its own streams, which are not ordered after torch's
    xs = [torch.zeros_like(fd) for _, fd in dev]
    torch.cuda.synchronize()
    for i, ((n, rho, f, prec, solver), (rd, fd)) in enumerate(zip(reqs, dev)):
        srv.submit((n, n), rho=rd, f=fd, x=xs[i], precision=prec, solver=solver, user_tag=i)
        if slots == 1:   # alone: wait for each before submitting the next
            while i not in infos:
                for r in srv.wait(timeout=60.0):
                    infos[r["user_tag"]] = r
    while len(infos) < len(reqs):
        for r in srv.wait(timeout=60.0):
            infos[r["user_tag"]] = r
    st = srv.stats()
    srv.close()
    return [to_host(x) for x in xs], infos, st


def test_alone_vs_mix_bitwise_and_oracle_checked():
    reqs = _requests()
    print(f"case serving: {len(reqs)} requests, sizes {sorted({r[0] for r in reqs})}", flush=True)
    alone, ia, _ = _run(reqs, 1)
    mix, im, st = _run(reqs, 6)
    assert st["peak_busy_slots"] > 1
    for i in range(len(reqs)):
        assert ia[i]["status"] == 0 and im[i]["status"] == 0, (ia[i], im[i])
        assert ia[i]["iterations"] == im[i]["iterations"]
        assert np.array_equal(alone[i], mix[i]), i
    # concurrency actually happened
    spans = sorted((im[i]["t_start"], im[i]["t_done"]) for i in range(len(reqs)))
    assert any(b[0] < a[1] for a, b in zip(spans, spans[1:]))
    # every served result: the oracle's operator gives a true relative
    # residual within 1e-10 (1% for the oracle's own rounding)
    seen = set()
    for i, (n, rho, f, prec, solver) in enumerate(reqs):
        b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))
        rr = rel2(operators.apply_pressure(mix[i], rho), b)
        print(f"  request {i}: {n}^2 {prec} {solver} it={im[i]['iterations']} oracle relres={rr:.3e}", flush=True)
        assert rr <= 1.01e-10, (i, n, prec, solver, rr)
        seen.add((n, prec))
    assert seen >= {(n, p) for n in SIZES for p in ("fp64", "fp32_refine")}


def test_velocity_requests_served():
    """Three-component velocity requests (ρu − δtν∇²u = g) through the
    server, several at once on shared slots: each result equals its solve on
    a grid of its own, and each component passes the oracle's residual."""
    from paper_2403_06654_amd.api import Grid, Server
    import torch
    from tests.gpu_util import smooth_density
    shape, nu = (32, 32, 32), 1e-3
    reqs = []
    for k in range(4):
        rho = smooth_density(shape, 60 + k, 0.5, 4.0 + k)
        g = np.stack([workloads.band_limited(shape, 6, seed=70 + 3 * k + c, keep_mean=True) for c in range(3)])
        reqs.append((rho, g))
    dev = [(to_dev(r), to_dev(g)) for r, g in reqs]
    xs = [torch.zeros_like(gd) for _, gd in dev]
    torch.cuda.synchronize()
    srv = Server(hbm_budget=8 << 30, max_slots=2)
    for i, (rd, gd) in enumerate(dev):
        srv.submit(shape, rho=rd, f=gd, x=xs[i], kind="helmholtz", dt_nu=nu, ncomp=3, user_tag=i)
    got = {}
    while len(got) < len(dev):
        for r in srv.wait(timeout=60.0):
            got[r["user_tag"]] = r
    st = srv.stats()
    srv.close()
    assert st["hbm_peak"] <= 2 * api_workspace_helmholtz(shape)
    for i, (rho, g) in enumerate(reqs):
        assert got[i]["status"] == 0
        grid = Grid(shape)
        grid.set_density(to_dev(rho))
        u, info = grid.solve_helmholtz(to_dev(g), nu)
        grid.close()
        assert info["iterations"] == got[i]["iterations"]
        assert np.array_equal(to_host(u), to_host(xs[i])), i
        served = to_host(xs[i])
        for c in range(3):
            assert rel2(operators.apply_helmholtz(served[c], rho, nu), g[c]) <= 1.01e-10, (i, c)


def api_workspace_helmholtz(shape):
    from paper_2403_06654_amd import api
    return api.workspace_bytes(shape, helmholtz_ncomp=3)
