"""The solve server on the GPU: every result is bitwise the same whether the
request ran alone or concurrently with others (fixed launch configurations
and reduction orders), and results pass the oracle's residual check."""
import numpy as np
import pytest

from oracle import operators
from paper_2403_06654_amd import workloads
from tests.gpu_util import rel2, to_dev, to_host

pytestmark = pytest.mark.gpu


def _requests():
    reqs = workloads.serving_requests(count=64, master_seed=7, sizes=(128, 256, 512))[:14]
    pool = workloads.serving_pool(sizes=(128, 256, 512), pool=3, seed=11)
    out = []
    for i, r in enumerate(reqs):
        S, f = pool[r["n"]][r["seed"] % 3]
        rho = workloads.serving_density(S, r["r"])
        prec = "fp32_refine" if i % 3 else "fp64"
        solver = ["gmres", "cg", "rmr"][i % 3]
        out.append((r["n"], rho, f, prec, solver))
    return out


def _run(reqs, slots):
    from paper_2403_06654_amd.api import Server
    import torch
    srv = Server(hbm_budget=8 << 30, max_slots=slots)
    xs, infos = [], {}
    dev = [(to_dev(rho), to_dev(f)) for (_, rho, f, _, _) in reqs]
    torch.cuda.synchronize()
    tickets = []
    for i, ((n, rho, f, prec, solver), (rd, fd)) in enumerate(zip(reqs, dev)):
        x = torch.zeros_like(fd)
        xs.append(x)
        tickets.append(srv.submit((n, n), rho=rd, f=fd, x=x, precision=prec, solver=solver, user_tag=i))
        if slots == 1:   # alone: wait for each before submitting the next
            for r in srv.wait(timeout=60.0):
                infos[r["user_tag"]] = r
    while len(infos) < len(reqs):
        for r in srv.wait(timeout=60.0):
            infos[r["user_tag"]] = r
    st = srv.stats()
    srv.close()
    return [to_host(x) for x in xs], infos, st


def test_alone_vs_mix_bitwise():
    reqs = _requests()
    print(f"case serving: {len(reqs)} requests", flush=True)
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
    # oracle check on the small ones
    for i, (n, rho, f, prec, solver) in enumerate(reqs):
        if n == 128:
            b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))
            assert rel2(operators.apply_pressure(mix[i], rho), b) <= 1.01e-10
