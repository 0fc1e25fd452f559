"""Host-side scheduling of the solve server, exercised without a GPU through
the scheduler's dry-run mode (no device work; each request occupies its
slot for a fixed time): FIFO admission, admission by HBM footprint,
rejection of requests larger than the budget, the slot limit, and release
of idle grids of other shapes under budget pressure."""
import time

import pytest

from paper_2403_06654_amd import api


def _drain(srv, count, timeout=30.0):
    out = []
    t_end = time.time() + timeout
    while len(out) < count and time.time() < t_end:
        out += srv.wait(timeout=0.5)
    assert len(out) == count, (len(out), count)
    return sorted(out, key=lambda r: r["ticket"])


def test_fifo_order_single_slot():
    srv = api.Server(hbm_budget=1 << 40, max_slots=1, dry_seconds=0.01, batch=1)
    tickets = [srv.submit((128, 128), user_tag=i, precision="fp32_refine") for i in range(8)]
    res = _drain(srv, 8)
    assert [r["ticket"] for r in res] == tickets
    starts = [r["t_start"] for r in res]
    assert starts == sorted(starts)
    for a, b in zip(res, res[1:]):
        assert b["t_start"] >= a["t_done"] - 1e-6
    assert all(r["status"] == -7 for r in res)      # dry run: nothing solved
    srv.close()


def test_admission_by_footprint_and_head_of_line():
    big = api.workspace_bytes((1024, 1024), precision="fp32_refine")
    small = api.workspace_bytes((128, 128), precision="fp32_refine")
    assert big > 40 * small
    srv = api.Server(hbm_budget=big + small // 2, max_slots=8, dry_seconds=0.05)
    t1 = srv.submit((1024, 1024), precision="fp32_refine")
    t2 = srv.submit((1024, 1024), precision="fp32_refine")   # same shape: reuses the grid after t1
    t3 = srv.submit((128, 128), precision="fp32_refine")     # does not fit next to the big grid
    res = {r["ticket"]: r for r in _drain(srv, 3)}
    assert res[t2]["t_start"] >= res[t1]["t_done"] - 1e-6
    assert res[t3]["t_start"] >= res[t2]["t_start"] - 1e-6     # FIFO: no overtaking
    st = srv.stats()
    assert st["hbm_peak"] <= big + small // 2
    srv.close()


def test_too_big_is_rejected():
    small = api.workspace_bytes((128, 128))
    srv = api.Server(hbm_budget=small, max_slots=2, dry_seconds=0.0)
    with pytest.raises(api.VdError) as e:
        srv.submit((256, 256))
    assert e.value.status == -6
    srv.submit((128, 128))
    _drain(srv, 1)
    srv.close()


def test_slot_limit_and_overlap():
    srv = api.Server(hbm_budget=1 << 40, max_slots=4, dry_seconds=0.05)
    t0 = time.time()
    for i in range(16):
        srv.submit((128, 128) if i % 2 else (256, 256))
    res = _drain(srv, 16)
    wall = time.time() - t0
    st = srv.stats()
    assert st["peak_busy_slots"] == 4
    assert wall < 16 * 0.05 * 0.6                   # requests overlapped
    # never more than 4 slots busy at any instant (a batch's requests share
    # their slot's start and end)
    slots = {(r["slot"], r["t_start"], r["t_done"]) for r in res}
    events = sorted([(a, 1) for _, a, _ in slots] + [(b, -1) for _, _, b in slots])
    run = peak = 0
    for _, d in events:
        run += d
        peak = max(peak, run)
    assert peak <= 4
    srv.close()


def _batches(res):
    """Requests grouped by the slot run that served them."""
    groups = {}
    for r in res:
        groups.setdefault((r["slot"], r["t_start"]), []).append(r)
    return sorted(groups.values(), key=lambda g: g[0]["t_start"])


def test_same_shape_requests_share_a_slot():
    """One slot: the first request starts alone (nothing else is queued yet);
    when the slot frees, the next three requests of its shape and options go
    together, then the next three.  Each keeps its own grid (charge)."""
    srv = api.Server(hbm_budget=1 << 40, max_slots=1, dry_seconds=0.05)
    tickets = [srv.submit((128, 128), user_tag=i) for i in range(7)]
    res = _drain(srv, 7)
    groups = _batches(res)
    assert [len(g) for g in groups] == [1, 3, 3]
    assert [sorted(r["ticket"] for r in g) for g in groups] == [tickets[:1], tickets[1:4], tickets[4:7]]
    for g in groups:
        assert len({(r["t_start"], r["t_done"], r["slot"]) for r in g}) == 1
    st = srv.stats()
    assert st["grids"] == 3 and st["hbm_used"] == 3 * api.workspace_bytes((128, 128))
    srv.close()


def test_free_slots_take_requests_alone():
    """While a slot is free for every waiting request, none is batched (a
    batch finishes with its slowest member); once requests outnumber the
    free slots, same-shape requests share a slot."""
    srv = api.Server(hbm_budget=1 << 40, max_slots=4, dry_seconds=0.1)
    first = [srv.submit((128, 128)) for _ in range(4)]      # four free slots: four runs of one
    later = [srv.submit((128, 128)) for _ in range(6)]      # all slots busy: these queue and batch
    res = _drain(srv, 10)
    groups = _batches(res)
    by_ticket = {r["ticket"]: g for g in groups for r in g}
    assert all(len(by_ticket[t]) == 1 for t in first)
    assert len({by_ticket[t][0]["slot"] for t in first}) == 4
    assert max(len(by_ticket[t]) for t in later) == 3
    srv.close()


def test_batches_group_only_what_can_share_launches():
    """Only pressure GMRES requests of one shape and options share a batch:
    another shape, another solver, a velocity request or a 1D grid each wait
    for a slot of their own; a batched request may overtake those."""
    srv = api.Server(hbm_budget=1 << 40, max_slots=1, dry_seconds=0.05)
    t0 = srv.submit((64, 64))                                  # starts alone
    others = [srv.submit((128, 128)), srv.submit((64, 64), solver="cg"),
              srv.submit((64, 64), kind="helmholtz", dt_nu=1e-3, ncomp=2), srv.submit((256,)),
              srv.submit((64, 64), rtol=1e-8)]
    t1 = srv.submit((64, 64))                                  # the rtol 1e-8 request's shape, not its options
    t2 = srv.submit((128, 128))                                # joins the queued 128^2 request
    res = _drain(srv, 8)
    by = {r["ticket"]: r for r in res}
    groups = _batches(res)
    sizes = [sorted(r["ticket"] for r in g) for g in groups]
    assert sizes[0] == [t0]
    assert sorted([others[0], t2]) in sizes                    # the two 128^2 requests together
    for t in others[1:]:
        assert [t] in sizes
    assert [t1] in sizes
    assert by[t2]["t_start"] < by[others[1]]["t_start"]        # batched past the queued CG request
    srv.close()


def test_batch_members_need_room_without_eviction():
    """A request joins a batch only if a grid for it fits next to those held;
    the budget here holds two 128^2 grids, so batches have two requests."""
    one = api.workspace_bytes((128, 128))
    srv = api.Server(hbm_budget=2 * one + one // 2, max_slots=1, dry_seconds=0.05)
    for _ in range(5):
        srv.submit((128, 128))
    res = _drain(srv, 5)
    assert [len(g) for g in _batches(res)] == [1, 2, 2]
    assert srv.stats()["hbm_peak"] <= 2 * one + one // 2
    with pytest.raises(api.VdError):
        api.Server(hbm_budget=1 << 30, max_slots=1, dry_seconds=0.0, batch=4)
    srv.close()


def test_idle_grids_released_under_pressure():
    a = api.workspace_bytes((512, 512))
    b = api.workspace_bytes((256, 256))
    srv = api.Server(hbm_budget=a + b // 2, max_slots=2, dry_seconds=0.0)
    srv.submit((512, 512))
    _drain(srv, 1)
    assert srv.stats()["grids"] == 1
    srv.submit((256, 256))                           # needs the 512^2 grid released
    _drain(srv, 1)
    st = srv.stats()
    assert st["grids"] == 1 and st["hbm_used"] == b
    srv.close()


def test_invalid_requests():
    srv = api.Server(hbm_budget=1 << 30, max_slots=1, dry_seconds=0.0)
    with pytest.raises(api.VdError):
        srv.submit((100, 100))
    with pytest.raises(api.VdError):
        srv.submit((128, 128), restart=99)
    # options a solve would reject are rejected at submit, not after queuing
    # (a shared batch would otherwise fall back to solves that never start)
    for bad in (dict(rho0=-1.0), dict(rho0=0.0), dict(kind="helmholtz", dt_nu=-1e-3),
                dict(kind="helmholtz", dt_nu=float("inf"))):
        with pytest.raises(api.VdError) as e:
            srv.submit((128, 128), **bad)
        assert e.value.status == -1, bad
    srv.submit((128, 128), rho0=2.0)                  # a valid constant is accepted
    assert len(_drain(srv, 1)) == 1
    srv.close()
    with pytest.raises(api.VdError):
        api.Server(hbm_budget=0, max_slots=1, dry_seconds=0.0)
    with pytest.raises(api.VdError):
        api.Server(hbm_budget=1 << 30, max_slots=0, dry_seconds=0.0)


def test_grids_are_reused_only_within_a_footprint_class():
    """A grid keeps every buffer it has allocated, so a grid charged for one
    set of options is not handed to a request whose options allocate other
    buffers: same-shape requests with different precisions get their own
    grid, and the charge of the grids held never exceeds the budget."""
    shape = (256, 256)
    b64 = api.workspace_bytes(shape, precision="fp64")
    b32 = api.workspace_bytes(shape, precision="fp32_refine")
    bcg = api.workspace_bytes(shape, precision="fp64", solver="cg")
    assert b64 != b32 and bcg < b64
    budget = max(b64, b32) + min(b64, b32) // 2     # room for one grid only
    srv = api.Server(hbm_budget=budget, max_slots=2, dry_seconds=0.0)
    srv.submit(shape, precision="fp64")
    _drain(srv, 1)
    assert srv.stats()["hbm_used"] == b64
    srv.submit(shape, precision="fp32_refine")      # not the FP64 grid: a new one, the old released
    _drain(srv, 1)
    st = srv.stats()
    assert st["grids"] == 1 and st["hbm_used"] == b32
    srv.submit(shape, precision="fp64", solver="cg")  # another class: a grid of its own
    _drain(srv, 1)
    st = srv.stats()
    expect = b32 + bcg if b32 + bcg <= budget else bcg
    assert st["grids"] == (2 if expect > bcg else 1) and st["hbm_used"] == expect
    srv.submit(shape, precision="fp64", solver="cg")  # same class: its grid is reused
    _drain(srv, 1)
    st2 = srv.stats()
    assert st2["grids"] == st["grids"] and st2["hbm_used"] == expect and st2["hbm_peak"] <= budget
    srv.close()


def test_velocity_requests_are_charged_for_their_components():
    """A velocity request of three components with GMRES holds three
    systems' Krylov vectors (the components are solved together): it is
    charged vd_workspace_bytes_helmholtz, and its grid is not handed to a
    one-component request (nor the other way round)."""
    shape = (64, 64, 64)
    one = api.workspace_bytes(shape)
    three = api.workspace_bytes(shape, helmholtz_ncomp=3)
    assert three > 2 * one
    srv = api.Server(hbm_budget=one + three, max_slots=1, dry_seconds=0.0)
    srv.submit(shape, kind="helmholtz", dt_nu=1e-3, ncomp=3)
    _drain(srv, 1)
    assert srv.stats()["hbm_used"] == three
    srv.submit(shape, kind="helmholtz", dt_nu=1e-3, ncomp=1)     # a grid of its own next to it
    _drain(srv, 1)
    st = srv.stats()
    assert st["grids"] == 2 and st["hbm_used"] == one + three
    srv.submit(shape, kind="helmholtz", dt_nu=1e-3, ncomp=3)     # reuses the three-component grid
    srv.submit(shape, kind="pressure")                            # reuses the one-system grid
    _drain(srv, 2)
    st = srv.stats()
    assert st["grids"] == 2 and st["hbm_used"] == one + three and st["hbm_peak"] == one + three
    with pytest.raises(api.VdError) as e:                         # larger than the whole budget
        srv.submit((256, 256, 256), kind="helmholtz", dt_nu=1e-3, ncomp=3)
    assert e.value.status == -6
    srv.close()


def test_submit_checks_tensors():
    """Tensors handed to the server are checked before submission (dtype,
    device, shape, layout; Helmholtz fields carry the component axis)."""
    import torch
    srv = api.Server(hbm_budget=1 << 30, max_slots=1, dry_seconds=0.0)
    with pytest.raises(TypeError):
        srv.submit((128, 128), rho=torch.ones(128, 128, dtype=torch.float32))
    with pytest.raises(TypeError):          # float64 but not on the device
        srv.submit((128, 128), f=torch.ones(128, 128, dtype=torch.float64))
    assert srv.stats()["in_flight"] == 0
    srv.close()
