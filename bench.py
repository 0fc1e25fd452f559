"""Throughput of the preconditioned variable-density Krylov solves on one MI355X.

Workload (one "step"): at 256^3 (triply periodic, [0, 2 pi)^3) with the
jet-like density rho = 1 + (rj-1)/2 (1 - tanh((r_perp - 0.5)/0.05)), rj
cycling over {0.5, 3, 5} from step to step, solve
  * the pressure equation L_rho p = f            (GMRES(30), rtol 1e-10),
  * the 3-component velocity system rho u - dt nu Lap u = g, dt nu = 1e-3
                                                 (GMRES(30), rtol 1e-10),
both preconditioned by the constant-density inverse.  Inputs are seeded
synthetic fields already resident in HBM.  The timed leg runs in plain FP64
(the headline `value`) and again with FP32 operator/preconditioner inside
FP64 iterative refinement at equal 1e-10 accuracy.

Prints one JSON line.  `value` = Krylov iterations per second (operator
applications inside the Krylov loops, summed over all solves of the FP64
leg) divided by the leg's wall time.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 256
RJS = (0.5, 3.0, 5.0)
DT_NU = 1e-3
PEAK_HBM_GBS = 8000.0
# Timed kernel classes (the library counts each launch's algorithmic bytes:
# fields read + written, a field being N^3 reals = N^3/2 complex).
PASS_NAMES = ["pressure z-first (k_col COL_P_FIRST)", "pressure y-inverse (k_col COL_P_MIDINV)",
              "pressure x pass (k_row ROW_P)", "pressure y-forward (k_col COL_P_MIDFWD)",
              "pressure z-last (k_col COL_P_LAST)", "helmholtz z-first (k_col COL_H_FIRST)",
              "helmholtz y-inverse (k_col COL_FFT_INV)", "helmholtz x pass (k_row ROW_H)",
              "helmholtz y-forward (k_col COL_FFT_FWD)", "helmholtz z-last (k_col COL_H_LAST)",
              "gmres gram-schmidt dots (k_mdot)", "gmres gram-schmidt update (k_gs_update)"]


def pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def run_leg(grid, rho_dev, f_dev, g_dev, precision, steps, warmup, torch, profile=False):
    """Warm-up steps, then `steps` timed steps.  With `profile`, the warm-up
    steps time every kernel class (per-pass table) and the timed steps time
    only the class that dominated the warm-up, so that events (about 5% of the
    step time when every launch is bracketed) barely perturb the timed region.
    Returns (result, warm-up profile, timed profile, timed class)."""
    lat_p, lat_u, iters, refin, worst, reorth = [], [], 0, 0, 0.0, 0
    p = torch.zeros_like(f_dev)
    u = torch.zeros_like(g_dev)

    def step(i):
        nonlocal iters, refin, worst, reorth
        grid.set_density(rho_dev[i % len(rho_dev)])
        t0 = time.perf_counter()
        _, ip = grid.solve_pressure(f_dev, p=p, precision=precision)
        t1 = time.perf_counter()
        _, iu = grid.solve_helmholtz(g_dev, DT_NU, u=u, precision=precision)
        t2 = time.perf_counter()
        for info in (ip, iu):
            if info["status"] != 0:
                raise RuntimeError(f"solve did not converge: {info}")
        return (t1 - t0, t2 - t1, ip, iu)

    prof_warm, cls = None, 11
    if profile:
        grid.profile_read()      # reset
        grid.profile_enable(True)
    for i in range(warmup):
        step(i)
    torch.cuda.synchronize()
    if profile:
        prof_warm = grid.profile_read()
        if warmup:
            cls = dominant_class(prof_warm)
        grid.profile_enable(1 << cls)
    t_start = time.perf_counter()
    for i in range(steps):
        tp, tu, ip, iu = step(i)
        lat_p.append(tp * 1e3)
        lat_u.append(tu * 1e3)
        iters += ip["iterations"] + iu["iterations"]
        refin += ip["refinements"] + iu["refinements"]
        reorth += ip["gs_second_passes"] + iu["gs_second_passes"]
        worst = max(worst, ip["rel_residual"], iu["rel_residual"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = None
    if profile:
        prof = grid.profile_read()
        grid.profile_enable(False)
    solves = steps * 4   # 1 pressure + 3 velocity components per step
    return {
        "elapsed_s": elapsed, "iters": iters, "iters_per_s": iters / elapsed, "solves_per_s": solves / elapsed,
        "pressure_p50_ms": pct(lat_p, 50), "pressure_p99_ms": pct(lat_p, 99),
        "velocity_p50_ms": pct(lat_u, 50), "velocity_p99_ms": pct(lat_u, 99),
        "iters_per_step": iters / steps, "refinements_per_step": refin / steps,
        "max_true_rel_residual": worst, "ms_per_step": elapsed * 1e3 / steps,
        "gs_second_passes_per_step": reorth / steps,
    }, (prof_warm, prof, cls)


def apply_timing(grid, x, precision, torch, reps=20):
    """The pressure operator alone: `reps` applications with the five pass
    classes event-timed; time per apply = the sum of the per-pass averages,
    bytes = their algorithmic bytes (23 field transfers of this precision)."""
    grid.profile_read()
    grid.profile_enable(0b11111)
    for _ in range(reps):
        grid.apply_operator("pressure", x, precision=precision)
    torch.cuda.synchronize()
    ms, cnt, nbytes = grid.profile_read()
    grid.profile_enable(False)
    t = sum(ms[c] / cnt[c] for c in range(5) if cnt[c])
    b = sum(nbytes[c] / cnt[c] for c in range(5) if cnt[c])
    gbs = b / (t * 1e-3) / 1e9
    return {"ms": round(t, 4), "bytes": round(b), "GB_s": round(gbs, 1), "frac_of_hbm_peak": round(gbs / PEAK_HBM_GBS, 4),
            "applies": reps}


def dominant_class(prof):
    """Kernel class with the largest total event time."""
    ms = prof[0]
    return max(range(len(ms)), key=lambda c: ms[c])


def pass_table(prof, field_bytes):
    """Per-class averages and the whole pressure operator application."""
    ms, cnt, nbytes = prof
    passes = {}
    for c in range(len(ms)):
        if cnt[c]:
            a = ms[c] / cnt[c]
            passes[PASS_NAMES[c]] = {"avg_us": round(a * 1e3, 2), "launches": cnt[c], "total_ms": round(ms[c], 3),
                                     "bytes_per_launch": round(nbytes[c] / cnt[c]),
                                     "GB_s": round(nbytes[c] / (ms[c] * 1e-3) / 1e9, 1)}
    # whole pressure operator application (5 passes, 23 field transfers)
    op_ms = sum(ms[c] / cnt[c] for c in range(5) if cnt[c])
    op_gbs = 23 * field_bytes / (op_ms * 1e-3) / 1e9 if op_ms else None
    op = {"avg_ms": round(op_ms, 4), "fields": 23, "GB_s": round(op_gbs, 1) if op_gbs else None,
          "frac_of_hbm_peak": round(op_gbs / PEAK_HBM_GBS, 4) if op_gbs else None}
    return passes, op


def roofline(prof, cls):
    """Achieved bandwidth of kernel class `cls` = its algorithmic bytes / its
    HIP-event time, from a profile that timed that class."""
    ms, cnt, nbytes = prof
    avg_ms = ms[cls] / max(cnt[cls], 1)
    bytes_per_launch = nbytes[cls] / max(cnt[cls], 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    return {
        "bound": "hbm", "kernel": PASS_NAMES[cls], "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
        "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
        "bytes_per_launch": round(bytes_per_launch), "avg_launch_us": round(avg_ms * 1e3, 2),
        "launches": cnt[cls],
    }


def traffic_from_profiles(best_name, fname="traffic_counters.json"):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("csrc_sha256_16") != csrc_hash():
        return None
    return rec.get("per_launch_bytes", {}).get(best_name)


# kernel sources of the 3D solves' passes and Krylov vector kernels: the
# stored counter readings are used only while these are unchanged
KERNEL_SOURCES_3D = ("fft_core.hpp", "passes.hip", "passes.hpp", "spectral.hpp", "vd_common.hpp", "vecops.hip",
                     "vecops.hpp", "vdsolve.cpp")  # the last decides which systems share a launch


def csrc_hash():
    """Hash of the kernel sources of the 3D solves (the operator passes and
    the Krylov vector kernels), so that stored counter readings are only used
    for the kernels they were taken on."""
    d = os.path.join(ROOT, "paper_2403_06654_amd", "csrc")
    h = hashlib.sha256()
    for fn in KERNEL_SOURCES_3D:
        h.update(fn.encode())
        h.update(open(os.path.join(d, fn), "rb").read())
    return h.hexdigest()[:16]


def pressure_forms(grid, rho_dev, f_dev, torch):
    """The paper's modified pressure form (Sec. 3.2, eq. VDINSE.Krho; the 3D choice of Sec. 4.2) beside
    the direct one on the same 256^3 pressure problems (FP64 GMRES(30), rtol
    1e-10, one solve per density after one untimed solve): iterations,
    milliseconds per solve and the relative difference of the two answers."""
    out = {}
    for i, rj in enumerate(RJS):
        grid.set_density(rho_dev[i])
        rec = {}
        sol = {}
        for form in ("L", "K"):
            grid.solve_pressure(f_dev, formulation=form)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            p, info = grid.solve_pressure(f_dev, formulation=form)
            torch.cuda.synchronize()
            rec[form] = {"iterations": info["iterations"], "ms": round(1e3 * (time.perf_counter() - t0), 2),
                         "rel_residual": info["rel_residual"]}
            sol[form] = p
        rec["rel_difference"] = float(torch.linalg.vector_norm(sol["K"] - sol["L"]) /
                                      torch.linalg.vector_norm(sol["L"]))
        out[f"rj={rj}"] = rec
    return out


def host_threads():
    """Threads for the all-cores oracle leg: the CPUs this process may run on,
    capped at the 16 a one-GPU share of the host provides."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(inp):
    """The oracle as it stands, on the host: GMRES on the same 256^3 pressure
    problem (rj = 3), stopped after a fixed number of iterations; once with
    numpy's one-thread FFTs and once with the same FFTs on all cores
    (operators.use_workers).  The all-cores figure is the reported baseline."""
    from oracle import krylov, operators
    rho, f = inp["rho"], inp["f"]
    b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))

    def leg(k, workers):
        operators.use_workers(workers)
        try:
            t0 = time.perf_counter()
            res = krylov.gmres(lambda u: operators.apply_pressure(u, rho), b,
                               lambda r: operators.precond_pressure(r, rho.mean()), max_iter=k)
            return res["iterations"], time.perf_counter() - t0
        finally:
            operators.use_workers(None)

    it1, dt1 = leg(2, None)
    nt = host_threads()
    itn, dtn = leg(4, nt)
    sample = ("oracle.krylov.gmres(restart 30) on the 256^3 pressure problem (rj=3), stopped after {k} "
              "iterations; {dt:.1f} s wall including its initial and final true-residual applications; {how}")
    return {"value": round(itn / dtn, 4), "unit": "Krylov iters/s", "cores": nt, "kind": "oracle",
            "sample": sample.format(k=itn, dt=dtn, how=f"FFTs on {nt} threads (scipy.fft), the rest of the "
                                                      "oracle's NumPy arithmetic as it stands"),
            "single_thread": {"value": round(it1 / dt1, 4), "unit": "Krylov iters/s", "cores": 1,
                              "sample": sample.format(k=it1, dt=dt1, how="NumPy FFTs on one thread")}}


def oracle_check(grid, rho_dev, dens, inp, f_dev, g_dev, torch):
    """Error against the FP64 oracle for a sample of the headline's results:
    the rj = 3 pressure solve and the first velocity component, each in FP64
    and FP32+refine, solved on the GPU as in the timed steps.  Per result: the
    oracle-evaluated true relative residual and ||x - x_oracle|| / ||x_oracle||,
    x_oracle the oracle's GMRES(30) solution to 1e-13 (FFTs on all cores)."""
    import numpy as np
    from oracle import krylov, operators
    rho, f, g0 = dens[3.0], inp["f"], inp["g"][0]
    basis = operators.nullspace_basis(f.shape)
    b, _ = operators.project_range(-f, basis)
    Ap = lambda u: operators.apply_pressure(u, rho)
    Ah = lambda u: operators.apply_helmholtz(u, rho, DT_NU)
    operators.use_workers(host_threads())
    try:
        t0 = time.perf_counter()
        ref_p = krylov.gmres(Ap, b, lambda r: operators.precond_pressure(r, rho.mean()), rtol=1e-13)
        ref_u = krylov.gmres(Ah, g0, lambda r: operators.precond_helmholtz(r, rho.mean(), DT_NU), rtol=1e-13)
        t_ref = time.perf_counter() - t0
        xp = operators.project_range(ref_p["x"], basis)[0]
        grid.set_density(rho_dev[RJS.index(3.0)])
        out = {"oracle_reference": {"pressure_iterations": ref_p["iterations"],
                                    "pressure_rel_residual": ref_p["rel_residual"],
                                    "velocity_iterations": ref_u["iterations"],
                                    "velocity_rel_residual": ref_u["rel_residual"], "seconds": round(t_ref, 1)}}
        for prec in ("fp64", "fp32_refine"):
            p, ip = grid.solve_pressure(f_dev, precision=prec)
            u, iu = grid.solve_helmholtz(g_dev[0].contiguous(), DT_NU, precision=prec)
            p, u = p.cpu().numpy(), u.cpu().numpy()
            nr = lambda a, c: float(np.linalg.norm(a - c) / np.linalg.norm(c))
            out[prec] = {
                "pressure_rj3": {"gpu_rel_residual": ip["rel_residual"], "oracle_rel_residual": nr(Ap(p), b),
                                 "rel_error_vs_oracle": nr(operators.project_range(p, basis)[0], xp),
                                 "iterations": ip["iterations"]},
                "velocity_rj3_component0": {"gpu_rel_residual": iu["rel_residual"],
                                            "oracle_rel_residual": nr(Ah(u), g0),
                                            "rel_error_vs_oracle": nr(u, ref_u["x"]), "iterations": iu["iterations"]}}
        return out
    finally:
        operators.use_workers(None)


def serving_oracle_check(reqs, rho_dev, f_dev, xs, got):
    """Oracle-evaluated true relative residual of served results: the first
    three requests of every grid size (FP32+refine, as served)."""
    import numpy as np
    from oracle import operators
    status = {g["user_tag"]: g for g in got}
    picked = {}
    for i, r in enumerate(reqs):
        if len(picked.setdefault(r["n"], [])) < 3:
            picked[r["n"]].append(i)
    out = {}
    for n, idx in sorted(picked.items()):
        worst = 0.0
        for i in idx:
            rho = rho_dev[i].cpu().numpy()
            f = f_dev[n][reqs[i]["seed"] % 8].cpu().numpy()
            x = xs[i].cpu().numpy()
            b, _ = operators.project_range(-f, operators.nullspace_basis(f.shape))
            rr = float(np.linalg.norm(operators.apply_pressure(x, rho) - b) / np.linalg.norm(b))
            worst = max(worst, rr)
            assert status[i]["status"] == 0
        out[f"{n}^2"] = {"requests": len(idx), "max_oracle_rel_residual": worst}
    return out


def bench_serving(args):
    """Serving stream of 2D periodic pressure solves (FP32+FP64-refine, rtol
    1e-10): closed-loop saturation throughput, then Poisson arrivals at 0.8x
    and 0.5x of it with p50/p99 arrival-to-completion latency; plain FP64
    single-slot solving of the same requests as the reference mode."""
    import numpy as np
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Server

    nreq = args.requests
    reqs = workloads.serving_requests(count=nreq)
    print(f"bench: serving pool for {nreq} requests", file=sys.stderr, flush=True)
    pool = workloads.serving_pool(pool=8)
    S_dev = {n: [torch.from_numpy(S).cuda() for S, _ in v] for n, v in pool.items()}
    f_dev = {n: [torch.from_numpy(f).cuda() for _, f in v] for n, v in pool.items()}
    # densities of every request (1 + (r-1)/2 S, the workload's formula) prepared in HBM up front
    rho = [1.0 + 0.5 * (r["r"] - 1.0) * S_dev[r["n"]][r["seed"] % 8] for r in reqs]
    xs = [torch.zeros_like(f_dev[r["n"]][0]) for r in reqs]
    torch.cuda.synchronize()
    budget = 64 << 30

    def submit(srv, i, prec="fp32_refine"):
        r = reqs[i]
        return srv.submit((r["n"], r["n"]), rho=rho[i], f=f_dev[r["n"]][r["seed"] % 8], x=xs[i],
                          precision=prec, user_tag=i)

    def closed(srv, idx, prec):
        t0 = time.perf_counter()
        for i in idx:
            submit(srv, i, prec)
        got = []
        while len(got) < len(idx):
            got += srv.wait(timeout=5.0)
        return time.perf_counter() - t0, got

    # the same closed loop with every request alone in its slot (no shared
    # launches), for comparison
    srv0 = Server(budget, max_slots=args.slots, batch=1)
    closed(srv0, list(range(min(16, nreq))), "fp32_refine")
    print("bench: closed loop, unbatched", file=sys.stderr, flush=True)
    wall0, got0 = closed(srv0, list(range(nreq)), "fp32_refine")
    lat0 = [g["t_done"] - g["t_arrive"] for g in got0]
    srv0.close()
    srv = Server(budget, max_slots=args.slots)
    closed(srv, list(range(min(16, nreq))), "fp32_refine")            # warm-up: grids of every size
    print("bench: closed loop", file=sys.stderr, flush=True)
    wall, got = closed(srv, list(range(nreq)), "fp32_refine")
    bad = [g for g in got if g["status"] != 0]
    if bad:
        raise RuntimeError(f"{len(bad)} serving requests failed, e.g. {bad[0]}")
    sat = nreq / wall
    lat_closed = [g["t_done"] - g["t_arrive"] for g in got]
    iters = sum(g["iterations"] for g in got)
    runs = {}
    for g in got:
        runs.setdefault((g["slot"], g["t_start"]), []).append(g)
    batch_sizes = [len(v) for v in runs.values()]
    oracle = None
    if not args.no_oracle_check:
        oracle = serving_oracle_check(reqs, rho, f_dev, xs, got)
    open_runs = {}
    for frac in (0.8, 0.5):
        qps = frac * sat
        arr = workloads.poisson_arrivals(nreq, qps)
        print(f"bench: open loop at {frac} x saturation ({qps:.0f} req/s)", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        got = []
        for i in range(nreq):
            while True:
                dt = arr[i] - (time.perf_counter() - t0)
                if dt <= 0:
                    break
                got += srv.poll()
                time.sleep(min(dt, 0.0005))
            submit(srv, i)
        while len(got) < nreq:
            got += srv.wait(timeout=5.0)
        el = time.perf_counter() - t0
        lat = [1e3 * (g["t_done"] - g["t_arrive"]) for g in got]
        open_runs[str(frac)] = {"qps_offered": round(qps, 1), "solves_per_s": round(nreq / el, 1),
                                "p50_ms": round(pct(lat, 50), 3), "p99_ms": round(pct(lat, 99), 3)}
    st = srv.stats()
    srv.close()
    # reference mode: plain FP64, one solve at a time, same requests (first 512)
    nref = min(512, nreq)
    srv1 = Server(budget, max_slots=1, batch=1)
    closed(srv1, list(range(min(16, nref))), "fp64")
    wall1, got1 = closed(srv1, list(range(nref)), "fp64")
    srv1.close()
    out = {
        "metric": "serving: solves/s at saturation and p50/p99 latency under Poisson arrivals (2D periodic, "
                  "mixed 128^2..1024^2, density ratio 1.5..10, FP32+FP64-refine, rtol 1e-10)",
        "value": round(sat, 2), "unit": "solves/s", "n_gpus": 1, "higher_is_better": True,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"{nreq} serving requests, grids uniform in {{128,256,512,1024}}^2, "
                               f"r log-uniform [1.5,10], tanh slab with 8-mode interface, GMRES(30)",
                   "slots": args.slots, "hbm_budget_GB": budget / 2 ** 30},
        "closed_loop": {"solves_per_s": round(sat, 2), "krylov_iters_per_s": round(iters / wall, 1),
                        "p50_ms": round(1e3 * pct(lat_closed, 50), 3), "p99_ms": round(1e3 * pct(lat_closed, 99), 3),
                        "slot_runs": len(batch_sizes),
                        "requests_per_slot_run": {str(k): batch_sizes.count(k) for k in sorted(set(batch_sizes))}},
        "closed_loop_unbatched": {"solves_per_s": round(nreq / wall0, 2), "p50_ms": round(1e3 * pct(lat0, 50), 3),
                                  "p99_ms": round(1e3 * pct(lat0, 99), 3)},
        "open_loop": open_runs,
        "oracle_check": oracle,
        "reference_fp64_single_slot": {"requests": nref, "solves_per_s": round(nref / wall1, 2),
                                       "mode": "plain FP64, one request at a time, no batching"},
        "speedup_vs_fp64_single_slot": round(sat / (nref / wall1), 2),
        "server": {"peak_busy_slots": st["peak_busy_slots"], "hbm_peak_GB": round(st["hbm_peak"] / 2 ** 30, 3),
                   "grids": st["grids"]},
    }
    print(json.dumps(out))


def bench_c5(args):
    """512^3, density ratio 10, 32-mode interface (width 0.02): GMRES(30)
    pressure solves to 1e-10 in FP64 and in FP32+FP64-refine."""
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid
    n = 512
    print("bench: generating 512^3 inputs", file=sys.stderr, flush=True)
    inp = workloads.c5_inputs(n, seed=0)
    rho = torch.from_numpy(inp["rho"]).cuda()
    f = torch.from_numpy(inp["f"]).cuda()
    grid = Grid((n, n, n))
    grid.set_density(rho)
    field_bytes = n * n * (n // 2) * 16
    out = {}
    for prec in ("fp64", "fp32_refine"):
        p = torch.zeros_like(f)
        if prec == "fp64":      # warm-up times every class, the timed solves only the dominant one
            grid.profile_read()
            grid.profile_enable(True)
        for _ in range(args.warmup):
            grid.solve_pressure(f, p=p, precision=prec)
        torch.cuda.synchronize()
        if prec == "fp64":
            prof_warm = grid.profile_read()
            best = dominant_class(prof_warm) if args.warmup else 11
            grid.profile_enable(1 << best)
        lat, iters = [], 0
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t1 = time.perf_counter()
            _, info = grid.solve_pressure(f, p=p, precision=prec)
            lat.append(1e3 * (time.perf_counter() - t1))
            if info["status"] != 0:
                raise RuntimeError(f"512^3 solve failed: {info}")
            iters += info["iterations"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[prec] = {"iters_per_s": round(iters / el, 2), "solves_per_s": round(args.steps / el, 3),
                     "iters_per_solve": iters / args.steps, "p50_ms": round(pct(lat, 50), 2),
                     "p99_ms": round(pct(lat, 99), 2), "rel_residual": info["rel_residual"],
                     "refinements": info["refinements"]}
        if prec == "fp64":
            prof = grid.profile_read()
            grid.profile_enable(False)
            roof = roofline(prof, best)
            roof["traffic"] = traffic_from_profiles(roof["kernel"], "traffic_counters_c5.json")
            passes, op = pass_table(prof_warm, field_bytes)
    grid.close()
    res = {
        "metric": "Krylov iters/s and solves/s at 512^3 (FP64 vs FP32+refine)",
        "value": out["fp64"]["iters_per_s"], "unit": "Krylov iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "512^3 triply periodic, density ratio 10, 32-mode interface width 0.02, "
                               "pressure L_rho p = f, GMRES(30), rtol 1e-10"},
        "fp64": out["fp64"], "fp32_refine": out["fp32_refine"], "roofline": roof, "operator_apply": op,
        "passes": passes,
    }
    print(json.dumps(res))


def bench_pmc5(args):
    """Short 512^3 run for hardware-counter passes: the 1 GiB calibration
    copy, then `--steps` FP64 and FP32 pressure-operator applications and
    one FP64 GMRES(30) pressure solve of the 512^3 workload, the solve that
    the c5 workload times (the same launches), without timing."""
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    n = 512
    inp = workloads.c5_inputs(n, seed=0)
    rho = torch.from_numpy(inp["rho"]).cuda()
    f = torch.from_numpy(inp["f"]).cuda()
    grid = Grid((n, n, n))
    grid.set_density(rho)
    for prec in ("fp64", "fp32"):
        for _ in range(args.steps):
            grid.apply_operator("pressure", f, precision=prec)
    _, info = grid.solve_pressure(f, p=torch.zeros_like(f), precision="fp64")
    torch.cuda.synchronize()
    grid.close()
    print(json.dumps({"pmc_run": True, "grid": n, "copy_bytes": nbytes, "applies": args.steps,
                      "solve_iterations": info["iterations"]}))


def bench_c2(args):
    """512 (Fourier x) x 257 (Chebyshev z, Neumann walls) pressure solves of
    the Rayleigh-Taylor-like configuration: PCG and GMRES(30) to 1e-10 in FP64
    and FP32+refine; per-kernel times come from rocprofv3 (the dense
    contractions are not event-timed)."""
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid
    inp = workloads.c2_inputs(nx=512, m=256, r=3.0, seed=0)
    rho = torch.from_numpy(inp["rho"]).cuda()
    f = torch.from_numpy(inp["f"]).cuda()
    grid = Grid((257, 512), lengths=(2.0, 2.0), cheb=True)
    grid.set_density(rho)
    out = {}
    for solver in ("cg", "gmres"):
        for prec in ("fp64", "fp32_refine"):
            p = torch.zeros_like(f)
            for _ in range(args.warmup):
                grid.solve_pressure(f, p=p, solver=solver, precision=prec)
            torch.cuda.synchronize()
            lat, iters = [], 0
            t0 = time.perf_counter()
            for _ in range(args.steps):
                t1 = time.perf_counter()
                _, info = grid.solve_pressure(f, p=p, solver=solver, precision=prec)
                lat.append(1e3 * (time.perf_counter() - t1))
                if info["status"] != 0:
                    raise RuntimeError(f"C2 solve failed: {info}")
                iters += info["iterations"]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[f"{solver}_{prec}"] = {"iters_per_s": round(iters / el, 1), "solves_per_s": round(args.steps / el, 2),
                                       "iters_per_solve": iters / args.steps, "p50_ms": round(pct(lat, 50), 3),
                                       "p99_ms": round(pct(lat, 99), 3), "rel_residual": info["rel_residual"]}
    grid.close()
    res = {"metric": "Krylov iters/s and solves/s, 512 x 257 Fourier-Chebyshev pressure (PCG and GMRES(30))",
           "value": out["gmres_fp64"]["iters_per_s"], "unit": "Krylov iters/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "x periodic 512 Fourier points on [0,2), z 257 Chebyshev-Gauss-Lobatto points "
                                  "with Neumann walls, rho = 1 + (1 + tanh((z - eta(x))/0.02)), 16-mode eta of "
                                  "amplitude 0.05, rtol 1e-10"},
           "results": out}
    print(json.dumps(res))


def bench_pmc(args):
    """Short run for hardware-counter passes: one 1 GiB plain device copy
    (calibration of the byte counters), then exactly the solve steps of the
    default run's timed FP64 leg (same densities, same order, so the same
    launches), without warm-up or timing."""
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid
    nbytes = 1 << 30
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)                      # calibration: reads and writes exactly 1 GiB
    torch.cuda.synchronize()
    del a, b
    dens = {rj: workloads.jet_density(N, rj) for rj in RJS}
    inp = workloads.c3_inputs(rj=3.0, n=N, seed=0, with_g=True)
    rho_dev = [torch.from_numpy(dens[rj]).cuda() for rj in RJS]
    f_dev = torch.from_numpy(inp["f"]).cuda()
    g_dev = torch.from_numpy(inp["g"]).cuda()
    grid = Grid((N, N, N))
    r, _ = run_leg(grid, rho_dev, f_dev, g_dev, "fp64", args.steps, 0, torch)
    grid.close()
    print(json.dumps({"pmc_run": True, "copy_bytes": nbytes, "iters": r["iters"]}))


VISC_FLOPS_PER_IT = 6   # x ni^2: V^-1 (ni x ni) and D1, D2 on the interior columns per iteration


def bench_visc1d(args):
    """Batched 1D viscous solves V_rho u = b (Sec. 3.1, Table 1 set-up: 257
    Chebyshev points, s = 1000): RMR and GMRES run for exactly 5/10/20/40
    iterations per system (rtol 1e-300, GMRES without restart), at batch 1
    (latency of one system) and at a full batch (throughput); then both
    methods to convergence at 1e-10 and a warm start from the converged
    solution after a small change of b."""
    import numpy as np
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Visc1d
    n, a, big = 257, 1e-3, args.batch
    ni = n - 2
    inp = workloads.visc1d_inputs(big, n=n, s=1000.0, seed=0)
    rho = torch.from_numpy(inp["rho"]).cuda()
    b = torch.from_numpy(inp["b"]).cuda()
    h = Visc1d("cheb", n, a)

    def timed(nb, its, solver, reps):
        u = torch.zeros((nb, n), dtype=torch.float64, device="cuda")
        kw = dict(solver=solver, rtol=1e-300, max_iter=its, restart=max(its, 1))
        h.solve(rho[:nb], b[:nb], u=u, **kw)
        t0 = time.perf_counter()
        dev = 0.0
        for k in range(reps):
            _, it, _, _ = h.solve(rho[:nb], b[:nb], u=u, **kw)
            dev += h.kernel_ms() * 1e-3   # HIP events around the kernel launch, on the handle's stream
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / reps
        dev /= reps
        assert int(it.min()) == its and int(it.max()) == its, (it.min(), it.max())
        return wall, dev

    table, roof = {}, None
    for its in (5, 10, 20, 40):
        row = {}
        for solver in ("rmr", "gmres"):
            w1, d1 = timed(1, its, solver, max(args.steps, 3))
            wb, db = timed(big, its, solver, max(args.steps, 3))
            row[solver] = {"one_system_ms": round(1e3 * w1, 3), "batch_ms": round(1e3 * wb, 3),
                           "per_system_us": round(1e6 * db / big, 3),
                           "system_iters_per_s": round(big * its / db, 1)}
            if its == 40 and solver == "rmr":
                fl = VISC_FLOPS_PER_IT * ni * ni * its * big
                roof = {"bound": "mfma", "achieved": round(fl / db / 1e12, 3), "peak": 78.6, "unit": "TFLOP/s",
                        "frac": round(fl / db / 1e12 / 78.6, 4), "traffic": None,
                        "kernel": "k_visc1d<4, RMR>", "launch_ms": round(1e3 * db, 3),
                        "per_unit": f"{VISC_FLOPS_PER_IT} ni^2 FP64 flops per system-iteration, ni = {ni}"}
            if its == 40 and solver == "gmres":
                # Gram-Schmidt over v_0..v_j: dots, update and check dots (3 (j + 1)
                # vector reads; the second pass's few selected vectors are not
                # counted), the new basis vector written, and the final
                # combination over 40 vectors
                vecs = sum(3 * (j + 1) + 1 for j in range(its)) + its
                by = vecs * ni * 8 * big
                row[solver]["basis_stream"] = {"bound": "hbm", "achieved": round(by / db / 1e9, 1), "peak": 8000.0,
                                               "unit": "GB/s", "frac": round(by / db / 8e12, 4),
                                               "per_unit": f"{vecs} basis vectors of {ni} doubles per system"}
        table[str(its)] = row
    conv = {}
    for solver in ("rmr", "gmres"):
        u = torch.zeros_like(b)
        t0 = time.perf_counter()
        _, it, rr, info = h.solve(rho, b, u=u, solver=solver, rtol=1e-10, max_iter=2000, restart=128)
        el = time.perf_counter() - t0
        b2 = b * (1.0 + 1e-4 * torch.sin(torch.arange(n, device="cuda", dtype=torch.float64)))
        t1 = time.perf_counter()
        _, it2, rr2, info2 = h.solve(rho, b2, u=u, solver=solver, rtol=1e-10, max_iter=2000, restart=128,
                                     use_x0=True)
        el2 = time.perf_counter() - t1
        conv[solver] = {"converged": int((np.asarray(rr) <= 1e-10).sum()), "of": big,
                        "iters_median": float(np.median(it)), "iters_max": int(it.max()),
                        "batch_ms": round(1e3 * el, 3),
                        "warm_iters_median": float(np.median(it2)), "warm_iters_max": int(it2.max()),
                        "warm_batch_ms": round(1e3 * el2, 3)}
    h.close()
    res = {"metric": "1D viscous solves: per-system time at fixed iteration counts (batched)",
           "value": table["40"]["rmr"]["system_iters_per_s"], "unit": "system-iterations/s (RMR, 40 its)",
           "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{big} systems, 257 Chebyshev-Gauss-Lobatto points with no-slip walls, "
                                  "a = 1e-3, top-hat rho with s = 1000, width 0.1, half-width uniform in [0.3, 0.5]"},
           "paper_table_seconds_one_cpu_core": {"5": [5.6e-3, 1.0e-2], "10": [1.1e-2, 3.4e-2],
                                                "20": [2.0e-2, 9.7e-2], "40": [4.2e-2, 2.2e-1]},
           "roofline": roof, "fixed_iterations": table, "to_convergence": conv}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = visc1d_cpu_baseline(inp, a)
    print(json.dumps(res))


def visc1d_cpu_baseline(inp, a):
    """The oracle's RMR (dense V^-1 and differentiation matrices, NumPy on
    one BLAS thread) for 40 iterations on a sample of the systems."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import krylov, viscous
    n = inp["rho"].shape[1]
    done, el = 0, 0.0
    with threadpool_limits(1):
        while done < 512 and el < 10.0:
            A, V = viscous.cheb_system(inp["rho"][done], a)
            Vi = np.linalg.inv(V)
            t0 = time.perf_counter()
            krylov.rmr(lambda u: A @ u, inp["b"][done, 1:n - 1], lambda r: Vi @ r, rtol=1e-300, max_iter=40)
            el += time.perf_counter() - t0
            done += 1
    return {"value": round(done * 40 / el, 1), "unit": "system-iterations/s (RMR, 40 its)",
            "cores": 1, "kind": "oracle",
            "sample": f"oracle.krylov.rmr, {done} systems x 40 iterations, {el:.2f} s (assembly and inversion "
                      f"of the dense matrices not timed), one BLAS thread"}

def bench_ns(args):
    """Fractional-step steps of the variable-density Navier-Stokes equations
    (Sec. 2) on the manufactured Taylor-Green solution (Sec. 4.1,
    eq. VDINSE.solexact): 128^3, Re = Sc = 1, s = 10.  (a) dt = 0.01 (the
    divergence-history set-up): time per step with warm-started solves,
    Krylov iterations, ||div u|| after every step up to t = pi/4; (b) errors
    at T = pi/4 for dt = T/8 .. T/64 and their orders (the temporal-error
    set-up); (c) event-timed classes over profiled steps for the roofline of
    the FFT transforms."""
    import numpy as np
    import torch
    from paper_2403_06654_amd.api import FractionalStep
    n, re, sc, s = args.ns_n, 1.0, 1.0, 10.0
    T = np.pi / 4
    ns = FractionalStep(n, re=re, sc=sc, dt=0.01, s=s)
    ns.init_taylor_green()
    print(f"bench: ns {n}^3 warm-up", file=sys.stderr, flush=True)
    ns.step(args.warmup)
    torch.cuda.synchronize()
    its_v, its_p = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        info = ns.step(1)
        its_v.append(info["visc_iters"])
        its_p.append(info["pres_iters"])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / args.steps
    # (c) profiled steps
    ns.profile_enable(True)
    ns.step(args.steps)
    prof = ns.profile_read()
    ns.profile_enable(False)
    tr = prof["transforms"]
    ach = tr["bytes"] / (tr["ms"] * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": 8000.0, "unit": "GB/s", "frac": round(ach / 8000.0, 4),
            "traffic": None, "kernel": "FFT transform passes (k_row R2C/C2R, k_col FFT_FWD/FFT_INV)",
            "per_unit": f"48 n^3 bytes per 3D transform (3 passes reading and writing the field), n = {n}; "
                        "a launch group is one transform or three batched",
            "launches": tr["count"], "transforms": int(round(tr["bytes"] / (48.0 * n ** 3))),
            "avg_us_per_transform": round(1e3 * tr["ms"] / max(tr["bytes"] / (48.0 * n ** 3), 1), 2)}
    ns.close()
    # (a) divergence history at dt = 0.01 up to t = pi/4
    print("bench: ns divergence history", file=sys.stderr, flush=True)
    ns = FractionalStep(n, re=re, sc=sc, dt=0.01, s=s)
    ns.init_taylor_green()
    divs = []
    for _ in range(int(round(T / 0.01))):
        ns.step(1)
        divs.append(ns.errors()["div"])
    ns.close()
    # (b) temporal errors
    errs = {}
    for K in (8, 16, 32, 64):
        print(f"bench: ns errors K={K}", file=sys.stderr, flush=True)
        ns = FractionalStep(n, re=re, sc=sc, dt=T / K, s=s)
        ns.init_taylor_green()
        ns.step(K)
        errs[K] = ns.errors()
        ns.close()
    Ks = sorted(errs)
    orders = {key: [round(float(np.log2(errs[Ks[i]][key] / errs[Ks[i + 1]][key])), 3) for i in range(len(Ks) - 1)]
              for key in ("u", "p", "rho")}
    res = {"metric": f"fractional-step time steps/s, {n}^3 manufactured Taylor-Green (Re = Sc = 1, s = 10)",
           "value": round(1e3 / ms_step, 3), "unit": "steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms_step, 3), "higher_is_better": True, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{n}^3 triply periodic box, eq. VDINSE.solexact forcing, Re = Sc = 1, s = 10, "
                                  "dt = 0.01, solves to 1e-12 warm-started"},
           "iterations_per_step": {"viscous_mean": float(np.mean(its_v)), "pressure_mean": float(np.mean(its_p)),
                                   "viscous_max": int(max(its_v)), "pressure_max": int(max(its_p))},
           "roofline": roof, "profile_classes": prof,
           "divergence_rms": {"max": max(divs), "last": divs[-1], "steps": len(divs)},
           "temporal_errors": {str(K): errs[K] for K in Ks}, "orders": orders}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = ns_cpu_baseline(n)
    print(json.dumps(res))


def ns_cpu_baseline(n):
    """One oracle step (NumPy FFTs, one BLAS thread) of the same problem."""
    from threadpoolctl import threadpool_limits
    from oracle import fractional_step as fs
    st = fs.taylor_green_state(n, 10.0, 0.01)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        fs.step(st, 0.01, 1.0, 1.0, s=10.0)
        el = time.perf_counter() - t0
    return {"value": round(1.0 / el, 5), "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle.fractional_step.step, 1 step at {n}^3 from the initial state, {el:.1f} s"}


def cheb_statements(out):
    """The paper's statements about the Chebyshev pressure operators (Sec.
    3.2), evaluated on the study's GPU-assembled numbers."""
    vs_s, vs_n = out["pressure_cheb_vs_s"], out["pressure_cheb_vs_N"]
    hist = out["pressure_cheb_histories_N256"]

    def first_below(h, t):
        for i, v in enumerate(h):
            if isinstance(v, float) and v <= t:
                return i
        return None

    big = {k: v for k, v in vs_n.items() if int(k) >= 32}
    pk = [v["PK"] for v in big.values()]
    kp = [v["KP"] for v in big.values()]
    pl = [v["PL"] for v in big.values()]
    return {
        # at s = 1 both preconditioned operators are the identity on the range (kappa 1)
        "kappa(P K) < kappa(P L) for 0.1 <= s <= 100, s != 1": all(v["PK"] < v["PL"] for k, v in vs_s.items()
                                                                     if float(k) != 1.0),
        "kappa(P K), kappa(K P) independent of N (max/min over N >= 32, s = 2)": [max(pk) / min(pk),
                                                                                   max(kp) / min(kp)],
        "kappa(P L) independent of N (max/min over N >= 32, s = 2; not the paper's picture)": max(pl) / min(pl),
        "GMRES 12 decades, iterations at s = 2, 10, 100 (paper: about 10)":
            [first_below(hist[f"s{s:g}_K_gmres"], 1e-12) for s in (2.0, 10.0, 100.0)],
        "RMR iterations to 1e-9 vs GMRES at s = 2 (paper: 4x)":
            [first_below(hist["s2_K_rmr"], 1e-9), first_below(hist["s2_K_gmres"], 1e-9)],
        "RMR converges for s = 10, 100 (paper: no)":
            [first_below(hist[f"s{s:g}_K_rmr"], 1e-9) is not None for s in (10.0, 100.0)],
        "CG smallest residual at s = 2, 10, 100 (paper: plateau near 0.5)":
            [min((v for v in hist[f"s{s:g}_K_cg"] if isinstance(v, float)), default=None) for s in (2.0, 10.0, 100.0)],
    }


def bench_kappa(args):
    """Condition-number study (Sec. 3.1 Figs. 1-3 set-ups for V_rho, Sec. 3.2
    Figs. 5-6 set-ups for L_rho and K_rho on periodic grids and on the
    paper's Chebyshev-collocation grid with Neumann walls) with every
    operator column computed by the library's GPU applications and kappa from
    an SVD on the host; GMRES, RMR and CG residual histories of the
    Chebyshev pressure systems (Fig. 7 set-up, N = 256, s = 2, 10, 100);
    RMR and GMRES residual histories of the batched 1D
    viscous solver (Fig. 4 set-up, N = 256, s = 2, a = 1e-3); and its
    iterations for a in {1e-4, 1e-3, 1e-2} and s in {10, 100, 1000} (App. A
    set-up)."""
    from paper_2403_06654_amd import conditioning as C
    t0 = time.perf_counter()
    out = {}
    print("bench: kappa V_rho vs N", file=sys.stderr, flush=True)
    out["visc_cheb_vs_N"] = {str(n): C.visc_kappa("cheb", n + 1, 1e-2, 2.0) for n in (16, 32, 64, 128, 256, 511)}
    out["visc_fourier_vs_N"] = {str(n): C.visc_kappa("fourier", n, 1e-2, 2.0) for n in (16, 32, 64, 128, 256, 512)}
    print("bench: kappa V_rho vs s, a", file=sys.stderr, flush=True)
    out["visc_cheb_vs_s"] = {str(s): C.visc_kappa("cheb", 257, 1e-2, s)
                             for s in (1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0, 200.0, 500.0, 1000.0)}
    out["visc_cheb_vs_a"] = {str(a): C.visc_kappa("cheb", 257, a, 2.0) for a in (1e-4, 1e-3, 1e-2, 1e-1, 1.0)}
    print("bench: kappa pressure", file=sys.stderr, flush=True)
    out["pressure_fourier_vs_N"] = {str(n): C.pressure_kappa(n, 2.0) for n in (32, 64, 128, 256, 512)}
    out["pressure_fourier_vs_s"] = {str(s): C.pressure_kappa(256, s)
                                    for s in (0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0)}
    print("bench: kappa pressure, Chebyshev collocation", file=sys.stderr, flush=True)
    out["pressure_cheb_vs_N"] = {str(n - 1): C.cheb_pressure_kappa(n, 2.0) for n in (17, 33, 65, 129, 257, 512)}
    out["pressure_cheb_vs_s"] = {str(s): C.cheb_pressure_kappa(257, s)
                                 for s in (0.1, 0.2, 0.5, 1.0, 2.0, 5.0, 10.0, 20.0, 50.0, 100.0)}
    print("bench: pressure histories, Chebyshev collocation", file=sys.stderr, flush=True)
    out["pressure_cheb_histories_N256"] = {f"s{s:g}_{form}_{solver}": C.cheb_pressure_history(257, s, form, solver)
                                           for s in (2.0, 10.0, 100.0) for form in ("K", "L")
                                           for solver in ("gmres", "rmr", "cg")}
    out["pressure_cheb_statements"] = cheb_statements(out)
    print("bench: viscous histories", file=sys.stderr, flush=True)
    out["visc_histories_N256_s2_a1e-3"] = {f"{basis}_{solver}": C.viscous_history(basis, 257 if basis == "cheb" else 256,
                                                                                 1e-3, 2.0, solver)
                                           for basis in ("cheb", "fourier") for solver in ("rmr", "gmres")}
    print("bench: viscous iterations", file=sys.stderr, flush=True)
    out["visc_iterations"] = {f"{solver}_a{a:g}": C.viscous_iterations(257, a, (10.0, 100.0, 1000.0), solver)
                              for solver in ("gmres", "rmr") for a in (1e-4, 1e-3, 1e-2)}
    el = time.perf_counter() - t0
    res = {"metric": "condition-number study wall time (GPU-assembled operators, host SVD)", "value": round(el, 2),
           "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "higher_is_better": False, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "top-hat densities of eq. VDINSE.rho.hat (d = 0.1, x0 a fifth of the domain); "
                                  "V_rho on Chebyshev (N+1 points, no-slip) and Fourier grids, a = dt/(2 Re); "
                                  "L_rho and K_rho on periodic 1D grids and on Chebyshev collocation with Neumann "
                                  "walls (N+1 points)"},
           "kappa": out}
    print(json.dumps(res))


def bench_table2(args):
    """Pressure solves inside the fractional-step run of the manufactured
    Taylor-Green solution, the set-up of Table 2: 128^3 Fourier, the modified
    form K_rho (eq. VDINSE.Krho), warm start from the previous phi, density
    ratios s = 2, 6, 10, RMR and GMRES, averaged over 10 steps of
    dt = pi/20 (10 dt ~ pi/2); both solves to 1e-10.  The L_rho form runs
    beside it.  The paper's times are for 8 cores of a Xeon E5-2670."""
    import numpy as np
    from paper_2403_06654_amd.api import FractionalStep
    n, dt, nsteps = args.ns_n, np.pi / 20, 10
    paper = {"2": {"rmr": {"iterations": 5, "seconds": 0.2124}, "gmres": {"iterations": 6, "seconds": 0.2480}},
             "6": {"rmr": {"iterations": 7, "seconds": 0.3045}, "gmres": {"iterations": 8, "seconds": 0.3573}},
             "10": {"rmr": {"iterations": 8, "seconds": 0.3477}, "gmres": {"iterations": 8, "seconds": 0.3547}}}
    rows = {}
    for form in ("K", "L"):
        for s in (2.0, 6.0, 10.0):
            for solver in ("rmr", "gmres"):
                print(f"bench: table2 form={form} s={s:g} {solver}", file=sys.stderr, flush=True)
                ns = FractionalStep(n, re=1.0, sc=1.0, dt=dt, s=s, visc_rtol=1e-10, pres_rtol=1e-10,
                                    pres_solver=solver, pres_form=form)
                ns.init_taylor_green()
                its, secs = [], []
                for _ in range(nsteps):
                    info = ns.step(1)
                    its.append(info["pres_iters"])
                    secs.append(info["pres_seconds"])
                err = ns.errors()
                ns.close()
                it_mean, t_mean = float(np.mean(its)), float(np.mean(secs))
                rows[f"{form}_s{s:g}_{solver}"] = {
                    "iterations_mean": it_mean, "iterations": its, "ms_per_solve": round(1e3 * t_mean, 3),
                    "ms_per_iteration": round(1e3 * t_mean / max(it_mean, 1e-9), 4),
                    "ns_per_iteration_per_cell": round(1e9 * t_mean / max(it_mean, 1e-9) / n ** 3, 5),
                    "eps_u_at_end": err["u"], "div_rms_at_end": err["div"]}
    k = rows["K_s10_gmres"]
    res = {"metric": f"pressure solve time inside the {n}^3 Taylor-Green run (Table 2 set-up), K_rho, GMRES, s = 10",
           "value": k["ms_per_solve"], "unit": "ms per solve", "n_gpus": 1, "steps": nsteps, "warmup": 0,
           "higher_is_better": False, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{n}^3 manufactured Taylor-Green (eq. VDINSE.solexact), Re = Sc = 1, dt = pi/20, "
                                  "10 steps, warm-started pressure solves to 1e-10, K_rho and L_rho forms"},
           "rows": rows, "paper_table_2_xeon_8_cores": paper}
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-oracle-check", action="store_true", help="skip the oracle check of sampled results")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--workload", choices=["c3", "serving", "c5", "c2", "pmc", "pmc5", "visc1d", "ns", "kappa", "table2"],
                    default="c3")
    ap.add_argument("--requests", type=int, default=4096)
    ap.add_argument("--slots", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--ns-n", type=int, default=128)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the slab-decomposition design for several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serving":
        bench_serving(args)
        return
    if args.workload == "c5":
        bench_c5(args)
        return
    if args.workload == "c2":
        bench_c2(args)
        return
    if args.workload == "pmc":
        bench_pmc(args)
        return
    if args.workload == "pmc5":
        bench_pmc5(args)
        return
    if args.workload == "visc1d":
        bench_visc1d(args)
        return
    if args.workload == "ns":
        bench_ns(args)
        return
    if args.workload == "kappa":
        bench_kappa(args)
        return
    if args.workload == "table2":
        bench_table2(args)
        return

    import numpy as np
    import torch
    from paper_2403_06654_amd import workloads
    from paper_2403_06654_amd.api import Grid

    print(f"bench: generating 256^3 inputs", file=sys.stderr, flush=True)
    dens = {rj: workloads.jet_density(N, rj) for rj in RJS}
    inp = workloads.c3_inputs(rj=3.0, n=N, seed=0, with_g=True)
    rho_dev = [torch.from_numpy(dens[rj]).cuda() for rj in RJS]
    f_dev = torch.from_numpy(inp["f"]).cuda()
    g_dev = torch.from_numpy(inp["g"]).cuda()
    grid = Grid((N, N, N))
    field_bytes = (N * N * (N // 2)) * 16

    print(f"bench: FP64 leg ({args.warmup} warmup + {args.steps} timed steps)", file=sys.stderr, flush=True)
    r64, (prof_warm, prof_timed, best) = run_leg(grid, rho_dev, f_dev, g_dev, "fp64", args.steps, args.warmup,
                                                 torch, profile=True)
    roof = roofline(prof_timed, best)
    roof["traffic"] = traffic_from_profiles(roof["kernel"])
    passes, op = pass_table(prof_warm, field_bytes)
    r32 = None
    if not args.no_fp32:
        print(f"bench: FP32+refine leg", file=sys.stderr, flush=True)
        r32, _ = run_leg(grid, rho_dev, f_dev, g_dev, "fp32_refine", args.steps, args.warmup, torch)
    print("bench: pressure forms (L_rho vs K_rho)", file=sys.stderr, flush=True)
    forms = pressure_forms(grid, rho_dev, f_dev, torch)
    print("bench: operator applies (FP64, FP32)", file=sys.stderr, flush=True)
    applies = {prec: apply_timing(grid, f_dev, prec, torch) for prec in ("fp64", "fp32")}
    ocheck = None
    if not args.no_oracle_check:
        print("bench: oracle check of sampled results (FP64, FP32+refine)", file=sys.stderr, flush=True)
        ocheck = oracle_check(grid, rho_dev, dens, inp, f_dev, g_dev, torch)
    grid.close()
    # one GPU's share of a z-slab decomposition over 8 GPUs (local passes only)
    slab = Grid((N // 8, N, N))
    slab.set_density(rho_dev[1][: N // 8].contiguous())
    applies["slab_share_fp64_32x256x256"] = apply_timing(slab, f_dev[: N // 8].contiguous(), "fp64", torch)
    slab.close()

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: oracle CPU baseline sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(inp)

    out = {
        "metric": "Krylov iters/s and solves/s at 256^3 (FP64 vs FP32+refine); p50/p99 solve latency",
        "value": round(r64["iters_per_s"], 2),
        "unit": "Krylov iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r64["ms_per_step"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("256^3 triply periodic jet-like density, rj cycling {0.5,3,5}; per step one "
                                "pressure solve L_rho p = f and one 3-component velocity solve rho u - 1e-3 Lap u "
                                "= g; GMRES(30), constant-density preconditioner, rtol 1e-10"),
                   "grid": [N, N, N], "solver": "gmres", "restart": 30, "rtol": 1e-10},
        "solves_per_s": round(r64["solves_per_s"], 3),
        "pressure_p50_ms": round(r64["pressure_p50_ms"], 3),
        "pressure_p99_ms": round(r64["pressure_p99_ms"], 3),
        "velocity_p50_ms": round(r64["velocity_p50_ms"], 3),
        "velocity_p99_ms": round(r64["velocity_p99_ms"], 3),
        "fp64": {k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in r64.items()},
        "fp32_refine": ({k: (float(f"{v:.6g}") if isinstance(v, float) else v) for k, v in r32.items()}
                        if r32 else None),
        "roofline": roof,
        "operator_apply": op,
        "operator_apply_direct": applies,
        "passes": passes,
        "passes_timed_over": "the warm-up steps (every class event-timed); the timed steps time only the roofline class",
        "pressure_forms": forms,
        "oracle_check": ocheck,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
