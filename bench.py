#!/usr/bin/env python3
"""Benchmark of the iPI hot path on one MI355X.

Workload (default): the epidemic-shaped birth-death MDP, S = 2,000,000
states, A = 16 actions, 24 banded nonzeros per row (768e6 nonzeros),
gamma = 0.999, synthetic and seeded, resident in HBM before timing.

One step = one full iPI solve to tolerance in FP64 plus one in the
FP32-mixed mode (float32 P values, FP64 everything else), both from V_0 = 0
with the Jacobi-preconditioned Richardson inner solver (the sweeps between
two stopping tests run as one temporally blocked launch, the library's
default), alpha = 0.1 and the certified stopping rule
||V - TV||_inf <= 1e-9 (1 - gamma) ||V||_inf.  On this chain it converges
fastest to that tolerance; plain Richardson (blocked and one launch per
sweep), GMRES(30), TFQMR and the fp32_inner mode are timed beside it
(other_solvers), and the fp32_inner mode once more on the MDP holding its
values as float32 hi + lo (8 bytes a value), whose Bellman pass alone is
bellman_series_split.

value = the metric's first part: the fused Bellman pass's algorithmic bytes
(BW_alg) over its measured time, FP64, averaged over every pass of the timed
steps (HIP events that the library records around each pass on the solve's
stream).  roofline = the dominant launches of the step (the blocked
Richardson launches of 16 sweeps), timed the same way; both are also set
beside a plain streaming read of 4 GiB (achievable).  roofline.traffic = HBM bytes per launch from the
committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary under profiles/, or null
when the kernel's sources changed since those counters were taken.
cpu_baseline = the oracle on this host: its Bellman pass over the whole MDP
(plain C, OpenMP) in GB/s, and its exact policy iteration to convergence;
rel_error_vs_fp64_oracle = each GPU result's distance to the oracle's V*.
c3_bellman = the pendulum's (2048 x 2048) Bellman pass in both precisions
and its time to tolerance;
c1 = the small random MDP's time to tolerance; c4_subset = the batched solve
of the first 128 of c4's 512 members; one_sweep_kernel = the HBM-bound
one-sweep product the blocked launches replace (--no-extras leaves these
out).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME]
  NAME: c2 (default), c3 (pendulum 2048 x 2048), amdahl (S = 1e5, A = 100,
  k = 150), maze (1000 x 1000); c1, c4 and c5 print their own JSON lines
  (time-to-tol of the small MDP, the batched solve, the serving stream);
  c3-bellman only the pendulum's Bellman pass series.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_VECTOR_PEAK_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_2507_22538_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_hash(names):
    import hashlib
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(CSRC, n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload, precision, sweeps=1):
    """HBM bytes per launch from a committed rocprofv3 counter summary, if the
    kernel's sources are unchanged since the counters were taken (else None);
    sweeps: of a blocked Richardson launch (a summary line without the field
    counts as 1)."""
    import glob
    for path in sorted(glob.glob(os.path.join(PROFILES, "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("counter-summary:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel"), kv.get("workload"), kv.get("precision")) != (kernel, workload, precision):
                    continue
                if int(kv.get("sweeps", "1")) != sweeps:
                    continue
                if sources_hash(kv["sources"].split(",")) != kv.get("sha256_16"):
                    return None
                return {"bytes_per_launch": int(kv["fetch_bytes"]) + int(kv["write_bytes"]),
                        "source": os.path.relpath(path, ROOT)}
    return None


def make_workload(name):
    """(MDP, config, inner solver, alpha, extra options) of a named workload."""
    from paper_2507_22538_amd import workloads as W
    if name == "c2":
        # Jacobi-preconditioned Richardson (Table 2's J-VI family): 18% fewer
        # sweeps than plain Richardson on this chain, the same kernels
        return (W.c2(), {"workload": "birth_death_S2e6_A16_k24_gamma0.999"}, "richardson", 0.1,
                {"pc": "jacobi"})
    if name == "c3":
        # Jacobi-preconditioned Richardson: the low-velocity states keep much
        # of their mass in their own cell, and the scaling cuts the sweeps to
        # a third (136,128 against 416,359 without it, FP64)
        return (W.c3(2048), {"workload": "pendulum_2048x2048_A11_k4_gamma0.9999"}, "richardson", 0.1,
                {"pc": "jacobi"})
    if name == "amdahl":  # the paper's parallel-efficiency MDP (Sec. IV-A): GMRES, alpha = 1e-4
        return W.amdahl(), {"workload": "random_sparse_S1e5_A100_k150_gamma0.69"}, "gmres", 1e-4, {}
    if name == "maze":  # the paper's largest maze (Sec. IV-D): TFQMR, alpha = 1e-4
        # the goal's value spreads one cell per policy improvement, so the
        # number of outer iterations grows with the path length to the goal
        return (W.maze(1000, 1000), {"workload": "maze_1000x1000_A5_gamma0.99"}, "tfqmr", 1e-4,
                {"max_outer": 100000})
    raise SystemExit(f"unknown config {name}")


def bellman_series(ipi, mdp, V, precision, solve_pass_bytes, warm=3, n=20):
    """Fused Bellman passes through the library's entry point on a fixed V
    (outside the timed steps): `warm` untimed, then `n`, each between two HIP
    events on the stream the library launches on (torch's current stream).
    The pass writes TV here, 8 S bytes more than inside a solve."""
    import numpy as np
    import torch
    S = V.numel()
    TV = torch.empty(S, dtype=torch.float64, device=V.device)
    pi = torch.empty(S, dtype=torch.int32, device=V.device)
    resid = torch.empty_like(TV)
    rho = torch.empty(1, dtype=torch.float64, device=V.device)
    code = ipi.IPI_FP64 if precision == "fp64" else ipi.IPI_FP32_MIXED
    for _ in range(warm):
        ipi.ipi_bellman(mdp.handle, V, TV, pi, resid, rho, code)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record()
        ipi.ipi_bellman(mdp.handle, V, TV, pi, resid, rho, code)
        b.record()
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    nbytes = solve_pass_bytes + 8.0 * S
    med = float(np.median(us))
    return {"passes": n, "warmup": warm, "median_us": round(med, 2), "min_us": round(float(us.min()), 2),
            "max_us": round(float(us.max()), 2), "bytes_per_pass": nbytes,
            "achieved_gbs": round(nbytes / (med * 1e-6) / 1e9, 1),
            "frac": round(nbytes / (med * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}


def cpu_baseline(d, budget_s=15.0):
    """The oracle's Bellman pass (numpy, FP64) on a prefix of the states."""
    import numpy as np

    from oracle import ipi_oracle as O
    from paper_2507_22538_amd import workloads as W

    k_mean = d.nnz / (d.S * d.A)
    S_s = int(max(1, min(d.S, 250_000, 1e8 / (d.A * k_mean))))
    R = S_s * d.A
    nnz = int(d.row_ptr[R])
    sub = W.MDPData(S_s, d.A, d.row_ptr[:R + 1].copy(), d.col[:nnz].copy(), d.val[:nnz].copy(), d.g[:R].copy(),
                    d.gamma)
    sub.col = np.minimum(sub.col, S_s - 1).astype(np.int32)  # keep the gathers inside the sample
    V = np.random.default_rng(0).random(S_s)
    bytes_pass = nnz * 12.0 + (R + 1) * 8.0 + 8.0 * R + 8.0 * S_s + 20.0 * S_s
    t0 = time.perf_counter()
    n = 0
    while True:
        O.bellman(sub, V)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    dt = (time.perf_counter() - t0) / n
    return {"value": round(bytes_pass / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle Bellman pass (numpy FP64, single thread) over the first {S_s} states "
                      f"({nnz} nonzeros) of the same MDP, {n} passes, {dt:.3f} s/pass"}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def run_c1(args):
    print(json.dumps(c1_result(args)), flush=True)


def c1_result(args):
    """c1: the small random MDP (S = 1000, A = 4, k = 8, gamma = 0.99): plain
    FP64 iPI with GMRES, outer atol 1e-10, alpha = 0.1.  L2-resident and
    latency bound, so reported as time-to-tol, per-pass time and iterations,
    beside the oracle's exact policy iteration on the host."""
    import numpy as np
    import torch

    from oracle import ipi_oracle as O
    from paper_2507_22538_amd import ipi
    from paper_2507_22538_amd import workloads as W

    dev = torch.device("cuda:0")
    d = W.c1()
    m = ipi.MDP.from_data(d)
    # timed solves without profiling (GMRES cycles replayed from a captured
    # HIP graph); one profiled solve (launches one by one, HIP events around
    # each pass) gives the per-pass times
    kw = dict(atol=1e-10, alpha=0.1, ksp_type="gmres", profile=0, device=dev)
    for _ in range(max(1, args.warmup)):
        m.solve(**kw)
    torch.cuda.synchronize()
    times, info = [], None
    for _ in range(args.steps):
        t0 = time.perf_counter()
        V, pi, info, st = m.solve(**kw)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
        if st != ipi.IPI_OK:
            raise RuntimeError(f"c1 solve did not converge: {info}")
    t0 = time.perf_counter()
    _, _, pinfo, _ = m.solve(**dict(kw, profile=1))
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3
    ref = O.policy_iteration(d)
    err = float(np.max(np.abs(V.cpu().numpy() - ref.V)) / np.max(np.abs(ref.V)))
    t0 = time.perf_counter()
    n_or = 0
    while time.perf_counter() - t0 < 3.0:
        O.policy_iteration(d)
        n_or += 1
    or_ms = (time.perf_counter() - t0) / n_or * 1e3
    out = {"metric": "c1 iPI time-to-tol (GMRES, FP64)", "value": round(float(np.median(times)), 3), "unit": "ms",
           "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "random_sparse_S1000_A4_k8_gamma0.99_seed0", "inner": "gmres", "alpha": 0.1,
                      "atol": 1e-10},
           "device_ms": round(info["device_ms"], 3), "outer_iters": info["outer_iters"],
           "inner_iters": info["inner_iters"], "final_rho": info["final_rho"],
           "eager_launch_ms": round(eager_ms, 3),
           "bellman_pass_us": round(pinfo["bellman_ms"] / max(1, pinfo["bellman_calls"]) * 1e3, 2),
           "product_us": round(pinfo["product_ms"] / max(1, pinfo["product_calls"]) * 1e3, 2),
           "rel_err_vs_oracle": err,
           "cpu_baseline": {"value": round(or_ms, 3), "unit": "ms", "cores": 1, "kind": "oracle",
                            "sample": f"oracle exact policy iteration on the same MDP, {n_or} runs"}}
    m.close()
    return out


def run_c4(args):
    print(json.dumps(c4_result(args)), flush=True)


def c4_result(args):
    """c4: independent random MDPs solved by one persistent launch
    (ipi_solve_batch), FP64 and FP32-mixed, alpha = 0.1, GMRES(30), the
    certified stop rtol_cert = 1e-9.  value = aggregate algorithmic GB/s of
    the whole batch solve.  The first members are re-solved alone (a batch
    of one) and compared bit for bit with their results in the batch."""
    import numpy as np
    import torch

    from paper_2507_22538_amd import ipi
    from paper_2507_22538_amd import workloads as W

    dev = torch.device("cuda:0")
    n = args.members
    t0 = time.perf_counter()
    mdps, nnz = [], 0
    for i in range(n):
        d = W.c4_member(i)
        nnz += d.nnz
        mdps.append(ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32))
        if (i + 1) % 32 == 0:
            torch.cuda.synchronize()
            log(f"c4: {i + 1}/{n} members resident ({nnz / 1e9:.2f}e9 nonzeros, {time.perf_counter() - t0:.1f}s)")
    torch.cuda.synchronize()
    res = {}
    for prec in args.precisions.split(","):
        kw = dict(atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="gmres", restart=30, precision=prec,
                  max_inner=1000)
        opts = [ipi.make_opts(**kw) for _ in mdps]
        Vs = [torch.empty(m.S, dtype=torch.float64, device=dev) for m in mdps]
        pis = [torch.empty(m.S, dtype=torch.int32, device=dev) for m in mdps]
        ipi.ipi_solve_batch([m.handle for m in mdps[:8]], opts[:8], Vs[:8], pis[:8])  # warm-up
        times = []
        # at least two calls: the first after a change of precision also
        # reallocates every member's workspace (FP32 / FP64 P_pi copies)
        for _ in range(max(2, args.steps)):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sts, infos = ipi.ipi_solve_batch([m.handle for m in mdps], opts, Vs, pis)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
            log(f"c4 {prec}: batch solve {times[-1]:.3f}s")
        ok = sum(1 for s in sts if s == ipi.IPI_OK)
        alg = sum(i["alg_bytes"] for i in infos)
        bitwise = True
        for j in range(min(4, n)):
            V1 = torch.empty_like(Vs[j])
            p1 = torch.empty_like(pis[j])
            ipi.ipi_solve_batch([mdps[j].handle], [opts[j]], [V1], [p1])
            torch.cuda.synchronize()
            bitwise &= bool(torch.equal(V1, Vs[j]) and torch.equal(p1, pis[j]))
        res[prec] = {"time_to_tol_ms": round(min(times) * 1e3, 3), "agg_gbs": round(alg / min(times) / 1e9, 1),
                     "converged": ok, "members": n, "outer_iters_total": sum(i["outer_iters"] for i in infos),
                     "inner_iters_total": sum(i["inner_iters"] for i in infos),
                     "alone_vs_batch_bitwise_first4": bitwise}
        del Vs, pis
    p0 = args.precisions.split(",")[0]
    out = {"metric": "c4 batched iPI: aggregate algorithmic GB/s, time-to-tol FP32-mixed vs FP64",
           "value": res[p0]["agg_gbs"], "unit": "GB/s", "higher_is_better": True, "n_gpus": 1,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"c4_batch_{n}_random_mdps", "nnz_total": nnz, "inner": "gmres(30)",
                      "alpha": 0.1, "stop": "rtol_cert 1e-9"},
           "detail": res}
    if "fp64" in res and "fp32_mixed" in res:
        out["fp32_mixed_speedup"] = round(res["fp64"]["time_to_tol_ms"] / res["fp32_mixed"]["time_to_tol_ms"], 3)
    for m in mdps:
        m.close()
    return out


def run_c5(args):
    """c5: a Poisson stream of solve requests (random MDPs, S log-uniform on
    [1e3, 5e6], A in {4..32}, k in {8..32}, 1 - gamma log-uniform on
    [1e-4, 5e-2]) into the serving loop (ipi_server_*), FP64, GMRES,
    alpha = 0.1, rtol_cert = 1e-9.  Requests are generated on the host by a
    separate thread a few requests ahead, so generation overlaps service.
    A closed-loop run (4 requests in flight) of the first requests measures
    the service capacity (16 requests); the open-loop stream of
    --requests requests (200 by default) then arrives at 0.7 of it.
    Reports p50 / p99 latency (done - arrival) and solves/s."""
    import queue
    import threading

    import numpy as np
    import torch

    from paper_2507_22538_amd import ipi
    from paper_2507_22538_amd import workloads as W

    torch.cuda.init()
    free, total = torch.cuda.mem_get_info()
    srv = ipi.ipi_server_create(hbm_budget_bytes=int(min(free * 0.85, 240e9)), max_slots=16, n_streams=4,
                                small_nnz_threshold=4_000_000, max_batch=16, backfill=8)
    opts = ipi.make_opts(atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="gmres", max_inner=1000)
    n_closed = 16
    n_total = n_closed + args.requests
    ready = queue.Queue(maxsize=4)

    def generator():
        for i in range(n_total):
            ready.put(W.c5_request(i))

    gen_th = threading.Thread(target=generator, daemon=True)
    gen_th.start()

    # closed loop: 4 requests in flight
    t0 = None
    inflight = []
    for i in range(n_closed):
        d = ready.get()
        if t0 is None:
            t0 = time.perf_counter()
        inflight.append((ipi.ipi_server_submit(srv, d, opts), d.S))
        del d
        if len(inflight) >= 4:
            tk, S = inflight.pop(0)
            ipi.ipi_server_wait(srv, tk, S)
    for tk, S in inflight:
        ipi.ipi_server_wait(srv, tk, S)
    cap = n_closed / (time.perf_counter() - t0)
    lam = 0.7 * cap
    log(f"c5: closed-loop capacity {cap:.3f} solves/s over {n_closed} requests; open loop at {lam:.3f}/s")
    # open loop: submit request j at its Poisson arrival time (later if its
    # generation is not done by then; the server records the actual submit)
    rng = np.random.default_rng(12345)
    gaps = rng.exponential(1.0 / lam, size=args.requests)
    tickets = []
    lock = threading.Lock()
    submitted = {"n": 0, "done": False}

    def submitter():
        t_next = time.perf_counter()
        t_first = t_next
        for j in range(args.requests):
            if time.perf_counter() - t_first > args.c5_seconds:
                log(f"c5: stream duration {args.c5_seconds}s reached after {j} requests")
                break
            d = ready.get()
            t_next += gaps[j]
            delay = t_next - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            tk = ipi.ipi_server_submit(srv, d, opts)
            with lock:
                tickets.append((tk, d.S, d.nnz))
            del d
            if (j + 1) % 8 == 0:
                log(f"c5: {j + 1}/{args.requests} submitted")
        with lock:
            submitted["done"] = True

    th = threading.Thread(target=submitter)
    t_open = time.perf_counter()
    th.start()
    lats, infos, batched, nnzs, sts = [], [], 0, [], []
    k = 0
    while True:
        with lock:
            item = tickets[k] if k < len(tickets) else None
            finished = submitted["done"] and k >= len(tickets)
        if finished:
            break
        if item is None:
            time.sleep(0.005)
            continue
        tk, S, nz = item
        st, V, pi, info, lat = ipi.ipi_server_wait(srv, tk, S)
        sts.append(st)
        lats.append(lat["done_ms"] - lat["arrival_ms"])
        infos.append(info)
        batched += int(lat["batched"])
        nnzs.append(nz)
        k += 1
        if k % 8 == 0:
            log(f"c5: {k}/{args.requests} done, latest latency {lats[-1]:.1f} ms")
    th.join()
    wall = time.perf_counter() - t_open
    ipi.ipi_server_destroy(srv)
    n_req = len(lats)
    out = {"metric": "c5 serving: p99 solve latency, p50, solves/s", "value": round(_pct(lats, 99), 1),
           "unit": "ms", "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"c5_poisson_{n_req}_random_mdp_requests", "arrival_rate_per_s": round(lam, 4),
                      "inner": "gmres", "alpha": 0.1, "stop": "rtol_cert 1e-9"},
           "p50_ms": round(_pct(lats, 50), 1), "p99_ms": round(_pct(lats, 99), 1),
           "mean_ms": round(float(np.mean(lats)), 1), "solves_per_s": round(n_req / wall, 4),
           "requests": n_req, "stream_s": round(wall, 1),
           "closed_loop_capacity_per_s": round(cap, 4), "ok": sum(1 for s in sts if s == ipi.IPI_OK),
           "batched": batched, "nnz_mean": int(np.mean(nnzs)), "nnz_max": int(np.max(nnzs)),
           "alg_gbs_mean": round(float(np.mean([i["alg_bytes"] / max(i["device_ms"], 1e-9) / 1e6 for i in infos])), 1)}
    print(json.dumps(out), flush=True)


def event_median_us(fn, warm=3, n=20):
    """Median of n launches of fn() (after warm untimed ones), each between two
    HIP events on torch's current stream (the stream fn launches on)."""
    import numpy as np
    import torch
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    us = np.array([a.elapsed_time(b) * 1e3 for a, b in ev])
    return float(np.median(us)), float(us.min()), float(us.max())


def achievable_lines(ipi, dev):
    """The achievable HBM rates the kernels are set beside: a plain streaming
    read (16-byte non-temporal loads, the way the P arrays are streamed) of
    4 GiB, and the runtime's device-to-device copy of 1 GiB (read + write)."""
    import torch
    nbytes = 4 << 30
    buf = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    x = torch.zeros(1, dtype=torch.int32, device=dev)
    med, lo, hi = event_median_us(lambda: ipi.ipi_stream_read(buf, nbytes, x))
    del buf
    src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    cmed, _, _ = event_median_us(lambda: dst.copy_(src))
    del src, dst
    torch.cuda.synchronize()
    read = nbytes / (med * 1e-6) / 1e9
    copy = 2.0 * (1 << 30) / (cmed * 1e-6) / 1e9
    return {"stream_read_gbs": round(read, 1), "stream_read_frac": round(read / HBM_PEAK_GBS, 4),
            "stream_read_us": round(med, 1), "stream_read_bytes": nbytes,
            "d2d_copy_gbs": round(copy, 1), "d2d_copy_bytes": 2 << 30,
            "kernel": "ipi_stream_read (k_stream_read), median of 20 after 3 warm-ups"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline_c2(d, gpu_V, gamma):
    """The oracle on the host: its Bellman pass over the whole MDP (plain C,
    OpenMP over all host threads; one pass on one thread) and its exact
    policy iteration (banded LU evaluation) timed to convergence; the GPU
    results' errors against the oracle's V*."""
    import numpy as np

    from oracle import ipi_oracle as O

    threads = O.host_threads()
    nnz = d.nnz
    R = d.S * d.A
    bytes_pass = nnz * 12.0 + (R + 1) * 8.0 + 8.0 * R + 8.0 * d.S + 20.0 * d.S
    V = np.random.default_rng(0).random(d.S)
    t0 = time.perf_counter()
    n = 0
    while True:
        O.bellman(d, V)
        n += 1
        if time.perf_counter() - t0 > 4.0 or n >= 20:
            break
    dt = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    ref = O.policy_iteration(d)
    pi_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.q_values_chunked(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, V, threads=1)
    dt1 = time.perf_counter() - t0
    O.q_values_chunked(d.S, d.A, d.row_ptr, d.col, d.val, d.g, d.gamma, V, threads=threads)  # restore the count
    scale = float(np.max(np.abs(ref.V)))
    errors = {p: float(np.max(np.abs(v - ref.V)) / scale) for p, v in gpu_V.items()}
    base = {"value": round(bytes_pass / dt / 1e9, 3), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"the oracle's Bellman pass (plain C, OpenMP, {threads} threads) over the whole MDP "
                      f"({nnz} nonzeros, {bytes_pass / 1e9:.2f} GB per pass), {n} passes, {dt:.3f} s/pass; "
                      f"then its exact policy iteration to convergence",
            "cpu_model": cpu_model(), "threads": threads,
            "single_thread_gbs": round(bytes_pass / dt1 / 1e9, 3),
            "time_to_tol_ms": round(pi_s * 1e3, 1), "tier": ref.tier, "pi_iterations": ref.iters,
            "oracle_rho": ref.rho}
    return base, errors


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (for profiling runs): no comparison solves, no c3 series")
    ap.add_argument("--precisions", default="fp64,fp32_mixed")
    ap.add_argument("--inner", default=None, help="inner solver (default: the workload's)")
    ap.add_argument("--richardson-block", type=int, default=1, help="0: one launch per Richardson sweep")
    ap.add_argument("--blocked-prefetch", type=int, default=0, choices=(0, -1),
                    help="FP64 blocked sweeps on long rows: 0 persistent with LDS prefetch, -1 one block per workgroup")
    ap.add_argument("--members", type=int, default=512, help="c4: batch members")
    ap.add_argument("--requests", type=int, default=200, help="c5: requests in the Poisson stream")
    ap.add_argument("--c5-seconds", type=float, default=900.0,
                    help="c5: stop submitting after this many seconds of the open-loop stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs is not "
              "built or measured", file=sys.stderr)
        sys.exit(2)

    if args.config == "c1":
        return run_c1(args)
    if args.config == "c4":
        return run_c4(args)
    if args.config == "c5":
        return run_c5(args)
    if args.config == "c3-bellman":
        from paper_2507_22538_amd import ipi
        print(json.dumps(c3_bellman_series(ipi)), flush=True)
        return None

    import numpy as np
    import torch

    from paper_2507_22538_amd import ipi

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    d, cfg, inner_default, alpha, extra = make_workload(args.config)
    log(f"generated {cfg['workload']}: S={d.S} A={d.A} nnz={d.nnz} in {time.perf_counter() - t:.1f}s")
    t = time.perf_counter()
    mdp = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    if args.blocked_prefetch != 0:
        mdp.set_tuning(blocked_prefetch=args.blocked_prefetch)
    torch.cuda.synchronize()
    log(f"resident on device in {time.perf_counter() - t:.1f}s: {mdp.describe()}")
    # the achievable lines; the 1 GiB device copy also calibrates the HBM
    # byte counters of profiling runs (its FETCH_SIZE / WRITE_SIZE)
    ach = achievable_lines(ipi, dev)
    log(f"achievable: {ach}")
    precs = args.precisions.split(",")
    gamma = d.gamma
    inner = args.inner or inner_default
    opts = {p: dict(dict(atol=0.0, rtol_cert=1e-9, alpha=alpha, precision=p, profile=1, max_inner=100000,
                         ksp_type=inner, richardson_block=args.richardson_block), **extra)
            for p in precs}
    S = d.S
    V = {p: torch.empty(S, dtype=torch.float64, device=dev) for p in precs}
    pi = {p: torch.empty(S, dtype=torch.int32, device=dev) for p in precs}

    def step(record):
        for p in precs:
            o = ipi.make_opts(**opts[p])
            st, info = ipi.ipi_solve(mdp.handle, o, V[p], pi[p])
            if st != ipi.IPI_OK:
                raise RuntimeError(f"solve did not converge ({p}): {info}")
            if record is not None:
                record.append((p, info))

    for i in range(args.warmup):
        t = time.perf_counter()
        step(None)
        log(f"warmup step {i} {time.perf_counter() - t:.3f}s")
    recs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(recs)
        log(f"timed step {i} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    total_bytes = sum(info["alg_bytes"] for _, info in recs)
    per_prec = {}
    for p in precs:
        infos = [info for q, info in recs if q == p]
        pp = {
            "time_to_tol_ms": round(float(np.median([i["device_ms"] for i in infos])), 3),
            "outer_iters": infos[-1]["outer_iters"], "inner_iters": infos[-1]["inner_iters"],
            "block_launches": infos[-1]["block_launches"],
            "final_rho": infos[-1]["final_rho"], "fp64_rho": infos[-1]["fp64_rho"],
            "err_bound_rel": infos[-1]["err_bound"] / max(1e-300, float(V[p].abs().max())),
            "bellman_calls": sum(i["bellman_calls"] for i in infos),
            "bellman_ms": sum(i["bellman_ms"] for i in infos),
            "bellman_bytes": infos[-1]["bellman_bytes"],
            "inner_ms": sum(i["inner_ms"] for i in infos),
            "product_calls": sum(i["product_calls"] for i in infos),
            "product_ms": sum(i["product_ms"] for i in infos),
            "product_bytes": sum(i["product_bytes"] for i in infos),
            # the blocked Richardson launches of the most sweeps (16 in long solves)
            "block_sweeps": max(i["block_sweeps"] for i in infos),
            "block_calls": sum(i["block_calls"] for i in infos),
            "block_ms": sum(i["block_ms"] for i in infos),
            "block_bytes": sum(i["block_bytes"] for i in infos),
            "alg_gbs": sum(i["alg_bytes"] for i in infos) / (sum(i["device_ms"] for i in infos) / 1e3) / 1e9,
            # P_pi loaded through the caches (bit 0: one-sweep products, bit 1: blocked sweeps)
            "ppi_cached": infos[-1]["ppi_cached"],
        }
        pp["bellman_avg_us"] = pp["bellman_ms"] / max(1, pp["bellman_calls"]) * 1e3
        pp["bellman_gbs"] = pp["bellman_bytes"] / (pp["bellman_avg_us"] * 1e-6) / 1e9 if pp["bellman_avg_us"] else None
        pp["product_avg_us"] = pp["product_ms"] / max(1, pp["product_calls"]) * 1e3
        pp["product_gbs"] = pp["product_bytes"] / (pp["product_ms"] * 1e-3) / 1e9 if pp["product_ms"] else None
        pp["block_avg_us"] = pp["block_ms"] / max(1, pp["block_calls"]) * 1e3
        pp["block_gbs"] = pp["block_bytes"] / (pp["block_ms"] * 1e-3) / 1e9 if pp["block_ms"] else None
        per_prec[p] = pp
    p0 = precs[0]
    pr = per_prec[p0]
    # which kernels the default tuning runs: the blocked Richardson sweeps when
    # the library ran them; else flat chunk streaming for rows of one length
    # (even for FP64) on wave tiles, or workgroup tiles; the Bellman pass runs
    # on wave tiles in the band form (A <= 64), else on workgroup tiles when
    # A k / E <= 2048
    desc = mdp.describe()
    kk = desc["k_max"]
    flat = bool(desc["uniform_k"]) and kk % 2 == 0
    blocked = pr["block_launches"] > 0 and pr["block_calls"] > 0
    if blocked:
        # the kernel of those launches: rows prefetched through LDS when every
        # wavefront's next rows fit the stage (rows staged one 16-byte piece
        # apart) or the rows are too long for a second copy in registers
        # (over 128 bytes), else prefetched in registers; in the LDS cases the
        # two-state kernel when it fits (pairs of rows staged 2 NP + 1 pieces
        # apart, at least half of its 8 wavefronts prefetched, both rows in
        # registers)
        row_bytes = kk * (4 if p0 == "fp32_mixed" else 8)
        waves = (160 * 1024 - 2 * 1024 * 8 - 16 * 8 - 256) // (64 * 16 * (row_bytes // 16 + 1))
        lds = waves >= 16 or row_bytes > 128
        pwaves = min(8, (160 * 1024 - 2 * (1024 + 8) * 8 - 8 * 8 - 256) // (64 * 16 * (2 * (row_bytes // 16) + 1)))
        pair = lds and pwaves >= 8 - pwaves and 2 * row_bytes <= 384
        pk = "k_rich_block_pair" if pair else ("k_rich_block_lds" if lds else "k_rich_block_pf")
    else:
        pk = "k_wave_flat" if flat else "k_tiled"
    if flat and desc["band"] and d.A <= 64:
        bk = "k_bellman_wave"
    elif bool(desc["uniform_k"]) and (kk == 1 or (flat and d.A * (kk // 2) <= 2048)):
        bk = "k_bellman_flat"
    else:
        bk = "k_bellman"
    if blocked:
        # the dominant launches: the blocked ones of the most sweeps
        gbs, avg_us, calls, nbytes = pr["block_gbs"], pr["block_avg_us"], pr["block_calls"], pr["block_bytes"]
        kname = f"{pk}, {pr['block_sweeps']} sweeps per launch ({p0}, {inner})"
        sweeps = pr["block_sweeps"]
    else:
        gbs, avg_us, calls, nbytes = pr["product_gbs"], pr["product_avg_us"], pr["product_calls"], pr["product_bytes"]
        kname = f"{pk} ({p0}, {inner})"
        sweeps = 1
    tr = measured_traffic(pk, cfg["workload"], p0, sweeps)
    roof = {"kernel": kname, "bound": "hbm",
            "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4),
            "traffic": tr["bytes_per_launch"] if tr else None, "traffic_unit": "bytes per launch (HBM, rocprofv3)",
            "traffic_source": tr["source"] if tr else None,
            "avg_us": round(avg_us, 2), "calls": calls,
            "bytes_per_call": round(nbytes / max(1, calls)),
            "frac_of_stream_read": round(gbs / ach["stream_read_gbs"], 4)}
    if blocked:
        # the rate the same sweeps would need launched one by one (each
        # streaming P_pi and the vectors): sweeps x bytes per launch / time
        roof["sweep_equivalent_gbs"] = round(nbytes / max(1, calls) * sweeps / (avg_us * 1e-6) / 1e9, 1)
    bell = {}
    for p in precs:
        btr = measured_traffic(bk, cfg["workload"], p)
        bell[p] = {"kernel": bk, "achieved": round(per_prec[p]["bellman_gbs"], 1),
                   "frac": round(per_prec[p]["bellman_gbs"] / HBM_PEAK_GBS, 4),
                   "frac_of_stream_read": round(per_prec[p]["bellman_gbs"] / ach["stream_read_gbs"], 4),
                   "avg_us": round(per_prec[p]["bellman_avg_us"], 2), "calls": per_prec[p]["bellman_calls"],
                   "bytes_per_call": per_prec[p]["bellman_bytes"],
                   "traffic": btr["bytes_per_launch"] if btr else None}
    # value: the metric's first part, the fused Bellman pass's algorithmic
    # bytes over its measured time, FP64, over every pass of the timed steps
    value = bell[p0]["achieved"]
    out = {
        "metric": "Bellman SpMV HBM GB/s; iPI time-to-tol FP32-mixed vs FP64; p99 solve latency",
        "value": value, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": dict(cfg, precisions=precs, inner=inner, richardson_block=args.richardson_block,
                       blocked_prefetch=args.blocked_prefetch, alpha=alpha,
                       stop="rtol_cert 1e-9", gamma=gamma),
        "value_kernel": f"{bk} ({p0}): BW_alg per pass / mean pass time, {bell[p0]['calls']} passes in the timed steps",
        "roofline": roof,
        "bellman_roofline": bell,
        "achievable": ach,
        "time_to_tol_ms": {p: per_prec[p]["time_to_tol_ms"] for p in precs},
        "whole_step_alg_gbs": round(total_bytes / elapsed / 1e9, 2),
        "detail": per_prec,
    }
    if "fp64" in per_prec and "fp32_mixed" in per_prec:
        out["fp32_mixed_speedup"] = round(per_prec["fp64"]["time_to_tol_ms"] / per_prec["fp32_mixed"]["time_to_tol_ms"], 3)
    if not args.no_extras:
        # the fused Bellman pass alone through its entry point (it also writes
        # T V: 8 S bytes more than in a solve), median of 20 after 3 warm-ups
        out["bellman_series"] = {p: bellman_series(ipi, mdp, V[p], p, per_prec[p]["bellman_bytes"]) for p in precs}
        log(f"bellman series: {out['bellman_series']}")
        # outside the timed steps: the same MDP with the other inner solvers and
        # the fp32_inner mode, one solve each
        others = {}
        # (the Krylov solvers with Table 1's inner cap of 1000: TFQMR stalls on
        # this chain and would otherwise run 1e5 steps per evaluation)
        cases = [("richardson_no_pc", dict(ksp_type="richardson", pc="none")),
                 ("richardson_one_sweep_no_pc", dict(ksp_type="richardson", pc="none", richardson_block=0)),
                 ("gmres30_no_pc", dict(ksp_type="gmres", pc="none", restart=30, max_inner=1000)),
                 ("tfqmr_no_pc", dict(ksp_type="tfqmr", pc="none", max_inner=1000))]
        for name, kw in cases:
            for p in precs:
                o = ipi.make_opts(**dict(opts[p], profile=0, **kw))
                Vx = torch.empty_like(V[p])
                px = torch.empty_like(pi[p])
                st, info = ipi.ipi_solve(mdp.handle, o, Vx, px)
                others[f"{name}_{p}"] = {"status": st, "time_to_tol_ms": round(info["device_ms"], 3),
                                         "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"],
                                         "final_rho": info["final_rho"]}
                log(f"{name} {p}: {others[f'{name}_{p}']}")
        # the one-sweep product kernel the blocked launches replace, timed
        # (one profiled solve, HIP events around every 16th launch): an
        # HBM-bound kernel, for comparison with the roofline above
        o = ipi.make_opts(**dict(opts[p0], profile=1, ksp_type="richardson", pc="none", richardson_block=0))
        st, info = ipi.ipi_solve(mdp.handle, o, torch.empty_like(V[p0]), torch.empty_like(pi[p0]))
        if info["product_calls"] and info["product_ms"]:
            g1 = info["product_bytes"] / (info["product_ms"] * 1e-3) / 1e9
            out["one_sweep_kernel"] = {
                "kernel": f"k_wave_flat ({p0}, richardson, one launch per sweep)", "bound": "hbm",
                "achieved": round(g1, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(g1 / HBM_PEAK_GBS, 4),
                "avg_us": round(info["product_ms"] / info["product_calls"] * 1e3, 2),
                "calls": info["product_calls"],
                "bytes_per_call": round(info["product_bytes"] / info["product_calls"])}
            log(f"one-sweep kernel: {out['one_sweep_kernel']}")
        V_inner = torch.empty_like(V[p0])
        o = ipi.make_opts(**dict(opts[p0], profile=0, precision="fp32_inner"))
        st, info = ipi.ipi_solve(mdp.handle, o, V_inner, torch.empty_like(pi[p0]))
        others["richardson_fp32_inner"] = {"status": st, "time_to_tol_ms": round(info["device_ms"], 3),
                                           "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"],
                                           "final_rho": info["final_rho"],
                                           "err_bound_rel": info["err_bound"] / float(V_inner.abs().max())}
        log(f"fp32_inner: {others['richardson_fp32_inner']}")
        # the same MDP with its values held as float32 hi + lo (8 bytes a value
        # instead of FP64 + float32, 12): the fp32_inner solve, whose Bellman
        # passes read hi + lo, and that pass alone
        sp = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_SPLIT)
        try:
            data_bytes = sp.describe()["device_bytes"]
            V_split = torch.empty_like(V[p0])
            st, info = ipi.ipi_solve(sp.handle, o, V_split, torch.empty_like(pi[p0]))
            others["richardson_fp32_inner_split"] = {
                "status": st, "time_to_tol_ms": round(info["device_ms"], 3), "outer_iters": info["outer_iters"],
                "inner_iters": info["inner_iters"], "final_rho": info["final_rho"],
                "err_bound_rel": info["err_bound"] / float(V_split.abs().max()), "mdp_device_bytes": data_bytes}
            log(f"fp32_inner on split values: {others['richardson_fp32_inner_split']}")
            if "fp64" in per_prec:
                out["bellman_series_split"] = bellman_series(ipi, sp, V["fp64"], "fp64",
                                                             per_prec["fp64"]["bellman_bytes"])
                log(f"bellman series, split values: {out['bellman_series_split']}")
        finally:
            sp.close()
        out["other_solvers"] = others
    if not args.no_cpu_baseline:
        gpu_V = {p: V[p].cpu().numpy() for p in precs}
        if not args.no_extras:
            gpu_V["fp32_inner"] = V_inner.cpu().numpy()
            gpu_V["fp32_inner_split"] = V_split.cpu().numpy()
        base, errors = cpu_baseline_c2(d, gpu_V, gamma) if args.config == "c2" else (cpu_baseline(d), {})
        out["cpu_baseline"] = base
        if errors:
            # relative error of each result against the oracle's exact V* of the FP64 MDP
            out["rel_error_vs_fp64_oracle"] = errors
        log(f"cpu baseline: {base}; errors {errors}")
    mdp.close()
    del V, pi
    if not args.no_extras and args.config == "c2":
        out["c3_bellman"] = c3_bellman_series(ipi, solve=True)
        # the other configurations' lines, smaller where the full one takes
        # minutes: c1 whole; c4 on its first 128 members (of 512), two batch
        # solves per precision; c5 (an 8-minute request stream) runs only as
        # --config c5
        import types
        out["c1"] = c1_result(types.SimpleNamespace(steps=args.steps, warmup=args.warmup))
        log(f"c1: {out['c1']['value']} ms")
        out["c4_subset"] = c4_result(types.SimpleNamespace(steps=2, members=128, precisions="fp64,fp32_mixed"))
        log(f"c4 subset: {out['c4_subset']['detail']}")
    print(json.dumps(out), flush=True)


def c3_bellman_series(ipi, solve=False):
    """The second GB/s workload, the pendulum (2048 x 2048 grid, A = 11, k = 4):
    the fused Bellman pass alone, median of 20 after 3 warm-ups per precision,
    on V = T^2(0); with solve, also one solve to the certified tolerance per
    precision (Jacobi-preconditioned Richardson, alpha = 0.1, outside any
    timed step)."""
    import torch

    from paper_2507_22538_amd import workloads as W
    dev = torch.device("cuda:0")
    d = W.c3(2048)
    m = ipi.MDP.from_data(d, flags=ipi.IPI_VAL_FP32)
    try:
        V = torch.zeros(d.S, dtype=torch.float64, device=dev)
        for _ in range(2):
            V, _, _, _ = m.bellman(V)
        torch.cuda.synchronize()
        desc = m.describe()
        R = d.S * d.A
        out = {"workload": "pendulum_2048x2048_A11_k4_gamma0.9999", "nnz": d.nnz}
        # the stencil form replaces the 4 column indices of a row by one word
        idx = 4.0 * R if desc["stencil_patterns"] > 0 else 4.0 * d.nnz
        for p, code, bv in (("fp64", ipi.IPI_FP64, 8.0), ("fp32_mixed", ipi.IPI_FP32_MIXED, 4.0)):
            # uniform rows: no row pointers read; values, indices, g, V, T V, pi, resid
            nbytes = d.nnz * bv + idx + 8.0 * R + 28.0 * d.S
            out[p] = bellman_series(ipi, m, V, p, nbytes - 8.0 * d.S)
            tr = measured_traffic("k_bellman_flat", out["workload"], p)
            out[p]["traffic"] = tr["bytes_per_launch"] if tr else None
        out["band"] = desc["band"]
        out["stencil_patterns"] = desc["stencil_patterns"]
        log(f"c3 bellman series: {out}")
        if solve:
            sol = {}
            for p in ("fp64", "fp32_mixed"):
                o = ipi.make_opts(atol=0.0, rtol_cert=1e-9, alpha=0.1, ksp_type="richardson", pc="jacobi",
                                  max_inner=1000000, precision=p)
                Vx = torch.empty(d.S, dtype=torch.float64, device=dev)
                st, info = ipi.ipi_solve(m.handle, o, Vx, torch.empty(d.S, dtype=torch.int32, device=dev))
                sol[p] = {"status": st, "time_to_tol_ms": round(info["device_ms"], 1),
                          "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters"],
                          "err_bound_rel": info["err_bound"] / float(Vx.abs().max())}
                log(f"c3 solve {p}: {sol[p]}")
            sol["fp32_mixed_speedup"] = round(sol["fp64"]["time_to_tol_ms"] / sol["fp32_mixed"]["time_to_tol_ms"], 3)
            out["time_to_tol"] = sol
        return out
    finally:
        m.close()


if __name__ == "__main__":
    main()
