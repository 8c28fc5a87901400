"""Benchmark of the fine-level two-level time stepping on one MI355X.

Workload (default): the single-track case at paper-like resolution -- a
2 x 1 x 0.5 mm plate with 50 x 25 x 13 coarse Q1 cells, a window of 10 x 5 x 3
coarse cells refined 8x (81 x 41 x 25 = 83,025 fine nodes), 8 micro steps per
25 us macro step, FP64 linear solves.  One benchmark step is one macro step
of the method (window update, coarse predictor, 7 fine micro steps, the
two-level correction with its fine and coarse solves, injection, ledger).

Metric: fine DOF-timesteps per second = (free fine nodes x micro steps) /
wall time of the timed macro steps, inputs resident in HBM.  The result is
checked against the FP64 CPU oracle by the parity tests, not here.

Prints one JSON line.  `roofline` reports the fine CG iteration kernel (one
Chronopoulos-Gear PCG iteration fused with the matrix-free Q1 apply):
algorithmic bytes per launch (read r, w, s_old, p, x, d, kappa, Dinv; write
r', w', s, p, x) over its average launch duration, timed with HIP events on
the library's stream for a sample of the launches that did work inside the
timed region.  `k2_sweep` times the bare operator apply (read v, d, kappa;
write y) at the workloads' fine shapes and at an HBM-resident grid.
`cpu_baseline` times the CPU oracle on one complete macro step of the same
workload.
"""
import argparse
import json
import os
import sys
import time
from dataclasses import replace

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100, help="timed macro steps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed macro steps (separate run)")
    ap.add_argument("--workload", default="single_track_2mm",
                    choices=["single_track_2mm", "single_track_1mm", "raster_5mm",
                             "served_tracks", "raster_10mm"])
    ap.add_argument("--requests", type=int, default=64, help="served_tracks: requests in the stream")
    ap.add_argument("--slots", type=int, default=64, help="served_tracks: server slots")
    ap.add_argument("--budget-mb", type=float, default=0.0,
                    help="served_tracks: HBM budget for active requests (0: room for every slot)")
    ap.add_argument("--load", type=float, default=1.5,
                    help="served_tracks: arrival rate as a multiple of the measured batched capacity")
    ap.add_argument("--precision", default=None, choices=[None, "fp64", "mixed"])
    ap.add_argument("--coupling", default=None, choices=[None, "dn", "composite"],
                    help="two-level correction: Dirichlet-Neumann iteration or one "
                         "composite-grid solve (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time every Nth fine operator launch with HIP events (0: off)")
    ap.add_argument("--k2-sweep", action="store_true",
                    help="also time the bare operator apply at several shapes")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB buffer 3 times (known-size "
                         "reference for HBM byte counters)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with measured HBM bytes per launch of the operator kernel")
    return ap.parse_args()


def measured_traffic(path, workload, elem):
    """HBM bytes per launch of the CG iteration kernel from the calibrated
    rocprofv3 FETCH_SIZE/WRITE_SIZE record in profiles/, or None when there
    is no record for this workload and precision or the kernel source has
    changed since the counters were taken."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    kname = "cg_iter_batched_kernel<%s, 0>" % ("double" if elem == 8 else "float")
    if path is None:
        path = os.path.join(root, "profiles", f"cg_iter_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = open(os.path.join(root, "paper_2110_12932_amd", "csrc", "tl_kernels.hip"), "rb").read()
    if rec.get("kernel") != kname or rec.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(wl, n_macro=2):
    """The oracle on the first `n_macro` complete macro steps of the same
    workload (about 10-20 s of CPU work at the benchmark size), one core."""
    from threadpoolctl import threadpool_limits
    import oracle
    el, dof_steps = 0.0, 0
    with threadpool_limits(1):
        sim = oracle.TwoLevel(wl)
        for _ in range(n_macro):
            t0 = time.perf_counter()
            sim.step()
            el += time.perf_counter() - t0
            dof_steps += int((~sim.win.dir_f).sum()) * wl.options.m_time
    return {"value": dof_steps / el, "unit": "fine DOF-timesteps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{wl.name} macro steps 0-{n_macro - 1} in full "
                      f"({n_macro * wl.options.m_time} micro steps, {dof_steps} fine "
                      f"DOF-steps, two-level correction included): "
                      f"{el:.1f} s on 1 core of {os.cpu_count()} "
                      f"(affinity {len(os.sched_getaffinity(0))})"}


def k2_sweep(tl, W, torch):
    """Bare operator apply y = d v + K[kappa] v, timed with events on the
    current stream (the library launches on it) over repeated launches."""
    import numpy as np
    out = []
    shapes = [("single_track_2mm fine", 80, 40, 24), ("raster_10mm fine", 120, 80, 30),
              ("mid-size 300x120x132", 300, 120, 132),
              ("HBM-resident 640x640x160", 640, 640, 160)]
    g = torch.Generator(device="cuda").manual_seed(0)
    for name, nx, ny, nz in shapes:
        for prec, dt, eb in ((W.FP64, torch.float64, 8), (W.MIXED, torch.float32, 4)):
            grid = tl.to_grid(nx, ny, nz, 5e-6, 5e-6, 4.8e-6)
            npad = tl.tl_op_padded_size(grid)
            nodes = (nx + 1) * (ny + 1) * (nz + 1)
            d = torch.rand(npad, dtype=dt, device="cuda", generator=g) * 1e-3
            kap = 10 + 20 * torch.rand(npad, dtype=dt, device="cuda", generator=g)
            v = torch.rand(npad, dtype=dt, device="cuda", generator=g) * 300
            y = torch.empty_like(v)
            reps = 20 if nodes > 1e7 else 200
            tl.tl_op_apply(grid, prec, d, kap, v, y, 3)
            # the median of 5 batches of `reps` launches
            batch_us = []
            for _ in range(5):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                tl.tl_op_apply(grid, prec, d, kap, v, y, reps)
                e1.record()
                torch.cuda.synchronize()
                batch_us.append(e0.elapsed_time(e1) * 1e3 / reps)
            us = float(np.median(batch_us))
            gbs = 4 * eb * nodes / (us * 1e-6) / 1e9
            out.append({"shape": name, "nodes": nodes, "dtype": "f64" if eb == 8 else "f32",
                        "us_per_launch": round(us, 3), "GB/s": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)})
            del d, kap, v, y
    # the practical HBM ceiling for reference: a device-to-device copy of
    # 1 GiB (read + write bytes over the time) and a read-only reduction
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").uniform_(generator=g)
    dst = torch.empty_like(src)
    for kind in ("copy", "sum"):
        for _ in range(2):
            dst.copy_(src) if kind == "copy" else src.sum()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            dst.copy_(src) if kind == "copy" else src.sum()
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / 10
        nbytes = (2 if kind == "copy" else 1) * src.numel() * 4
        out.append({"shape": f"torch {kind}, 1 GiB fp32", "dtype": "f32",
                    "us_per_launch": round(us, 3), "GB/s": round(nbytes / (us * 1e-6) / 1e9, 1),
                    "frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)})
    del src, dst
    return out


def serve_stream(tl, W, torch, reqs, slots, budget, arrivals=None, profile_every=0):
    """Run a request stream through a server.  arrivals: seconds after the
    start at which each request is submitted (None: all at once).  Returns
    (wall seconds, per-request latencies, per-request stats, profile)."""
    pool = sum(tl.tl_workspace_bytes(w.mesh, w.options) + 4096 for w in reqs)
    pool += tl.tl_server_overhead_bytes(slots) + (1 << 20)
    sv = tl.Server(pool, hbm_budget=budget if budget else pool, max_slots=slots)
    if profile_every:
        tl.tl_server_set_profiling(sv.h, profile_every)
    arr = [0.0] * len(reqs) if arrivals is None else list(arrivals)
    order = sorted(range(len(reqs)), key=lambda q: arr[q])
    ids, done_t = {}, {}
    nxt = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while len(done_t) < len(reqs):
        now = time.perf_counter() - t0
        while nxt < len(order) and arr[order[nxt]] <= now:
            q = order[nxt]
            ids[sv.submit(reqs[q])] = q
            nxt += 1
        active, queued, finished = sv.tick()
        if finished:
            t = time.perf_counter() - t0
            for rid, q in ids.items():
                if q not in done_t and sv.info(rid)["state"] >= 2:
                    done_t[q] = t
        if active == 0 and queued == 0 and nxt < len(order):
            time.sleep(max(0.0, arr[order[nxt]] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    stats = []
    for rid, q in ids.items():
        _, _, st, _, info = sv.result(rid)
        if info["state"] != 2:
            raise RuntimeError(f"request {q} failed")
        stats.append(st)
    lat = [done_t[q] - arr[q] for q in range(len(reqs))]
    prof = tl.tl_server_get_profile(sv.h) if profile_every else (0, 0.0)
    sv.close()
    return wall, lat, stats, prof


def main_serving(args):
    """The served workload: a seeded stream of single-track requests through the
    continuous-batching server.  A closed-loop run (all requests at t = 0)
    measures the batched capacity; the stream then arrives as a Poisson
    process at `--load` times that capacity, and throughput (fine
    DOF-timesteps/s over the stream's wall time) and p50/p99 latency come
    from that run."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2110_12932_amd import tl
    tl.load()
    stream = W.served_tracks(args.requests, seed=0, mean_interarrival=1.0)
    reqs = [w for _, w in stream]
    unit_gaps = np.diff([0.0] + [a for a, _ in stream])   # Exp(1) draws, in order
    budget = int(args.budget_mb * 2 ** 20) if args.budget_mb else 0
    # warm-up: two short requests
    serve_stream(tl, W, torch, [replace(reqs[0], n_macro=2), replace(reqs[1], n_macro=2)],
                 2, 0)
    wall_c, _, _, _ = serve_stream(tl, W, torch, reqs, args.slots, budget)
    capacity = len(reqs) / wall_c                      # requests per second
    mean_gap = 1.0 / (args.load * capacity)
    arrivals = np.cumsum(unit_gaps * mean_gap)
    wall, lat, stats, prof = serve_stream(tl, W, torch, reqs, args.slots, budget,
                                          arrivals, args.profile_every)
    dof = sum(st["fine_dof_steps"] for st in stats)
    fine_bytes = sum(st["fine_op_bytes"] for st in stats)
    roofline = None
    if prof[0] > 0:
        # fused CG iteration: 13 arrays of FP32 per fine node and iteration
        fine_iters = sum(st["fine_op_applies"] for st in stats)
        launches_work = prof[0] * max(1, args.profile_every)
        achieved = fine_bytes / (prof[1] * 1e-3 * max(1, args.profile_every)) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "cg_iter_batched_kernel<float, 0> (all requests of a tick)",
                    "avg_launch_us": prof[1] * 1e3 / prof[0],
                    "bytes_per_launch": fine_bytes / max(1.0, launches_work),
                    "launches_timed": prof[0], "fine_cg_item_iterations": fine_iters}
    lat = np.array(lat)
    out = {
        "metric": "fine DOF-timesteps/s", "value": dof / wall, "unit": "fine DOF-timesteps/s",
        "n_gpus": 1, "steps": int(sum(st["macro_steps"] for st in stats)), "warmup": 1,
        "ms_per_step": wall * 1e3 / max(1, int(sum(st["macro_steps"] for st in stats))),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "served_tracks", "requests": len(reqs), "slots": args.slots,
                   "hbm_budget_bytes": budget or "unbounded",
                   "fine_nodes_per_request": list(stats[0]["fine_nodes"]),
                   "arrivals": f"Poisson, {args.load}x the closed-loop capacity "
                               f"({capacity:.2f} req/s), mean gap {mean_gap * 1e3:.1f} ms"},
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "closed_loop": {"wall_s": wall_c, "fine_dof_steps_per_s": dof / wall_c},
        "roofline": roofline,
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.workload == "served_tracks" and args.gpus == 1:
        main_serving(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2110_12932_amd import tl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    kw = {}
    if args.precision:
        kw["precision"] = W.FP64 if args.precision == "fp64" else W.MIXED
    wl = W.by_name(args.workload, **kw)
    if args.coupling:
        from dataclasses import replace
        wl = replace(wl, options=replace(
            wl.options, coupling=W.COMPOSITE if args.coupling == "composite" else W.DN))
    steps = min(args.steps, wl.n_macro)
    tl.load()

    # warm-up on its own handle (first launches, code objects, caches)
    if args.warmup > 0:
        s = tl.Sim(wl)
        s.step(min(args.warmup, wl.n_macro))
        s.close()
    torch.cuda.synchronize()

    sim = tl.Sim(wl)
    if args.profile_every > 0:
        tl.tl_set_profiling(sim.h, args.profile_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = sim.stats()
    led = sim.ledger()
    sim.close()

    value = st["fine_dof_steps"] / el
    fine_nodes = st["fine_nodes"][0] * st["fine_nodes"][1] * st["fine_nodes"][2]
    elem = 8 if wl.options.precision == W.FP64 else 4
    # fused CG iteration: read r, w, s_old, p, x, d, kappa, Dinv; write r', w',
    # s, p, x -- 13 arrays of the CG precision per node
    bytes_per_launch = 13 * elem * fine_nodes
    roofline = None
    if st["fine_op_timed"] > 0:
        avg_s = st["fine_op_timed_ms"] / st["fine_op_timed"] * 1e-3
        achieved = bytes_per_launch / avg_s / 1e9
        traffic = measured_traffic(args.traffic, wl.name, elem)
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "kernel": "cg_iter_batched_kernel<%s, 0>" % ("double" if elem == 8 else "float"),
                    "bytes_per_launch": bytes_per_launch, "avg_launch_us": avg_s * 1e6,
                    "launches_timed": st["fine_op_timed"]}
    out = {
        "metric": "fine DOF-timesteps/s",
        "value": value,
        "unit": "fine DOF-timesteps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl.options.precision == W.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "fine_nodes": list(st["fine_nodes"]),
                   "coarse_nodes": list(st["coarse_nodes"]), "m_time": wl.options.m_time,
                   "dt_coarse": wl.options.dt_coarse,
                   "precision": "fp64" if wl.options.precision == W.FP64 else "mixed",
                   "coupling": "composite" if wl.options.coupling == W.COMPOSITE else "dn",
                   "macro_steps_timed": steps},
        "roofline": roofline,
        "counters": {k: st[k] for k in ("micro_steps", "newton_fine", "newton_coarse", "cg_fine",
                                        "cg_coarse", "dn_iters", "window_moves", "fine_solves",
                                        "coarse_solves", "line_search_halvings")},
        "ledger_rel_defect": abs((led["stored"] - led["stored0"])
                                 - (led["absorbed"] - led["bottom"] - led["surface"] + led["remap"]))
                             / max(abs(led["absorbed"]), 1e-300),
    }
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.rand(n, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibrate_copy_bytes"] = n * 4
    if args.k2_sweep:
        out["k2_sweep"] = k2_sweep(tl, W, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
