"""Benchmark of the fine-level two-level time stepping on one MI355X.

Workload (default): the large multi-track build -- a 10 x 10 x 2 mm plate
with 200 x 200 x 40 coarse Q1 cells (1.66 M coarse nodes), 20 alternating
raster tracks at 100 um hatch, a window of 12 x 8 x 3 coarse cells refined
10x (121 x 81 x 31 = 303,831 fine nodes), 8 micro steps per 25 us macro
step, FP64 linear solves.  One benchmark step is one macro step of the
method (window update, coarse predictor, 7 fine micro steps, the composite
two-level correction, injection, ledger).

Metric: fine DOF-timesteps per second = (free fine nodes x micro steps) /
wall time of the timed macro steps, inputs resident in HBM.  The timed run
starts from the initial state, so its fields are compared with the oracle's
fields for the same number of macro steps where tests/golden holds them
(`oracle_rel_err`: max-norm error relative to the largest temperature, and
to the largest rise above the plate).  `mixed` repeats the run with the
mixed-precision path (FP32 operator and CG on both levels under an FP64
residual, Newton iteration and ledger) and reports its speedup over the
FP64 path.
`serving` runs the served stream of 64 single-track requests (closed loop,
then Poisson arrivals at 1.5x that capacity) with its p50/p99 latency.

Prints one JSON line.  `roofline` reports the fine CG iteration kernel (one
Chronopoulos-Gear PCG iteration fused with the matrix-free Q1 apply):
algorithmic bytes per launch (read r, w, s_old, p, x, d, kappa, Dinv; write
r', w', s, p, x) over its average launch duration, timed with HIP events on
the library's stream for a sample of the fine micro steps' launches that
did work inside the timed region (CG iterations after the first of each
direction, which read and write all 13 arrays).  `k2_sweep` times the bare operator apply
(read v, d, kappa; write y) at the workloads' fine shapes and at an
HBM-resident grid.  `cpu_baseline` times the CPU oracle on a bounded sample
of the same workload: whole macro steps where one takes a few seconds, else
the first fine micro steps of the first macro step (the fine-level implicit
solves alone; the oracle's coarse predictor and correction on the 1.66 M-node
plate take several times longer and are left out).
"""
import argparse
import json
import os
import sys
import time
from dataclasses import replace

HBM_PEAK_GBS = 8000.0
DEFAULT_WORKLOAD = "raster_10mm"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed macro steps")
    ap.add_argument("--warmup", type=int, default=2, help="untimed macro steps (separate run)")
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD,
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
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-precision run of the FP64 workload")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the served stream of the default run")
    ap.add_argument("--profile-every", type=int, default=8,
                    help="time every Nth fine operator launch with HIP events (0: off)")
    ap.add_argument("--k2-sweep", action="store_true",
                    help="also time the bare operator apply at several shapes")
    ap.add_argument("--sync-probe", action="store_true",
                    help="also measure a device-wide barrier against a kernel boundary "
                         "between dependent sweeps, at the served and the large-window scale")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-MiB buffer 3 times (known-size "
                         "reference for HBM byte counters)")
    ap.add_argument("--traffic", default=None,
                    help="JSON file with measured HBM bytes per launch of the operator kernel")
    return ap.parse_args()


def measured_traffic(path, workload, elem):
    """(HBM bytes per launch, kernel instance) of the CG iteration kernel from
    the calibrated rocprofv3 FETCH_SIZE/WRITE_SIZE record in profiles/, or
    (None, None) when there is no record for this workload and precision or
    the kernel source has changed since the counters were taken.  The
    instance names the stack depth the library chose for the workload's
    window (`<R, 0, 2>`: stacks of two tiles)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    prefix = "cg_iter_batched_kernel<%s, 0," % ("double" if elem == 8 else "float")
    if path is None:
        path = os.path.join(root, "profiles", f"cg_iter_{workload}_traffic.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path))
    src = open(os.path.join(root, "paper_2110_12932_amd", "csrc", "tl_kernels.hip"), "rb").read()
    if (not str(rec.get("kernel", "")).startswith(prefix)
            or rec.get("kernel_source_sha256") != hashlib.sha256(src).hexdigest()):
        return None, None
    return rec.get("bytes_per_launch"), rec["kernel"]


def cpu_baseline(wl, n_macro=2, budget_s=15.0):
    """The oracle, one core, on a bounded sample of the same workload:
    `n_macro` complete macro steps when the plate is small (about 10-20 s of
    CPU work at the single-track size), else the first fine micro steps of
    macro step 0 until `budget_s` has passed (at least one), with Dirichlet
    data from the initial coarse field."""
    from threadpoolctl import threadpool_limits
    import oracle
    from oracle import laser as OL
    from oracle.twolevel import micro_time
    el, dof_steps, what = 0.0, 0, ""
    with threadpool_limits(1):
        sim = oracle.TwoLevel(wl)
        free = int((~sim.win.dir_f).sum())
        if sim.coarse.n_nodes <= 100_000:
            for _ in range(n_macro):
                t0 = time.perf_counter()
                sim.step()
                el += time.perf_counter() - t0
                dof_steps += free * wl.options.m_time
            what = (f"macro steps 0-{n_macro - 1} in full ({n_macro * wl.options.m_time} "
                    "micro steps, two-level correction included)")
        else:
            m, dt = wl.options.m_time, wl.options.dt_coarse / wl.options.m_time
            g = sim.win.P @ sim.Tc
            T = sim.Tf
            j = 0
            while j < m - 1 and (j == 0 or el < budget_s):
                j += 1
                t0 = time.perf_counter()
                Ff = sim.fine_load(OL.laser_at(wl.scan, micro_time(wl.scan, wl.options, 0, j)))
                T, _ = sim.fine_step(T, dt, Ff, g)
                el += time.perf_counter() - t0
                dof_steps += free
            what = (f"fine micro steps 1-{j} of macro step 0 ({sim.win.fine.n_nodes} fine "
                    "nodes; coarse predictor and correction not included)")
    return {"value": dof_steps / el, "unit": "fine DOF-timesteps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{wl.name} {what}: {dof_steps} fine DOF-steps in {el:.1f} s on 1 core "
                      f"of {os.cpu_count()} (affinity {len(os.sched_getaffinity(0))})"}


def k2_sweep(tl, W, torch):
    """Bare operator apply y = d v + K[kappa] v with each of its two kernels
    (3D LDS tiles, z-marching columns), timed with events on the current
    stream (the library launches on it) over repeated launches; `auto` marks
    the kernel the library picks for the grid."""
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
            auto = tl.OP_ZMARCH if nodes > 4 * 2**20 and nz >= 8 else tl.OP_TILED
            for kern in (tl.OP_TILED, tl.OP_ZMARCH):
                tl.tl_op_apply(grid, prec, d, kap, v, y, 3, kernel=kern)
                # the median of 5 batches of `reps` launches
                batch_us = []
                for _ in range(5):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    tl.tl_op_apply(grid, prec, d, kap, v, y, reps, kernel=kern)
                    e1.record()
                    torch.cuda.synchronize()
                    batch_us.append(e0.elapsed_time(e1) * 1e3 / reps)
                us = float(np.median(batch_us))
                gbs = 4 * eb * nodes / (us * 1e-6) / 1e9
                out.append({"shape": name, "nodes": nodes, "dtype": "f64" if eb == 8 else "f32",
                            "kernel": "tiled" if kern == tl.OP_TILED else "zmarch",
                            "auto": kern == auto,
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


def sync_probe(tl, torch):
    """Per-sweep time of `rounds` dependent sweeps with one launch per sweep
    against one cooperative launch with a grid barrier per sweep, over the
    bytes one fine CG launch moves: the served batch (64 requests of
    81 x 49 x 25 nodes, 13 FP32 arrays) and the large window (121 x 81 x 31
    nodes, 13 FP64 arrays)."""
    out = []
    ctl = torch.zeros(1024, dtype=torch.uint8, device="cuda")
    for name, nbytes in (("served batch, FP32", 13 * 4 * 64 * 81 * 49 * 25),
                         ("large window, FP64", 13 * 8 * 121 * 81 * 31)):
        n = nbytes // 16       # a sweep reads and writes each double: 16 B
        data = torch.zeros(n, dtype=torch.float64, device="cuda")
        for blocks in (256, 1024):
            row = {"data": name, "bytes_per_sweep": 16 * n, "blocks": blocks}
            for barrier in (0, 1):
                tl.tl_op_sync_probe(blocks, 2, barrier, data, ctl)     # warm-up
                t1 = tl.tl_op_sync_probe(blocks, 1, barrier, data, ctl)
                t21 = tl.tl_op_sync_probe(blocks, 21, barrier, data, ctl)
                key = "barrier" if barrier else "launches"
                row[key + "_us_per_sweep"] = round((t21 - t1) / 20, 2)
            out.append(row)
        del data
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


def serving_run(args, tl, W, torch, profile_every=0):
    """The served workload: a seeded stream of single-track requests through the
    continuous-batching server.  A closed-loop run (all requests at t = 0)
    measures the batched capacity; the stream then arrives as a Poisson
    process at `--load` times that capacity, and throughput (fine
    DOF-timesteps/s over the stream's wall time) and p50/p99 latency come
    from that run."""
    import numpy as np
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
                                          arrivals, profile_every)
    dof = sum(st["fine_dof_steps"] for st in stats)
    lat = np.array(lat)
    return {"wall": wall, "wall_closed": wall_c, "dof": dof, "stats": stats, "prof": prof,
            "capacity": capacity, "mean_gap": mean_gap, "budget": budget, "n": len(reqs),
            "p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}


def serving_summary(args, tl, W, torch):
    r = serving_run(args, tl, W, torch)
    return {"workload": "served_tracks", "requests": r["n"], "slots": args.slots,
            "precision": "mixed", "hbm_budget_bytes": r["budget"] or "unbounded",
            "fine_dof_steps_per_s": r["dof"] / r["wall"],
            "latency_p50_s": r["p50"], "latency_p99_s": r["p99"],
            "arrivals": f"Poisson, {args.load}x the closed-loop capacity "
                        f"({r['capacity']:.2f} req/s)",
            "closed_loop_fine_dof_steps_per_s": r["dof"] / r["wall_closed"]}


def main_serving(args):
    """The served workload as the headline line (--workload served_tracks)."""
    import torch
    import workloads as W
    from paper_2110_12932_amd import tl
    r = serving_run(args, tl, W, torch, args.profile_every)
    stats, prof, wall = r["stats"], r["prof"], r["wall"]
    fine_bytes = sum(st["fine_op_bytes"] for st in stats)
    roofline = None
    if prof[0] > 0:
        # fused CG iteration: 13 arrays of FP32 per fine node and iteration
        fine_iters = sum(st["fine_op_applies"] for st in stats)
        launches_work = prof[0] * max(1, args.profile_every)
        achieved = fine_bytes / (prof[1] * 1e-3 * max(1, args.profile_every)) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                    "kernel": "cg_iter_batched_kernel<float, 0, S> (all requests of a tick)",
                    "avg_launch_us": prof[1] * 1e3 / prof[0],
                    "bytes_per_launch": fine_bytes / max(1.0, launches_work),
                    "launches_timed": prof[0], "fine_cg_item_iterations": fine_iters}
    n_steps = int(sum(st["macro_steps"] for st in stats))
    out = {
        "metric": "fine DOF-timesteps/s", "value": r["dof"] / wall, "unit": "fine DOF-timesteps/s",
        "n_gpus": 1, "steps": n_steps, "warmup": 1,
        "ms_per_step": wall * 1e3 / max(1, n_steps),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "served_tracks", "requests": r["n"], "slots": args.slots,
                   "hbm_budget_bytes": r["budget"] or "unbounded",
                   "fine_nodes_per_request": list(stats[0]["fine_nodes"]),
                   "arrivals": f"Poisson, {args.load}x the closed-loop capacity "
                               f"({r['capacity']:.2f} req/s), mean gap {r['mean_gap'] * 1e3:.1f} ms"},
        "latency_p50_s": r["p50"],
        "latency_p99_s": r["p99"],
        "closed_loop": {"wall_s": r["wall_closed"],
                        "fine_dof_steps_per_s": r["dof"] / r["wall_closed"]},
        "roofline": roofline,
    }
    print(json.dumps(out), flush=True)


def golden_error(name, steps, Tc, Tf, origin):
    """Max-norm error of a run's fields against the oracle fields stored for
    the same workload and macro-step count (tests/golden, written by the
    oracle only), or None when there is none."""
    import numpy as np
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        f"{name}_n{steps}.npz")
    if not os.path.exists(path):
        return None
    g = np.load(path, allow_pickle=False)
    if tuple(int(v) for v in g["origin"]) != tuple(origin):
        return {"golden": os.path.relpath(path), "window_origin_differs": True}
    out = {"golden": os.path.relpath(path, os.path.dirname(os.path.abspath(__file__)))}
    for lvl, a, b in (("coarse", Tc, g["Tc"]), ("fine", Tf, g["Tf"])):
        d = float(np.max(np.abs(a - b)))
        out[lvl] = d / float(np.max(np.abs(b)))
        # the stricter norm: relative to the largest rise above the plate
        out[lvl + "_vs_rise"] = d / float(np.max(np.abs(b - 300.0)))
    return out


def timed_run(tl, torch, wl, steps, warmup, profile_every):
    """Warm-up on a handle of its own, then `steps` macro steps from the
    initial state on a fresh handle, bracketed by device synchronisation."""
    if warmup > 0:
        s = tl.Sim(wl)
        s.step(min(warmup, wl.n_macro))
        s.close()
    torch.cuda.synchronize()
    sim = tl.Sim(wl)
    try:
        if profile_every > 0:
            tl.tl_set_profiling(sim.h, profile_every)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        st, led = sim.stats(), sim.ledger()
        Tc, _ = sim.temperature(0)
        Tf, origin = sim.temperature(1)
    finally:
        sim.close()
    return {"el": el, "st": st, "led": led, "err": golden_error(wl.name, steps, Tc, Tf, origin)}


def ledger_defect(led):
    return abs((led["stored"] - led["stored0"])
               - (led["absorbed"] - led["bottom"] - led["surface"] + led["remap"])) \
        / max(abs(led["absorbed"]), 1e-300)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; the path's sharding across "
                                   "GPUs is a design only, so --gpus must be 1"}))
        sys.exit(2)
    if args.workload == "served_tracks":
        main_serving(args)
        return
    import torch
    import workloads as W
    from paper_2110_12932_amd import tl

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    prec = W.FP64 if args.precision in (None, "fp64") else W.MIXED

    def make_wl(p):
        w = W.by_name(args.workload, precision=p)
        if args.coupling:
            w = replace(w, options=replace(
                w.options, coupling=W.COMPOSITE if args.coupling == "composite" else W.DN))
        return w

    wl = make_wl(prec)
    steps = min(args.steps, wl.n_macro)
    tl.load()

    run = timed_run(tl, torch, wl, steps, args.warmup, args.profile_every)
    el, st, led = run["el"], run["st"], run["led"]
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
        traffic, kname = measured_traffic(args.traffic, wl.name, elem)
        if kname is None:   # S: the stack depth of the CG work units
            kname = "cg_iter_batched_kernel<%s, 0, S>" % ("double" if elem == 8 else "float")
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kname,
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
        "oracle_rel_err": run["err"],
        "roofline": roofline,
        "counters": {k: st[k] for k in ("micro_steps", "newton_fine", "newton_coarse", "cg_fine",
                                        "cg_coarse", "dn_iters", "window_moves", "fine_solves",
                                        "coarse_solves", "line_search_halvings")},
        "ledger_rel_defect": ledger_defect(led),
    }
    if args.profile_every > 0:
        # GPU time per macro step of each phase (HIP events at the phase
        # boundaries; the sampled CG-launch events run at the same time)
        out["phase_ms_per_step"] = dict(zip(
            ("window_loads_predictor", "micro_steps", "correction", "ledger_commit"),
            (round(v / steps, 4) for v in st["phase_ms"])))
    if prec == W.FP64 and not args.no_mixed:
        # the mixed-precision path (FP32 operator and CG on both levels under
        # an FP64 residual, Newton iteration and ledger) on the same workload
        # and steps
        wm = make_wl(W.MIXED)
        mr = timed_run(tl, torch, wm, steps, min(args.warmup, 1), 0)
        mv = mr["st"]["fine_dof_steps"] / mr["el"]
        out["mixed"] = {"value": mv, "ms_per_step": mr["el"] * 1e3 / steps,
                        "speedup_vs_fp64": mv / value, "oracle_rel_err": mr["err"],
                        "newton_fine": mr["st"]["newton_fine"], "cg_fine": mr["st"]["cg_fine"],
                        "ledger_rel_defect": ledger_defect(mr["led"])}
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
    if args.sync_probe:
        out["sync_probe"] = sync_probe(tl, torch)
    if not args.no_serving and args.workload == DEFAULT_WORKLOAD:
        out["serving"] = serving_summary(args, tl, W, torch)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
