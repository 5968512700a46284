"""Benchmark of the local noise filter on one MI355X.

    python bench.py [--steps K] [--warmup W] [--radius 3] [--rule mean9]

A step is one filter pass (all steps of the hot path: tile + halo staging,
x-, y- and z-passes, combine, gate, store) over one device-resident
512x512x512 uint16 CT phantom holding 12-bit data, at radius 3 with the
paper's nine-cluster mean.  The W warm-up steps are untimed and continue
until the device has been busy for at least 0.1 s (its clocks ramp up under
load; "warmup_launches" in the line counts them).  Prints one JSON line with
Gvoxel/s, the HBM roofline fraction of the kernel (timed with HIP events on
the launch stream) and the CPU oracle's rate on a bounded sample of the same
volume.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak, GB/s
# VALU peak in 32-bit lane operations per second: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz (the MINVAR9 kernel is bound by its VALU work, not by HBM)
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9
DIMS = (512, 512, 512)
SEED = 2000
WARM_SECONDS = 0.1  # least device time of the untimed warm-up before the timed steps
# rocprofv3 summaries of the kernels this script times (512^3 uint16, r = 3),
# with the measured HBM bytes per launch (FETCH_SIZE and WRITE_SIZE, each scaled
# by what it reads for the device copy of known size this script times) and the
# VALU lane operations per voxel.  Each records a hash of the kernel's sources;
# a figure is used only while the sources still hash the same (else null).
PROFILES = {
    "mean9": ("profiles/mean9_stream_r3_512cube_u16.txt",
              ["mean9.hip", "mean9_tile.h", "device_common.h", "lnf_internal.h"]),
    "minvar9": ("profiles/minvar9_planes_r3_512cube_u16.txt",
                ["minvar9.hip", "plane_tile.h", "device_common.h",
                 "lnf_internal.h"]),
}


def sources_sha256(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1807_03119_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled(rule):
    """(traffic bytes per launch, VALU lane ops per voxel) from the committed
    profile of `rule`'s kernel, or (None, None) if the kernel changed since."""
    path, files = PROFILES[rule]
    vals = {}
    try:
        with open(os.path.join(ROOT, path)) as fh:
            for line in fh:
                k, _, v = line.strip().partition(":")
                if k in ("sources_sha256", "traffic_bytes_per_launch", "valu_lane_ops_per_voxel"):
                    vals[k] = v.strip()
    except OSError:
        return None, None
    if vals.get("sources_sha256") != sources_sha256(files):
        return None, None
    t = vals.get("traffic_bytes_per_launch")
    v = vals.get("valu_lane_ops_per_voxel")
    return (int(t) if t else None), (float(v) if v else None)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def warm_up(fn, steps, min_seconds):
    """`steps` untimed launches, continued until the device has been busy for
    `min_seconds`: an idle MI355X takes some tens of milliseconds of load to
    reach its working clocks (a 512^3 MEAN9 launch runs about 190 us in the
    first 10 ms, 160 us from 20 ms on).  Synchronises every 16 launches, so
    host time tracks device time.  Returns the launches made."""
    import torch
    n = 0
    t0 = time.perf_counter()
    while n < steps or time.perf_counter() - t0 < min_seconds:
        fn()
        n += 1
        if n % 16 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return n


def time_launches(fn, steps, warmup, stream, min_warm_seconds=0.0):
    import torch
    warm_up(fn, warmup, min_warm_seconds)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def copy_bandwidth(nbytes, stream):
    """Device-to-device copy rate (read + write bytes / s) for context."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    ms, _ = time_launches(lambda: b.copy_(a), 20, 5, stream)
    return 2 * nbytes / (ms * 1e-3) / 1e9


def batch_benchmark(rule_code, stream, steps=5):
    """64 mixed volumes (axes 64..384, uint8/uint16, r in 1..3): one batch call
    as a per-tile grid, as a persistent tile queue, and the grid call captured
    in a HIP graph and replayed, against one tuned launch per volume, all on
    the same stream.  Every mode's bytes are checked against the singles."""
    import torch
    from paper_1807_03119_amd import _lib, phantom
    from paper_1807_03119_amd.api import Filter
    jobs = phantom.batch_jobs()
    vols = [phantom.batch_volume(j, device="cuda") for j in jobs]
    outs = [torch.empty_like(v) for v in vols]
    ref = [torch.empty_like(v) for v in vols]
    nvox = sum(v.numel() for v in vols)
    nbytes = sum(2 * v.numel() * v.element_size() for v in vols)
    f = Filter(rule_code, 0)
    f.tune([(v, o, j.radius) for v, o, j in zip(vols, outs, jobs)])
    triples = [(v, o, j.radius) for v, o, j in zip(vols, outs, jobs)]

    def singles():
        for v, o, j in zip(vols, ref, jobs):
            f(v, j.radius, out=o)
    ms_s, _ = time_launches(singles, steps, 2, stream)

    def same():
        torch.cuda.synchronize()
        return all(torch.equal(a.view(torch.uint8), b.view(torch.uint8)) for a, b in zip(outs, ref))
    res = {"jobs": len(jobs), "voxels": nvox, "singles_ms": ms_s,
           "singles_Gvox_s": nvox / (ms_s * 1e-3) / 1e9}
    for name, mode in (("grid", _lib.LNF_BATCH_GRID), ("queue", _lib.LNF_BATCH_PERSISTENT)):
        for o in outs:
            o.zero_()
        ms, _ = time_launches(lambda: f.batch(triples, mode=mode), steps, 2, stream)
        res[f"{name}_ms"] = ms
        res[f"{name}_Gvox_s"] = nvox / (ms * 1e-3) / 1e9
        res[f"{name}_GBps"] = nbytes / (ms * 1e-3) / 1e9
        res[f"{name}_bytes_equal_singles"] = same()
    f.close()
    # the grid call captured once in a graph (a context of its own, so no
    # earlier call left a table slot pending), replayed `steps` times
    try:
        g = Filter(rule_code, 0)
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            g.batch(triples)
        graph.replay()
        ok = same()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        cur = torch.cuda.current_stream()
        start.record(cur)
        for _ in range(steps):
            graph.replay()
        stop.record(cur)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / steps
        ok = ok and same()
        res.update({"graph_ms": ms, "graph_Gvox_s": nvox / (ms * 1e-3) / 1e9,
                    "graph_bytes_equal_singles": ok})
        del graph
        g.close()
    except Exception as e:  # capture unsupported: report, do not fail the run
        res["graph_error"] = f"{type(e).__name__}: {e}"[:200]
    res["grid_vs_singles"] = ms_s / res["grid_ms"]
    res["queue_vs_singles"] = ms_s / res["queue_ms"]
    return res


def surface_benchmark(vol, radius, threshold, stream):
    """First-hit pass (z-rays, both directions) at Otsu's threshold and the
    surface pipeline (first hit, then both rules at the hits) on the benchmark
    volume.  Algorithmic bytes of the first-hit pass: every ray reads its
    column up to and including its hit (the whole column for a miss) and
    writes 12 bytes."""
    import torch
    from paper_1807_03119_amd import _lib
    from paper_1807_03119_amd.api import Filter
    nz, ny, nx = vol.shape
    esize = vol.element_size()
    out = {"threshold": int(threshold), "rays": nx * ny}
    g = Filter(_lib.LNF_MEAN9, 0)
    for direction, name in ((1, "front"), (-1, "back")):
        hits = g.first_hit(vol, threshold, direction)
        z = hits[:, 2].to(torch.int64)
        depth = torch.where(z < 0, torch.full_like(z, nz), z + 1 if direction == 1 else nz - z)
        alg = int(depth.sum().item()) * esize + 12 * nx * ny
        ms, _ = time_launches(lambda: g.first_hit(vol, threshold, direction), 20, 3, stream)
        out[f"first_hit_{name}"] = {"ms": ms, "alg_bytes": alg, "GBps": alg / (ms * 1e-3) / 1e9,
                                    "frac_of_hbm": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                    "hit_rays": int((z >= 0).sum().item()),
                                    "mean_depth": float(depth.double().mean().item())}
    g.close()
    for rule_name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9)):
        g = Filter(rc, 0)
        ms, _ = time_launches(lambda: g.surface(vol, radius, threshold, 1), 10, 2, stream)
        out[f"pipeline_{rule_name}_r{radius}_ms"] = ms
        g.close()
    return out


def serve_benchmark(rule_code, seconds, rate=300.0, pool_n=8, side=512):
    """Open-loop Poisson replay of the serving trace against the server, once
    with continuous batching and once with one lnf_filter per request in FIFO
    order (same trace).  30% of requests re-filter a resident volume at a new
    radius; the others upload a new volume dense from a contiguous chunk of a
    pinned pool of 512^3 uint16 phantoms (the phantom's value statistics, the
    request's cube size).  Latency = completion - scheduled arrival."""
    import torch
    from paper_1807_03119_amd import _lib, phantom
    from paper_1807_03119_amd.api import Filter, Server
    pool = []
    for i in range(pool_n):
        v = phantom.ct_u12((side, side, side), seed=5100 + i, device="cuda")
        hbuf = torch.empty(v.shape, dtype=torch.uint16, pin_memory=True)
        hbuf.copy_(v)
        pool.append(hbuf)
        del v
    torch.cuda.synchronize()
    log(f"  serve: pool of {pool_n} pinned phantoms ready")
    trace = phantom.serve_trace(rate=rate, duration=seconds)
    offered = sum(r.side ** 3 for r in trace)
    out = {"requests": len(trace), "seconds": seconds, "rate_per_s": rate,
           "offered_Gvox_s": offered / seconds / 1e9, "pool_volumes": pool_n,
           "cap_bytes": 200 << 30}
    for name, mode in (("batched", _lib.LNF_SERVE_BATCHED), ("fifo", _lib.LNF_SERVE_FIFO)):
        f = Filter(rule_code, 0)
        srv = Server(f, cap_bytes=200 << 30, n_streams=4, max_batch=256, mode=mode)
        residents, rejected, lag_max = [], 0, 0.0
        t0 = _lib.lnf_server_now_ns() + 200_000_000
        wall0 = time.perf_counter()
        for k, req in enumerate(trace):
            due = t0 + int(req.t_arrival * 1e9)
            while True:
                now = _lib.lnf_server_now_ns()
                if now >= due:
                    break
                if due - now > 1_000_000:
                    time.sleep((due - now - 500_000) * 1e-9)
            lag_max = max(lag_max, (now - due) * 1e-6)
            if k % 500 == 0:
                log(f"  serve[{name}] request {k}/{len(trace)} trace t={req.t_arrival:.1f}s "
                    f"wall {time.perf_counter() - wall0:.1f}s lag {(now - due) * 1e-6:.1f} ms")
            if req.refilter and residents:
                vid = residents[int(req.pick * len(residents))]
                rc, _t = srv.submit(vid, req.radius, arrival_ns=due)
                if rc == 0:
                    continue
                residents.remove(vid)
            # a new volume arrives dense: a contiguous chunk of pinned phantom data
            src = pool[req.pool_index % pool_n]
            nvox = req.side ** 3
            o = int(req.pick * (src.numel() - nvox)) // 256 * 256
            rc, vid = srv.put(src.data_ptr() + 2 * o, dims=(req.side,) * 3, dtype=_lib.LNF_U16)
            if rc != 0:
                rejected += 1
                continue
            residents.append(vid)
            rc, _t = srv.submit(vid, req.radius, arrival_ns=due)
            if rc != 0:
                rejected += 1
        srv.sync()
        st = srv.stats()
        out[name] = {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
                     "mean_ms": st["mean_ms"], "completed": st["completed"],
                     "failed": st["failed"], "rejected": rejected, "batches": st["batches"],
                     "uploads": st["uploads"], "evictions": st["evictions"],
                     "served_Gvox_s": st["gvox_per_s"], "peak_GB": st["peak_bytes"] / 1e9,
                     "client_lag_max_ms": lag_max}
        srv.close()
        f.close()
    return out


SWEEPS = {
    # cube sides log-uniform in [lo, hi]; request rates (per second)
    "large": (128, 512, (300, 1000, 3000, 10000, 20000)),
    "small": (48, 160, (1000, 10000, 30000, 60000, 100000)),
}


def serve_sweep(rule_code, regime="large", seconds=1.5, n_vols=24, max_requests=20000):
    """Open-loop Poisson re-filter requests on device-resident volumes (no
    upload in the loop): cube sides log-uniform in the regime's range, r in
    1..3, at each of its rates, served with continuous batching and with one
    launch per request in FIFO order.  Reports p50/p99 latency (from the
    scheduled arrival) and the served rate per rate, and the rates at which
    batching has the lower p99."""
    import math

    import numpy as np
    import torch
    from paper_1807_03119_amd import _lib, phantom
    from paper_1807_03119_amd.api import Filter, Server
    lo, hi, rates = SWEEPS[regime]
    rng = np.random.default_rng(5700)
    sides = [int(round(math.exp(rng.uniform(math.log(lo), math.log(hi))))) for _ in range(n_vols)]
    hosts = []
    for i, sd in enumerate(sides):
        v = phantom.ct_u12((sd, sd, sd), seed=5800 + i, device="cuda")
        hbuf = torch.empty(v.shape, dtype=torch.uint16, pin_memory=True)
        hbuf.copy_(v)
        hosts.append(hbuf)
        del v
    torch.cuda.synchronize()
    out = {"side_range": [lo, hi], "volumes": n_vols,
           "voxels_per_volume_mean": float(np.mean([sd ** 3 for sd in sides])),
           "seconds_per_rate": seconds, "rates": {}}
    for rate in rates:
        n = min(max_requests, int(rate * seconds))
        gaps = rng.exponential(1.0 / rate, n)
        arrivals = np.cumsum(gaps)
        picks = rng.integers(0, n_vols, n)
        radii = rng.integers(1, 4, n)
        vox = float(sum(sides[int(i)] ** 3 for i in picks))
        row = {"requests": n, "offered_Gvox_s": vox / float(arrivals[-1]) / 1e9}
        for name, mode in (("batched", _lib.LNF_SERVE_BATCHED), ("fifo", _lib.LNF_SERVE_FIFO)):
            f = Filter(rule_code, 0)
            srv = Server(f, n_streams=4, max_batch=256, mode=mode)
            ids = [srv.put(h)[1] for h in hosts]
            srv.sync()
            srv.stats(reset=True)
            t0 = _lib.lnf_server_now_ns() + 50_000_000
            lag = 0.0
            for k in range(n):
                due = t0 + int(arrivals[k] * 1e9)
                while True:
                    now = _lib.lnf_server_now_ns()
                    if now >= due:
                        break
                    if due - now > 1_000_000:
                        time.sleep((due - now - 500_000) * 1e-9)
                lag = max(lag, (now - due) * 1e-6)
                srv.submit(ids[int(picks[k])], int(radii[k]), arrival_ns=due)
            srv.sync()
            st = srv.stats()
            row[name] = {"p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "max_ms": st["max_ms"],
                         "served_Gvox_s": st["gvox_per_s"], "batches": st["batches"],
                         "completed": st["completed"], "client_lag_max_ms": lag}
            srv.close()
            f.close()
        out["rates"][str(rate)] = row
        log(f"  sweep {regime} {rate}/s: batched p50/p99 {row['batched']['p50_ms']:.2f}/"
            f"{row['batched']['p99_ms']:.2f} ms {row['batched']['served_Gvox_s']:.1f} Gvox/s, "
            f"fifo {row['fifo']['p50_ms']:.2f}/{row['fifo']['p99_ms']:.2f} ms "
            f"{row['fifo']['served_Gvox_s']:.1f} Gvox/s")
    out["batched_p99_lower_at"] = [int(k) for k, v in out["rates"].items()
                                   if v["batched"]["p99_ms"] < v["fifo"]["p99_ms"]]
    return out


def burst_benchmark(rule_code, n_vols=32, n_req=2048, side_lo=48, side_hi=160):
    """Closed burst: n_req re-filter requests on resident volumes submitted at
    once (sides log-uniform in [side_lo, side_hi], r in 1..3), served with
    continuous batching and with one launch per request; wall time to drain."""
    import math

    import numpy as np
    import torch
    from paper_1807_03119_amd import _lib, phantom
    from paper_1807_03119_amd.api import Filter, Server
    rng = np.random.default_rng(5500)
    sides = [int(round(math.exp(rng.uniform(math.log(side_lo), math.log(side_hi)))))
             for _ in range(n_vols)]
    hosts = []
    for i, sd in enumerate(sides):
        v = phantom.ct_u12((sd, sd, sd), seed=5600 + i, device="cuda")
        hbuf = torch.empty(v.shape, dtype=torch.uint16, pin_memory=True)
        hbuf.copy_(v)
        hosts.append(hbuf)
    torch.cuda.synchronize()
    picks = rng.integers(0, n_vols, n_req)
    radii = rng.integers(1, 4, n_req)
    vox = int(sum(sides[i] ** 3 for i in picks))
    out = {"requests": n_req, "volumes": n_vols, "side_range": [side_lo, side_hi]}
    for name, mode in (("batched", _lib.LNF_SERVE_BATCHED), ("fifo", _lib.LNF_SERVE_FIFO)):
        f = Filter(rule_code, 0)
        srv = Server(f, n_streams=4, max_batch=256, mode=mode)
        ids = [srv.put(h)[1] for h in hosts]
        srv.sync()
        srv.stats(reset=True)
        t = time.perf_counter()
        for i, r in zip(picks, radii):
            srv.submit(ids[int(i)], int(r))
        srv.sync()
        wall = time.perf_counter() - t
        st = srv.stats()
        out[name] = {"wall_ms": wall * 1e3, "Gvox_s": vox / wall / 1e9, "batches": st["batches"],
                     "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"]}
        srv.close()
        f.close()
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(vol_np, radius, rule, got_np, budget_s=12.0, single_s=4.0):
    """Time the oracle on whole z-slices of the same volume, on all host threads
    and on one; verify the slices against the GPU output too."""
    import numpy as np
    import oracle
    nz, ny, nx = vol_np.shape
    orule = oracle.MEAN9 if rule == "mean9" else oracle.MINVAR9

    def run(z0, k, rows=None):
        rows = ny if rows is None else rows
        zz, yy, xx = np.meshgrid(np.arange(z0, z0 + k), np.arange(rows), np.arange(nx),
                                 indexing="ij")
        pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)
        t = time.perf_counter()
        vals = oracle.filter_points(vol_np, radius, pts, orule)
        dt = time.perf_counter() - t
        ok = np.array_equal(vals, got_np[z0:z0 + k, :rows].ravel().astype(np.uint32))
        return dt, ok

    threads = oracle.threads()
    z0 = nz // 2
    dt1, ok1 = run(z0, 1)
    k = int(max(1, min(nz - z0 - 1, budget_s / max(dt1, 1e-6))))
    dt, ok = run(z0 + 1, k)
    vox = k * ny * nx
    # one thread: rows of one slice, about single_s seconds
    oracle.set_threads(1)
    try:
        dr, okr = run(z0, 1, rows=8)
        rows = int(max(8, min(ny, single_s / max(dr, 1e-6) * 8)))
        ds, oks = run(z0, 1, rows=rows)
    finally:
        oracle.set_threads(threads)
    return {
        "value": vox / dt / 1e9, "unit": "Gvoxel/s", "cores": threads, "kind": "oracle",
        "sample": f"{k} whole z-slices ({vox} voxels) of the same {nx}x{ny}x{nz} volume, "
                  f"brute-force oracle, r={radius}, {rule.upper()}, {threads} threads; took {dt:.1f} s",
        "single_core": {"value": rows * nx / ds / 1e9, "unit": "Gvoxel/s", "cores": 1,
                        "sample": f"{rows} rows of one z-slice ({rows * nx} voxels); took {ds:.1f} s"},
        "cpu_model": cpu_model(),
        "sample_matches_gpu": bool(ok and ok1 and okr and oks),
    }


def valu_info(gvox, lane_ops):
    """The kernel against its VALU bound: lane operations per voxel (profiled)
    and the voxel rate at 100 % VALU issue."""
    if not lane_ops:
        return None
    bound = VALU_PEAK_LANE_OPS / lane_ops / 1e9
    return {"lane_ops_per_voxel": lane_ops, "bound_Gvox_s": bound, "frac": gvox / bound}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--radius", type=int, default=3)
    ap.add_argument("--rule", choices=["mean9", "minvar9"], default="mean9")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the served-mode trace (0 skips it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(volumes shard by z-slab with one halo exchange; not built here)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1807_03119_amd import _lib, phantom
    from paper_1807_03119_amd.api import Filter

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    log(f"generating {DIMS} uint16 phantom on the device (seed {SEED})")
    vol = phantom.ct_u12(DIMS, seed=SEED, device="cuda")
    out = torch.empty_like(vol)
    nvox = vol.numel()
    rule_code = _lib.LNF_MEAN9 if args.rule == "mean9" else _lib.LNF_MINVAR9
    f = Filter(rule_code, 0)

    def step():
        f(vol, args.radius, out=out)

    log(f"timing {args.steps} steps ({args.warmup} warm-up, at least {WARM_SECONDS} s), "
        f"{args.rule} r={args.radius}")
    warm_n = warm_up(step, args.warmup, WARM_SECONDS)
    ms, wall = time_launches(step, args.steps, 0, stream)
    gvox = nvox / (ms * 1e-3) / 1e9
    alg_bytes = 4 * nvox  # read + write of one uint16 per voxel
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    traffic, lane_ops = profiled(args.rule) if args.radius == 3 else (None, None)
    res = {
        "metric": "filtered Gvoxel/s + % of HBM roofline; p50/p99 latency in served mode",
        "value": gvox, "unit": "Gvoxel/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "warmup_launches": warm_n, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"single {DIMS[0]}x{DIMS[1]}x{DIMS[2]} uint16 (12-bit) CT "
                               f"phantom, radius {args.radius}, {args.rule.upper()}",
                   "dims": list(DIMS), "voxel": "uint16", "radius": args.radius,
                   "rule": args.rule.upper(), "seed": SEED},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "valu": valu_info(gvox, lane_ops),
        "timed_wall_s": wall,
    }
    torch.cuda.synchronize()
    # reference copy of known size: read alg_bytes/2, write alg_bytes/2 (also the
    # yardstick the HBM byte counters are scaled by)
    res["copy_GBps"] = copy_bandwidth(alg_bytes // 2, stream)
    if not args.no_extras:
        extras = {}
        for rule_name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9)):
            g = Filter(rc, 0)
            for r in (1, 2, 3, 4):
                if rule_name == args.rule and r == args.radius:
                    continue
                ms2, _ = time_launches(lambda: g(vol, r, out=out), 10, 2, stream)
                extras[f"{rule_name}_r{r}_Gvox_s"] = nvox / (ms2 * 1e-3) / 1e9
                if r == 3:
                    gv = nvox / (ms2 * 1e-3) / 1e9
                    t3, ops3 = profiled(rule_name)
                    extras[f"{rule_name}_r3"] = {"Gvox_s": gv, "hbm_frac": gv * 4 / HBM_PEAK_GBS,
                                                 "valu": valu_info(gv, ops3)}
            g.close()
        log("timing the cluster geometry variants")
        geoms = {"box_d1": _lib.LNF_GEOM_OFFSET_1, "box_d2r1": _lib.LNF_GEOM_OFFSET_2R1,
                 "cross_dr": _lib.LNF_GEOM_CROSS,
                 "cross_d1": _lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_1,
                 "cross_d2r1": _lib.LNF_GEOM_CROSS | _lib.LNF_GEOM_OFFSET_2R1}
        for gname, gflags in geoms.items():
            for rule_name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9)):
                g = Filter(rc, 0, geometry=gflags)
                for r in (1, 3):
                    ms2, _ = time_launches(lambda: g(vol, r, out=out), 5, 1, stream)
                    extras[f"geom_{gname}_{rule_name}_r{r}_Gvox_s"] = nvox / (ms2 * 1e-3) / 1e9
                g.close()
        log("timing the paper's comparison filters at M = 3 (r = 1)")
        g = Filter(_lib.LNF_MEAN9, 0)
        _, hw = g.sigma(vol, 1, -1, out=out)  # floor(2 sigma) of the phantom, once
        cmp = {"ours_mean9": lambda: g(vol, 1, out=out),
               "mean": lambda: g.mean(vol, 1, out=out),
               "sigma": lambda: g.sigma(vol, 1, hw, out=out),
               "okada": lambda: g.okada(vol, 64, out=out),
               "entropy_incl_histogram": lambda: g.entropy(vol, 1, 2.0, out=out)}
        for name, fn in cmp.items():
            ms2, _ = time_launches(fn, 5, 1, stream)
            extras[f"compare_r1_{name}_ms"] = ms2
        extras["compare_r1_sigma_half_width"] = hw
        g.close()
        log("timing the at-scale volume 1024 x 1024 x 1536 (r=3, both rules)")
        big_dims = (1024, 1024, 1536)
        big = phantom.ct_u12(big_dims, seed=3000, device="cuda")
        big_out = torch.empty_like(big)
        extras["scale_1024x1024x1536"] = {}
        for rule_name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9)):
            g = Filter(rc, 0)
            ms2, _ = time_launches(lambda: g(big, 3, out=big_out), 5, 1, stream)
            gv = big.numel() / (ms2 * 1e-3) / 1e9
            extras["scale_1024x1024x1536"][rule_name] = {
                "ms": ms2, "Gvox_s": gv, "hbm_frac": gv * 4 / HBM_PEAK_GBS}
            g.close()
        del big, big_out
        torch.cuda.empty_cache()
        log("timing the Otsu pipeline and the surface-point mode")
        g = Filter(_lib.LNF_MEAN9, 0)
        ms2, _ = time_launches(lambda: g.histogram(vol), 10, 2, stream)
        extras["otsu"] = {"histogram_ms": ms2, "histogram_GBps": nvox * 2 / (ms2 * 1e-3) / 1e9}
        _, t_otsu = g.filter_otsu(vol, args.radius, out=out)
        ms2, _ = time_launches(lambda: g.filter_otsu(vol, args.radius, out=out), 5, 1, stream)
        extras["otsu"].update({"threshold": int(t_otsu), "pipeline_ms": ms2,
                               "pipeline_Gvox_s": nvox / (ms2 * 1e-3) / 1e9,
                               "pipeline": "histogram, exact Otsu on the host, gated MEAN9 "
                                           f"r={args.radius}"})
        g.close()
        gen = torch.Generator(device="cuda").manual_seed(SEED + 1)
        npts = 1 << 20  # one value per pixel of a 1024 x 1024 view
        xyz = torch.randint(0, DIMS[0], (npts, 3), generator=gen, device="cuda", dtype=torch.int32)
        extras["points"] = {"points": npts, "sample": "uniform random voxels of the volume"}
        for rule_name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9)):
            g = Filter(rc, 0)
            ms2, _ = time_launches(lambda: g.points(vol, args.radius, xyz), 5, 1, stream)
            extras["points"][f"{rule_name}_r{args.radius}_ms"] = ms2
            extras["points"][f"{rule_name}_r{args.radius}_Mpoints_s"] = npts / (ms2 * 1e-3) / 1e6
            g.close()
        extras["surface"] = surface_benchmark(vol, args.radius, t_otsu, stream)
        log("timing the 64-volume mixed batch, both rules")
        extras["batch64"] = {name: batch_benchmark(rc, stream)
                             for name, rc in (("mean9", _lib.LNF_MEAN9), ("minvar9", _lib.LNF_MINVAR9))}
        res["extras"] = extras
        if args.serve_seconds > 0:
            log(f"serving trace: {args.serve_seconds:.0f} s at 300 req/s, batched then FIFO")
            res["served"] = serve_benchmark(rule_code, args.serve_seconds)
            log("serving burst of small re-filter requests")
            res["served"]["burst"] = burst_benchmark(rule_code)
            log("serving rate sweep on resident volumes")
            res["served"]["sweep"] = {k: serve_sweep(rule_code, k) for k in SWEEPS}
    if not args.no_cpu_baseline:
        f(vol, args.radius, out=out)
        torch.cuda.synchronize()
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(vol.cpu().numpy(), args.radius, args.rule,
                                           out.cpu().numpy())
    f.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
