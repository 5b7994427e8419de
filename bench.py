"""Throughput benchmark: points mapped per second on one MI355X.

Workload: 220,900 jittered grid blocks (470 x 470, ~24 vertices each) under a
4-level hierarchy (50 regions / 3,000 counties / 70,000 tracts), 100M int32
points from a 200-component Gaussian mixture plus 5% uniform outliers. One
step maps all 100M points (inputs resident in HBM). Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

# MI355X published figures: 256 CUs at 2.4 GHz, 64 lanes per CU-cycle of
# integer vector ALU; HBM3E 8 TB/s.
PEAK_INT_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.32 T lane-ops/s
PEAK_HBM_GBS = 8000.0

# Work per point of the method on this workload, from the oracle's instrumented
# counts over the workload's first 2M points: 140.38 box tests, 34.98 ring-edge
# tests and 0.239 exact cross products per point. Lane-operation cost model:
# 5 per box test (4 compares + and), 7 per edge test (2 compares, straddle,
# x-range, parity), 12 per cross product -> 949.7 integer lane-ops per point.
OPS_PER_POINT = 5 * 140.38 + 7 * 34.98 + 12 * 0.239
# Algorithmic HBM bytes per point: 8 in + 4 out. The 158 MB index is left
# out: it fits the 256 MB last-level cache, and read once per 100M-point step
# it would add 1.6 B/pt.
BYTES_PER_POINT = 12.0


def read_traffic(kernel, pts_per_launch):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_grid221k_100m.json" % kernel)
    src = os.path.join(ROOT, "paper_2005_03156_amd", "csrc", "map_kernels.hip")
    try:
        d = json.load(open(path))
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if d.get("kernel_source_sha256") != h:
            return None
        return d["hbm_bytes_per_point"] * pts_per_launch
    except (OSError, ValueError, KeyError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--sweep", action="store_true", help="also time every launch shape (stderr)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a known-size kernel for counter calibration)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form leg")
    ap.add_argument("--no-cover", action="store_true", help="skip the cell-cover (fast approach) leg")
    ap.add_argument("--no-served", action="store_true", help="skip the served-form leg")
    ap.add_argument("--no-all-levels", action="store_true",
                    help="skip the leg that keeps every hierarchy level (its launches would mix into a profile)")
    ap.add_argument("--served-requests", type=int, default=20_000)
    ap.add_argument("--quadtree8m", action="store_true",
                    help="also measure the 8M-block graded mesh streamed over 1B points (stderr)")
    ap.add_argument("--quadtree8m-kernel", action="store_true",
                    help="only map one resident 2^26-point chunk over the 8M-block mesh a few times and "
                         "print its timing (a short run for the profiler)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the mapping path has no multi-GPU form here (points are "
              "independent, so several GPUs would each map their own range against a copy of the "
              "index); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2005_03156_amd as bm

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.quadtree8m_kernel:
        profile_quadtree8m(bm, torch, args)
        return
    t0 = time.time()
    g = synth.geometry("grid221k")
    n = synth.n_points("grid221k")
    pts = synth.points("grid221k", n)
    log("generated %d blocks, %d points in %.1fs" % (g.n_blocks, n, time.time() - t0))
    ix = bm.Index.from_geometry(g)
    xy = torch.from_numpy(pts).to(dev)
    out = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.sweep:
        for ch in (4, 8, 16):
            for bpc in (2, 3, 4, 5, 6, 8):
                t = bm.Tuning(ch, bpc, 2048, 1)
                bm.map_points(ix, xy, out, stream, tuning=t)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(3):
                    bm.map_points(ix, xy, out, stream, tuning=t)
                e1.record(stream)
                torch.cuda.synchronize()
                log("sweep chunk=%d blocks/cu=%d: %.3f ms" % (ch, bpc, e0.elapsed_time(e1) / 3))
    for _ in range(args.warmup):
        bm.map_points(ix, xy, out, stream)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[2 * k].record(stream)
        bm.map_points(ix, xy, out, stream)
        ev[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kern_ms = [ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(args.steps)]
    avg_ms = float(np.mean(kern_ms))
    value = n * args.steps / wall
    log("plain: %.3f ms/launch (events), wall %.3f ms/step, %.3g points/s" %
        (avg_ms, wall * 1e3 / args.steps, value))

    # the dominant kernel (the mapping kernel) timed live with HIP events on
    # the stream it runs on, over a few more steps of the same workload
    tm = {"map_ms": 0.0, "sort_ms": 0.0, "map_launches": 0, "sort_launches": 0}
    reps = 3
    for _ in range(reps):
        r = bm.map_points_timed(ix, xy, out, stream)
        for k in tm:
            tm[k] += r[k]
    map_ms_per_step = tm["map_ms"] / reps
    launches = max(1, tm["map_launches"] // reps)
    kernel_ms = map_ms_per_step / launches
    pts_per_launch = n / launches
    achieved = OPS_PER_POINT * pts_per_launch / (kernel_ms * 1e-3) / 1e12
    step_ms = wall * 1e3 / args.steps
    hbm_gbs = BYTES_PER_POINT * n / (step_ms * 1e-3) / 1e9
    traffic = read_traffic("map_sorted_kernel", pts_per_launch)
    log("dominant kernel: %d launches/step, %.3f ms each (%.0f points), sort phases %.3f ms/step; "
        "%.2f T algorithmic ops/s" % (launches, kernel_ms, pts_per_launch, tm["sort_ms"] / reps, achieved))
    res = {
        "metric": "points mapped/sec on 1 GPU, served/batched vs plain kernel; p50/p99 latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "census-scale plain mapping: 220,900 blocks (470x470 jittered grid, "
                               "~24 vertices/block), hierarchy 50 regions / 3,000 counties / 70,000 "
                               "tracts / 220,900 blocks (the index merges the ~3-block tracts into "
                               "their counties; all_levels_kept times all four), "
                               "100M int32 points (200-Gaussian mixture + 5% uniform)",
                   "points_per_step": n, "blocks": g.n_blocks},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                     "frac": achieved / PEAK_INT_TOPS, "traffic": traffic,
                     "kernel": "map_sorted_kernel" if tm["sort_launches"] else "map_kernel",
                     "kernel_ms": kernel_ms, "launches_per_step": launches, "points_per_launch": pts_per_launch,
                     "ops_per_point": OPS_PER_POINT,
                     "sort_ms_per_step": tm["sort_ms"] / reps,
                     "step_frac": OPS_PER_POINT * n / (step_ms * 1e-3) / 1e12 / PEAK_INT_TOPS},
        "hbm": {"achieved_GBs": hbm_gbs, "peak_GBs": PEAK_HBM_GBS, "frac": hbm_gbs / PEAK_HBM_GBS,
                "bytes_per_point": BYTES_PER_POINT},
    }
    if not args.no_all_levels:
        res["all_levels_kept"] = bench_all_levels(bm, torch, g, xy, out, args.steps)
    if not args.no_cover:
        res["cover"] = bench_cover(bm, torch, g, ix, xy, out, args.steps)
    res["count_per_block"] = bench_count(bm, torch, out, g.n_blocks, args.steps)
    del xy, out
    torch.cuda.empty_cache()
    res["quantize"] = bench_quantize(bm, torch, n, args.steps)
    if not args.no_batched:
        res["batched"] = bench_batched(bm, torch, g, ix)
    if args.quadtree8m or not args.no_served:
        g3 = synth.geometry("quadtree8m")
        ix3 = bm.Index.from_geometry(g3)
        if args.quadtree8m:
            res["quadtree8m"] = bench_quadtree8m(bm, torch, g3, ix3)
        if not args.no_served:
            res["served"] = bench_served(bm, torch, g3, ix3, args.served_requests)
        ix3.close()
        del g3
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline(g, pts)
    print(json.dumps(res), flush=True)


def bench_all_levels(bm, torch, g, xy, ref, steps):
    """The same plain mapping with every level of the hierarchy kept
    (regions, counties, tracts, blocks): the thin tract level, which the
    default index leaves out, costs each point one more round of group
    items. `ref` holds the default index's output for the same points."""
    ix4 = bm.Index.from_geometry(g, keep_all_levels=True)
    out = torch.empty_like(ref)
    s = torch.cuda.current_stream()
    bm.map_points(ix4, xy, out, s)
    torch.cuda.synchronize()
    same = bool(torch.equal(out, ref))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = time.perf_counter()
    e0.record(s)
    for _ in range(steps):
        bm.map_points(ix4, xy, out, s)
    e1.record(s)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t) / steps
    n = xy.shape[0]
    r = {"group_levels": ix4.info()["n_levels"], "points_per_s": n / wall, "ms_per_step": wall * 1e3,
         "events_ms": e0.elapsed_time(e1) / steps, "same_ids_as_default_index": same}
    log("every level kept (%d group levels): %.3f ms/step, %.3g points/s, same ids: %s" %
        (r["group_levels"], wall * 1e3, n / wall, same))
    ix4.close()
    del out
    return r


def bench_cover(bm, torch, g, ix, xy, ref, steps):
    """The cell cover (the paper's fast approach) over the same 100M resident
    points: build time and size, exact and approximate throughput. `ref` holds
    the plain path's output for the same points."""
    t0 = time.time()
    cv = bm.Cover.from_geometry(ix, g)
    info = cv.info()
    log("cover: built in %.1fs (wall %.1fs): %s" % (info["build_seconds"], time.time() - t0, info))
    n = xy.shape[0]
    out = torch.empty_like(ref)
    s = torch.cuda.current_stream()
    r = {"build_seconds": info["build_seconds"], "device_bytes": info["device_bytes"],
         "cell_log2": info["cell_log2"], "trie_levels": info["trie_levels"],
         "boundary_cells": info["boundary_cells"], "trie_entries": info["trie_entries"]}
    for mode in ("exact", "approx"):
        approx = mode == "approx"
        bm.map_points_cover(cv, xy, out, approx=approx, stream=s)
        torch.cuda.synchronize()
        same = float((out == ref).float().mean().item())
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t = time.perf_counter()
        e0.record(s)
        for _ in range(steps):
            bm.map_points_cover(cv, xy, out, approx=approx, stream=s)
        e1.record(s)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t) / steps
        r[mode] = {"points_per_s": n / wall, "ms_per_step": wall * 1e3,
                   "kernel_ms": e0.elapsed_time(e1) / steps, "agree_with_plain": same}
        log("cover %s: %.3f ms/step, %.3g points/s, agrees with the plain path on %.6f of the points" %
            (mode, wall * 1e3, n / wall, same))
    cv.close()
    return r


def bench_count(bm, torch, ids, n_blocks, steps):
    """Points per block over the plain path's 100M ids (the aggregation the
    mapping feeds), checked against torch's bincount."""
    counts = torch.zeros(n_blocks + 1, dtype=torch.int64, device=ids.device)
    bm.count_per_block(ids, n_blocks, counts)
    torch.cuda.synchronize()
    ref = torch.bincount(torch.where(ids >= 0, ids, torch.full_like(ids, n_blocks)).long(),
                         minlength=n_blocks + 1)
    ok = bool(torch.equal(counts, ref))
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        bm.count_per_block(ids, n_blocks, counts, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    log("count per block: %.3f ms per 100M ids (%.3g ids/s), equal to bincount: %s" % (ms, ids.shape[0] / ms * 1e3, ok))
    return {"ms": ms, "ids_per_s": ids.shape[0] / ms * 1e3, "equal_to_bincount": ok}


def bench_quantize(bm, torch, n, steps):
    """The quantiser on n resident (lon, lat) doubles, uniform over the globe:
    16 bytes read and 8 written per point, against the HBM peak; checked
    against torch's round-half-even of v * 2^22, plus 2^30."""
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    ll = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    ll[:, 0].uniform_(-180.0, 180.0, generator=gen)
    ll[:, 1].uniform_(-90.0, 90.0, generator=gen)
    q = torch.empty((n, 2), dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    bm.quantize_lonlat(ll, q, s)
    want = (torch.round(ll * 4194304.0).to(torch.int64) + (1 << 30)).to(torch.int32)
    ok = bool(torch.equal(q, want))
    del want
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        bm.quantize_lonlat(ll, q, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    gbs = 24.0 * n / (ms * 1e-3) / 1e9
    log("quantize: %.3f ms per %d points (%.3g points/s, %.0f GB/s = %.1f%% of HBM peak), exact: %s" %
        (ms, n, n / ms * 1e3, gbs, 100 * gbs / PEAK_HBM_GBS, ok))
    del ll, q
    torch.cuda.empty_cache()
    return {"points": n, "ms": ms, "points_per_s": n / ms * 1e3, "achieved_GBs": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS, "bytes_per_point": 24, "exact": ok}


def bench_batched(bm, torch, g, ix, nb=10_000):
    """Batched form: 10,000 batches over this index, sizes log-uniform on
    [1, 1e6], each batch one Gaussian cluster (centre uniform, sigma
    log-uniform on [0.1%, 5%] of the extent). One graph replay (and one eager
    persistent launch) against one plain launch per batch."""
    t0 = time.time()
    sizes = synth.sizes(synth.key("batches10k", 2, 0), nb, 0, 0.0, 0.0, 1e6)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    total = int(off[-1])
    host = np.empty((total, 2), np.int32)
    for b in range(nb):
        m = synth.Mixture(synth.key("batches10k", 2, b + 1), 1, g.W, 0.0, 0.001, 0.05, 0.0)
        m.sample(synth.key("batches10k", 3, b + 1), 0, int(sizes[b]), out=host[off[b]:off[b + 1]])
    xy = torch.from_numpy(host).cuda()
    del host
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    ref = torch.empty(total, dtype=torch.int32, device="cuda")
    log("batched: %d batches, %d points (sizes %d..%d), generated in %.1fs" %
        (nb, total, sizes.min(), sizes.max(), time.time() - t0))
    base_x, base_o, base_r = xy.data_ptr(), out.data_ptr(), ref.data_ptr()
    rows = [(base_x + 8 * int(off[b]), base_o + 4 * int(off[b]), int(sizes[b])) for b in range(nb)]
    s = torch.cuda.current_stream()
    tune = bm.autotune(ix, xy[: min(total, 1 << 22)], s)
    log("batched: autotuned %s" % tune.as_dict())
    # per-batch plain launches (the library's plain entry point, one call per batch)
    lib, sh = bm.lib, bm._stream_handle(s)
    import ctypes as C

    def plain_all():
        for b in range(nb):
            lib.map_points(ix.handle, C.c_void_p(base_x + 8 * int(off[b])), int(sizes[b]),
                           C.c_void_p(base_r + 4 * int(off[b])), sh)
    plain_all()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_all()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    # eager persistent launch over a device table
    table = torch.tensor(rows, dtype=torch.int64).cuda()
    bm.map_batches(ix, table, s, tune)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t = time.perf_counter()
    e0.record(s)
    bm.map_batches(ix, table, s, tune)
    e1.record(s)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t
    eager_ms = e0.elapsed_time(e1)
    ok_eager = bool(torch.equal(out, ref))
    # captured graph, replayed
    out.fill_(-7)
    plan = bm.BatchPlan(ix, nb, tune)
    crow = bm.make_rows(rows)
    plan.run_rows(crow, nb, s)
    torch.cuda.synchronize()
    ok_graph = bool(torch.equal(out, ref))
    reps = 3
    t = time.perf_counter()
    e0.record(s)
    for _ in range(reps):
        plan.run_rows(crow, nb, s)
    e1.record(s)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t) / reps
    graph_ms = e0.elapsed_time(e1) / reps
    plan.close()
    res = {"batches": nb, "points": total, "tuning": tune.as_dict(),
           "graph_points_per_s": total / t_graph, "graph_ms": graph_ms,
           "eager_points_per_s": total / t_eager, "eager_kernel_ms": eager_ms,
           "plain_per_batch_points_per_s": total / t_plain, "plain_per_batch_ms": t_plain * 1e3,
           "identical_to_plain": ok_eager and ok_graph,
           "hbm_frac": BYTES_PER_POINT * total / (graph_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    log("batched: graph %.1f ms (%.3g pts/s), eager %.1f ms, per-batch plain %.1f ms (%.3g pts/s), identical=%s" %
        (graph_ms, res["graph_points_per_s"], eager_ms, t_plain * 1e3, res["plain_per_batch_points_per_s"],
         res["identical_to_plain"]))
    del xy, out, ref, table
    torch.cuda.empty_cache()
    return res


def bench_served(bm, torch, g, ix, nreq):
    """Served form over the 8M-block graded mesh resident in HBM: requests of
    lognormal size (median 10k points, sigma 2, at most 10M), each a Gaussian
    cluster plus 20% uniform points, in page-locked host memory. Baseline: the
    same request loop with coalescing and overlap switched off (one request
    per batch, one slot, one stream), i.e. the plain kernel request by
    request. Both see the same Poisson arrivals at 50% and 90% of the
    baseline's capacity, and all at once."""
    t0 = time.time()
    npool = 1000
    sizes = synth.sizes(synth.key("requests20k", 2, 0), npool, 1, 10_000.0, 2.0, 10_000_000)
    pool, outs, ref = [], [], []
    for r in range(npool):
        m = synth.Mixture(synth.key("requests20k", 2, r + 1), 1, g.W, 0.0, 0.001, 0.02, 0.2)
        x = torch.empty((int(sizes[r]), 2), dtype=torch.int32, pin_memory=True).numpy()
        m.sample(synth.key("requests20k", 3, r + 1), 0, int(sizes[r]), out=x)
        pool.append(x)
        outs.append(torch.empty(int(sizes[r]), dtype=torch.int32, pin_memory=True).numpy())
        ref.append(bm.map_points(ix, torch.from_numpy(x).cuda()).cpu().numpy())
    rng = np.random.default_rng(5)
    order = rng.integers(0, npool, nreq)
    mean_pts = float(sizes[order].mean())
    reqs = [(pool[i], outs[i]) for i in order]
    log("served: %d distinct requests (mean %.0f points, max %d), %d submissions, prepared in %.1fs" %
        (npool, sizes.mean(), sizes.max(), nreq, time.time() - t0))

    def run(cfg, arrivals, nr):
        for o in outs:
            o.fill(-7)
        srv = bm.Server(ix, cfg)
        t = time.perf_counter()
        srv.run_trace(reqs[:nr], arrivals[:nr])
        wall = time.perf_counter() - t
        st = srv.stats()
        srv.close()
        same = all(np.array_equal(outs[i], ref[i]) for i in set(order[:nr].tolist()))
        return {"points_per_s": st["points_per_s"], "requests_per_s": st["completed"] / wall,
                "p50_us": st["p50_us"], "p99_us": st["p99_us"], "mean_us": st["mean_us"],
                "mean_requests_per_batch": st["mean_requests_per_batch"], "batches": st["batches"],
                "identical_to_alone": bool(same),
                "hbm_frac": BYTES_PER_POINT * st["points_per_s"] / 1e9 / PEAK_HBM_GBS}

    base_cfg = bm.server_cfg(mem_budget_bytes=2 << 30, max_batch_points=1 << 24, max_slots=1, n_streams=1,
                             flags=bm.BM_SERVER_ONE_PER_BATCH)
    srv_cfg = bm.server_cfg(mem_budget_bytes=2 << 30, max_batch_points=1 << 23, max_slots=6, n_streams=4)
    nsat = min(nreq, 5000)
    zero = np.zeros(nreq)
    res = {"requests": nreq, "mean_points_per_request": mean_pts}
    res["baseline_saturated"] = run(base_cfg, zero, nsat)
    cap = res["baseline_saturated"]["requests_per_s"]
    res["server_saturated"] = run(srv_cfg, zero, nreq)
    for name, frac in (("50pct", 0.5), ("90pct", 0.9)):
        arr = np.cumsum(rng.exponential(1e6 / (frac * cap), nreq))
        res["baseline_" + name] = run(base_cfg, arr, nreq)
        res["server_" + name] = run(srv_cfg, arr, nreq)
        res["baseline_" + name]["offered_qps"] = res["server_" + name]["offered_qps"] = frac * cap
    for k, v in res.items():
        if isinstance(v, dict):
            log("served %-19s %.3g pts/s, %.0f req/s, p50 %.0f us, p99 %.0f us, %.1f req/batch, identical=%s" %
                (k, v["points_per_s"], v["requests_per_s"], v["p50_us"], v["p99_us"], v["mean_requests_per_batch"],
                 v["identical_to_alone"]))
    return res


def profile_quadtree8m(bm, torch, args):
    """One resident 2^26-point chunk of the 1B-point stream over the 8M-block
    mesh, mapped once to warm up and then `steps` times, each call timed per
    launch with HIP events on its stream. Prints one JSON line."""
    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    t0 = time.time()
    g = synth.geometry("quadtree8m")
    ix = bm.Index.from_geometry(g)
    CH = synth.QUADTREE["chunk"]
    xy = torch.from_numpy(synth.points("quadtree8m", CH, 0)).cuda()
    out = torch.empty(CH, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    log("quadtree8m: %d blocks, index %.2f GB, chunk of %d points ready in %.1fs" % (
        g.n_blocks, ix.info()["device_bytes"] / 1e9, CH, time.time() - t0))
    bm.map_points(ix, xy, out, s)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 5))
    tm = {"map_ms": 0.0, "sort_ms": 0.0, "map_launches": 0, "sort_launches": 0}
    for _ in range(steps):
        r = bm.map_points_timed(ix, xy, out, s)
        for k in tm:
            tm[k] += r[k]
    launches = max(1, tm["map_launches"] // steps)
    kernel_ms = tm["map_ms"] / steps / launches
    res = {"workload": "8M-block graded quadtree mesh, one resident 2^26-point chunk", "points": CH,
           "calls": steps, "map_launches_per_call": launches, "map_kernel_ms": kernel_ms,
           "sort_ms_per_call": tm["sort_ms"] / steps,
           "points_per_s_per_call": CH / ((tm["map_ms"] + tm["sort_ms"]) / steps * 1e-3)}
    log("quadtree8m chunk: %d mapping launch(es) of %.3f ms, sort %.3f ms per call" % (
        launches, kernel_ms, res["sort_ms_per_call"]))
    ix.close()
    print(json.dumps(res), flush=True)


def bench_quadtree8m(bm, torch, g, ix):
    """8M blocks, 1B points streamed in 2^26-point chunks from pinned host
    memory: kernel-only rate (chunk resident) and end-to-end rate with the
    copies in and out overlapped with the mapping."""
    t0 = time.time()
    info = ix.info()
    q = synth.QUADTREE
    N, CH = q["n_points"], q["chunk"]
    nch = (N + CH - 1) // CH
    dxy = [torch.empty((CH, 2), dtype=torch.int32, device="cuda") for _ in range(2)]
    dout = [torch.empty(CH, dtype=torch.int32, device="cuda") for _ in range(2)]
    # all chunks generated into pinned host memory first (not timed)
    hin = torch.empty((N, 2), dtype=torch.int32, pin_memory=True)
    hres = torch.empty(N, dtype=torch.int32, pin_memory=True)
    for k in range(nch):
        n = min(CH, N - k * CH)
        synth.points("quadtree8m", n, k * CH, out=hin[k * CH:k * CH + n].numpy())
    log("quadtree8m: %d blocks, %.2f GB index; %d points generated into pinned host memory in %.1fs" % (
        g.n_blocks, info["device_bytes"] / 1e9, N, time.time() - t0))
    # kernel only: chunk 0 resident
    dxy[0].copy_(hin[:CH])
    s = torch.cuda.current_stream()
    bm.map_points(ix, dxy[0], dout[0], s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(5):
        bm.map_points(ix, dxy[0], dout[0], s)
    e1.record(s)
    torch.cuda.synchronize()
    kern_ms = e0.elapsed_time(e1) / 5
    first = dout[0].clone()
    # end to end: copy-in, mapping and copy-out on three streams with two
    # device buffers, so chunk k+1 comes in and chunk k-1 goes out while chunk
    # k is mapped
    cin, cout = torch.cuda.Stream(), torch.cuda.Stream()
    comp = torch.cuda.current_stream()
    ev_in = [torch.cuda.Event() for _ in range(2)]
    ev_map = [torch.cuda.Event() for _ in range(2)]
    ev_out = [torch.cuda.Event() for _ in range(2)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(nch):
        n, b, lo = min(CH, N - k * CH), k & 1, k * CH
        with torch.cuda.stream(cin):
            if k >= 2:
                cin.wait_event(ev_map[b])  # buffer b was mapped (chunk k-2)
            dxy[b][:n].copy_(hin[lo:lo + n], non_blocking=True)
            ev_in[b].record(cin)
        comp.wait_event(ev_in[b])
        if k >= 2:
            comp.wait_event(ev_out[b])  # chunk k-2's results were copied out
        bm.map_points(ix, dxy[b][:n], dout[b][:n], comp)
        ev_map[b].record(comp)
        with torch.cuda.stream(cout):
            cout.wait_event(ev_map[b])
            hres[lo:lo + n].copy_(dout[b][:n], non_blocking=True)
            ev_out[b].record(cout)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t
    same = bool(torch.equal(hres[:CH], first.cpu()))
    res = {"blocks": g.n_blocks, "vertices": int(g.verts.shape[0]), "points": N,
           "kernel_points_per_s": CH / (kern_ms * 1e-3), "kernel_ms_per_chunk": kern_ms,
           "end_to_end_points_per_s": N / t_wall, "end_to_end_first_chunk_identical": same,
           "index_device_bytes": info["device_bytes"],
           "kernel_hbm_frac": BYTES_PER_POINT * CH / (kern_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    log("quadtree8m: kernel %.3f ms per 2^26 chunk (%.3g pts/s); end-to-end with PCIe %.3g pts/s "
        "(first chunk identical to the resident run: %s)" %
        (kern_ms, res["kernel_points_per_s"], res["end_to_end_points_per_s"], same))
    return res


def cpu_baseline(g, pts):
    """The CPU oracle (hierarchy route, C + OpenMP) on the host cores: whole
    passes over the workload's 100M points until at least 10 s have passed;
    plus one thread on the first 2M points."""
    import oracle
    H = oracle.Hier.from_geometry(g)
    H.map(pts[:100_000])  # warm
    t = time.perf_counter()
    passes = 0
    while True:
        H.map(pts)
        passes += 1
        dt = time.perf_counter() - t
        if dt >= 10.0 or passes >= 20:
            break
    cores = oracle.threads()
    oracle.set_threads(1)
    t1 = time.perf_counter()
    H.map(pts[:2_000_000])
    single = 2_000_000 / (time.perf_counter() - t1)
    oracle.set_threads(cores)
    return {"value": passes * pts.shape[0] / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "%d full passes over the workload's %d points (%.1f s), hierarchy route, C + OpenMP"
                      % (passes, pts.shape[0], dt),
            "single_thread_points_per_s": single, "host": host_cpus()}


def host_cpus():
    """The host's CPUs as the OS reports them: logical CPUs, those this
    process may run on, and physical cores (distinct (package, core) pairs)."""
    r = {"logical": os.cpu_count()}
    try:
        r["usable"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        pairs, phys, core = set(), None, None
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "physical id":
                    phys = v.strip()
                elif k == "core id":
                    core = v.strip()
                elif not k and phys is not None and core is not None:
                    pairs.add((phys, core))
                    phys = core = None
        if phys is not None and core is not None:
            pairs.add((phys, core))
        if pairs:
            r["physical_cores"] = len(pairs)
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    r["model"] = line.partition(":")[2].strip()
                    break
    except OSError:
        pass
    return r


if __name__ == "__main__":
    main()
