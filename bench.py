"""Throughput benchmark: points mapped per second on one MI355X.

Headline workload: 220,900 jittered grid blocks (470 x 470, ~24 vertices each)
under a 4-level hierarchy (50 regions / 3,000 counties / 70,000 tracts), 100M
int32 points from a 200-component Gaussian mixture plus 5% uniform outliers.
One step maps all 100M points (inputs resident in HBM). Beside it, in the same
JSON line: the small 1,024-block grid, the 8M-block graded mesh over 1B points
(kernel and streamed end to end), the batched and served forms, the cell
cover, the aggregation and the quantiser, and the CPU oracle on the host.

  python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--only LEG[,LEG]]

--only runs just the named legs (for profiling) and prints their results:
plain, grid1k, all-levels, cover, aggregate, quantize, batched, served,
quadtree8m, quadtree8m-kernel.
"""
from __future__ import annotations

import argparse
import hashlib
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

# Lane-operation cost of one unit of the method's work (Sec. III's box tests,
# Sec. III-A's ring-edge tests and the exact cross products of x-ambiguous
# straddling edges): 4 compares + and per box test; 2 compares, straddle,
# x-range and parity per edge test; 12 for a 64-bit cross product and sign.
# The counts per point come from the oracle's instrumented hierarchy route on
# the workload's own points, taken in the CPU leg.
COST = {"bbox_tests": 5, "edge_tests": 7, "x_ambiguous": 12}
# Algorithmic HBM bytes per point: 8 in + 4 out for a call; the sorted mapping
# kernel reads the sorted point and writes its result in sorted order (8 + 4).
BYTES_PER_POINT = 12.0
SORTED_KERNEL_BYTES_PER_POINT = 12.0
KERNEL_SRC = os.path.join(ROOT, "paper_2005_03156_amd", "csrc", "map_kernels.hip")
LEGS = ["plain", "grid1k", "all-levels", "cover", "aggregate", "quantize", "batched", "served", "quadtree8m",
        "quadtree8m-kernel"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()


def read_traffic(name):
    """Counter-measured HBM bytes per point from a committed summary
    (profiles/traffic_<name>.json), if it was taken on the current kernel
    source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic_%s.json" % name)
    try:
        d = json.load(open(path))
        if d.get("kernel_source_sha256") != kernel_sha():
            return None
        return float(d["hbm_bytes_per_point"])
    except (OSError, ValueError, KeyError):
        return None


def ops_per_point(counts, n):
    return sum(COST[k] * counts[k] for k in COST) / n


def timed_calls(torch, fn, reps, stream):
    """Wall time and event time per call of fn() over reps calls."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / reps, e0.elapsed_time(e1) / reps


def launch_times(bm, ix, xy, out, stream, reps=3):
    """Mapping-kernel launches and sort phases of map_points, timed with HIP
    events on the stream they run on."""
    tm = {"map_ms": 0.0, "sort_ms": 0.0, "unsort_ms": 0.0, "map_launches": 0, "sort_launches": 0}
    for _ in range(reps):
        r = bm.map_points_timed(ix, xy, out, stream)
        for k in tm:
            tm[k] += r[k]
    launches = max(1, tm["map_launches"] // reps)
    return {"kernel_ms": tm["map_ms"] / reps / launches, "launches_per_call": launches,
            "sort_ms_per_call": tm["sort_ms"] / reps, "unsort_ms_per_call": tm["unsort_ms"] / reps,
            "kernel": "map_sorted_kernel" if tm["sort_launches"] else "map_kernel"}


def copy_calibration(torch):
    """One 1 GiB device-to-device copy: a kernel of known size for scaling the
    HBM counters."""
    a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--only", default="", help="comma-separated legs to run alone: " + ", ".join(LEGS))
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (a known-size kernel for counter calibration)")
    ap.add_argument("--served-requests", type=int, default=20_000)
    ap.add_argument("--served-runs", default="all", help="all, or saturated (the server alone, for profiling)")
    ap.add_argument("--quadtree8m-kernel", action="store_true", help="same as --only quadtree8m-kernel")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the mapping path has no multi-GPU form here (points are "
              "independent, so several GPUs would each map their own range against a copy of the "
              "index); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    only = [x for x in args.only.split(",") if x] + (["quadtree8m-kernel"] if args.quadtree8m_kernel else [])
    for x in only:
        if x not in LEGS:
            ap.error("unknown leg %r" % x)

    import torch
    import paper_2005_03156_amd as bm

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration(torch)
    if only:
        res = run_legs(bm, torch, args, only)
        print(json.dumps(res), flush=True)
        return

    res = headline(bm, torch, args)
    g, ix, pts = res.pop("_g"), res.pop("_ix"), res.pop("_pts")
    xy, out = res.pop("_xy"), res.pop("_out")
    res["grid1k"] = bench_grid1k(bm, torch, args.steps)
    all_levels = bench_all_levels(bm, torch, g, xy, out, args.steps)
    res["all_levels_kept"] = all_levels
    res["cover"] = bench_cover(bm, torch, g, ix, xy, out, args.steps)
    res["aggregate"] = bench_aggregate(bm, torch, g, out, args.steps)
    del xy, out
    torch.cuda.empty_cache()
    res["quantize"] = bench_quantize(bm, torch, synth.n_points("grid221k"), args.steps)
    res["batched"] = bench_batched(bm, torch, g, ix)
    g3 = synth.geometry("quadtree8m")
    ix3 = bm.Index.from_geometry(g3)
    res["quadtree8m"] = bench_quadtree8m(bm, torch, g3, ix3)
    res["served"] = bench_served(bm, torch, g3, ix3, args.served_requests, args.served_runs)
    ix3.close()
    del g3
    torch.cuda.empty_cache()
    if not args.no_cpu:
        cpu = cpu_baseline(g, pts)
        res["cpu_baseline"] = cpu
        fill_roofline(res, cpu)
    print(json.dumps(res), flush=True)


def run_legs(bm, torch, args, only):
    """Only the named legs, each on its own workload (for profiler runs)."""
    res = {"legs": only}
    need_grid = [x for x in only if x in ("plain", "all-levels", "cover", "aggregate", "batched")]
    g = ix = xy = out = None
    if need_grid:
        g = synth.geometry("grid221k")
        ix = bm.Index.from_geometry(g)
    if "plain" in only or "all-levels" in only or "cover" in only or "aggregate" in only:
        n = synth.n_points("grid221k")
        xy = torch.from_numpy(synth.points("grid221k", n)).cuda()
        out = torch.empty(n, dtype=torch.int32, device="cuda")
        bm.map_points(ix, xy, out)
    if "plain" in only:
        s = torch.cuda.current_stream()
        for _ in range(args.warmup):
            bm.map_points(ix, xy, out, s)
        wall, ev = timed_calls(torch, lambda: bm.map_points(ix, xy, out, s), args.steps, s)
        res["plain"] = {"points_per_s": xy.shape[0] / wall, "ms_per_step": wall * 1e3, "events_ms": ev,
                        **launch_times(bm, ix, xy, out, s)}
    if "grid1k" in only:
        res["grid1k"] = bench_grid1k(bm, torch, args.steps)
    if "all-levels" in only:
        res["all_levels_kept"] = bench_all_levels(bm, torch, g, xy, out, args.steps)
    if "cover" in only:
        res["cover"] = bench_cover(bm, torch, g, ix, xy, out, args.steps)
    if "aggregate" in only:
        res["aggregate"] = bench_aggregate(bm, torch, g, out, args.steps)
    if "quantize" in only:
        res["quantize"] = bench_quantize(bm, torch, synth.n_points("grid221k"), args.steps)
    if "batched" in only:
        res["batched"] = bench_batched(bm, torch, g, ix, reps=max(1, min(args.steps, 3)))
    if any(x.startswith("quadtree8m") or x == "served" for x in only):
        g3 = synth.geometry("quadtree8m")
        ix3 = bm.Index.from_geometry(g3)
        if "quadtree8m-kernel" in only:
            res["quadtree8m_kernel"] = profile_quadtree8m(bm, torch, g3, ix3, max(1, min(args.steps, 5)))
        if "quadtree8m" in only:
            res["quadtree8m"] = bench_quadtree8m(bm, torch, g3, ix3)
        if "served" in only:
            res["served"] = bench_served(bm, torch, g3, ix3, args.served_requests, args.served_runs)
        ix3.close()
    return res


def headline(bm, torch, args):
    """The census-scale workload: 100M resident points per step through
    map_points, wall-clock timed; the mapping kernel timed per launch."""
    t0 = time.time()
    g = synth.geometry("grid221k")
    n = synth.n_points("grid221k")
    pts = synth.points("grid221k", n)
    log("generated %d blocks, %d points in %.1fs" % (g.n_blocks, n, time.time() - t0))
    ix = bm.Index.from_geometry(g)
    # the index leaves out the tract level (3.2 blocks per tract on average):
    # it filters regions -> counties -> blocks
    assert ix.info()["n_levels"] == 2
    xy = torch.from_numpy(pts).cuda()
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        bm.map_points(ix, xy, out, stream)
    torch.cuda.synchronize()
    # exactly `steps` steps between two synchronisations
    t_start = time.perf_counter()
    for _ in range(args.steps):
        bm.map_points(ix, xy, out, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    value = n * args.steps / wall
    step_ms = wall * 1e3 / args.steps
    log("plain: wall %.3f ms/step, %.3g points/s" % (step_ms, value))
    lt = launch_times(bm, ix, xy, out, stream)
    pts_per_launch = n / lt["launches_per_call"]
    bpp = read_traffic("map_sorted_kernel_grid221k_100m")
    traffic = bpp * pts_per_launch if bpp is not None else None
    log("dominant kernel: %d launch(es)/step, %.3f ms each (%.0f points), sort passes %.3f ms/step, unsort "
        "passes %.3f ms/step" % (lt["launches_per_call"], lt["kernel_ms"], pts_per_launch, lt["sort_ms_per_call"],
                                  lt["unsort_ms_per_call"]))
    hbm_gbs = BYTES_PER_POINT * n / (step_ms * 1e-3) / 1e9
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
        "roofline": {"bound": "alu", "achieved": None, "peak": PEAK_INT_TOPS, "unit": "TOP/s", "frac": None,
                     "traffic": traffic,
                     "kernel": lt["kernel"], "kernel_ms": lt["kernel_ms"],
                     "launches_per_step": lt["launches_per_call"], "points_per_launch": pts_per_launch,
                     "sort_ms_per_step": lt["sort_ms_per_call"], "unsort_ms_per_step": lt["unsort_ms_per_call"],
                     "ops_basis": "method-equivalent integer lane-ops: the oracle's counts of the paper's "
                                  "work on this workload's points (box tests per level, ring-edge tests, "
                                  "exact cross products) over the workload's four-level hierarchy, priced "
                                  "5/7/12 lane-ops each; filtered_hierarchy gives the same over the three "
                                  "levels the index filters; the kernel issues far fewer operations (slot "
                                  "tables, y-slabs) and is bound by the latency of dependent gathers of "
                                  "index lines, whose counter-measured bytes are in traffic / hbm_measured"},
        "hbm": {"achieved_GBs": hbm_gbs, "peak_GBs": PEAK_HBM_GBS, "frac": hbm_gbs / PEAK_HBM_GBS,
                "bytes_per_point": BYTES_PER_POINT},
        "_g": g, "_ix": ix, "_pts": pts, "_xy": xy, "_out": out,
    }
    if traffic is not None:
        gbs = traffic / (lt["kernel_ms"] * 1e-3) / 1e9
        res["hbm_measured"] = {"kernel_bytes_per_point": bpp, "kernel_GBs": gbs, "kernel_frac": gbs / PEAK_HBM_GBS}
    return res


def fill_roofline(res, cpu):
    """The ALU roofline of the dominant kernel from the oracle's counts: the
    paper's method over the workload's full four-level hierarchy (regions,
    counties, tracts, blocks), about 950 lane-ops per point at 5 per box
    test, 7 per ring-edge test and 12 per exact cross product; beside it the
    same over the three levels the default index
    filters (its counties hold the tracts' blocks, so the method scans more
    boxes per point there)."""
    rf = res["roofline"]
    w = cpu["work_per_point"]
    ops = w["every_level"]["ops_per_point"]
    ops3 = w["default_index"]["ops_per_point"]
    per_s = rf["points_per_launch"] / (rf["kernel_ms"] * 1e-3)
    achieved = ops * per_s / 1e12
    rf.update({"achieved": achieved, "frac": achieved / PEAK_INT_TOPS, "ops_per_point": ops,
               "step_frac": ops * res["config"]["points_per_step"] / (res["ms_per_step"] * 1e-3) / 1e12
               / PEAK_INT_TOPS,
               "filtered_hierarchy": {"ops_per_point": ops3, "achieved": ops3 * per_s / 1e12,
                                      "frac": ops3 * per_s / 1e12 / PEAK_INT_TOPS}})
    al = res.get("all_levels_kept")
    if al and "kernel_ms" in al:
        a4 = ops * al["points_per_launch"] / (al["kernel_ms"] * 1e-3) / 1e12
        al["roofline"] = {"bound": "alu", "achieved": a4, "peak": PEAK_INT_TOPS, "unit": "TOP/s",
                          "frac": a4 / PEAK_INT_TOPS, "ops_per_point": ops}
    log("roofline: %.1f method ops/point, %.2f T ops/s = %.1f%% of %.2f T" % (
        ops, achieved, 100 * achieved / PEAK_INT_TOPS, PEAK_INT_TOPS))


def bench_grid1k(bm, torch, steps):
    """The small workload: 1,024 blocks, 100,000 points per call (below the
    pre-sort threshold: one launch of the unsorted mapping kernel)."""
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    xy = torch.from_numpy(synth.points("grid1k")).cuda()
    out = torch.empty(xy.shape[0], dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    bm.map_points(ix, xy, out, s)
    reps = max(50, steps)
    wall, ev = timed_calls(torch, lambda: bm.map_points(ix, xy, out, s), reps, s)
    lt = launch_times(bm, ix, xy, out, s)
    n = xy.shape[0]
    r = {"blocks": g.n_blocks, "points": n, "points_per_s": n / wall, "ms_per_call": wall * 1e3,
         "events_ms": ev, "kernel_ms": lt["kernel_ms"], "kernel": lt["kernel"],
         "note": "launch-bound: 100k points fill 1,563 of the 64-point tiles"}
    log("grid1k: %.4f ms per call (kernel %.4f ms), %.3g points/s" % (wall * 1e3, lt["kernel_ms"], n / wall))
    ix.close()
    return r


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
    wall, ev = timed_calls(torch, lambda: bm.map_points(ix4, xy, out, s), steps, s)
    lt = launch_times(bm, ix4, xy, out, s)
    n = xy.shape[0]
    r = {"group_levels": ix4.info()["n_levels"], "points_per_s": n / wall, "ms_per_step": wall * 1e3,
         "events_ms": ev, "same_ids_as_default_index": same, "kernel_ms": lt["kernel_ms"],
         "points_per_launch": n / lt["launches_per_call"]}
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
        wall, ev = timed_calls(torch, lambda: bm.map_points_cover(cv, xy, out, approx=approx, stream=s), steps, s)
        r[mode] = {"points_per_s": n / wall, "ms_per_step": wall * 1e3, "kernel_ms": ev, "agree_with_plain": same}
        bpp = read_traffic("cover_map_kernel_%s_grid221k_100m" % mode)
        if bpp is not None:
            gbs = bpp * n / (ev * 1e-3) / 1e9
            r[mode]["hbm_measured"] = {"bytes_per_point": bpp, "GBs": gbs, "frac": gbs / PEAK_HBM_GBS}
        log("cover %s: %.3f ms/step, %.3g points/s, agrees with the plain path on %.6f of the points" %
            (mode, wall * 1e3, n / wall, same))
    cv.close()
    return r


def bench_aggregate(bm, torch, g, ids, steps):
    """What the mapping feeds: points per block over the 100M ids (checked
    against torch's bincount) and the per-point join of a per-block code table
    (checked against a torch gather)."""
    n_blocks = g.n_blocks
    s = torch.cuda.current_stream()
    counts = torch.zeros(n_blocks + 1, dtype=torch.int64, device=ids.device)
    bm.count_per_block(ids, n_blocks, counts)
    torch.cuda.synchronize()
    ref = torch.bincount(torch.where(ids >= 0, ids, torch.full_like(ids, n_blocks)).long(),
                         minlength=n_blocks + 1)
    ok = bool(torch.equal(counts, ref))
    del ref
    _, ms = timed_calls(torch, lambda: bm.count_per_block(ids, n_blocks, counts, stream=s), steps, s)
    n = ids.shape[0]
    table = torch.from_numpy(synth.block_codes(g)).cuda()
    codes = torch.empty(n, dtype=torch.int64, device="cuda")
    bm.join_per_block(ids, table, out=codes, fill=-1)
    torch.cuda.synchronize()
    want = torch.where(ids >= 0, table[ids.clamp(min=0).long()], torch.full_like(codes, -1))
    ok_join = bool(torch.equal(codes, want))
    del want
    _, jms = timed_calls(torch, lambda: bm.join_per_block(ids, table, out=codes, fill=-1, stream=s), steps, s)
    jgbs = 12.0 * n / (jms * 1e-3) / 1e9
    log("count per block: %.3f ms per 100M ids (%.3g ids/s), equal to bincount: %s" % (ms, n / ms * 1e3, ok))
    log("join per block: %.3f ms per 100M ids (%.0f GB/s = %.1f%% of HBM peak), equal to a gather: %s" % (
        jms, jgbs, 100 * jgbs / PEAK_HBM_GBS, ok_join))
    del codes, table
    return {"count": {"ms": ms, "ids_per_s": n / ms * 1e3, "equal_to_bincount": ok},
            "join": {"ms": jms, "ids_per_s": n / jms * 1e3, "achieved_GBs": jgbs, "hbm_frac": jgbs / PEAK_HBM_GBS,
                     "bytes_per_point": 12, "equal_to_gather": ok_join}}


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
    _, ms = timed_calls(torch, lambda: bm.quantize_lonlat(ll, q, s), steps, s)
    gbs = 24.0 * n / (ms * 1e-3) / 1e9
    log("quantize: %.3f ms per %d points (%.3g points/s, %.0f GB/s = %.1f%% of HBM peak), exact: %s" %
        (ms, n, n / ms * 1e3, gbs, 100 * gbs / PEAK_HBM_GBS, ok))
    del ll, q
    torch.cuda.empty_cache()
    return {"points": n, "ms": ms, "points_per_s": n / ms * 1e3, "achieved_GBs": gbs,
            "hbm_frac": gbs / PEAK_HBM_GBS, "bytes_per_point": 24, "exact": ok}


def bench_batched(bm, torch, g, ix, nb=10_000, reps=3):
    """Batched form: 10,000 batches lying back to back (sizes log-uniform on
    [1, 1e6], each batch one Gaussian cluster) over this index, given as
    device offsets. One graph replay (and one eager persistent launch)
    against one plain launch per batch."""
    t0 = time.time()
    sizes = synth.batch_sizes(nb)
    host, off = synth.batch_points(g, sizes)
    total = int(off[-1])
    xy = torch.from_numpy(host).cuda()
    doff = torch.from_numpy(off).cuda()
    del host
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    ref = torch.empty(total, dtype=torch.int32, device="cuda")
    log("batched: %d batches, %d points (sizes %d..%d), generated in %.1fs" %
        (nb, total, sizes.min(), sizes.max(), time.time() - t0))
    s = torch.cuda.current_stream()
    tune = bm.autotune(ix, xy[: min(total, 1 << 22)], s)
    log("batched: autotuned %s" % tune.as_dict())
    lib, sh = bm.lib, bm._stream_handle(s)
    import ctypes as C
    base_x, base_r = xy.data_ptr(), ref.data_ptr()

    def plain_all():  # the library's plain entry point, one call per batch
        for b in range(nb):
            lib.map_points(ix.handle, C.c_void_p(base_x + 8 * int(off[b])), int(sizes[b]),
                           C.c_void_p(base_r + 4 * int(off[b])), sh)
    plain_all()
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain_all()
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    # eager persistent launch over the offsets
    bm.map_batches(ix, xy, doff, out, s, tune)
    _, eager_ms = timed_calls(torch, lambda: bm.map_batches(ix, xy, doff, out, s, tune), 1, s)
    ok_eager = bool(torch.equal(out, ref))
    # captured graph, replayed
    out.fill_(-7)
    plan = bm.BatchPlan(ix, nb, tune, max_points=total)
    plan.run_offsets(xy, doff, out, s)
    torch.cuda.synchronize()
    ok_graph = bool(torch.equal(out, ref))
    t_graph, graph_ms = timed_calls(torch, lambda: plan.run_offsets(xy, doff, out, s), reps, s)
    plan.close()
    res = {"batches": nb, "points": total, "tuning": tune.as_dict(),
           "graph_points_per_s": total / t_graph, "graph_ms": graph_ms,
           "eager_kernel_ms": eager_ms, "eager_points_per_s": total / (eager_ms * 1e-3),
           "plain_per_batch_points_per_s": total / t_plain, "plain_per_batch_ms": t_plain * 1e3,
           "speedup_vs_plain_per_batch": t_plain / t_graph,
           "identical_to_plain": ok_eager and ok_graph,
           "hbm_algorithmic_frac": BYTES_PER_POINT * total / (graph_ms * 1e-3) / 1e9 / PEAK_HBM_GBS}
    bpp = read_traffic("batch_map_kernel_batches10k")
    if bpp is not None:
        gbs = bpp * total / (graph_ms * 1e-3) / 1e9
        res["hbm_measured"] = {"bytes_per_point": bpp, "GBs": gbs, "frac": gbs / PEAK_HBM_GBS}
        res["hbm_frac"] = gbs / PEAK_HBM_GBS
    log("batched: graph %.1f ms (%.3g pts/s), eager %.1f ms, per-batch plain %.1f ms (%.3g pts/s), identical=%s" %
        (graph_ms, res["graph_points_per_s"], eager_ms, t_plain * 1e3, res["plain_per_batch_points_per_s"],
         res["identical_to_plain"]))
    del xy, out, ref, doff
    torch.cuda.empty_cache()
    return res


def bench_served(bm, torch, g, ix, nreq, runs="all"):
    """Served form over the 8M-block graded mesh resident in HBM: requests of
    lognormal size (median 10k points, sigma 2, at most 10M), each a Gaussian
    cluster plus 20% uniform points, in page-locked host memory; every
    submission writes its own output buffer. Baseline: the same request loop
    with coalescing and overlap switched off (one request per batch, one slot,
    one stream), i.e. the plain kernel request by request. Both see the same
    Poisson arrivals at 50% and 90% of the baseline's capacity, and all at
    once."""
    t0 = time.time()
    npool = 1000
    sizes = synth.request_sizes(npool)
    pool, ref = [], []
    for r in range(npool):
        x = torch.empty((int(sizes[r]), 2), dtype=torch.int32, pin_memory=True).numpy()
        synth.request_points(g, r, int(sizes[r]), out=x)
        pool.append(x)
        ref.append(bm.map_points(ix, torch.from_numpy(x).cuda()).cpu().numpy())
    rng = np.random.default_rng(5)
    order = rng.integers(0, npool, nreq)
    osz = sizes[order]
    ooff = np.concatenate([[0], np.cumsum(osz)]).astype(np.int64)
    outbuf = torch.empty(int(ooff[-1]), dtype=torch.int32, pin_memory=True).numpy()
    outs = [outbuf[ooff[i]:ooff[i + 1]] for i in range(nreq)]
    want = np.concatenate([ref[i] for i in order])
    reqs = [(pool[order[i]], outs[i]) for i in range(nreq)]
    mean_pts = float(osz.mean())
    log("served: %d distinct payloads (mean %.0f points, max %d), %d submissions with %d output points, "
        "prepared in %.1fs" % (npool, sizes.mean(), sizes.max(), nreq, int(ooff[-1]), time.time() - t0))
    bpp = read_traffic("served_requests20k")

    def run(cfg, arrivals, nr):
        outbuf[: ooff[nr]] = -7
        srv = bm.Server(ix, cfg)
        t = time.perf_counter()
        srv.run_trace(reqs[:nr], arrivals[:nr])
        wall = time.perf_counter() - t
        st = srv.stats()
        srv.close()
        same = bool(np.array_equal(outbuf[: ooff[nr]], want[: ooff[nr]]))
        r = {"points_per_s": st["points_per_s"], "requests_per_s": st["completed"] / wall,
             "p50_us": st["p50_us"], "p99_us": st["p99_us"], "mean_us": st["mean_us"],
             "mean_requests_per_batch": st["mean_requests_per_batch"], "batches": st["batches"],
             "identical_to_alone": same,
             "hbm_algorithmic_frac": BYTES_PER_POINT * st["points_per_s"] / 1e9 / PEAK_HBM_GBS}
        if bpp is not None:
            r["hbm_frac"] = bpp * st["points_per_s"] / 1e9 / PEAK_HBM_GBS
        return r

    base_cfg = bm.server_cfg(mem_budget_bytes=2 << 30, max_batch_points=1 << 24, max_slots=1, n_streams=1,
                             flags=bm.BM_SERVER_ONE_PER_BATCH)
    srv_cfg = bm.server_cfg(mem_budget_bytes=2 << 30, max_batch_points=1 << 22, max_slots=8, n_streams=8)
    zero = np.zeros(nreq)
    res = {"requests": nreq, "mean_points_per_request": mean_pts, "output_buffers": "one per submission"}
    if bpp is not None:
        res["hbm_bytes_per_point_measured"] = bpp
    res["server_saturated"] = run(srv_cfg, zero, nreq)
    if runs == "all":
        nsat = min(nreq, 5000)
        res["baseline_saturated"] = run(base_cfg, zero, nsat)
        cap = res["baseline_saturated"]["requests_per_s"]
        for name, frac in (("50pct", 0.5), ("90pct", 0.9)):
            arr = np.cumsum(rng.exponential(1e6 / (frac * cap), nreq))
            res["baseline_" + name] = run(base_cfg, arr, nreq)
            res["server_" + name] = run(srv_cfg, arr, nreq)
            res["baseline_" + name]["offered_qps"] = res["server_" + name]["offered_qps"] = frac * cap
        res["speedup_saturated"] = (res["server_saturated"]["points_per_s"] /
                                    res["baseline_saturated"]["points_per_s"])
    for k, v in res.items():
        if isinstance(v, dict):
            log("served %-19s %.3g pts/s, %.0f req/s, p50 %.0f us, p99 %.0f us, %.1f req/batch, identical=%s" %
                (k, v["points_per_s"], v["requests_per_s"], v["p50_us"], v["p99_us"], v["mean_requests_per_batch"],
                 v["identical_to_alone"]))
    del outbuf, outs, want
    return res


def profile_quadtree8m(bm, torch, g, ix, steps):
    """One resident 2^26-point chunk of the 1B-point stream over the 8M-block
    mesh, mapped once to warm up and then `steps` times, each call timed per
    launch with HIP events on its stream (a short run for the profiler)."""
    CH = synth.QUADTREE["chunk"]
    xy = torch.from_numpy(synth.points("quadtree8m", CH, 0)).cuda()
    out = torch.empty(CH, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    bm.map_points(ix, xy, out, s)
    torch.cuda.synchronize()
    lt = launch_times(bm, ix, xy, out, s, reps=steps)
    res = {"workload": "8M-block graded quadtree mesh, one resident 2^26-point chunk", "points": CH,
           "calls": steps, "map_launches_per_call": lt["launches_per_call"], "map_kernel_ms": lt["kernel_ms"],
           "sort_ms_per_call": lt["sort_ms_per_call"], "unsort_ms_per_call": lt["unsort_ms_per_call"],
           "points_per_s_per_call": CH / ((lt["kernel_ms"] * lt["launches_per_call"] + lt["sort_ms_per_call"] +
                                           lt["unsort_ms_per_call"]) * 1e-3)}
    log("quadtree8m chunk: %d mapping launch(es) of %.3f ms, sort %.3f ms, unsort %.3f ms per call" % (
        lt["launches_per_call"], lt["kernel_ms"], lt["sort_ms_per_call"], lt["unsort_ms_per_call"]))
    return res


def bench_quadtree8m(bm, torch, g, ix):
    """8M blocks, 1B points in 2^26-point chunks: kernel-only rate (chunk
    resident, every launch timed), and end-to-end rate streamed from pinned
    host memory with the copies in and out overlapped with the mapping."""
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
    _, kern_ms = timed_calls(torch, lambda: bm.map_points(ix, dxy[0], dout[0], s), 5, s)
    lt = launch_times(bm, ix, dxy[0], dout[0], s)
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
    launch_pts = CH / lt["launches_per_call"]
    alg = SORTED_KERNEL_BYTES_PER_POINT * launch_pts
    achieved = alg / (lt["kernel_ms"] * 1e-3) / 1e9
    bpp = read_traffic("map_sorted_kernel_quadtree8m_chunk")
    res = {"blocks": g.n_blocks, "vertices": int(g.verts.shape[0]), "points": N, "chunk": CH,
           "kernel_points_per_s": CH / (kern_ms * 1e-3), "kernel_ms_per_chunk": kern_ms,
           "map_kernel_ms": lt["kernel_ms"], "sort_ms_per_chunk": lt["sort_ms_per_call"],
           "unsort_ms_per_chunk": lt["unsort_ms_per_call"],
           "end_to_end_points_per_s": N / t_wall, "end_to_end_first_chunk_identical": same,
           "index_device_bytes": info["device_bytes"], "sort_bins": info["sort_bins"],
           "sort_bins_adaptive": bool(info["sort_adaptive"]),
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": achieved / PEAK_HBM_GBS,
                        "traffic": bpp * launch_pts if bpp is not None else None,
                        "kernel": lt["kernel"], "algorithmic_bytes_per_point": SORTED_KERNEL_BYTES_PER_POINT}}
    if bpp is not None:
        gbs = bpp * launch_pts / (lt["kernel_ms"] * 1e-3) / 1e9
        res["roofline"].update({"traffic_bytes_per_point": bpp, "traffic_GBs": gbs,
                                "traffic_frac": gbs / PEAK_HBM_GBS})
    log("quadtree8m: kernel %.3f ms per 2^26 chunk (%.3g pts/s; mapping launch %.3f ms); end-to-end with PCIe "
        "%.3g pts/s (first chunk identical to the resident run: %s)" %
        (kern_ms, res["kernel_points_per_s"], lt["kernel_ms"], res["end_to_end_points_per_s"], same))
    del hin, hres, dxy, dout
    return res


def cpu_baseline(g, pts):
    """The CPU oracle (hierarchy route, C + OpenMP) on the host cores: whole
    passes over the workload's 100M points until at least 10 s have passed;
    one thread on the first 2M points; and the oracle's counts of the
    method's work on the first 2M points, over the hierarchy the index
    filters (regions, counties, blocks: the tract level merged into counties,
    as the paper's own state / county / block) and over all four levels."""
    import tempfile

    import oracle
    # the oracle's source built for this host's CPU (-O3 -march=native), in a
    # temporary directory; the in-tree copy is built for any x86-64 host
    flags = "gcc -O3 -march=native, OpenMP"
    tmpdir = tempfile.mkdtemp(prefix="bm_oracle_")
    try:
        oracle.use(oracle.build_native(tmpdir))
    except Exception as e:  # no compiler on this host: the portable build
        log("cpu baseline: native build failed (%s); timing the portable build" % e)
        flags = "gcc -O3 (portable x86-64), OpenMP"
    H = oracle.Hier.from_geometry(g)
    sample = pts[:2_000_000]
    _, c4 = H.map(sample, with_counts=True)
    par = g.parents  # county -> region, tract -> county, block -> tract
    H3 = oracle.Hier(g.vert_off, g.verts, [g.n_groups[0], g.n_groups[1]],
                     [par[0], np.asarray(par[1])[np.asarray(par[2])]])
    _, c3 = H3.map(sample, with_counts=True)
    del H3
    n = sample.shape[0]
    work = {}
    for name, c in (("default_index", c3), ("every_level", c4)):
        work[name] = {k: v / n for k, v in c.items()}
        work[name]["ops_per_point"] = ops_per_point(c, n)
    work["cost_lane_ops"] = COST
    work["sample_points"] = n
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
    H.map(sample)
    single = n / (time.perf_counter() - t1)
    oracle.set_threads(cores)
    return {"value": passes * pts.shape[0] / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "%d full passes over the workload's %d points (%.1f s), hierarchy route, C, %s"
                      % (passes, pts.shape[0], dt, flags),
            "single_thread_points_per_s": single, "host": host_cpus(), "work_per_point": work}


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
