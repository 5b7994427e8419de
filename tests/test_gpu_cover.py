"""GPU parity for the cell cover (the paper's fast approach, Sec. IV): exact
mode gives the oracle's block ids bit for bit; approximate mode gives, at
every point, the oracle's answer at the point or at the centre of the point's
finest cell (which bounds its error by half a cell diagonal)."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_map import boundary_points, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def bm():
    import paper_2005_03156_amd as bm
    return bm


def cover_map(bm, torch, cv, pts, approx=False):
    xy = torch.from_numpy(np.ascontiguousarray(pts, np.int32)).cuda()
    out = bm.map_points_cover(cv, xy, approx=approx)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def centres(info, pts):
    cl = info["cell_log2"]
    x = pts[:, 0].astype(np.int64) - info["origin_x"]
    y = pts[:, 1].astype(np.int64) - info["origin_y"]
    cx = info["origin_x"] + ((x >> cl) << cl) + (1 << (cl - 1))
    cy = info["origin_y"] + ((y >> cl) << cl) + (1 << (cl - 1))
    return np.stack([np.clip(cx, 0, 2**31 - 1), np.clip(cy, 0, 2**31 - 1)], 1).astype(np.int32)


def grid_points(info, rng, n):
    cl, L = info["cell_log2"], info["log2_side"]
    k = rng.integers(0, 1 << (L - cl), size=(n, 2), dtype=np.int64)
    off = rng.choice(np.array([0, 0, 1, -1, (1 << cl) - 1], np.int64), size=(n, 2))
    x = info["origin_x"] + (k[:, 0] << cl) + off[:, 0]
    y = info["origin_y"] + (k[:, 1] << cl) + off[:, 1]
    return np.stack([np.clip(x, 0, 2**31 - 1), np.clip(y, 0, 2**31 - 1)], 1).astype(np.int32)


def check(bm, torch, cv, pts, exact_fn, approx_sample=None):
    """Exact mode against exact_fn (the oracle); approximate mode's contract
    on all points (or a sample)."""
    got = cover_map(bm, torch, cv, pts)
    want = exact_fn(pts)
    assert (got == want).all(), int((got != want).sum())
    apx = cover_map(bm, torch, cv, pts, approx=True)
    sub = np.arange(len(pts)) if approx_sample is None else \
        np.random.default_rng(0).choice(len(pts), approx_sample, replace=False)
    at_centre = exact_fn(centres(cv.info(), pts[sub]))
    ok = (apx[sub] == want[sub]) | (apx[sub] == at_centre)
    assert ok.all(), int((~ok).sum())
    return got, apx


def test_cover_grid1k_exact_and_approx(torch_cuda, bm):
    say("cover grid1k")
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    cv = bm.Cover.from_geometry(ix, g)
    info = cv.info()
    assert info["boundary_cells"] > 0 and info["interior_entries"] > 0 and info["device_bytes"] > 0
    rng = np.random.default_rng(3)
    out = np.array([[-1, -1], [-2**31, 5], [2**31 - 1, 2**31 - 1], [0, 2**31 - 1], [5, -7]], np.int32)
    pts = np.concatenate([synth.points("grid1k"), boundary_points(g), grid_points(info, rng, 30_000), out])
    got, apx = check(bm, torch_cuda, cv, pts, lambda p: oracle.brute(g.vert_off, g.verts, p, box_reject=True))
    assert (got == -1).any() and (got >= 0).any()
    assert (apx != got).any()  # points in boundary cells really are answered from the cell
    # the plain path agrees
    xy = torch_cuda.from_numpy(pts).cuda()
    assert (bm.map_points(ix, xy).cpu().numpy() == got).all()


def test_cover_over_an_index_that_keeps_a_thin_level(torch_cuda, bm):
    """The cover reads the leaf order from the index it is built on: over an
    index that keeps a thin level (pairs of blocks under 16 groups), exact
    cover lookups equal brute force and the index's own plain path."""
    say("cover over an index with a kept thin level")
    g = synth.geometry("grid1k")
    pair = (np.arange(g.n_blocks) // 2).astype(np.int32)
    top = (np.arange(g.n_blocks // 2) % 16).astype(np.int32)
    ix = bm.Index(g.vert_off, g.verts, [16, g.n_blocks // 2], [top, pair], keep_all_levels=True)
    assert ix.info()["n_levels"] == 2
    cv = bm.Cover(ix, g.vert_off, g.verts)
    rng = np.random.default_rng(5)
    pts = np.concatenate([synth.points("grid1k", 30_000), boundary_points(g),
                          grid_points(cv.info(), rng, 10_000)])
    got, _ = check(bm, torch_cuda, cv, pts, lambda p: oracle.brute(g.vert_off, g.verts, p, box_reject=True))
    xy = torch_cuda.from_numpy(pts).cuda()
    assert (bm.map_points(ix, xy).cpu().numpy() == got).all()


@pytest.mark.parametrize("cl", [7, 13])
def test_cover_cell_sizes(torch_cuda, bm, cl):
    say("cover cell size", cl)
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    cv = bm.Cover.from_geometry(ix, g, cell_log2=cl)
    assert cv.info()["cell_log2"] == cl
    rng = np.random.default_rng(cl)
    pts = np.concatenate([synth.points("grid1k", 30_000), grid_points(cv.info(), rng, 10_000), boundary_points(g, 1000)])
    check(bm, torch_cuda, cv, pts, lambda p: oracle.brute(g.vert_off, g.verts, p, box_reject=True))


def test_cover_grid221k_two_million(torch_cuda, bm):
    say("cover grid221k: build")
    g = synth.geometry("grid221k")
    ix = bm.Index.from_geometry(g)
    cv = bm.Cover.from_geometry(ix, g)
    H = oracle.Hier.from_geometry(g)
    say("cover grid221k:", cv.info())
    rng = np.random.default_rng(9)
    pts = np.concatenate([synth.points("grid221k", 2_000_000), boundary_points(g, 20_000, seed=4),
                          grid_points(cv.info(), rng, 50_000)])
    got, _ = check(bm, torch_cuda, cv, pts, H.map, approx_sample=300_000)
    xy = torch_cuda.from_numpy(pts).cuda()
    assert (bm.map_points(ix, xy).cpu().numpy() == got).all()


def _rings(rings):
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    return off, np.concatenate([np.asarray(r, np.int32) for r in rings])


def test_cover_overlaps_nested_and_flat(torch_cuda, bm):
    """Overlapping rectangles (smallest id wins), 600 nested squares (boundary
    cells listing hundreds of blocks: the list overflow falls back to the
    per-point walk), both without a hierarchy and with one."""
    rng = np.random.default_rng(6)
    rects = []
    for _ in range(300):
        x, y = rng.integers(0, 9000, 2)
        w, h = rng.integers(50, 2000, 2)
        rects.append([(x, y), (x + w, y), (x + w, y + h), (x, y + h)])
    nested = [[(0, 0), (10 + k, 0), (10 + k, 10 + k), (0, 10 + k)] for k in range(600)]
    for name, rings, pts in [
            ("overlaps", rects, rng.integers(-10, 11000, (50_000, 2))),
            ("nested", nested, rng.integers(-5, 620, (20_000, 2)))]:
        off, verts = _rings(rings)
        for L in (0, 1):
            say("cover", name, "levels", L)
            m = len(rings)
            ix = bm.Index(off, verts, [5] if L else (), [np.arange(m, dtype=np.int32) % 5] if L else ())
            cv = bm.Cover(ix, off, verts)
            check(bm, torch_cuda, cv, pts.astype(np.int32), lambda p: oracle.brute(off, verts, p))


def test_cover_heavy_ring(torch_cuda, bm):
    say("cover heavy ring")
    rng = np.random.default_rng(4)
    m = 20000
    ang = (np.arange(m) + rng.uniform(0.1, 0.9, m)) * 2 * np.pi / m
    rad = rng.uniform(4e5, 5e5, m)
    star = np.stack([1_000_000 + rad * np.cos(ang), 1_000_000 + rad * np.sin(ang)], 1).round().astype(np.int32)
    tri = [[(10 * i, 0), (10 * i + 9, 0), (10 * i, 9)] for i in range(100)]
    off, verts = _rings([star] + tri)
    ix = bm.Index(off, verts)
    cv = bm.Cover(ix, off, verts, cell_log2=10)
    pts = np.concatenate([rng.integers(4e5, 1.6e6, (30000, 2)), rng.integers(-2, 1001, (5000, 2)),
                          star[:2000], star[:2000] + 1]).astype(np.int32)
    check(bm, torch_cuda, cv, pts, lambda p: oracle.brute(off, verts, p))


def test_cover_ragged_sizes_and_errors(torch_cuda, bm):
    torch = torch_cuda
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    cv = bm.Cover.from_geometry(ix, g)
    pts = synth.points("grid1k", 5000, i0=777)
    want = oracle.brute(g.vert_off, g.verts, pts)
    for n in [0, 1, 63, 64, 65, 127, 128, 129, 1000, 4097]:
        say("cover ragged", n)
        got = cover_map(bm, torch, cv, pts[:n])
        assert got.shape == (n,) and (got == want[:n]).all()
    # a descriptor whose rings differ from the index's, and a bad mode
    bad = g.verts.copy()
    bad[5] += 1
    with pytest.raises(bm.BlockmapError):
        bm.Cover(ix, g.vert_off, bad)
    xy = torch.from_numpy(pts).cuda()
    out = torch.empty(len(pts), dtype=torch.int32, device="cuda")
    import ctypes as C
    rc = bm.lib.map_points_cover(cv.handle, C.c_void_p(xy.data_ptr()), len(pts), C.c_void_p(out.data_ptr()), 2,
                                 C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == bm.BM_EINVAL


def test_count_per_block(torch_cuda, bm):
    """Points per block equal numpy's bincount of the ids (the last slot for
    ids outside [0, n_blocks)); counts accumulate over calls."""
    torch = torch_cuda
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    pts = synth.points("grid1k", 100_000)
    ids = bm.map_points(ix, torch.from_numpy(pts).cuda())
    rng = np.random.default_rng(2)
    odd = torch.from_numpy(rng.choice(np.array([-1, -7, g.n_blocks, 2**31 - 1, 0, 5], np.int32), 3000)).cuda()
    for name, t in [("mapped", ids), ("sorted", torch.sort(ids).values), ("odd", odd),
                    ("ragged", ids[:777]), ("empty", ids[:0])]:
        say("count per block", name)
        got = bm.count_per_block(t, g.n_blocks).cpu().numpy()
        a = t.cpu().numpy().astype(np.int64)
        a = np.where((a >= 0) & (a < g.n_blocks), a, g.n_blocks)
        assert np.array_equal(got, np.bincount(a, minlength=g.n_blocks + 1)), name
    c = bm.count_per_block(ids, g.n_blocks)
    bm.count_per_block(ids, g.n_blocks, counts=c)
    assert np.array_equal(c.cpu().numpy(), 2 * bm.count_per_block(ids, g.n_blocks).cpu().numpy())
    assert np.array_equal(c.cpu().numpy().view(np.uint64), 2 * oracle.count_per_block(ids.cpu().numpy(), g.n_blocks))


@pytest.mark.parametrize("nb", [1024, 220_900, 3_000_001])
def test_count_per_block_bucketed(torch_cuda, bm, nb):
    """Large calls take the bucketed route (counting sort by id >> 13, LDS
    histograms per slice, summed rows): the same counts as bincount."""
    torch = torch_cuda
    rng = np.random.default_rng(nb)
    a = rng.integers(-3, nb + 3, size=3_000_000).astype(np.int32)
    a[:1000] = nb - 1  # a crowded block
    for order in ("random", "sorted"):
        say("bucketed count", nb, order)
        t = torch.from_numpy(np.sort(a) if order == "sorted" else a).cuda()
        got = bm.count_per_block(t, nb).cpu().numpy()
        b = np.where((a >= 0) & (a < nb), a, nb).astype(np.int64)
        assert np.array_equal(got, np.bincount(b, minlength=nb + 1)), order
