"""GPU parity: block ids from the HIP kernels equal the CPU oracle's, bit for
bit, on seeded inputs; plus edge cases and launch-shape invariance."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


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


def gpu_map(bm, torch, ix, pts, tuning=None):
    xy = torch.from_numpy(np.ascontiguousarray(pts, np.int32)).cuda()
    out = bm.map_points(ix, xy, tuning=tuning)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def boundary_points(g, k=3000, seed=0):
    rng = np.random.default_rng(seed)
    v = g.verts[rng.choice(g.verts.shape[0], min(k, g.verts.shape[0]), replace=False)]
    offs = np.array([[0, 0], [-1, 0], [0, -1], [1, 0], [0, 1], [-1, -1], [1, 1]], np.int32)
    return (v[:, None, :] + offs[None]).reshape(-1, 2).astype(np.int32)


# ------------------------------------------------------------ grid1k ----

def test_grid1k_full_vs_brute_force(torch_cuda, bm):
    say("grid1k: 100k points + boundary points vs brute force")
    g = synth.geometry("grid1k")
    pts = np.concatenate([synth.points("grid1k"), boundary_points(g)])
    ix = bm.Index.from_geometry(g)
    got = gpu_map(bm, torch_cuda, ix, pts)
    want = oracle.brute(g.vert_off, g.verts, pts)
    assert (got == want).all(), int((got != want).sum())
    assert (want == -1).any() and (want >= 0).any()


@pytest.mark.parametrize("chunk", [4, 8, 16])
@pytest.mark.parametrize("bpc", [1, 3])
def test_launch_shape_never_changes_results(torch_cuda, bm, chunk, bpc):
    say("grid1k tuning", chunk, bpc)
    g = synth.geometry("grid1k")
    pts = np.concatenate([synth.points("grid1k", 30_001), boundary_points(g, 500)])
    ix = bm.Index.from_geometry(g)
    t = bm.Tuning(chunk, bpc, 65536)
    got = gpu_map(bm, torch_cuda, ix, pts, tuning=t)
    want = oracle.brute(g.vert_off, g.verts, pts)
    assert (got == want).all()


def test_ragged_sizes_and_empty(torch_cuda, bm):
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    pts = synth.points("grid1k", 5000)
    want = oracle.brute(g.vert_off, g.verts, pts)
    for n in [0, 1, 2, 63, 64, 65, 255, 257, 1000, 4999]:
        say("ragged n =", n)
        got = gpu_map(bm, torch_cuda, ix, pts[:n])
        assert got.shape == (n,) and (got == want[:n]).all(), n


def test_extreme_coordinates(torch_cuda, bm):
    say("extreme coordinates")
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    I32 = np.iinfo(np.int32)
    vals = [I32.min, I32.min + 1, -1, 0, 1, g.W - 1, g.W, I32.max - 1, I32.max]
    pts = np.array([[a, b] for a in vals for b in vals], np.int32)
    got = gpu_map(bm, torch_cuda, ix, pts)
    assert (got == oracle.brute(g.vert_off, g.verts, pts)).all()


def _cell_grid_points(vert_off, verts):
    """Every corner of every cell of every block's 16 x 16 cell map (cell
    sides: the smallest powers of two with 16 cells covering each side of the
    block's box), and the points one unit below and left of each: the
    borders between cells a crossing test may skip and cells it must run."""
    box = oracle.ring_boxes(vert_off, verts).astype(np.int64)
    out = []
    for x0, x1, y0, y1 in box:
        if x1 <= x0 or y1 <= y0:
            continue
        sx = max(0, int(np.ceil(np.log2(x1 - x0))) - 4) if x1 - x0 > 1 else 0
        sy = max(0, int(np.ceil(np.log2(y1 - y0))) - 4) if y1 - y0 > 1 else 0
        xs = np.minimum(x0 + (np.arange(17) << sx), x1)
        ys = np.minimum(y0 + (np.arange(17) << sy), y1)
        gx, gy = np.meshgrid(xs, ys)
        c = np.stack([gx.ravel(), gy.ravel()], 1)
        out += [c, c - 1, c - [1, 0], c - [0, 1]]
    return np.concatenate(out).astype(np.int32)


def test_cell_map_borders_vs_brute_force(torch_cuda, bm):
    """Points on the corners of every block's cell map, and one unit off
    them, for the 1,024-block grid and for rings whose cells are a few units
    wide (a comb, a notched spiral, a triangle): the mapping kernel, which
    decides pairs in settled cells from the map, equals brute force."""
    say("cell map borders")
    g = synth.geometry("grid1k")
    pts = _cell_grid_points(g.vert_off, g.verts)
    ix = bm.Index.from_geometry(g)
    got = gpu_map(bm, torch_cuda, ix, pts)
    want = oracle.brute(g.vert_off, g.verts, pts, box_reject=True)
    assert (got == want).all(), int((got != want).sum())
    rings = [
        [(0, 0), (60, 0), (60, 40), (45, 40), (45, 10), (30, 10), (30, 40), (15, 40), (15, 10), (5, 10), (5, 40),
         (0, 40)],
        [(100, 100), (170, 100), (170, 160), (110, 160), (110, 120), (150, 120), (150, 140), (130, 140),
         (130, 150), (160, 150), (160, 110), (100, 110)],
        [(200, 5), (255, 5), (213, 47)],
    ]
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    verts = np.concatenate([np.asarray(r, np.int32) for r in rings])
    ix2 = bm.Index(off, verts)
    xs, ys = np.meshgrid(np.arange(-2, 260), np.arange(-2, 175))
    pts2 = np.concatenate([np.stack([xs.ravel(), ys.ravel()], 1), _cell_grid_points(off, verts)]).astype(np.int32)
    got2 = gpu_map(bm, torch_cuda, ix2, pts2)
    assert (got2 == oracle.brute(off, verts, pts2)).all()


# ------------------------------------------------------------ grid221k ----

@pytest.fixture(scope="module")
def grid221k(bm, torch_cuda):
    g = synth.geometry("grid221k")
    return g, bm.Index.from_geometry(g), oracle.Hier.from_geometry(g)


def test_grid221k_two_million_vs_hierarchy_oracle(torch_cuda, bm, grid221k):
    say("grid221k: 2M points vs hierarchy oracle; sample vs brute force")
    g, ix, H = grid221k
    pts = np.concatenate([synth.points("grid221k", 2_000_000), boundary_points(g, 20_000, seed=3)])
    got = gpu_map(bm, torch_cuda, ix, pts)
    want = H.map(pts)
    assert (got == want).all(), int((got != want).sum())
    sub = np.random.default_rng(1).choice(pts.shape[0], 1000, replace=False)
    assert (got[sub] == oracle.brute(g.vert_off, g.verts, pts[sub], box_reject=True)).all()


def test_grid221k_every_level_kept(torch_cuda, bm, grid221k):
    """The full four-level filter (regions, counties, tracts, blocks; the thin
    tract level kept): the same ids as the oracle on 2M points plus boundary
    points, and the same as the default index on a pre-sorted call of 5M."""
    torch = torch_cuda
    g, ix, H = grid221k
    ix4 = bm.Index.from_geometry(g, keep_all_levels=True)
    assert ix4.info()["n_levels"] == 3 and ix.info()["n_levels"] == 2
    say("grid221k, every level kept: 2M points vs hierarchy oracle")
    pts = np.concatenate([synth.points("grid221k", 2_000_000, i0=9_000_000), boundary_points(g, 20_000, seed=4)])
    got = gpu_map(bm, torch, ix4, pts)
    assert (got == H.map(pts)).all()
    say("grid221k, every level kept: 5M pre-sorted points vs the default index")
    xy = torch.from_numpy(synth.points("grid221k", 5_000_000, i0=20_000_000)).cuda()
    a = bm.map_points(ix4, xy)
    b = bm.map_points(ix, xy)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    ix4.close()


def test_spatial_presort_never_changes_results(torch_cuda, bm, grid221k):
    """Calls above the pre-sort threshold, sorted or not, several chunks with
    a ragged tail: identical outputs, equal to the oracle on a sample."""
    torch = torch_cuda
    g, ix, H = grid221k
    n = 3 * (1 << 22) + 12345
    pts = synth.points("grid221k", n, i0=5_000_000)
    xy = torch.from_numpy(pts).cuda()
    say("presort on/off", n)
    a = bm.map_points(ix, xy, tuning=bm.Tuning(4, 5, 2048, 1))
    b = bm.map_points(ix, xy, tuning=bm.Tuning(8, 3, 2048, 0))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    sub = np.random.default_rng(8).choice(n, 100_000, replace=False)
    assert (a.cpu().numpy()[sub] == H.map(pts[sub])).all()


def test_concurrent_calls_on_several_streams(torch_cuda, bm, grid221k):
    """The index is read-only and each call's scratch is its own (stream
    ordered): calls queued on three streams at once, two of them pre-sorted,
    give the ids of the same calls made one at a time, three times over."""
    torch = torch_cuda
    g, ix, H = grid221k
    sizes = [(1 << 21) + 333, 50_000, (1 << 20) + 7]
    xs = [torch.from_numpy(synth.points("grid221k", n, i0=30_000_000 + 5_000_000 * k)).cuda()
          for k, n in enumerate(sizes)]
    ref = [bm.map_points(ix, x) for x in xs]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in sizes]
    outs = [torch.empty_like(r) for r in ref]
    for rep in range(3):
        say("three streams, round", rep)
        for o in outs:
            o.fill_(-7)
        torch.cuda.synchronize()
        for st, x, o in zip(streams, xs, outs):
            bm.map_points(ix, x, o, st)
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r)
    sub = np.random.default_rng(12).choice(sizes[0], 20_000, replace=False)
    assert (ref[0].cpu().numpy()[sub] == H.map(xs[0].cpu().numpy()[sub])).all()


@pytest.mark.parametrize("kind", ["one_point_inside", "one_point_outside", "vertical_line", "two_clusters"])
def test_spatial_presort_degenerate_distributions(torch_cuda, bm, kind):
    """Pre-sorted calls whose points all fall in one bin (a single bin cut
    into many refinement pieces), on one line, or in two tight clusters: the
    same ids as unsorted, and as brute force on a sample."""
    torch = torch_cuda
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    n = (1 << 21) + 77
    rng = np.random.default_rng(len(kind))
    if kind == "one_point_inside":
        pts = np.tile(np.array([[g.W // 3, g.W // 5]], np.int32), (n, 1))
    elif kind == "one_point_outside":
        pts = np.tile(np.array([[g.W + 10, -3]], np.int32), (n, 1))
    elif kind == "vertical_line":
        pts = np.stack([np.full(n, g.W // 2), rng.integers(-5, g.W + 5, n)], 1).astype(np.int32)
    else:
        c = rng.integers(0, 2, n)
        pts = (np.array([[g.W // 7, g.W // 9], [g.W - 11, g.W - 13]])[c] + rng.integers(-2, 3, (n, 2))).astype(np.int32)
    xy = torch.from_numpy(pts).cuda()
    say("presort degenerate", kind, n)
    a = bm.map_points(ix, xy, tuning=bm.Tuning(4, 8, 2048, 1))
    b = bm.map_points(ix, xy, tuning=bm.Tuning(4, 8, 2048, 0))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    sub = rng.choice(n, 5_000, replace=False)
    assert (a.cpu().numpy()[sub] == oracle.brute(g.vert_off, g.verts, pts[sub])).all()


@pytest.mark.parametrize("side", [40, 3000])
def test_spatial_presort_small_root_box(torch_cuda, bm, side):
    """Pre-sorted calls over indexes whose root box is narrower than the
    1024 x 1024 sort grid (side 40: bins only, no refinement; side 3000: both),
    with points outside the box too: the same ids as unsorted, and as brute
    force on a sample."""
    torch = torch_cuda
    rng = np.random.default_rng(side)
    k = 30
    rings = [[(0, 0), (side * (j + 1) // k, 0), (side * (j + 1) // k, side * (j + 1) // k), (0, side * (j + 1) // k)]
             for j in range(k)]
    off, verts, ix = _rings_index(bm, rings)
    n = (1 << 20) + 321
    pts = rng.integers(-3, side + 4, size=(n, 2)).astype(np.int32)
    xy = torch.from_numpy(pts).cuda()
    say("presort small root box", side, n)
    a = bm.map_points(ix, xy, tuning=bm.Tuning(4, 8, 2048, 1))
    b = bm.map_points(ix, xy, tuning=bm.Tuning(4, 8, 2048, 0))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    sub = rng.choice(n, 20_000, replace=False)
    assert (a.cpu().numpy()[sub] == oracle.brute(off, verts, pts[sub])).all()


def test_large_index_small_extent_uniform_bins(torch_cuda, bm):
    """An index over 256 MB whose extent is too small for the adaptive sort
    bins (3.24M squares of side 36 filling a 64,800-unit square) sorts over
    the uniform 64 x 64 grid of bins: a pre-sorted call equals the squares'
    closed form (square (i, j), block i * 1800 + j, holds [36 j, 36 j + 36) x
    [36 i, 36 i + 36)) at every point and brute force on a sample."""
    torch = torch_cuda
    n, s = 1800, 36
    j, i = np.meshgrid(np.arange(n), np.arange(n))
    x0, y0 = (j.ravel() * s).astype(np.int32), (i.ravel() * s).astype(np.int32)
    verts = np.stack([np.stack([x0, y0], 1), np.stack([x0 + s, y0], 1), np.stack([x0 + s, y0 + s], 1),
                      np.stack([x0, y0 + s], 1)], 1).reshape(-1, 2)
    off = np.arange(0, 4 * n * n + 1, 4, dtype=np.int64)
    grp = ((i.ravel() // 15) * (n // 15) + j.ravel() // 15).astype(np.int32)
    say("large index, small extent: building", n * n, "squares")
    ix = bm.Index(off, verts, [(n // 15) ** 2], [grp])
    info = ix.info()
    assert info["device_bytes"] > 256 << 20 and info["sort_adaptive"] == 0 and info["sort_bins"] == 4096, info
    rng = np.random.default_rng(44)
    pts = rng.integers(-100, n * s + 100, (1 << 21, 2)).astype(np.int32)
    got = bm.map_points(ix, torch.from_numpy(pts).cuda()).cpu().numpy()
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    inside = (x >= 0) & (x < n * s) & (y >= 0) & (y < n * s)
    assert (got == np.where(inside, (y // s) * n + x // s, -1)).all()
    sub = rng.choice(len(pts), 500, replace=False)
    assert (got[sub] == oracle.brute(off, verts, pts[sub], box_reject=True)).all()
    ix.close()


def test_grid221k_full_size_every_point(torch_cuda, bm, grid221k):
    """100M points in the benchmark's launch shape: every output equals the
    hierarchy oracle's, the partition property holds at every point (an id
    exactly when the point lies in [0, W)^2), and a sample equals brute force."""
    torch = torch_cuda
    g, ix, H = grid221k
    n = synth.n_points("grid221k")
    say("grid221k full size: generating", n)
    pts = synth.points("grid221k", n)
    xy = torch.from_numpy(pts).cuda()
    out = bm.map_points(ix, xy)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    say("grid221k full size: oracle over every point")
    want = H.map(pts)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (bad.size, bad[:5], got[bad[:5]], want[bad[:5]])
    x, y = pts[:, 0], pts[:, 1]
    inside = (x >= 0) & (x < g.W) & (y >= 0) & (y < g.W)
    assert ((got >= 0) == inside).all()
    sub = np.random.default_rng(7).choice(n, 2000, replace=False)
    assert (got[sub] == oracle.brute(g.vert_off, g.verts, pts[sub], box_reject=True)).all()
    # a repeat run gives identical bytes
    out2 = bm.map_points(ix, xy)
    torch.cuda.synchronize()
    assert torch.equal(out, out2)
    # one call over more than 2^27 points: two rounds of sort passes, the
    # second with a ragged last chunk
    extra = 40_012_345
    say("grid221k full size: one call of", n + extra)
    out3 = bm.map_points(ix, torch.cat([xy, xy[:extra]]))
    torch.cuda.synchronize()
    assert torch.equal(out3[:n], out) and torch.equal(out3[n:], out[:extra])


# ----------------------------------------------------- hard inputs ----

def _rings_index(bm, rings, n_groups=(), parents=(), keep_all_levels=False):
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    verts = np.concatenate([np.asarray(r, np.int32) for r in rings])
    return off, verts, bm.Index(off, verts, n_groups, parents, keep_all_levels=keep_all_levels)


def test_nested_squares_overflow_fallback(torch_cuda, bm):
    """600 nested squares: every point has hundreds of candidates, more than
    the per-wave lists hold, so the per-point fallback walk decides."""
    say("nested squares")
    K = 600
    rings = [[(0, 0), (10 + k, 0), (10 + k, 10 + k), (0, 10 + k)] for k in range(K)]
    rng = np.random.default_rng(2)
    pts = rng.integers(-5, 620, (20000, 2)).astype(np.int32)
    for L in (0, 1):
        off, verts, ix = _rings_index(bm, rings, [7] if L else (),
                                      [np.arange(K, dtype=np.int32) % 7] if L else ())
        got = gpu_map(bm, torch_cuda, ix, pts)
        want = oracle.brute(off, verts, pts)
        assert (got == want).all(), L
        assert (want > 300).any()
    # two group levels, the finer one thin (pairs of squares): left out by
    # default, kept on request, so the walk climbs one or two group levels
    for keep in (False, True):
        say("nested squares, thin level kept:", keep)
        pair = (np.arange(K) // 2).astype(np.int32)
        top = (np.arange(K // 2) % 7).astype(np.int32)
        off, verts, ix = _rings_index(bm, rings, [7, K // 2], [top, pair], keep_all_levels=keep)
        assert ix.info()["n_levels"] == (2 if keep else 1)
        got = gpu_map(bm, torch_cuda, ix, pts)
        assert (got == oracle.brute(off, verts, pts)).all(), keep


def test_heavy_ring_and_many_small(torch_cuda, bm):
    say("heavy ring")
    rng = np.random.default_rng(4)
    m = 20000
    ang = (np.arange(m) + rng.uniform(0.1, 0.9, m)) * 2 * np.pi / m
    rad = rng.uniform(4e5, 5e5, m)
    star = np.stack([1_000_000 + rad * np.cos(ang), 1_000_000 + rad * np.sin(ang)], 1).round().astype(np.int32)
    tri = [[(10 * i, 0), (10 * i + 9, 0), (10 * i, 9)] for i in range(100)]
    rings = [star] + tri
    off, verts, ix = _rings_index(bm, rings)
    pts = np.concatenate([rng.integers(4e5, 1.6e6, (30000, 2)), rng.integers(-2, 1001, (5000, 2)),
                          star[:2000], star[:2000] + 1]).astype(np.int32)
    got = gpu_map(bm, torch_cuda, ix, pts)
    assert (got == oracle.brute(off, verts, pts)).all()


def _comb(T=1500, H=10000, o=1000):
    """A comb: a base [0, 20(T-1)+10) x [0, 100) with T teeth [20i, 20i+10) x
    [100, H), shifted by (o, o). Every tooth edge straddles every height above
    the base, so the ring's y-slabs list ~2T edges each."""
    v = [(0, 0), (20 * (T - 1) + 10, 0)]
    for i in range(T - 1, -1, -1):
        v += [(20 * i + 10, H), (20 * i, H)]
        if i > 0:
            v += [(20 * i, 100), (20 * (i - 1) + 10, 100)]
    return np.array(v, np.int32) + o


def _comb_inside(pts, T=1500, H=10000, o=1000):
    x, y = pts[:, 0].astype(np.int64) - o, pts[:, 1].astype(np.int64) - o
    return (x >= 0) & (x < 20 * (T - 1) + 10) & (y >= 0) & (y < H) & ((y < 100) | (x % 20 < 10))


def test_long_slab_lists(torch_cuda, bm):
    """A comb of 1,500 teeth: each point inside its box pairs with slab lists
    of 3,000 edges, so a round deals tens of thousands of edge chunks over
    many windows. Equal to brute force (20k points and boundary points, edge
    chunks of 4 and 16), and a pre-sorted call of 2^20 + 100 points equal to
    the comb's closed form (which the oracle matches on the small set)."""
    torch = torch_cuda
    comb = _comb()
    off, verts, ix = _rings_index(bm, [comb])
    rng = np.random.default_rng(9)
    pts = np.stack([rng.integers(900, 31100, 20000), rng.integers(900, 11100, 20000)], 1).astype(np.int32)
    pts = np.concatenate([pts, comb, comb - 1, comb + 1]).astype(np.int32)
    want = oracle.brute(off, verts, pts)
    assert np.array_equal(want == 0, _comb_inside(pts))
    for chunk in (4, 16):
        say("comb, edge chunk", chunk)
        got = gpu_map(bm, torch, ix, pts, tuning=bm.Tuning(chunk, 3, 2048, 1))
        assert (got == want).all(), int((got != want).sum())
    n = (1 << 20) + 100
    big = np.stack([rng.integers(900, 31100, n), rng.integers(900, 11100, n)], 1).astype(np.int32)
    say("comb, pre-sorted call of", n)
    got = gpu_map(bm, torch, ix, big)
    assert np.array_equal(got, np.where(_comb_inside(big), 0, -1).astype(got.dtype))


def test_random_hierarchies_and_empty_groups(torch_cuda, bm):
    g = synth.geometry("grid1k")
    pts = np.concatenate([synth.points("grid1k", 20000), boundary_points(g, 500)])
    want = oracle.brute(g.vert_off, g.verts, pts)
    rng = np.random.default_rng(5)
    for t in range(3):
        sizes = sorted(rng.integers(1, 300, 4).tolist())
        pars = [rng.integers(0, sizes[l], sizes[l + 1]).astype(np.int32) for l in range(3)]
        pars.append(rng.integers(0, sizes[3], g.n_blocks).astype(np.int32))
        say("random hierarchy", sizes)
        ix = bm.Index(g.vert_off, g.verts, sizes, pars)
        assert (gpu_map(bm, torch_cuda, ix, pts) == want).all()
    say("flat index")
    ix = bm.Index(g.vert_off, g.verts)
    assert (gpu_map(bm, torch_cuda, ix, pts) == want).all()


@pytest.mark.parametrize("per_group", [65, 100, 200, 256, 257])
def test_wide_groups(torch_cuda, bm, per_group):
    """Groups of 65..256 children use slot tables with several 64-bit words per
    row; 257 and more have none. Children in id order (row strips) and
    scattered at random."""
    g = synth.geometry("grid1k")
    pts = np.concatenate([synth.points("grid1k", 20000), boundary_points(g, 500)])
    want = oracle.brute(g.vert_off, g.verts, pts)
    rng = np.random.default_rng(per_group)
    for name, order in [("strips", np.arange(g.n_blocks)), ("scattered", rng.permutation(g.n_blocks))]:
        parent = np.empty(g.n_blocks, np.int32)
        parent[order] = np.arange(g.n_blocks) // per_group
        say("wide groups", per_group, name)
        ix = bm.Index(g.vert_off, g.verts, [int(parent.max()) + 1], [parent])
        assert (gpu_map(bm, torch_cuda, ix, pts) == want).all()


def test_overlapping_blocks_smallest_id(torch_cuda, bm):
    say("overlaps")
    rng = np.random.default_rng(6)
    rings = []
    for k in range(300):
        x, y = rng.integers(0, 9000, 2)
        w, h = rng.integers(50, 2000, 2)
        rings.append([(x, y), (x + w, y), (x + w, y + h), (x, y + h)])
    off, verts, ix = _rings_index(bm, rings, [4], [rng.integers(0, 4, 300).astype(np.int32)])
    pts = rng.integers(-10, 11000, (50000, 2)).astype(np.int32)
    got = gpu_map(bm, torch_cuda, ix, pts)
    assert (got == oracle.brute(off, verts, pts)).all()


def test_save_load_roundtrip(torch_cuda, bm, tmp_path):
    say("save/load")
    g = synth.geometry("grid1k")
    ix = bm.Index.from_geometry(g)
    p = str(tmp_path / "grid1k.bmi")
    ix.save(p)
    ix2 = bm.Index.load(p)
    assert ix2.info()["n_blocks"] == g.n_blocks
    pts = synth.points("grid1k", 10000)
    assert (gpu_map(bm, torch_cuda, ix2, pts) == gpu_map(bm, torch_cuda, ix, pts)).all()
    with open(p, "r+b") as f:
        f.seek(12)
        f.write(b"\xff\xff\xff\x7f")
    with pytest.raises(bm.BlockmapError):
        bm.Index.load(p)


# ----------------------------------------------------------- quantiser ----

def test_quantizer_matches_reference(torch_cuda, bm):
    import json
    import os
    from oracle import pyref
    say("quantiser")
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "quantize_hand.json")))
    hand = np.array([[float(v) for v in c["lonlat"]] for c in d["cases"]])
    rng = np.random.default_rng(9)
    rnd = np.stack([rng.uniform(-181, 181, 100000), rng.uniform(-91, 91, 100000)], 1)
    ties = (rng.integers(-180 * 2**23, 180 * 2**23, (2000, 2)) / 2**23)  # exact half-steps
    ties[:, 1] /= 2
    ll = np.concatenate([hand, rnd, ties])
    out = bm.quantize_lonlat(torch_cuda.from_numpy(ll).cuda())
    torch_cuda.cuda.synchronize()
    got = out.cpu().numpy()
    assert (got[: len(hand)] == np.array([c["xy"] for c in d["cases"]])).all()
    assert (got == pyref.quantize_lonlat(ll)).all()


def test_quantized_points_map_like_the_oracle(torch_cuda, bm):
    """Quantiser and mapper chained on the device, against the oracle on the
    reference quantiser's output."""
    from oracle import pyref
    say("quantise + map")
    g = synth.geometry("grid1k")
    # a grid of blocks laid over lon/lat: scale grid1k into [2^30, 2^30 + 1e6)
    off, verts = g.vert_off, (g.verts.astype(np.int64) + 2**30).astype(np.int32)
    ix = bm.Index(off, verts, g.n_groups, g.parents)
    rng = np.random.default_rng(10)
    ll = rng.uniform(-0.01, 0.26, (50000, 2))
    xy = bm.quantize_lonlat(torch_cuda.from_numpy(ll).cuda())
    got = bm.map_points(ix, xy).cpu().numpy()
    want = oracle.brute(off, verts, pyref.quantize_lonlat(ll))
    assert (got == want).all()
    assert (want >= 0).any() and (want == -1).any()


# ------------------------------------------------------------ quadtree8m ----

QT_CHUNKS = (synth.QUADTREE["n_points"] + synth.QUADTREE["chunk"] - 1) // synth.QUADTREE["chunk"]


@pytest.fixture(scope="module")
def quadtree8m(bm, torch_cuda):
    say("quadtree8m: generating geometry, index and oracle hierarchy")
    g = synth.geometry("quadtree8m")
    return g, bm.Index.from_geometry(g), oracle.Hier.from_geometry(g)


@pytest.mark.parametrize("k", range(QT_CHUNKS))
def test_quadtree8m_chunk_every_point(torch_cuda, bm, quadtree8m, k):
    """Chunk k of the 1B-point stream over the 8M-block graded mesh (2^26
    points, one resident call as the benchmark maps it): every output equals
    the hierarchy oracle's, the partition property holds at every point, and a
    sample equals brute force. Together the chunks cover all 1B points."""
    torch = torch_cuda
    g, ix, H = quadtree8m
    q = synth.QUADTREE
    N, CH = q["n_points"], q["chunk"]
    n = min(CH, N - k * CH)
    say("quadtree8m chunk", k, "of", QT_CHUNKS, ":", n, "points")
    pts = synth.points("quadtree8m", n, i0=k * CH)
    got = bm.map_points(ix, torch.from_numpy(pts).cuda()).cpu().numpy()
    want = H.map(pts)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (k, bad.size, bad[:5], got[bad[:5]], want[bad[:5]])
    x, y = pts[:, 0], pts[:, 1]
    inside = (x >= 0) & (x < g.W) & (y >= 0) & (y < g.W)
    assert ((got >= 0) == inside).all(), k
    sub = np.random.default_rng(12 + k).choice(n, 100, replace=False)
    assert (got[sub] == oracle.brute(g.vert_off, g.verts, pts[sub], box_reject=True)).all(), k


def test_quadtree8m_one_call_over_several_chunks(torch_cuda, bm, quadtree8m):
    """One call over two chunks and a ragged tail (2^27 + 12,345 points): with
    this index's size the sort runs in 2^26-point chunks, two rounds of sort
    passes; the result equals the per-chunk calls and, on the tail, the
    oracle."""
    torch = torch_cuda
    g, ix, H = quadtree8m
    CH, extra = synth.QUADTREE["chunk"], 12_345
    xs = [torch.from_numpy(synth.points("quadtree8m", CH, i0=k * CH)).cuda() for k in range(2)]
    per = [bm.map_points(ix, x) for x in xs]
    say("quadtree8m: one call of", 2 * CH + extra)
    both = bm.map_points(ix, torch.cat([xs[0], xs[1], xs[0][:extra]]))
    torch.cuda.synchronize()
    assert torch.equal(both[:CH], per[0]) and torch.equal(both[CH:2 * CH], per[1])
    assert torch.equal(both[2 * CH:], per[0][:extra])
    tail = xs[0][:extra].cpu().numpy()
    assert (both[2 * CH:].cpu().numpy() == H.map(tail)).all()


def test_quadtree8m_adaptive_sort_bins(torch_cuda, bm, quadtree8m):
    """The 8M-block mesh's index (over 256 MB) sorts over adaptive bins: a
    32 x 32 grid of coarse cells, each cut into 4^d bins where blocks are
    dense. A pre-sorted call over points that crowd the mesh's dense part, lie
    on every possible bin border (and one unit off it) and lie outside the
    square on every side (clamped into border bins) equals the oracle; the
    census-scale grid's smaller index keeps the uniform 32 x 32 bins."""
    torch = torch_cuda
    g, ix, H = quadtree8m
    info = ix.info()
    assert info["sort_adaptive"] == 1 and 1024 < info["sort_bins"] <= 4096, info
    small = bm.Index.from_geometry(synth.geometry("grid1k")).info()
    assert small["sort_adaptive"] == 0 and small["sort_bins"] == 1024, small
    rng = np.random.default_rng(31)
    W = int(g.W)
    L = max(W - 1, 1).bit_length()
    step = 1 << (L - 11)  # the finest bin border spacing (5 coarse bits + depth 6)
    n_line = 1 << 18
    lines = rng.integers(0, W // step + 1, n_line) * step + rng.integers(-1, 2, n_line)
    other = rng.integers(-(1 << 20), W + (1 << 20), n_line)
    on_x = np.stack([lines, other], 1)
    on_y = np.stack([other[::-1], lines[::-1]], 1)
    far = rng.integers(1 << 20, 1 << 28, (1 << 17, 2))
    outside = np.concatenate([np.stack([-far[:, 0], far[:, 1] % (W + 1)], 1),
                              np.stack([W + far[:, 0], far[:, 1] % (W + 1)], 1),
                              np.stack([far[:, 1] % (W + 1), -far[:, 0]], 1),
                              np.stack([far[:, 1] % (W + 1), W + far[:, 0]], 1)])
    dense = synth.points("quadtree8m", 1 << 19, i0=123_456_789)
    pts = np.concatenate([dense, on_x, on_y, outside]).astype(np.int64)
    pts = np.clip(pts, -(1 << 31), (1 << 31) - 1).astype(np.int32)
    pts = pts[rng.permutation(len(pts))]
    say("quadtree8m adaptive bins:", len(pts), "points")
    got = bm.map_points(ix, torch.from_numpy(pts).cuda()).cpu().numpy()
    assert (got == H.map(pts)).all()


# ------------------------------------------------------- batched form ----

def _cluster_batches(g, sizes, seed):
    """One Gaussian cluster per batch (the batched workload's recipe)."""
    allp, off = synth.batch_points(g, np.asarray(sizes), first=seed * 100000)
    return [allp[off[b]:off[b + 1]] for b in range(len(sizes))]


def test_batched_equals_oracle_and_plain(torch_cuda, bm, grid221k):
    """Batches of 0 to 200k points in one persistent launch, for three tile
    sizes, through both batched calls (offsets into one concatenated array,
    and a device table of descriptors): every output equals the hierarchy
    oracle's, and the plain path's per-batch result."""
    torch = torch_cuda
    g, ix, H = grid221k
    sizes = synth.sizes(synth.key("batches10k", 2, 0), 300, 0, 0, 0, 200_000)
    sizes[:5] = [0, 1, 63, 64, 65]
    say("batched: %d batches, %d points" % (len(sizes), sizes.sum()))
    allp, off = synth.batch_points(g, np.asarray(sizes), first=100000)
    want = H.map(allp)
    xy = torch.from_numpy(allp).cuda()
    doff = torch.from_numpy(off).cuda()
    xys = [xy[off[b]:off[b + 1]] for b in range(len(sizes))]
    plain = torch.cat([bm.map_points(ix, x) for x in xys]).cpu().numpy()
    assert np.array_equal(plain, want)
    for tile in (64, 1024, 8192):
        out = torch.full((allp.shape[0],), -7, dtype=torch.int32, device="cuda")
        bm.map_batches(ix, xy, doff, out, tuning=bm.Tuning(8, 4, tile))
        outs = [torch.full((x.shape[0],), -7, dtype=torch.int32, device="cuda") for x in xys]
        bm.map_batch_table(ix, bm.batch_table(xys, outs), tuning=bm.Tuning(8, 4, tile))
        torch.cuda.synchronize()
        for name, got in (("offsets", out.cpu().numpy()), ("table", torch.cat(outs).cpu().numpy())):
            bad = np.flatnonzero(got != want)
            assert bad.size == 0, (name, tile, bad.size, bad[:5])


def test_batched_full_size_every_point(torch_cuda, bm, grid221k):
    """The batched workload at full size (10,000 batches of 1 to 1M points,
    729M points over the census-scale index), through the captured graph of
    the offset form as the benchmark replays it: every output equals the
    hierarchy oracle's."""
    torch = torch_cuda
    g, ix, H = grid221k
    sizes = synth.batch_sizes()
    say("batched full size: generating", int(sizes.sum()), "points")
    host, off = synth.batch_points(g, sizes)
    xy = torch.from_numpy(host).cuda()
    doff = torch.from_numpy(off).cuda()
    out = torch.full((host.shape[0],), -7, dtype=torch.int32, device="cuda")
    plan = bm.BatchPlan(ix, len(sizes), bm.Tuning(4, 8, 512), max_points=host.shape[0])
    plan.run_offsets(xy, doff, out)
    torch.cuda.synchronize()
    plan.close()
    got = out.cpu().numpy()
    del xy, out
    say("batched full size: oracle over every point")
    want = H.map(host)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, (bad.size, bad[:5], got[bad[:5]], want[bad[:5]])


def test_batch_plan_graph_replays(torch_cuda, bm, grid221k):
    """Both captured graphs replayed with different batches, eager work and
    syncs in between: every replay equals the plain result. The offset form
    skips batches whose offsets decrease or end beyond max_points, leaving
    their outputs untouched."""
    torch = torch_cuda
    g, ix, H = grid221k
    plan = bm.BatchPlan(ix, 64, bm.Tuning(8, 4, 512), max_points=1_000_000)
    for rep in range(4):
        sizes = synth.sizes(synth.key("batches10k", 2, 10 + rep), 10 + 13 * rep, 0, 0, 0, 50_000)
        say("plan replay", rep, len(sizes), sizes.sum())
        pts = _cluster_batches(g, sizes, 20 + rep)
        xys = [torch.from_numpy(p).cuda() for p in pts]
        outs = [torch.full((p.shape[0],), -7, dtype=torch.int32, device="cuda") for p in pts]
        plan.run(xys, outs)
        torch.cuda.synchronize()
        for xy, o in zip(xys, outs):
            assert torch.equal(bm.map_points(ix, xy), o), rep
        allp = np.concatenate(pts)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        xy = torch.from_numpy(allp).cuda()
        out = torch.full((allp.shape[0],), -7, dtype=torch.int32, device="cuda")
        plan.run_offsets(xy, torch.from_numpy(off).cuda(), out)
        torch.cuda.synchronize()
        assert torch.equal(bm.map_points(ix, xy), out), rep
    # guarded offsets: batch 1 decreases, batch 3 ends beyond max_points
    pts = synth.points("grid221k", 300_000, i0=70_000_000)
    xy = torch.from_numpy(pts).cuda()
    off = torch.tensor([0, 1000, 900, 5000, 300_000], dtype=torch.int64, device="cuda")
    small = bm.BatchPlan(ix, 8, bm.Tuning(8, 4, 512), max_points=200_000)
    out = torch.full((300_000,), -7, dtype=torch.int32, device="cuda")
    small.run_offsets(xy, off, out)
    torch.cuda.synchronize()
    ref = bm.map_points(ix, xy)
    torch.cuda.synchronize()
    assert torch.equal(out[:900], ref[:900]) and (out[900:1000] == ref[900:1000]).all()
    assert torch.equal(out[900:5000], ref[900:5000])
    assert (out[5000:] == -7).all()
    small.close()
    with pytest.raises(bm.BlockmapError):
        plan.run([xys[0]] * 65, [outs[0]] * 65)
    plan.close()


def test_autotune_never_changes_results(torch_cuda, bm, grid221k, tmp_path, monkeypatch):
    torch = torch_cuda
    g, ix, H = grid221k
    monkeypatch.setenv("BM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    pts = synth.points("grid221k", 2_000_000)
    xy = torch.from_numpy(pts).cuda()
    say("autotune")
    t = bm.autotune(ix, xy)
    assert t.edge_chunk in (4, 8) and t.blocks_per_cu in (4, 6, 8) and t.tile_points in (512, 2048, 8192)
    assert t.presort in (0, 1)
    t2 = bm.autotune(ix, xy)  # from the cache
    assert t2.as_dict() == t.as_dict()
    assert torch.equal(bm.map_points(ix, xy, tuning=t), bm.map_points(ix, xy))


# -------------------------------------------------------- served form ----

def _requests(g, sizes, seed):
    out = []
    for r, n in enumerate(sizes):
        m = synth.Mixture(synth.key("requests20k", 2, seed * 100000 + r), 1, g.W, 0.0, 0.001, 0.02, 0.2)
        out.append(m.sample(synth.key("requests20k", 3, seed * 100000 + r), 0, int(n)))
    return out


def test_server_results_same_alone_and_in_the_mix(torch_cuda, bm, grid221k):
    """Requests submitted together, coalesced into shared device batches (and
    split across batches when large), give exactly the ids each gets alone."""
    torch = torch_cuda
    g, ix, H = grid221k
    sizes = list(synth.sizes(synth.key("requests20k", 2, 0), 300, 1, 2000.0, 1.5, 300_000))
    sizes[:4] = [0, 1, 64, 250_000]
    reqs = _requests(g, sizes, 1)
    alone = [gpu_map(bm, torch, ix, p) for p in reqs]
    for cfg in (bm.server_cfg(mem_budget_bytes=64 << 20, max_batch_points=100_000, max_slots=4, n_streams=3),
                bm.server_cfg(mem_budget_bytes=12 * 70_000 + 4096, max_batch_points=70_000, max_slots=2,
                              n_streams=1, coalesce_us=200)):
        say("server mix", cfg.max_batch_points, cfg.max_slots, cfg.n_streams)
        srv = bm.Server(ix, cfg)
        outs = [np.full(p.shape[0], -7, np.int32) for p in reqs]
        tickets = [srv.submit(p, o) for p, o in zip(reqs, outs)]
        for t in tickets:
            srv.wait(t)
        st = srv.stats()
        srv.close()
        for a, o in zip(alone, outs):
            assert (a == o).all()
        assert st["completed"] == len(reqs) and st["p50_us"] <= st["p99_us"] <= st["max_us"]
        assert st["mean_requests_per_batch"] > 1.0  # requests really shared batches


@pytest.mark.parametrize("threads, direct_log2", [(1, 10), (5, 14), (8, 40)])
def test_server_pinned_buffers_copy_paths(torch_cuda, bm, grid221k, threads, direct_log2):
    """Requests and outputs in page-locked memory: pieces of at least
    direct_min_points are copied by DMA straight to and from their place in
    the device pool, the others packed and unpacked by `copy_threads` host
    threads (1: the server's own threads alone). Every request's ids equal
    those it gets alone, whatever the split."""
    torch = torch_cuda
    g, ix, H = grid221k
    sizes = list(synth.sizes(synth.key("requests20k", 2, 7), 200, 1, 3000.0, 1.5, 200_000))
    sizes[:6] = [0, 1, 1023, 1024, 16_383, 16_384]

    def pinned(a):
        t = torch.empty(a.shape, dtype=torch.int32, pin_memory=True)
        t.numpy()[...] = a
        return t.numpy()
    reqs = [pinned(p) for p in _requests(g, sizes, 4)]
    alone = [gpu_map(bm, torch, ix, p) for p in reqs]
    cfg = bm.server_cfg(mem_budget_bytes=64 << 20, max_batch_points=150_000, max_slots=4, n_streams=3,
                        copy_threads=threads, direct_min_points=1 << direct_log2)
    say("server, pinned buffers", threads, direct_log2)
    outs = [pinned(np.full(p.shape[0], -7, np.int32)) for p in reqs]
    srv = bm.Server(ix, cfg)
    tickets = [srv.submit(p, o) for p, o in zip(reqs, outs)]
    for t in tickets:
        srv.wait(t)
    st = srv.stats()
    srv.close()
    for k, (a, o) in enumerate(zip(alone, outs)):
        assert (a == o).all(), (k, sizes[k])
    assert st["completed"] == len(reqs)


def test_server_backpressure_timeout_and_failure(torch_cuda, bm, grid221k):
    g, ix, H = grid221k
    pts = _requests(g, [1000, 1000, 1000], 2)
    outs = [np.empty(1000, np.int32) for _ in pts]
    # a long coalescing window keeps the first pieces queued: the queue fills
    srv = bm.Server(ix, bm.server_cfg(queue_capacity=2, coalesce_us=300_000, max_batch_points=1 << 20))
    t1 = srv.submit(pts[0], outs[0])
    t2 = srv.submit(pts[1], outs[1])
    with pytest.raises(bm.BlockmapError) as e:
        srv.submit(pts[2], outs[2])
    assert e.value.code == bm.BM_EBUSY
    with pytest.raises(bm.BlockmapError) as e:
        srv.wait(t1, timeout_us=1000)
    assert e.value.code == bm.BM_ETIMEDOUT
    srv.wait(t1)
    srv.wait(t2)
    assert (outs[0] == gpu_map(bm, torch_cuda, ix, pts[0])).all()
    with pytest.raises(bm.BlockmapError) as e:
        srv.wait(t1)  # consumed
    assert e.value.code == bm.BM_EINVAL
    srv.close()
    with pytest.raises(bm.BlockmapError) as e:
        bm.Server(ix, bm.server_cfg(flags=bm.BM_SERVER_FAIL_ALLOC))
    assert e.value.code == bm.BM_ENOMEM
    with pytest.raises(bm.BlockmapError) as e:
        bm.Server(ix, bm.server_cfg(mem_budget_bytes=1000, max_batch_points=1000))
    assert e.value.code == bm.BM_EINVAL
    for bad in (dict(copy_threads=0), dict(copy_threads=65), dict(direct_min_points=0)):
        with pytest.raises(bm.BlockmapError) as e:
            bm.Server(ix, bm.server_cfg(**bad))
        assert e.value.code == bm.BM_EINVAL, bad


def test_server_poisson_trace(torch_cuda, bm, grid221k):
    g, ix, H = grid221k
    sizes = synth.sizes(synth.key("requests20k", 2, 7), 2000, 1, 10_000.0, 2.0, 2_000_000)
    reqs = _requests(g, sizes, 3)
    outs = [np.full(p.shape[0], -7, np.int32) for p in reqs]
    rng = np.random.default_rng(0)
    arrivals = np.cumsum(rng.exponential(1e6 / 5000.0, len(reqs)))  # 5,000 requests/s
    srv = bm.Server(ix, bm.server_cfg(mem_budget_bytes=256 << 20, max_batch_points=1 << 21))
    say("server trace", len(reqs), int(sizes.sum()))
    srv.run_trace(list(zip(reqs, outs)), arrivals)
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs)
    allp = np.concatenate(reqs)
    allo = np.concatenate(outs)
    sub = np.random.default_rng(1).choice(allp.shape[0], 50_000, replace=False)
    assert (allo[sub] == H.map(allp[sub])).all()


def test_server_over_quadtree8m_every_point(torch_cuda, bm, quadtree8m):
    """The served workload's setting: the 8M-block mesh resident in HBM,
    requests of lognormal size (median 10k points, sigma_ln 2, capped at 2M
    here), each a cluster plus 20% uniform points with its own output buffer,
    under Poisson arrivals and all at once. Every output equals the hierarchy
    oracle's, and the server really coalesced requests."""
    g, ix, H = quadtree8m
    sizes = synth.request_sizes(600, first=3, hi=2_000_000)
    reqs = [synth.request_points(g, 50_000 + r, n) for r, n in enumerate(sizes)]
    say("server over quadtree8m: %d requests, %d points; oracle" % (len(reqs), int(sizes.sum())))
    want = H.map(np.concatenate(reqs))
    rng = np.random.default_rng(3)
    cfg = bm.server_cfg(mem_budget_bytes=1 << 30, max_batch_points=1 << 22, max_slots=6, n_streams=4)
    for name, arrivals in [("poisson", np.cumsum(rng.exponential(1e6 / 4000.0, len(reqs)))),
                           ("all at once", np.zeros(len(reqs)))]:
        say("server over quadtree8m:", name)
        outs = [np.full(p.shape[0], -7, np.int32) for p in reqs]
        srv = bm.Server(ix, cfg)
        srv.run_trace(list(zip(reqs, outs)), arrivals)
        st = srv.stats()
        srv.close()
        got = np.concatenate(outs)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, (name, bad.size, bad[:5])
        assert st["completed"] == len(reqs)
        if name == "all at once":
            assert st["mean_requests_per_batch"] > 2.0


def test_server_budget_covers_presort_scratch(torch_cuda, bm, grid221k):
    """Batches of 2^20 points or more are pre-sorted, and their sort scratch
    comes out of the server's memory budget: a budget of 12 bytes per point
    alone (points and results) is refused; one that also holds the scratch
    (20 bytes per point more) serves requests of 2^21 points (pre-sorted in
    the pool) with the ids each gets alone."""
    torch = torch_cuda
    g, ix, H = grid221k
    mb = 1 << 21
    with pytest.raises(bm.BlockmapError) as e:
        bm.Server(ix, bm.server_cfg(mem_budget_bytes=12 * mb + 4096, max_batch_points=mb))
    assert e.value.code == bm.BM_EINVAL and "scratch" in str(e.value)
    sizes = [mb - 5, 1000, mb, 70_000, mb - 64]
    reqs = [synth.points("grid221k", n, i0=90_000_000 + 3_000_000 * k) for k, n in enumerate(sizes)]
    alone = [gpu_map(bm, torch, ix, p) for p in reqs]
    srv = bm.Server(ix, bm.server_cfg(mem_budget_bytes=34 * mb, max_batch_points=mb, max_slots=4, n_streams=2))
    outs = [np.full(p.shape[0], -7, np.int32) for p in reqs]
    say("server, pre-sort scratch in the budget")
    tickets = [srv.submit(p, o) for p, o in zip(reqs, outs)]
    for t in tickets:
        srv.wait(t)
    srv.close()
    for a, o in zip(alone, outs):
        assert (a == o).all()
    assert (np.concatenate(outs) == H.map(np.concatenate(reqs))).all()
