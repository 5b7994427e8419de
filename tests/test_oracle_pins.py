"""Pins for the CPU oracle: checks against facts fixed by the paper and by
geometry, not against the oracle's own formula. CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import pyref

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _lattice(x0, x1, y0, y1):
    xs, ys = np.meshgrid(np.arange(x0, x1 + 1), np.arange(y0, y1 + 1), indexing="ij")
    return np.stack([xs.ravel(), ys.ravel()], 1).astype(np.int32)


def _inside_all(ring, pts):
    """oracle.brute over a single-ring index, as a boolean per point."""
    ring = np.asarray(ring, np.int32)
    off = np.array([0, ring.shape[0]], np.int64)
    return oracle.brute(off, ring, pts) == 0


# ------------------------------------------------------------ hand cases ----

def test_hand_cases_golden():
    d = json.load(open(os.path.join(GOLD, "hand_cases.json")))
    for case in d["cases"]:
        pts = np.array([p for p, _ in case["points"]], np.int32)
        want = np.array([w for _, w in case["points"]])
        got = _inside_all(case["ring"], pts)
        assert (got == want).all(), (case["name"], pts[got != want])
        for (p, w) in case["points"]:
            assert pyref.crossing_inside(case["ring"], *p) == w, (case["name"], p)
    s = d["smallest_id"]
    rings = [np.asarray(r, np.int32) for r in s["rings"]]
    off = np.concatenate([[0], np.cumsum([r.shape[0] for r in rings])]).astype(np.int64)
    verts = np.concatenate(rings)
    pts = np.array([p for p, _ in s["points"]], np.int32)
    want = np.array([w for _, w in s["points"]], np.int32)
    assert (oracle.brute(off, verts, pts) == want).all()
    assert (oracle.brute(off, verts, pts, box_reject=True) == want).all()
    h = oracle.Hier(off, verts, [1], [np.zeros(len(rings), np.int32)])
    assert (h.map(pts) == want).all()


# ----------------------------------------------------- closed forms ----

RECTS = [(0, 10, 0, 10), (-7, 3, 5, 6), (100, 101, -50, 40), (-2**31 + 5, -2**31 + 9, 2**31 - 9, 2**31 - 2)]


@pytest.mark.parametrize("rect", RECTS)
def test_rectangle_closed_form(rect):
    """Axis-aligned rectangle: inside exactly on [x0, x1) x [y0, y1), for every
    orientation and start vertex."""
    x0, x1, y0, y1 = rect
    ccw = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    pts = _lattice(max(x0 - 2, -2**31), min(x1 + 2, 2**31 - 1), max(y0 - 2, -2**31), min(y1 + 2, 2**31 - 1))
    if pts.shape[0] > 5000:
        pts = pts[np.random.default_rng(0).choice(pts.shape[0], 5000, replace=False)]
    want = (pts[:, 0] >= x0) & (pts[:, 0] < x1) & (pts[:, 1] >= y0) & (pts[:, 1] < y1)
    for ring in (ccw, ccw[::-1]):
        for s in range(4):
            r = ring[s:] + ring[:s]
            assert (_inside_all(r, pts) == want).all(), (rect, r)


# rectilinear shapes as (ring, disjoint half-open rectangles covering the region)
RECTILINEAR = {
    "L": ([(0, 0), (20, 0), (20, 5), (5, 5), (5, 20), (0, 20)],
          [(0, 20, 0, 5), (0, 5, 5, 20)]),
    "U": ([(0, 0), (30, 0), (30, 30), (20, 30), (20, 10), (10, 10), (10, 30), (0, 30)],
          [(0, 30, 0, 10), (0, 10, 10, 30), (20, 30, 10, 30)]),
    "comb": ([(0, 0), (25, 0), (25, 20), (20, 20), (20, 5), (15, 5), (15, 20), (10, 20), (10, 5),
              (5, 5), (5, 20), (0, 20)],
             [(0, 25, 0, 5), (0, 5, 5, 20), (10, 15, 5, 20), (20, 25, 5, 20)]),
    "spiral": ([(0, 0), (30, 0), (30, 30), (0, 30), (0, 10), (20, 10), (20, 20), (10, 20), (10, 15),
                (15, 15), (15, 17), (17, 17), (17, 13), (5, 13), (5, 25), (25, 25), (25, 5), (0, 5)],
               [(0, 30, 0, 5), (25, 30, 5, 25), (0, 30, 25, 30), (0, 5, 10, 25), (5, 20, 10, 13),
                (17, 20, 13, 20), (10, 17, 17, 20), (10, 15, 15, 17)]),
}


@pytest.mark.parametrize("name", sorted(RECTILINEAR))
def test_rectilinear_closed_form(name):
    ring, rects = RECTILINEAR[name]
    pts = _lattice(-2, 32, -2, 32)
    want = np.zeros(pts.shape[0], bool)
    for (x0, x1, y0, y1) in rects:
        m = (pts[:, 0] >= x0) & (pts[:, 0] < x1) & (pts[:, 1] >= y0) & (pts[:, 1] < y1)
        assert not (want & m).any(), "rectangles must be disjoint"
        want |= m
    for r in (ring, ring[::-1], ring[3:] + ring[:3]):
        assert (_inside_all(r, pts) == want).all(), name


def _star(rng, m, cx, cy, r0, r1):
    ang = (np.arange(m) + rng.uniform(0.1, 0.9, m)) * 2 * math.pi / m
    rad = rng.uniform(r0, r1, m)
    return [(int(round(cx + r * math.cos(a))), int(round(cy + r * math.sin(a)))) for a, r in zip(ang, rad)]


NONRECT = {
    "star": [(0, 30), (7, 9), (29, 9), (11, -4), (18, -25), (0, -12), (-18, -25), (-11, -4), (-29, 9), (-7, 9)],
    "chevron": [(0, 0), (10, 8), (20, 0), (20, 6), (10, 17), (0, 6)],
    "notched triangle": [(0, 0), (24, 0), (12, 21), (12, 9), (9, 15)],
    "self-touching bowtie": [(0, 0), (10, 10), (20, 0), (20, 20), (10, 10), (0, 20)],
}


@pytest.mark.parametrize("name", sorted(NONRECT))
def test_exact_rational_reference(name):
    ring = NONRECT[name]
    xs = [p[0] for p in ring]
    ys = [p[1] for p in ring]
    pts = _lattice(min(xs) - 2, max(xs) + 2, min(ys) - 2, max(ys) + 2)
    want = np.array([pyref.crossing_inside(ring, int(x), int(y)) for x, y in pts])
    assert want.any() and not want.all()
    assert (_inside_all(ring, pts) == want).all()


def test_random_star_polygons_rational_and_winding():
    """Random simple (star-shaped) rings: the oracle equals the exact rational
    evaluation, and equals 'winding number != 0' (independent formula)."""
    rng = np.random.default_rng(11)
    for t in range(40):
        m = int(rng.integers(3, 40))
        ring = _star(rng, m, 0, 0, 300, 3000)
        pts = np.stack([rng.integers(-3200, 3200, 400), rng.integers(-3200, 3200, 400)], 1).astype(np.int32)
        pts = np.concatenate([pts, np.asarray(ring, np.int32)])  # vertices themselves
        got = _inside_all(ring, pts)
        want = np.array([pyref.crossing_inside(ring, int(x), int(y)) for x, y in pts])
        wn = np.array([pyref.winding_number(ring, int(x), int(y)) for x, y in pts])
        assert (got == want).all(), t
        assert (got == (wn != 0)).all(), t
        assert set(np.unique(wn)) <= {0, 1}  # counter-clockwise simple ring


def test_box_is_conservative():
    """inside(ring, p) implies p in the half-open box [min x, max x) x [min y, max y)."""
    rng = np.random.default_rng(5)
    for t in range(30):
        ring = np.asarray(_star(rng, int(rng.integers(3, 30)), 50, -20, 10, 500), np.int32)
        pts = np.stack([rng.integers(-600, 700, 3000), rng.integers(-700, 600, 3000)], 1).astype(np.int32)
        pts = np.concatenate([pts, ring, ring + 1, ring - 1])
        box = oracle.ring_boxes(np.array([0, ring.shape[0]]), ring)[0]
        inb = (pts[:, 0] >= box[0]) & (pts[:, 0] < box[1]) & (pts[:, 1] >= box[2]) & (pts[:, 1] < box[3])
        got = _inside_all(ring, pts)
        assert not (got & ~inb).any()
        assert got.any()


# --------------------------------------------------------- metamorphic ----

def test_metamorphic_invariances():
    rng = np.random.default_rng(3)
    for t in range(20):
        ring = _star(rng, int(rng.integers(4, 25)), 0, 0, 200, 2000)
        pts = np.stack([rng.integers(-2100, 2100, 800), rng.integers(-2100, 2100, 800)], 1).astype(np.int32)
        pts = np.concatenate([pts, np.asarray(ring, np.int32)])
        base = _inside_all(ring, pts)
        dx, dy = int(rng.integers(-10**6, 10**6)), int(rng.integers(-10**6, 10**6))
        shifted = [(x + dx, y + dy) for x, y in ring]
        assert (_inside_all(shifted, pts + np.array([dx, dy], np.int32)) == base).all(), "translation"
        s = int(rng.integers(2, 50))
        assert (_inside_all([(x * s, y * s) for x, y in ring], pts * s) == base).all(), "scaling"
        assert (_inside_all(ring[::-1], pts) == base).all(), "reversal"
        k = int(rng.integers(1, len(ring)))
        assert (_inside_all(ring[k:] + ring[:k], pts) == base).all(), "start vertex"
        dup = ring[:k] + [ring[k]] + ring[k:]
        assert (_inside_all(dup, pts) == base).all(), "duplicated vertex"
        closed = ring + [ring[0]]
        assert (_inside_all(closed, pts) == base).all(), "stored closing vertex"
        # exactly collinear midpoint (scale by 2 so the midpoint is integral)
        r2 = [(2 * x, 2 * y) for x, y in ring]
        a, b = r2[k - 1], r2[k]
        mid = ((a[0] + b[0]) // 2, (a[1] + b[1]) // 2)
        r3 = r2[:k] + [mid] + r2[k:]
        assert (_inside_all(r3, pts * 2) == base).all(), "collinear vertex"


def test_block_permutation():
    g = synth.geometry("grid1k")
    pts = synth.points("grid1k", 3000)
    base = oracle.brute(g.vert_off, g.verts, pts)
    rng = np.random.default_rng(9)
    perm = rng.permutation(g.n_blocks)  # new block q holds old block perm[q]
    rings = [g.verts[g.vert_off[b]:g.vert_off[b + 1]] for b in perm]
    off = np.concatenate([[0], np.cumsum([r.shape[0] for r in rings])]).astype(np.int64)
    got = oracle.brute(off, np.concatenate(rings), pts)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    want = np.where(base >= 0, inv[np.maximum(base, 0)], -1)
    assert (got == want).all()  # the partition has no overlaps, so the id is unique


# ----------------------------------------- partitions and hierarchy ----

def test_unjittered_grid_closed_form():
    """No jitter: every block is the square cell [i c, (i+1) c) x [j c, (j+1) c)
    (extra vertices on its sides are collinear), so id = floor(y/c)*n + floor(x/c)."""
    n, c = 12, 1000
    off, verts = synth.jittered_grid(n, c, kmin=1, kmax=5, vjit=0.0, pjit=0.0, key_=77)
    W = n * c
    rng = np.random.default_rng(1)
    pts = rng.integers(-300, W + 300, (20000, 2)).astype(np.int32)
    corners = np.stack(np.meshgrid(np.arange(0, W + 1, c), np.arange(0, W + 1, c)), -1).reshape(-1, 2)
    near = (corners[:, None, :] + np.array([[0, 0], [-1, 0], [0, -1], [-1, -1], [1, 1], [0, 1], [1, 0]])).reshape(-1, 2)
    pts = np.concatenate([pts, near]).astype(np.int32)
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    inside = (x >= 0) & (x < W) & (y >= 0) & (y < W)
    want = np.where(inside, (y // c) * n + (x // c), -1)
    assert (oracle.brute(off, verts, pts) == want).all()
    ng, par = synth.band_hierarchy(n, [(2, 3), (4, 6)])
    assert (oracle.Hier(off, verts, ng, par).map(pts) == want).all()


@pytest.mark.parametrize("workload", ["grid1k", "grid221k"])
def test_partition_invariant(workload):
    """Watertight partition of [0, W)^2: a point inside the square lies in exactly
    one block, a point outside in none."""
    g = synth.geometry(workload)
    pts = synth.points(workload, 100_000 if workload == "grid1k" else 2000)
    # extra points on the hull, its corners and grid vertices
    W = g.W
    edge = np.array([[0, 5], [5, 0], [W - 1, 7], [7, W - 1], [W, 3], [3, W], [0, 0], [W - 1, W - 1],
                     [W, W], [-1, 0], [0, -1]], np.int32)
    v = g.verts[np.random.default_rng(2).choice(g.verts.shape[0], 400, replace=False)]
    pts = np.concatenate([pts, edge, v, v + 1, v - 1]).astype(np.int32)
    out, hits = oracle.brute(g.vert_off, g.verts, pts, box_reject=(workload != "grid1k"), count_hits=True)
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    inside = (x >= 0) & (x < W) & (y >= 0) & (y < W)
    assert (hits[inside] == 1).all()
    assert (hits[~inside] == 0).all()
    assert ((out >= 0) == inside).all()


def test_overlapping_rectangles_smallest_id():
    """Overlapping axis-aligned rectangles (not a partition): containment has a
    closed form (the half-open box), so the answer at every point is the
    smallest id among the rectangles whose box holds it, or -1. Both routes,
    with and without box rejection, under a random grouping."""
    rng = np.random.default_rng(21)
    m = 200
    x0 = rng.integers(0, 900, m)
    y0 = rng.integers(0, 900, m)
    x1 = x0 + rng.integers(1, 300, m)
    y1 = y0 + rng.integers(1, 300, m)
    rings = [np.array([[a, c], [b, c], [b, d], [a, d]], np.int32) for a, b, c, d in zip(x0, x1, y0, y1)]
    off = np.concatenate([[0], np.cumsum([4] * m)]).astype(np.int64)
    verts = np.concatenate(rings)
    pts = np.concatenate([rng.integers(-5, 1250, (20_000, 2)),
                          np.stack([x0, y0], 1), np.stack([x1 - 1, y1 - 1], 1), np.stack([x1, y0], 1)]).astype(np.int32)
    px, py = pts[:, :1].astype(np.int64), pts[:, 1:].astype(np.int64)
    hit = (x0 <= px) & (px < x1) & (y0 <= py) & (py < y1)
    want = np.where(hit.any(1), hit.argmax(1), -1)
    assert (oracle.brute(off, verts, pts) == want).all()
    assert (oracle.brute(off, verts, pts, box_reject=True) == want).all()
    ids, hits = oracle.brute(off, verts, pts, count_hits=True)  # scans every block
    assert (ids == want).all() and (hits == hit.sum(1)).all()
    g = rng.integers(0, 7, m).astype(np.int32)
    assert (oracle.Hier(off, verts, [7], [g]).map(pts) == want).all()


def test_hier_equals_brute_grid1k():
    g = synth.geometry("grid1k")
    pts = synth.points("grid1k")
    want = oracle.brute(g.vert_off, g.verts, pts)
    got, cnt = oracle.Hier.from_geometry(g).map(pts, with_counts=True)
    assert (got == want).all()
    assert cnt["hits"] == int((want >= 0).sum())


def test_hier_equals_brute_grid221k_sample():
    g = synth.geometry("grid221k")
    pts = synth.points("grid221k", 200_000)
    got = oracle.Hier.from_geometry(g).map(pts)
    sub = np.random.default_rng(4).choice(pts.shape[0], 1500, replace=False)
    want = oracle.brute(g.vert_off, g.verts, pts[sub], box_reject=True)
    assert (got[sub] == want).all()


def test_hier_any_grouping_is_exact():
    """Group boxes are unions of their children's boxes, so the hierarchy never
    loses a containing block, whatever the grouping: random regroupings and
    extra levels give the definition's answer."""
    g = synth.geometry("grid1k")
    pts = synth.points("grid1k", 20000)
    want = oracle.brute(g.vert_off, g.verts, pts)
    rng = np.random.default_rng(6)
    for t in range(4):
        G1 = int(rng.integers(1, 40))
        G0 = int(rng.integers(1, G1 + 1))
        par_blocks = rng.integers(0, G1, g.n_blocks).astype(np.int32)
        par_groups = rng.integers(0, G0, G1).astype(np.int32)
        got = oracle.Hier(g.vert_off, g.verts, [G0, G1], [par_groups, par_blocks]).map(pts)
        assert (got == want).all()
    assert (oracle.Hier(g.vert_off, g.verts, [], []).map(pts) == want).all()


# ----------------------------------------------------------- quantiser ----

def test_quantizer_hand_values():
    d = json.load(open(os.path.join(GOLD, "quantize_hand.json")))
    ll = np.array([[float(v) for v in c["lonlat"]] for c in d["cases"]])
    want = np.array([c["xy"] for c in d["cases"]], np.int32)
    assert (pyref.quantize_lonlat(ll) == want).all()


def test_quantizer_monotone_and_resolution():
    rng = np.random.default_rng(8)
    lon = np.sort(rng.uniform(-180, 180, 20000))
    lat = np.sort(rng.uniform(-90, 90, 20000))
    q = pyref.quantize_lonlat(np.stack([lon, lat], 1)).astype(np.int64)
    assert (np.diff(q[:, 0]) >= 0).all() and (np.diff(q[:, 1]) >= 0).all()
    back = (q - 2**30) / 2**22
    assert np.abs(back[:, 0] - lon).max() <= 2.0**-23
    assert np.abs(back[:, 1] - lat).max() <= 2.0**-23


# ------------------------------------------------------- work counters ----
#
# The hierarchy route counts its work (Sec. III's box tests level by level,
# Sec. III-A's edge tests), and those counts price the method per point. On a
# sheared grid every count has a closed form: cell (i, j) is the
# parallelogram with corners (i c + j s, j c), ((i+1) c + j s, j c),
# ((i+1) c + (j+1) s, (j+1) c), (i c + (j+1) s, (j+1) c), each side cut into
# k + 1 equal collinear pieces. Its half-open box is
# [i c + j s, (i+1) c + (j+1) s) x [j c, (j+1) c); a group of g x g cells has
# the same shape with c, s scaled by g.

SHEAR = dict(n=24, c=600, s=240, k=2, mid=3, top=2)  # c and s divisible by k + 1


def _sheared_grid(n, c, s, k, mid, top):
    rings = []
    for j in range(n):
        for i in range(n):
            A = (i * c + j * s, j * c)
            B = ((i + 1) * c + j * s, j * c)
            Cc = ((i + 1) * c + (j + 1) * s, (j + 1) * c)
            D = (i * c + (j + 1) * s, (j + 1) * c)
            ring = []
            for P, Q in ((A, B), (B, Cc), (Cc, D), (D, A)):
                for q in range(k + 1):  # P and the k interior points of side P->Q
                    ring.append((P[0] + (Q[0] - P[0]) * q // (k + 1), P[1] + (Q[1] - P[1]) * q // (k + 1)))
            rings.append(ring)
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    verts = np.asarray([v for r in rings for v in r], np.int32)
    nm, nt = n // mid, n // (mid * top)
    jj, ii = np.divmod(np.arange(n * n), n)
    par_cells = ((jj // mid) * nm + ii // mid).astype(np.int32)
    mj, mi = np.divmod(np.arange(nm * nm), nm)
    par_mid = ((mj // top) * nt + mi // top).astype(np.int32)
    return off, verts, [nt * nt, nm * nm], [par_mid, par_cells]


def _boxes_holding(px, py, C, S, nI, nJ):
    """Number of boxes [I C + J S, (I+1) C + (J+1) S) x [J C, (J+1) C),
    0 <= I < nI, 0 <= J < nJ, that hold each point, and the first such I."""
    J = py // C
    lo = (px - (J + 1) * S) // C  # smallest I with (I+1) C + (J+1) S > px
    hi = (px - J * S) // C        # largest I with I C + J S <= px
    lo_c, hi_c = np.maximum(lo, 0), np.minimum(hi, nI - 1)
    cnt = np.where((py >= 0) & (J < nJ), np.maximum(hi_c - lo_c + 1, 0), 0)
    return cnt, lo_c


def _closed_form_counts(pts, n, c, s, k, mid, top):
    px, py = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    nm, nt = n // mid, n // (mid * top)
    top_hit, _ = _boxes_holding(px, py, c * mid * top, s * mid * top, nt, nt)
    mid_hit, _ = _boxes_holding(px, py, c * mid, s * mid, nm, nm)
    leaf, first = _boxes_holding(px, py, c, s, n, n)
    m = 4 * (k + 1)
    bbox = nt * nt + top * top * top_hit + mid * mid * mid_hit
    # one piece of each slanted side straddles the point's row: piece q of
    # the left side of cell i spans x in [i c + j s + q s', i c + j s + (q+1) s']
    sp = s // (k + 1)
    j = py // c
    q = (py - j * c) * (k + 1) // c
    xamb = np.zeros_like(px)
    for d in range(2):  # s < c: at most two candidate cells per point
        i = first + d
        valid = d < leaf
        for side in (0, 1):  # left side of cell i, then its right side
            lo = (i + side) * c + j * s + q * sp
            xamb += (valid & (lo <= px) & (px < lo + sp)).astype(np.int64)
    inside = (py >= 0) & (py < n * c) & (px * c >= py * s) & (px * c < py * s + n * c * c)
    return {"bbox_tests": bbox, "leaf_cands": leaf, "edge_tests": leaf * m, "straddles": 2 * leaf,
            "x_ambiguous": xamb, "hits": inside.astype(np.int64)}


def _shear_points(n, c, s, **_):
    rng = np.random.default_rng(31)
    W = n * c + n * s
    pts = rng.integers(-200, W + 200, (6000, 2))
    pts[:, 1] = rng.integers(-200, n * c + 200, 6000)
    # lattice corners, interior side points and their neighbours
    jj, ii = np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij")
    corner = np.stack([ii * c + jj * s, jj * c], -1).reshape(-1, 2)
    near = (corner[:, None, :] + np.array([[0, 0], [-1, 0], [0, -1], [1, 0], [0, 1], [1, 1], [-1, -1]])).reshape(-1, 2)
    piece = corner[:, None, :] + np.array([[s // 3, c // 3], [s // 3 - 1, c // 3], [2 * s // 3, 2 * c // 3]])
    return np.concatenate([pts, near, piece.reshape(-1, 2)]).astype(np.int32)


def test_hierarchy_work_counts_closed_form():
    """Every counter of the hierarchy route (box tests at each level, blocks
    reaching the crossing test, ring edges examined, straddling edges, edges
    whose x-range holds the point, hits) equals its closed form on a sheared
    grid, point by point on a sample and in total over all points."""
    off, verts, ng, par = _sheared_grid(**SHEAR)
    pts = _shear_points(**SHEAR)
    want = _closed_form_counts(pts, **SHEAR)
    H = oracle.Hier(off, verts, ng, par)
    ids, tot = H.map(pts, with_counts=True)
    for key, arr in want.items():
        assert tot[key] == int(arr.sum()), (key, tot[key], int(arr.sum()))
    assert (want["x_ambiguous"] > 0).sum() > 100 and (want["leaf_cands"] == 2).sum() > 100
    sub = np.random.default_rng(2).choice(pts.shape[0], 400, replace=False)
    for i in sub:
        _, one = H.map(pts[i:i + 1], with_counts=True)
        for key, arr in want.items():
            assert one[key] == int(arr[i]), (key, pts[i], one[key], int(arr[i]))
    assert ((ids >= 0) == (want["hits"] == 1)).all()


# ------------------------------------------------- per-block aggregation ----

def test_count_and_join_per_block_closed_form():
    """On the un-jittered grid, a lattice of q x q points inside every cell puts
    exactly q^2 points in each block, and points outside land in the last
    entry; a per-block code table joined per point gives the code of the
    point's cell, floor(y/c) * 1000 + floor(x/c), or the fill value."""
    n, c, q = 10, 1000, 3
    off, verts = synth.jittered_grid(n, c, kmin=1, kmax=4, vjit=0.0, pjit=0.0, key_=5)
    u = (np.arange(q) * (c // q) + 7)
    cx, cy = np.meshgrid(np.arange(n) * c, np.arange(n) * c)
    ux, uy = np.meshgrid(u, u)
    lattice = np.stack([(cx.ravel()[:, None] + ux.ravel()[None]).ravel(),
                        (cy.ravel()[:, None] + uy.ravel()[None]).ravel()], 1)
    outside = np.array([[-1, 5], [n * c, 3], [4, n * c], [-7, -7], [n * c + 9, n * c + 9]])
    pts = np.concatenate([lattice, outside]).astype(np.int32)
    pts = pts[np.random.default_rng(3).permutation(pts.shape[0])]
    ids = oracle.brute(off, verts, pts)
    counts = oracle.count_per_block(ids, n * n)
    assert (counts[:-1] == q * q).all() and counts[-1] == outside.shape[0]
    assert counts.sum() == pts.shape[0]
    # accumulation: a second call adds
    ids2 = np.array([0, 0, -1, n * n, 5], np.int32)
    c2 = oracle.count_per_block(ids2, n * n)
    assert c2[0] == 2 and c2[5] == 1 and c2[-1] == 2 and c2.sum() == 5
    table = np.array([(b // n) * 1000 + b % n for b in range(n * n)], np.int64)
    got = oracle.join_per_block(ids, table, fill=-99)
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    ins = (x >= 0) & (x < n * c) & (y >= 0) & (y < n * c)
    assert (got == np.where(ins, (y // c) * 1000 + x // c, -99)).all()
