"""The host-side index builder without a GPU: the file written by
bm_index_build_file is parsed here and its derived structures are checked
against their definitions (half-open boxes, unions, children ranges, slot
tables as supersets, y-slab edge lists as supersets of the straddling
edges, per-leaf cell maps whose In and Out cells hold the oracle's answer at
every point)."""
import numpy as np
import pytest

import oracle
import synth


GROUP = np.dtype([("box", np.int32, 4), ("child", np.int32, 4)])
LEAF = np.dtype([("box", np.int32, 4), ("ent", np.int64), ("leaf_id", np.int32), ("packed", np.int32),
                 ("off", np.uint8, 32), ("cell", np.uint32, 16)])
assert LEAF.itemsize == 128
EXT = 1 << 24


def read_index(path):
    with open(path, "rb") as f:
        buf = f.read()
    assert buf[:8] == b"BMIDX003"
    sc = np.frombuffer(buf, np.int32, 12, 8)
    pos = 8 + 48 + 8
    out = {"n_verts": int(np.frombuffer(buf, np.int64, 1, 56)[0])}
    for name, dt, w in [("grp", GROUP, 1), ("leaf", LEAF, 1), ("ent", np.int32, 4), ("slot_mask", np.uint64, 1),
                        ("parent", np.int32, 1)]:
        n = int(np.frombuffer(buf, np.int64, 1, pos)[0])
        pos += 8
        a = np.frombuffer(buf, dt, n * w, pos)
        pos += a.nbytes
        out[name] = a.reshape(n, w) if w > 1 else a
    assert pos == len(buf)
    out.update(n_levels=int(sc[0]), g0=int(sc[1]), leaf_base=int(sc[2]), n_leaves=int(sc[3]),
               root_child=sc[4:8].copy(), root_box=sc[8:12].copy())
    lb = out["leaf_base"]
    out["box"] = np.concatenate([out["grp"]["box"], out["leaf"]["box"]]) if lb else out["leaf"]["box"]
    out["child"] = out["grp"]["child"]
    return out


def slab_of(ix, nb, py):
    """Entries (a.x, a.y, b.x, b.y) listed for height py in leaf nb."""
    r = ix["leaf"][nb]
    sh, logK = int(r["packed"]) & 0xFF, (int(r["packed"]) >> 8) & 0xFF
    K = 1 << logK
    s = (int(py) - int(r["box"][2])) >> sh
    assert 0 <= s < K
    if int(r["packed"]) & EXT:
        nq = (K + 1 + 3) // 4
        offs = ix["ent"][int(r["ent"]) - nq:int(r["ent"])].ravel().view(np.uint32)[:K + 1]
    else:
        offs = r["off"][:K + 1]
    e0 = int(r["ent"])
    return ix["ent"][e0 + int(offs[s]):e0 + int(offs[s + 1])]


@pytest.fixture(scope="module")
def grid221k_index(tmp_path_factory):
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid221k")
    p = str(tmp_path_factory.mktemp("idx") / "c2.bmi")
    bm.build_index_file(p, g.vert_off, g.verts, g.n_groups, g.parents)
    return g, read_index(p)


def test_structure_and_boxes(grid221k_index):
    g, ix = grid221k_index
    B, lb = ix["n_leaves"], ix["leaf_base"]
    # the tract level (about 3 blocks per tract) is left out: each county holds
    # the blocks of its tracts
    assert B == g.n_blocks and lb == g.n_groups[0] + g.n_groups[1] and ix["g0"] == g.n_groups[0]
    county_of_block = g.parents[1][g.parents[2]]
    per_county = ix["child"][g.n_groups[0]:lb, 1] - ix["child"][g.n_groups[0]:lb, 0]
    assert np.array_equal(np.sort(per_county), np.sort(np.bincount(county_of_block, minlength=g.n_groups[1])))
    assert ix["n_verts"] == g.verts.shape[0]
    # leaf ids are a permutation; leaf boxes are the ring extents (oracle's own)
    lid = ix["leaf"]["leaf_id"]
    assert np.array_equal(np.sort(lid), np.arange(B))
    want = oracle.ring_boxes(g.vert_off, g.verts)[lid]
    assert np.array_equal(ix["leaf"]["box"], want)
    # children ranges are contiguous, consecutive and consistent with parents
    child = ix["child"]
    for gnode in np.random.default_rng(1).choice(lb, 300, replace=False):
        c0, c1 = child[gnode, 0], child[gnode, 1]
        assert np.all(ix["parent"][c0:c1] == gnode)
        # group box = smallest box holding the children's boxes
        cb = ix["box"][c0:c1]
        assert np.array_equal(ix["box"][gnode], [cb[:, 0].min(), cb[:, 1].max(), cb[:, 2].min(), cb[:, 3].max()])
    # every level's children ranges tile the next level in order
    starts = child[:, 0]
    assert np.all(starts[1:] >= starts[:-1])


@pytest.mark.parametrize("top, kept", [(4, False), (2, True)])
def test_thin_levels(tmp_path, top, kept):
    """A group level whose groups hold fewer than 4 children on average is left
    out (its parents adopt the children) unless a parent would then hold more
    than 256 children. 1,024 blocks in 400 groups of ~2.6 under `top` groups:
    with 4 top groups each adopts 256 blocks; with 2 each would get 512."""
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    mid = (np.arange(g.n_blocks) * 400 // g.n_blocks).astype(np.int32)
    up = (np.arange(400) * top // 400).astype(np.int32)
    p = str(tmp_path / "t.bmi")
    bm.build_index_file(p, g.vert_off, g.verts, [top, 400], [up, mid])
    ix = read_index(p)
    assert ix["g0"] == top and ix["leaf_base"] == (top + 400 if kept else top)
    child = ix["child"][:top]
    if not kept:
        assert np.all(child[:, 1] - child[:, 0] == g.n_blocks // top) and np.all(child[:, 0] >= top)
        assert np.all(child[:, 2] >= 0)  # 256 children: still a slot table


def test_keep_all_levels(tmp_path):
    """keep_all_levels keeps a thin level: the 220,900-block grid's tracts
    (~3 blocks each) stay as a level of their own between counties and blocks,
    and every group's children are the entities the caller assigned to it."""
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid221k")
    p = str(tmp_path / "k.bmi")
    bm.build_index_file(p, g.vert_off, g.verts, g.n_groups, g.parents, keep_all_levels=True)
    ix = read_index(p)
    sizes = [int(s) for s in g.n_groups]
    assert ix["n_levels"] == len(sizes) == 3
    assert ix["g0"] == sizes[0] and ix["leaf_base"] == sum(sizes)
    # the tracts: node ids [s0 + s1, s0 + s1 + s2), their children are blocks
    t0 = sizes[0] + sizes[1]
    tr = ix["child"][t0:t0 + sizes[2]]
    assert tr[:, 0].min() >= ix["leaf_base"] and tr[:, 1].max() == ix["leaf_base"] + g.n_blocks
    assert int((tr[:, 1] - tr[:, 0]).sum()) == g.n_blocks
    # the blocks under one tract are the ones whose parent is that tract
    lid = ix["leaf"]["leaf_id"]
    node_of_tract = {}
    for k in range(0, sizes[2], 997):
        blocks = lid[tr[k, 0] - ix["leaf_base"]:tr[k, 1] - ix["leaf_base"]]
        parents = set(int(t) for t in g.parents[2][blocks])
        assert len(parents) <= 1
        if parents:
            node_of_tract[parents.pop()] = k
    assert len(node_of_tract) > 50
    # the default build leaves the tracts out
    p2 = str(tmp_path / "d.bmi")
    bm.build_index_file(p2, g.vert_off, g.verts, g.n_groups, g.parents)
    assert read_index(p2)["n_levels"] == 2


def _table_candidates(ix, crec, gbox, px, py):
    """Candidate set of a point from a group's slot table, as one Python int
    (bit k = child k): x-rows then y-rows of W words each."""
    c0, c1, off, packed = (int(v) for v in crec)
    logS, shx, shy, W = packed & 0xFF, (packed >> 8) & 0xFF, (packed >> 16) & 0xFF, (packed >> 24) & 0xFF
    assert W == (c1 - c0 + 63) // 64
    S = 1 << logS
    sx, sy = (px - int(gbox[0])) >> shx, (py - int(gbox[2])) >> shy
    if not (0 <= sx < S and 0 <= sy < S):
        return 0
    mx = sum(int(ix["slot_mask"][off + sx * W + w]) << (64 * w) for w in range(W))
    my = sum(int(ix["slot_mask"][off + (S + sy) * W + w]) << (64 * w) for w in range(W))
    return mx & my


def test_slot_tables_are_supersets(grid221k_index):
    g, ix = grid221k_index
    rng = np.random.default_rng(2)
    groups = [(ix["root_child"], ix["root_box"])]
    tabbed = np.flatnonzero(ix["child"][:, 2] >= 0)
    assert tabbed.size > 3000  # regions and counties carry tables
    groups += [(ix["child"][k], ix["box"][k]) for k in rng.choice(tabbed, 400, replace=False)]
    for crec, gb in groups:
        c0, c1 = int(crec[0]), int(crec[1])
        assert int(crec[2]) >= 0
        for _ in range(40):
            px = int(rng.integers(gb[0], gb[1]))
            py = int(rng.integers(gb[2], gb[3]))
            cand = _table_candidates(ix, crec, gb, px, py)
            cb = ix["box"][c0:c1]
            inside = (cb[:, 0] <= px) & (px < cb[:, 1]) & (cb[:, 2] <= py) & (py < cb[:, 3])
            for k in np.flatnonzero(inside):
                assert cand >> int(k) & 1
            assert cand >> (c1 - c0) == 0


def _check_tables(ix, groups, rng, tries=40):
    for crec, gb in groups:
        c0, c1 = int(crec[0]), int(crec[1])
        assert int(crec[2]) >= 0
        for _ in range(tries):
            px = int(rng.integers(gb[0], gb[1]))
            py = int(rng.integers(gb[2], gb[3]))
            cand = _table_candidates(ix, crec, gb, px, py)
            cb = ix["box"][c0:c1]
            inside = (cb[:, 0] <= px) & (px < cb[:, 1]) & (cb[:, 2] <= py) & (py < cb[:, 3])
            for k in np.flatnonzero(inside):
                assert cand >> int(k) & 1
            assert cand >> (c1 - c0) == 0


@pytest.mark.parametrize("per_group", [200, 1024])
def test_slot_tables_with_several_words_per_row(tmp_path, per_group):
    """Groups of 65..256 children keep a table whose rows hold one 64-bit word
    per 64 children; larger groups have none (their children are all tested)."""
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    parent = (np.arange(g.n_blocks) // per_group).astype(np.int32)
    ng = int(parent.max()) + 1
    p = str(tmp_path / "w.bmi")
    bm.build_index_file(p, g.vert_off, g.verts, [ng], [parent])
    ix = read_index(p)
    child = ix["child"][:ng]
    m = child[:, 1] - child[:, 0]
    has = child[:, 2] >= 0
    assert np.array_equal(has, (m >= 2) & (m <= 256))
    rng = np.random.default_rng(per_group)
    _check_tables(ix, [(child[k], ix["box"][k]) for k in np.flatnonzero(has)], rng, tries=300)


def test_slot_tables_of_small_groups(tmp_path):
    """Groups of up to 8 children get 8 slots per axis, up to 16 get 16, larger
    ones 128; every table starts on a 128-byte boundary, tables do not overlap,
    and each is a superset of the children containing a point. 1,024 blocks in
    consecutive groups of 2..40."""
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    sizes, left = [], g.n_blocks
    rng = np.random.default_rng(11)
    while left > 0:
        k = min(left, int(rng.integers(2, 41)))
        sizes.append(k)
        left -= k
    parent = np.repeat(np.arange(len(sizes)), sizes).astype(np.int32)
    p = str(tmp_path / "s.bmi")
    bm.build_index_file(p, g.vert_off, g.verts, [len(sizes)], [parent])
    ix = read_index(p)
    child = ix["child"][:len(sizes)]
    m = child[:, 1] - child[:, 0]
    has = child[:, 2] >= 0
    assert np.array_equal(has, m >= 2)
    logS = child[:, 3] & 0xFF
    assert np.array_equal(logS[has], np.where(m[has] <= 8, 3, np.where(m[has] <= 16, 4, 7)))
    assert {3, 4, 7} <= set(logS[has].tolist())
    off = child[has, 2].astype(np.int64)
    assert np.all(off % 16 == 0)
    span = 2 * (1 << logS[has].astype(np.int64))  # words: one per row (W = 1)
    order = np.argsort(off)
    assert np.all(off[order][:-1] + span[order][:-1] <= off[order][1:])
    _check_tables(ix, [(child[k], ix["box"][k]) for k in np.flatnonzero(has)], rng, tries=300)


def test_y_slabs_list_every_straddling_edge(grid221k_index):
    """For any height in a leaf's y-extent, its slab lists (as vertex pairs)
    every edge of the caller's ring that straddles that height, and only
    edges of that ring."""
    g, ix = grid221k_index
    rng = np.random.default_rng(3)
    for nb in rng.choice(ix["n_leaves"], 300, replace=False):
        b = int(ix["leaf"]["leaf_id"][nb])
        ring = g.verts[g.vert_off[b]:g.vert_off[b + 1]].astype(np.int64)
        a, c = ring, np.roll(ring, -1, axis=0)
        edges = {tuple(e) for e in np.concatenate([a, c], 1).tolist()}
        box = ix["leaf"]["box"][nb]
        for py in list(rng.integers(box[2], box[3], 20)) + [int(box[2]), int(box[3]) - 1]:
            listed = slab_of(ix, nb, py)
            lset = {tuple(e) for e in listed.tolist()}
            assert lset <= edges
            strad = np.flatnonzero((a[:, 1] > py) != (c[:, 1] > py))
            for k in strad:
                assert (a[k, 0], a[k, 1], c[k, 0], c[k, 1]) in lset
            assert len(listed) <= len(ring)


def test_y_slab_parity_equals_oracle(grid221k_index):
    """Crossing parity over the listed slab edges only (intersections computed
    with exact rationals) equals the oracle's parity over the full ring."""
    from fractions import Fraction
    g, ix = grid221k_index
    rng = np.random.default_rng(4)
    for nb in rng.choice(ix["n_leaves"], 60, replace=False):
        b = int(ix["leaf"]["leaf_id"][nb])
        ring = g.verts[g.vert_off[b]:g.vert_off[b + 1]]
        box = ix["leaf"]["box"][nb]
        for _ in range(10):
            px, py = int(rng.integers(box[0], box[1])), int(rng.integers(box[2], box[3]))
            cnt = 0
            for ax, ay, bx, by in slab_of(ix, nb, py).tolist():
                if (ay > py) != (by > py) and Fraction(ax) + Fraction((py - ay) * (bx - ax), by - ay) > px:
                    cnt += 1
            assert (cnt & 1) == int(oracle.inside(ring, px, py))


def test_build_file_rejects_bad_input(tmp_path):
    import paper_2005_03156_amd as bm
    with pytest.raises(bm.BlockmapError) as e:
        bm.build_index_file(str(tmp_path / "x.bmi"), [0, 3], [[0, 0], [5, -2], [0, 5]])
    assert e.value.code == bm.BM_ERANGE


def test_load_rejects_malformed_files(tmp_path):
    """bm_index_load checks a file before anything reaches the device: a
    truncated file, a wrong magic, a decreasing slab offset, an edge list
    past the end, a child range past the nodes and a slot table of 2^8 slots
    all give BM_EIO; the unmodified file passes the checks (on a machine
    without a GPU it then fails only at the upload)."""
    import ctypes as C
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    good = str(tmp_path / "good.bmi")
    bm.build_index_file(good, g.vert_off, g.verts, g.n_groups, g.parents)
    buf = bytearray(open(good, "rb").read())
    ix = read_index(good)
    n_grp = len(ix["grp"])
    grp_at = 64 + 8                     # after magic, scalars, n_verts and the count
    leaf_at = grp_at + 32 * n_grp + 8   # first leaf record

    def load(data):
        path = str(tmp_path / "x.bmi")
        open(path, "wb").write(bytes(data))
        h = C.c_void_p()
        rc = bm.lib.bm_index_load(path.encode(), C.byref(h))
        if rc == bm.BM_OK:
            bm.lib.bm_index_destroy(h)
        return rc, bm.lib.bm_last_error().decode()

    rc, _ = load(buf)
    assert rc != bm.BM_EIO
    cases = {}
    cases["truncated"] = buf[:-5]
    bad = bytearray(buf); bad[7:8] = b"9"; cases["magic"] = bad
    # a leaf with inline offsets and at least two slabs: make them decrease
    leaf = ix["leaf"]
    k = next(i for i in range(len(leaf)) if not (int(leaf[i]["packed"]) & EXT) and (int(leaf[i]["packed"]) >> 8) & 0xFF >= 1)
    bad = bytearray(buf); o = leaf_at + 64 * k + 32
    bad[o + 1] = 200; bad[o + 2] = 100; cases["decreasing slab offsets"] = bad
    bad = bytearray(buf); o = leaf_at + 64 * k + 16
    bad[o:o + 8] = np.int64(len(ix["ent"]) + 1).tobytes(); cases["edge list past the end"] = bad
    bad = bytearray(buf); o = grp_at + 32 * 0 + 16 + 4
    bad[o:o + 4] = np.int32(len(ix["box"]) + 5).tobytes(); cases["child range past the nodes"] = bad
    t = next(i for i in range(n_grp) if int(ix["child"][i][2]) >= 0)
    bad = bytearray(buf); o = grp_at + 32 * t + 16 + 12
    packed = int(ix["child"][t][3])
    bad[o:o + 4] = np.int32((packed & ~0xFF) | 8).tobytes(); cases["slot table of 2^8 slots"] = bad
    for name, data in cases.items():
        rc, msg = load(data)
        assert rc == bm.BM_EIO, (name, rc, msg)


# ---- per-leaf cell maps -------------------------------------------------

def cell_shift(w):
    """The smallest s >= 0 with 16 << s >= w (w >= 1)."""
    s = 0
    while (16 << s) < w:
        s += 1
    return s


def cell_class(rec, px, py):
    """Class of the cell holding (px, py) in a leaf record: 0 out, 1 in, 2 test."""
    b = rec["box"]
    col = (int(px) - int(b[0])) >> cell_shift(int(b[1]) - int(b[0]))
    row = (int(py) - int(b[2])) >> cell_shift(int(b[3]) - int(b[2]))
    return (int(rec["cell"][row]) >> (2 * col)) & 3


def _rings_file(tmp_path, rings):
    import paper_2005_03156_amd as bm
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    verts = np.concatenate([np.asarray(r, np.int32) for r in rings])
    p = str(tmp_path / "rings.bmi")
    bm.build_index_file(p, off, verts)
    return off, verts, read_index(p)


def test_cell_maps_exact_on_every_point(tmp_path):
    """Small rings (boxes of 20 to 70 units, so cells are 2 to 8 units a side):
    every integer point of every In cell is inside its ring and every point of
    every Out cell outside, by the oracle's crossing test; rings include a
    comb, a spiral-like notch, a triangle, a square with a long horizontal
    edge on a cell border and a ring with a zero-length edge."""
    rng = np.random.default_rng(3)
    rings = [
        [(0, 0), (60, 0), (60, 40), (45, 40), (45, 10), (30, 10), (30, 40), (15, 40), (15, 10), (5, 10), (5, 40),
         (0, 40)],                                                            # comb
        [(100, 100), (170, 100), (170, 160), (110, 160), (110, 120), (150, 120), (150, 140), (130, 140),
         (130, 150), (160, 150), (160, 110), (100, 110)],                      # notched spiral
        [(200, 5), (255, 5), (213, 47)],                                       # triangle
        [(300, 0), (332, 0), (332, 32), (316, 32), (316, 32), (300, 32)],      # duplicate vertex, border edge
    ]
    for _ in range(6):  # random star-shaped rings
        cx, cy = rng.integers(400, 4000, 2)
        k = int(rng.integers(5, 14))
        ang = np.sort(rng.uniform(0, 2 * np.pi, k))
        rad = rng.uniform(8, 35, k)
        rings.append(list(zip((cx + rad * np.cos(ang)).round().astype(int), (cy + rad * np.sin(ang)).round().astype(int))))
    off, verts, ix = _rings_file(tmp_path, rings)
    L = ix["leaf"]
    settled = [0, 0]
    for nb in range(L.shape[0]):
        rec = L[nb]
        b = rec["box"]
        ring = verts[off[rec["leaf_id"]]:off[rec["leaf_id"] + 1]]
        for py in range(int(b[2]), int(b[3])):
            for px in range(int(b[0]), int(b[1])):
                c = cell_class(rec, px, py)
                if c == 2:
                    continue
                settled[c] += 1
                assert int(oracle.inside(ring, px, py)) == c, (nb, px, py, c)
    assert settled[0] > 1000 and settled[1] > 1000, settled


def test_cell_maps_exact_on_sampled_points(grid221k_index):
    """220,900-block grid: for 3,000 leaves, points drawn in every In and Out
    cell (its corners, centre and random points) get the class as their
    crossing-test answer; and the maps settle a large share of the cells."""
    g, ix = grid221k_index
    L = ix["leaf"]
    rng = np.random.default_rng(11)
    counts = np.zeros(4, np.int64)
    for nb in rng.choice(L.shape[0], 3000, replace=False):
        rec = L[nb]
        b = [int(v) for v in rec["box"]]
        sx, sy = cell_shift(b[1] - b[0]), cell_shift(b[3] - b[2])
        ring = g.verts[g.vert_off[rec["leaf_id"]]:g.vert_off[rec["leaf_id"] + 1]]
        for r in range(16):
            for c in range(16):
                x0, y0 = b[0] + (c << sx), b[2] + (r << sy)
                x1, y1 = min(b[1], x0 + (1 << sx)), min(b[3], y0 + (1 << sy))
                if x0 >= x1 or y0 >= y1:
                    continue
                cls = (int(rec["cell"][r]) >> (2 * c)) & 3
                counts[cls] += 1
                if cls == 2:
                    continue
                pts = [(x0, y0), (x1 - 1, y1 - 1), (x0, y1 - 1), (x1 - 1, y0), ((x0 + x1) // 2, (y0 + y1) // 2)]
                pts += list(zip(rng.integers(x0, x1, 3), rng.integers(y0, y1, 3)))
                for px, py in pts:
                    assert int(oracle.inside(ring, int(px), int(py))) == cls, (nb, r, c, px, py)
    assert counts[3] == 0
    assert (counts[0] + counts[1]) > 0.5 * counts.sum(), counts
