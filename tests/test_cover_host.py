"""The cell cover (the paper's fast approach, Sec. IV) built on the host only:
the file written by bm_cover_build_file is parsed here, the radix trie is
walked in numpy, and every kind of cell is checked against the oracle:
interior cells give the exact answer, empty cells mean no block, a boundary
cell lists every block that holds a point of it, and the stored centre answer
of a boundary cell is the exact answer there (which makes the approximate
mode's error bound hold)."""
import numpy as np
import pytest

import oracle
import synth
from test_index_host import read_index

EMPTY = 0xFFFFFFFF
PAY = (1 << 30) - 1


def read_cover(path):
    with open(path, "rb") as f:
        buf = f.read()
    assert buf[:8] == b"BMCOV001"
    sh = np.frombuffer(buf, np.int32, 6, 8)
    counts = np.frombuffer(buf, np.int64, 4, 32)
    pos = 64
    out = {}
    for name, dt in [("ent", np.uint32), ("cell_off", np.uint32), ("cell_leaf", np.uint32), ("cell_rep", np.int32)]:
        n = int(np.frombuffer(buf, np.int64, 1, pos)[0])
        pos += 8
        out[name] = np.frombuffer(buf, dt, n, pos)
        pos += out[name].nbytes
    assert pos == len(buf)
    out.update(ox=int(sh[0]), oy=int(sh[1]), log_side=int(sh[2]), n_levels=int(sh[3]), last_bits=int(sh[4]),
               cell_log2=int(sh[5]), counts=counts.copy())
    return out


def walk(cv, xy):
    """Trie entry of the cell holding each point (EMPTY off the square), and
    the trie level where the walk stopped."""
    px, py = xy[:, 0].astype(np.int64), xy[:, 1].astype(np.int64)
    dx, dy = px - cv["ox"], py - cv["oy"]
    L = cv["log_side"]
    act = (dx >= 0) & (dy >= 0) & ((dx >> L) == 0) & ((dy >> L) == 0)
    res = np.full(len(xy), EMPTY, np.uint32)
    lev = np.full(len(xy), -1, np.int64)
    node = np.zeros(len(xy), np.int64)
    shift = L
    for t in range(cv["n_levels"]):
        bits = cv["last_bits"] if t == cv["n_levels"] - 1 else 4
        shift -= bits
        m = (1 << bits) - 1
        e = ((dx >> shift) & m) | (((dy >> shift) & m) << bits)
        v = np.where(act, cv["ent"][np.where(act, node + e, 0)], EMPTY).astype(np.uint32)
        isnode = act & ((v >> 30) == 1)
        stop = act & ~isnode
        res[stop] = v[stop]
        lev[stop] = t
        node = np.where(isnode, (v & PAY).astype(np.int64), node)
        act = isnode
    assert not act.any(), "a walk ended on a node entry"
    return res, lev


def cell_centres(cv, xy):
    cl = cv["cell_log2"]
    px, py = xy[:, 0].astype(np.int64), xy[:, 1].astype(np.int64)
    cx = cv["ox"] + (((px - cv["ox"]) >> cl) << cl) + (1 << (cl - 1))
    cy = cv["oy"] + (((py - cv["oy"]) >> cl) << cl) + (1 << (cl - 1))
    return np.stack([np.minimum(cx, 2**31 - 1), np.minimum(cy, 2**31 - 1)], 1).astype(np.int32)


def grid_points(cv, rng, n):
    """Points on the finest cell grid's lines and corners (where a cover is
    most easily wrong), inside the covered square."""
    cl, L = cv["cell_log2"], cv["log_side"]
    k = rng.integers(0, 1 << (L - cl), size=(n, 2), dtype=np.int64)
    off = rng.choice(np.array([0, 0, 1, -1, (1 << cl) - 1], np.int64), size=(n, 2))
    x = cv["ox"] + (k[:, 0] << cl) + off[:, 0]
    y = cv["oy"] + (k[:, 1] << cl) + off[:, 1]
    return np.stack([np.clip(x, 0, 2**31 - 1), np.clip(y, 0, 2**31 - 1)], 1).astype(np.int32)


def vertex_points(g, rng, n):
    """Block vertices and their unit neighbours."""
    i = rng.integers(0, g.verts.shape[0], n)
    d = rng.integers(-1, 2, size=(n, 2))
    return np.clip(g.verts[i].astype(np.int64) + d, 0, 2**31 - 1).astype(np.int32)


def check_cover(g, cv, ix, xy):
    want = oracle.brute(g.vert_off, g.verts, xy, box_reject=True)
    v, lev = walk(cv, xy)
    tag = np.where(v == EMPTY, 3, v >> 30)
    # interior: the exact answer; empty: no block
    assert np.array_equal(want[tag == 0], (v[tag == 0] & PAY).astype(np.int32))
    assert np.all(want[tag == 3] == -1)
    # boundary cells only at the finest trie level, and their list holds the answer
    b = np.nonzero(tag == 2)[0]
    assert np.all(lev[b] == cv["n_levels"] - 1)
    lid = ix["leaf"]["leaf_id"]
    for k in b:
        c = int(v[k] & PAY)
        listed = lid[cv["cell_leaf"][cv["cell_off"][c]:cv["cell_off"][c + 1]]]
        if want[k] >= 0:
            assert want[k] in listed, (xy[k], want[k], listed)
    # approximate mode: the cell's stored answer is the exact answer at its centre
    if len(b):
        cen = cell_centres(cv, xy[b])
        assert np.array_equal(cv["cell_rep"][(v[b] & PAY).astype(np.int64)],
                              oracle.brute(g.vert_off, g.verts, cen, box_reject=True))
    return tag


@pytest.fixture(scope="module")
def grid1k_cover(tmp_path_factory):
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    d = tmp_path_factory.mktemp("cov")
    bm.build_cover_file(str(d / "c1.bmc"), g.vert_off, g.verts, g.n_groups, g.parents)
    bm.build_index_file(str(d / "c1.bmi"), g.vert_off, g.verts, g.n_groups, g.parents)
    return g, read_cover(str(d / "c1.bmc")), read_index(str(d / "c1.bmi"))


def test_structure(grid1k_cover):
    g, cv, ix = grid1k_cover
    ent = cv["ent"]
    tag = np.where(ent == EMPTY, 3, ent >> 30)
    assert np.all(tag <= 3)
    nodes = (ent[tag == 1] & PAY).astype(np.int64)
    assert np.all(nodes < len(ent)) and np.all(nodes > 0)
    assert np.all((ent[tag == 2] & PAY) < len(cv["cell_rep"]))
    assert np.all((ent[tag == 0] & PAY) < g.n_blocks)
    off = cv["cell_off"].astype(np.int64)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(cv["cell_leaf"])
    assert np.all(cv["cell_leaf"] < ix["n_leaves"])
    assert [int(c) for c in cv["counts"]] == [int(np.sum(tag == t)) for t in range(4)]
    # the finest level's side is 2^cell_log2 and the square covers the root box
    assert cv["log_side"] - 4 * (cv["n_levels"] - 1) - cv["last_bits"] == cv["cell_log2"]
    assert 1 <= cv["last_bits"] <= 4
    rb = ix["root_box"]
    assert cv["ox"] == rb[0] and cv["oy"] == rb[2]
    assert max(rb[1] - rb[0], rb[3] - rb[2]) <= 1 << cv["log_side"]


def test_random_points(grid1k_cover):
    g, cv, ix = grid1k_cover
    xy = synth.points("grid1k", 100_000)
    tag = check_cover(g, cv, ix, xy)
    # the cover does its job: most points need no crossing test
    assert np.mean(tag == 2) < 0.25


def test_grid_and_vertex_points(grid1k_cover):
    g, cv, ix = grid1k_cover
    rng = np.random.default_rng(5)
    check_cover(g, cv, ix, grid_points(cv, rng, 30_000))
    check_cover(g, cv, ix, vertex_points(g, rng, 30_000))


def test_outside_points(grid1k_cover):
    g, cv, ix = grid1k_cover
    xy = np.array([[-1, -1], [0, -5], [-7, 100], [2**31 - 1, 2**31 - 1], [cv["ox"] + (1 << cv["log_side"]), 0]],
                  np.int32)
    v, _ = walk(cv, xy)
    assert np.all(v[:3] == EMPTY)
    check_cover(g, cv, ix, xy)


@pytest.mark.parametrize("cl", [6, 13])
def test_cell_sizes(tmp_path, cl):
    """A fine and a coarse finest side both give a correct cover."""
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    bm.build_cover_file(str(tmp_path / "c.bmc"), g.vert_off, g.verts, g.n_groups, g.parents, cell_log2=cl)
    bm.build_index_file(str(tmp_path / "c.bmi"), g.vert_off, g.verts, g.n_groups, g.parents)
    cv, ix = read_cover(str(tmp_path / "c.bmc")), read_index(str(tmp_path / "c.bmi"))
    assert cv["cell_log2"] == cl
    rng = np.random.default_rng(cl)
    check_cover(g, cv, ix, np.concatenate([synth.points("grid1k", 20_000), grid_points(cv, rng, 10_000)]))


def test_overlapping_blocks(tmp_path):
    """Blocks that overlap (not a partition): a boundary cell must list every
    containing block, an interior cell must store the smallest one."""
    import paper_2005_03156_amd as bm
    rng = np.random.default_rng(11)
    rings = []
    for _ in range(60):
        cx, cy = rng.integers(10000, 60000, 2)
        r = int(rng.integers(500, 9000))
        k = int(rng.integers(3, 9))
        ang = np.sort(rng.uniform(0, 2 * np.pi, k))
        rad = r * rng.uniform(0.4, 1.0, k)
        rings.append(np.stack([cx + rad * np.cos(ang), cy + rad * np.sin(ang)], 1).round().astype(np.int32))
    vo = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    vv = np.concatenate(rings).astype(np.int32)

    class G:
        pass
    g = G()
    g.vert_off, g.verts, g.n_blocks = vo, vv, len(rings)
    bm.build_cover_file(str(tmp_path / "o.bmc"), vo, vv, cell_log2=7)
    bm.build_index_file(str(tmp_path / "o.bmi"), vo, vv)
    cv, ix = read_cover(str(tmp_path / "o.bmc")), read_index(str(tmp_path / "o.bmi"))
    xy = rng.integers(0, 70000, size=(40_000, 2)).astype(np.int32)
    check_cover(g, cv, ix, np.concatenate([xy, vertex_points(g, rng, 5000), grid_points(cv, rng, 5000)]))


def test_bad_config(tmp_path):
    import paper_2005_03156_amd as bm
    g = synth.geometry("grid1k")
    with pytest.raises(bm.BlockmapError):
        bm.build_cover_file(str(tmp_path / "x.bmc"), g.vert_off, g.verts, cell_log2=31)
    with pytest.raises(bm.BlockmapError):
        bm.build_cover_file(str(tmp_path / "x.bmc"), g.vert_off, g.verts, cell_log2=-1)
