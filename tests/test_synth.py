"""Generator checks (CPU): the synthetic partitions are watertight and have
the stated shape, so the oracle's partition property is a real pin."""
import numpy as np
import pytest

import oracle
import synth


def _small_quadtree():
    q = dict(synth.QUADTREE)
    q.update(R=64, target_leaves=60_000, n_points=10_000_000)
    return q, synth.quadtree_geometry(**q)


def _vertex_probes(g, k, seed):
    rng = np.random.default_rng(seed)
    v = g.verts[rng.choice(g.verts.shape[0], k, replace=False)]
    offs = np.array([[0, 0], [1, 0], [-1, 0], [0, 1], [0, -1], [1, -1], [-1, 1]], np.int32)
    return (v[:, None, :] + offs[None]).reshape(-1, 2)


def test_quadtree_mesh_is_watertight_and_hierarchy_exact():
    q, g = _small_quadtree()
    pts = np.concatenate([synth.quadtree_mixture(q).sample(synth.key("quadtree8m", 1, 1), 0, 20000),
                          _vertex_probes(g, 3000, 0)]).astype(np.int32)
    out, hits = oracle.brute(g.vert_off, g.verts, pts, box_reject=True, count_hits=True)
    x, y = pts[:, 0].astype(np.int64), pts[:, 1].astype(np.int64)
    inside = (x >= 0) & (x < g.W) & (y >= 0) & (y < g.W)
    assert (hits[inside] == 1).all() and (hits[~inside] == 0).all()
    assert (oracle.Hier.from_geometry(g).map(pts) == out).all()
    # the mesh is graded: several depths present, neighbours within one level
    d = g.meta["depth"].astype(int)
    assert len(np.unique(d)) >= 3
    assert np.abs(np.diff(d, axis=0)).max() <= 1 and np.abs(np.diff(d, axis=1)).max() <= 1


def test_quadtree_t_junctions_present():
    """Some rings carry the corner of a finer neighbour on a side (the
    T-junction vertex that keeps the mesh watertight)."""
    q, g = _small_quadtree()
    d = g.meta["depth"]
    assert (np.abs(np.diff(d.astype(int), axis=1)) == 1).any()


def test_quadtree8m_shape():
    g = synth.geometry("quadtree8m")
    nv = np.diff(g.vert_off)
    assert abs(g.n_blocks - 8_000_000) < 80_000
    assert nv.min() >= 4 and nv.max() <= 2000
    assert 27 <= nv.mean() <= 33
    assert (nv > 1000).sum() > 100  # heavy tail present
    d = g.meta["depth"]
    assert d.min() == 0 and d.max() == 5  # leaf areas differ by 4^5 = 1024x
    for l, p in enumerate(g.parents):
        assert p.min() >= 0 and p.max() < g.n_groups[l]
        assert np.bincount(p).max() <= 64  # fan-out <= 64 at every level


@pytest.mark.parametrize("workload", ["grid1k", "grid221k"])
def test_grid_shape(workload):
    g = synth.geometry(workload)
    nv = np.diff(g.vert_off)
    if workload == "grid1k":
        assert g.n_blocks == 1024 and nv.min() >= 16 and nv.max() <= 28
    else:
        assert g.n_blocks == 220_900 and 23 <= nv.mean() <= 25 and nv.max() <= 4 + 4 * 40
        assert g.n_groups == [50, 3000, 70000]


def test_points_are_counter_based():
    """Any slice of a point stream can be regenerated on its own."""
    a = synth.points("grid221k", 10_000)
    b = synth.points("grid221k", 4_000, i0=6_000)
    assert (a[6_000:] == b).all()
    c = synth.points("quadtree8m", 1000, i0=(1 << 26) * 3)
    assert c.shape == (1000, 2)
