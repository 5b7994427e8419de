"""Seeded synthetic inputs for the point -> block mapping workloads.

Generates watertight block partitions, their group hierarchy and query points.
Inputs only: nothing here computes bounding boxes or crossing tests, so the GPU
library and the CPU oracle can both consume these arrays without sharing any of
the mapping arithmetic. The arrays stand in for the census shapefiles and the
mobile-location points of the paper (Sec. II, Sec. V), which are not available.

The heavy lifting is in ``synth.c`` (counter-based splitmix64 streams, OpenMP),
built into ``libsynth.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
SEED = 200503156


def build(force: bool = False) -> str:
    """Compile libsynth.so with gcc (OpenMP, no FP contraction)."""
    src = os.path.join(_HERE, "synth.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-ffp-contract=off", "-fPIC",
                               "-shared", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        u64, i64, i32, dbl, P = C.c_uint64, C.c_int64, C.c_int32, C.c_double, C.c_void_p
        lib.syn_key.restype = u64
        lib.syn_key.argtypes = [u64, u64, u64, u64]
        lib.syn_rand_u64.restype = u64
        lib.syn_rand_u64.argtypes = [u64, u64]
        lib.syn_rand_u01.restype = dbl
        lib.syn_rand_u01.argtypes = [u64, u64]
        lib.syn_grid_offsets.restype = i64
        lib.syn_grid_offsets.argtypes = [P, P]
        lib.syn_grid_fill.restype = None
        lib.syn_grid_fill.argtypes = [P, P, P]
        lib.syn_band_hierarchy.restype = None
        lib.syn_band_hierarchy.argtypes = [i32, i32, P, P, P]
        lib.syn_mixture_setup.restype = None
        lib.syn_mixture_setup.argtypes = [u64, i32, dbl, dbl, dbl, dbl, P, P, P, P]
        lib.syn_mixture_points.restype = None
        lib.syn_mixture_points.argtypes = [u64, i64, i64, i32, P, P, P, P, dbl, dbl, dbl, P]
        lib.syn_sizes.restype = None
        lib.syn_sizes.argtypes = [u64, i64, i32, dbl, dbl, dbl, P]
        lib.syn_qt_offsets.restype = i64
        lib.syn_qt_offsets.argtypes = [P, i64, P]
        lib.syn_qt_fill.restype = None
        lib.syn_qt_fill.argtypes = [P, i64, P, P]
        lib.syn_qt_groups.restype = i64
        lib.syn_qt_groups.argtypes = [P, i64, P, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# Each workload draws from its own seed stream (a small integer folded into
# every key), so adding a workload never changes another one's data.
SEED_STREAM = {"grid1k": 1, "grid221k": 2, "quadtree8m": 3, "batches10k": 4, "requests20k": 5}


def key(workload, stream: int, k: int = 0) -> int:
    """Counter-based key for (workload, stream, k); workload is a name of
    SEED_STREAM (or its integer seed stream)."""
    wid = SEED_STREAM[workload] if isinstance(workload, str) else int(workload)
    return int(_L().syn_key(SEED, wid, stream, k))


class _GridParams(C.Structure):
    _fields_ = [("n", C.c_int32), ("c", C.c_int64), ("klaw", C.c_int32), ("kmin", C.c_int32),
                ("kmax", C.c_int32), ("kp", C.c_double), ("vjit", C.c_double), ("pjit", C.c_double),
                ("taper", C.c_double), ("key", C.c_uint64)]


@dataclass
class Geometry:
    """A block partition plus its hierarchy.

    vert_off: int64 [n_blocks+1]; ring b is verts[vert_off[b]:vert_off[b+1]] (no closing duplicate)
    verts:    int32 [V, 2] (x, y)
    n_groups: group counts per level, coarse -> fine (blocks excluded)
    parents:  parents[l][i] = level-l group of entity i of level l+1 (blocks for the last)
    W:        the partition covers exactly [0, W)^2 (see the generator)
    """
    vert_off: np.ndarray
    verts: np.ndarray
    n_groups: list
    parents: list
    W: int
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_blocks(self) -> int:
        return int(self.vert_off.shape[0] - 1)


def jittered_grid(n: int, c: int, *, klaw: int = 0, kmin: int = 3, kmax: int = 6, kp: float = 0.25,
                  vjit: float = 0.3, pjit: float = 0.1, taper: float = 0.2, key_: int = 1):
    """Shared-edge jittered grid: n x n blocks over [0, n*c]^2, block id = row*n + col."""
    g = _GridParams(n, c, klaw, kmin, kmax, kp, vjit, pjit, taper, key_)
    off = np.empty(n * n + 1, np.int64)
    total = _L().syn_grid_offsets(C.byref(g), _p(off))
    verts = np.empty((total, 2), np.int32)
    _L().syn_grid_fill(C.byref(g), _p(off), _p(verts))
    return off, verts


def band_hierarchy(n: int, bands):
    """Nested bands: bands = [(rows, cols), ...] coarse -> fine."""
    L = len(bands)
    rows = np.array([b[0] for b in bands], np.int32)
    cols = np.array([b[1] for b in bands], np.int32)
    sizes = [bands[l + 1][0] * bands[l + 1][1] for l in range(L - 1)] + [n * n]
    parents = [np.empty(s, np.int32) for s in sizes]
    arr = (C.c_void_p * L)(*[p.ctypes.data for p in parents])
    _L().syn_band_hierarchy(n, L, _p(rows), _p(cols), arr)
    return [int(r * c) for r, c in bands], parents


# ---------------------------------------------------------- the workloads ----

# grid1k: 32 x 32 jittered grid over [0, 1e6]^2 (1,024 blocks), 3..6 points per
# shared edge, 8 x 8 groups of 4 x 4 blocks; 100,000 points.
# grid221k: 470 x 470 grid (220,900 blocks), 2 + Geometric(1/4) (<= 40) points
# per edge; 50 regions / 3,000 counties / 70,000 tracts; 100M points.
# quadtree8m: the graded quadtree mesh below (about 8M blocks); 1B points.
WORKLOADS = {
    "grid1k": dict(n=32, c=31_250, klaw=0, kmin=3, kmax=6, kp=0.0, bands=[(8, 8)], n_points=100_000,
            K=5, wsig=0.0, sig=(0.05, 0.05), p_unif=0.20),
    "grid221k": dict(n=470, c=2_000_000, klaw=1, kmin=2, kmax=40, kp=0.25,
            bands=[(5, 10), (50, 60), (250, 280)], n_points=100_000_000,
            K=200, wsig=1.0, sig=(0.005, 0.05), p_unif=0.05),
}


def geometry(workload: str) -> Geometry:
    """The block partition and hierarchy of a workload ("grid1k", "grid221k",
    "quadtree8m")."""
    if workload == "quadtree8m":
        return quadtree_geometry(**QUADTREE)
    p = WORKLOADS[workload]
    off, verts = jittered_grid(p["n"], p["c"], klaw=p["klaw"], kmin=p["kmin"], kmax=p["kmax"],
                               kp=p["kp"], key_=key(workload, 0, 0))
    n_groups, parents = band_hierarchy(p["n"], p["bands"])
    return Geometry(off, verts, n_groups, parents, W=p["n"] * p["c"], name=workload,
                    meta=dict(grid_n=p["n"], cell=p["c"]))


def n_points(workload: str) -> int:
    """Size of a workload's point stream."""
    return QUADTREE["n_points"] if workload == "quadtree8m" else WORKLOADS[workload]["n_points"]


class Mixture:
    """Gaussian mixture plus a uniform share over the 10%-enlarged extent."""

    def __init__(self, key_: int, K: int, W: float, wsig: float, sig_lo: float, sig_hi: float,
                 p_unif: float):
        self.K, self.W, self.p_unif = K, W, p_unif
        self.cumw, self.cx, self.cy, self.sig = (np.empty(K) for _ in range(4))
        _L().syn_mixture_setup(key_, K, W, wsig, sig_lo, sig_hi, _p(self.cumw), _p(self.cx),
                               _p(self.cy), _p(self.sig))

    def sample(self, key_: int, i0: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
        out = np.empty((n, 2), np.int32) if out is None else out
        assert out.shape == (n, 2) and out.dtype == np.int32 and out.flags.c_contiguous
        lo, hi = -0.05 * self.W, 1.05 * self.W
        _L().syn_mixture_points(key_, i0, n, self.K, _p(self.cumw), _p(self.cx), _p(self.cy),
                                _p(self.sig), self.p_unif, lo, hi, _p(out))
        return out


def points(workload: str, n: int | None = None, i0: int = 0, out: np.ndarray | None = None) -> np.ndarray:
    """Points i0 .. i0+n-1 of a workload's point stream (int32 [n, 2])."""
    if workload == "quadtree8m":
        q = QUADTREE
        n = q["n_points"] if n is None else n
        return quadtree_mixture(q).sample(key(workload, 1, 1), i0, n, out)
    p = WORKLOADS[workload]
    W = p["n"] * p["c"]
    n = p["n_points"] if n is None else n
    m = Mixture(key(workload, 1, 0), p["K"], W, p["wsig"], p["sig"][0], p["sig"][1], p["p_unif"])
    return m.sample(key(workload, 1, 1), i0, n, out)


def sizes(key_: int, nb: int, law: int, median: float, s: float, hi: float) -> np.ndarray:
    out = np.empty(nb, np.int64)
    _L().syn_sizes(key_, nb, law, median, s, hi, _p(out))
    return out


# ------------------------------------------------ graded quadtree mesh ----

class _QtParams(C.Structure):
    _fields_ = [("R", C.c_int32), ("lg_cell", C.c_int32), ("maxd", C.c_int32), ("depth", C.c_void_p),
                ("leaf_off", C.c_void_p), ("vjit", C.c_double), ("pjit", C.c_double),
                ("taper", C.c_double), ("k_lambda", C.c_double), ("k_alpha", C.c_double),
                ("vmax", C.c_int32), ("key", C.c_uint64), ("factor", C.c_void_p)]


# quadtree8m: 2^30 square of 512 x 512 root cells, each cut into 4^d equal
# leaves (d <= 5, neighbours differ by <= 1) following the point density, to
# about 8M leaves; per-segment interior points from a Lomax(2) law (block
# mean about 30, 4..2000 vertices); hierarchy 64 / 4,096 / 262,144 root cells
# / depth-2 quadtree nodes / leaves; 1B points in chunks of 2^26.
QUADTREE = dict(R=512, lg_cell=21, maxd=5, target_leaves=8_000_000, vjit=0.25, pjit=0.10, taper=0.2,
                k_lambda=7.0, k_alpha=2.0, vmax=2000, K=64, wsig=1.0, sig=(0.002, 0.03), p_unif=0.03,
                n_points=1_000_000_000, chunk=1 << 26, workload="quadtree8m")


def quadtree_mixture(q) -> Mixture:
    W = float(q["R"] << q["lg_cell"])
    return Mixture(key(q["workload"], 1, 0), q["K"], W, q["wsig"], q["sig"][0], q["sig"][1], q["p_unif"])


def _balance(d: np.ndarray) -> np.ndarray:
    """Raise depths until 8-neighbours differ by at most one."""
    d = d.copy()
    while True:
        p = np.pad(d, 1, constant_values=-1)
        m = np.max(np.stack([p[1 + a:p.shape[0] - 1 + a, 1 + b:p.shape[1] - 1 + b]
                             for a in (-1, 0, 1) for b in (-1, 0, 1)]), 0)
        nd = np.maximum(d, m - 1)
        if (nd == d).all():
            return d
        d = nd


def quadtree_depths(q) -> np.ndarray:
    """Depth per root cell from the expected point count of the density the
    points are drawn from: deeper where points are denser."""
    from scipy.special import ndtr
    R, cell = q["R"], float(1 << q["lg_cell"])
    W = R * cell
    mix = quadtree_mixture(q)
    w = np.diff(np.concatenate([[0.0], mix.cumw]))
    edges = np.arange(R + 1) * cell
    px = ndtr((edges[None, :] - mix.cx[:, None]) / mix.sig[:, None])
    py = ndtr((edges[None, :] - mix.cy[:, None]) / mix.sig[:, None])
    px, py = np.diff(px, axis=1), np.diff(py, axis=1)  # [K, R]
    prob = (1 - q["p_unif"]) * np.einsum("k,ki,kj->ji", w, px, py)
    prob += q["p_unif"] * (cell * cell) / (1.1 * W) ** 2
    E = prob * q["n_points"]

    def depths(T):
        d = np.clip(np.ceil(np.log(np.maximum(E / T, 1e-30)) / np.log(4.0)), 0, q["maxd"]).astype(np.int8)
        return _balance(d)

    lo, hi = np.log(1e-3), np.log(1e12)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        n = int((4 ** depths(np.exp(mid)).astype(np.int64)).sum())
        if n > q["target_leaves"]:
            lo = mid
        else:
            hi = mid
    return depths(np.exp(hi))


def quadtree_geometry(**q) -> Geometry:
    R = q["R"]
    depth = np.ascontiguousarray(quadtree_depths(q), np.int8).ravel()
    leaf_off = np.concatenate([[0], np.cumsum(4 ** depth.astype(np.int64))]).astype(np.int64)
    nl = int(leaf_off[-1])
    factor = np.empty(nl, np.float32)
    qp = _QtParams(R, q["lg_cell"], q["maxd"], depth.ctypes.data, leaf_off.ctypes.data, q["vjit"],
                   q["pjit"], q["taper"], q["k_lambda"], q["k_alpha"], q["vmax"], key(q["workload"], 0, 0),
                   factor.ctypes.data)
    off = np.empty(nl + 1, np.int64)
    total = _L().syn_qt_offsets(C.byref(qp), nl, _p(off))
    verts = np.empty((total, 2), np.int32)
    _L().syn_qt_fill(C.byref(qp), nl, _p(off), _p(verts))
    # hierarchy: 64 tiles / 4096 tiles / root cells / depth-2 quadtree nodes / leaves
    leaf_group = np.empty(nl, np.int32)
    group_cell = np.empty(nl, np.int32)
    ng = int(_L().syn_qt_groups(C.byref(qp), nl, _p(leaf_group), _p(group_cell)))
    group_cell = group_cell[:ng].copy()
    cy, cx = np.divmod(np.arange(R * R), R)
    t1 = (cy // 8) * (R // 8) + cx // 8
    ty, tx = np.divmod(np.arange((R // 8) ** 2), R // 8)
    t0 = (ty // 8) * (R // 64) + tx // 8
    parents = [t0.astype(np.int32), t1.astype(np.int32), group_cell, leaf_group]
    n_groups = [(R // 64) ** 2, (R // 8) ** 2, R * R, ng]
    return Geometry(off, verts, n_groups, parents, W=R << q["lg_cell"], name="quadtree8m",
                    meta=dict(depth=depth.reshape(R, R), leaf_off=leaf_off))


def block_codes(g: Geometry) -> np.ndarray:
    """A numeric code per block composed like a census FIPS code: the top
    group's number (from 1), then at every level the entity's rank among its
    parent's children in index order, each level in as many decimal digits as
    its largest family needs. A per-block attribute table for the join; it
    depends only on the hierarchy arrays."""
    if not g.parents:
        return np.arange(g.n_blocks, dtype=np.int64)
    code = np.arange(1, int(g.n_groups[0]) + 1, dtype=np.int64)
    total_digits = len(str(int(g.n_groups[0])))
    for par in g.parents:
        par = np.asarray(par, np.int64)
        counts = np.bincount(par, minlength=code.shape[0])
        digits = len(str(max(int(counts.max()) - 1, 0)))
        total_digits += digits
        if total_digits > 18:
            raise ValueError("codes would not fit in 63 bits")
        order = np.argsort(par, kind="stable")
        first = np.concatenate([[0], np.cumsum(counts)[:-1]])
        rank = np.empty(par.shape[0], np.int64)
        rank[order] = np.arange(par.shape[0]) - first[par[order]]
        code = code[par] * (10 ** digits) + rank
    return code

# ------------------------------------------- batched and served workloads ----

def batch_sizes(nb: int = 10_000, hi: float = 1e6) -> np.ndarray:
    """Sizes of the batched workload's batches: round(exp(U[0, ln hi]))."""
    return sizes(key("batches10k", 2, 0), nb, 0, 0.0, 0.0, hi)


def batch_points(g: Geometry, sizes_: np.ndarray, first: int = 1, out: np.ndarray | None = None):
    """The batched workload's points: batch b (key first + b) is one Gaussian
    cluster (centre uniform over the extent, sigma log-uniform on [0.1%, 5%]
    of it). Returns the concatenation (int32 [sum, 2]) and the batch offsets
    (int64 [nb + 1])."""
    off = np.concatenate([[0], np.cumsum(sizes_)]).astype(np.int64)
    out = np.empty((int(off[-1]), 2), np.int32) if out is None else out
    for b in range(len(sizes_)):
        m = Mixture(key("batches10k", 2, first + b), 1, g.W, 0.0, 0.001, 0.05, 0.0)
        m.sample(key("batches10k", 3, first + b), 0, int(sizes_[b]), out=out[off[b]:off[b + 1]])
    return out, off


def request_sizes(n: int, first: int = 0, median: float = 10_000.0, s: float = 2.0, hi: float = 10_000_000):
    """Sizes of served requests: lognormal (median 10k, sigma_ln 2), clamped
    to [1, hi]."""
    return sizes(key("requests20k", 2, first), n, 1, median, s, hi)


def request_points(g: Geometry, r: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
    """Request r of the served workload: one Gaussian cluster (sigma
    log-uniform on [0.1%, 2%] of the extent) plus 20% uniform points."""
    m = Mixture(key("requests20k", 2, r + 1), 1, g.W, 0.0, 0.001, 0.02, 0.2)
    return m.sample(key("requests20k", 3, r + 1), 0, int(n), out)
