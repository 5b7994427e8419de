"""CPU oracle for point -> block mapping -- TEST INFRASTRUCTURE ONLY.

Used by the unit tests, the smoke check and the benchmark's CPU-baseline leg.
The GPU library does not import, link or call anything in this package, and
this package shares no code with it.

``oracle.c`` (built with gcc into ``liboracle.so``) holds the two plain routes:
the definition (every block for every point) and the paper's hierarchy of
bounding boxes (Sec. III) followed by the crossing-number test (Sec. III-A).
``pyref.py`` holds a pure-Python evaluation with exact rationals for small
hand-made cases, and the reference quantiser.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")


FLAGS = ["-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """The in-tree library, built for any x86-64 host (it travels with the
    tree to other machines)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc"] + FLAGS + [src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def build_native(directory: str) -> str:
    """The same source built for the CPU it is built on (-march=native), into
    `directory` (outside the tree: the result only runs on this machine's CPU
    model). Returns the library path; use() switches to it."""
    src = os.path.join(_HERE, "oracle.c")
    path = os.path.join(directory, "liboracle_native.so")
    subprocess.check_call(["gcc"] + FLAGS + ["-march=native", src, "-o", path])
    return path


def use(path: str) -> None:
    """Load the oracle from `path` for every later call (objects made before
    keep working only while the earlier library stays loaded)."""
    global _LIB_PATH, _lib
    _LIB_PATH = path
    _lib = None
    _L()


class Counts(C.Structure):
    _fields_ = [("bbox_tests", C.c_int64), ("leaf_cands", C.c_int64), ("edge_tests", C.c_int64),
                ("straddles", C.c_int64), ("x_ambiguous", C.c_int64), ("hits", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        P, i64, i32 = C.c_void_p, C.c_int64, C.c_int32
        lib.orc_inside.restype = C.c_int
        lib.orc_inside.argtypes = [P, i64, i32, i32]
        lib.orc_ring_boxes.restype = None
        lib.orc_ring_boxes.argtypes = [i64, P, P, P]
        lib.orc_brute.restype = None
        lib.orc_brute.argtypes = [i64, P, P, P, i64, P, P, P]
        lib.orc_hier_create.restype = P
        lib.orc_hier_create.argtypes = [i64, P, P, i32, P, P]
        lib.orc_hier_destroy.restype = None
        lib.orc_hier_destroy.argtypes = [P]
        lib.orc_hier_map.restype = None
        lib.orc_hier_map.argtypes = [P, i64, P, P, C.POINTER(Counts)]
        lib.orc_count_per_block.restype = None
        lib.orc_count_per_block.argtypes = [i64, P, i64, P]
        lib.orc_join_per_block.restype = None
        lib.orc_join_per_block.argtypes = [i64, P, i64, P, i64, P]
        lib.orc_threads.restype = C.c_int
        lib.orc_threads.argtypes = []
        lib.orc_set_threads.restype = None
        lib.orc_set_threads.argtypes = [C.c_int]
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def threads() -> int:
    return int(_L().orc_threads())


def set_threads(t: int) -> None:
    _L().orc_set_threads(int(t))


def inside(ring, px: int, py: int) -> bool:
    """Crossing-number test of one point against one ring ([m, 2] int32)."""
    r = _c(ring, np.int32)
    return bool(_L().orc_inside(_p(r), r.shape[0], int(px), int(py)))


def ring_boxes(vert_off, verts) -> np.ndarray:
    vo, vv = _c(vert_off, np.int64), _c(verts, np.int32)
    nb = vo.shape[0] - 1
    box = np.empty((max(nb, 0), 4), np.int32)
    _L().orc_ring_boxes(nb, _p(vo), _p(vv), _p(box))
    return box


def brute(vert_off, verts, xy, *, box_reject: bool = False, count_hits: bool = False):
    """Smallest containing block per point (or -1), scanning every block.

    box_reject skips blocks whose half-open box misses the point; count_hits
    also returns the number of containing blocks per point.
    """
    vo, vv, pts = _c(vert_off, np.int64), _c(verts, np.int32), _c(xy, np.int32)
    nb, n = vo.shape[0] - 1, pts.shape[0]
    box = ring_boxes(vo, vv) if box_reject else None
    out = np.empty(n, np.int32)
    hits = np.empty(n, np.int32) if count_hits else None
    _L().orc_brute(nb, _p(vo), _p(vv), _p(box), n, _p(pts), _p(out), _p(hits))
    return (out, hits) if count_hits else out


def count_per_block(ids, n_blocks: int) -> np.ndarray:
    """Points per block: entry b counts the ids equal to b, entry n_blocks the
    others (-1, no block)."""
    a = _c(ids, np.int32)
    counts = np.zeros(int(n_blocks) + 1, np.uint64)
    _L().orc_count_per_block(a.shape[0], _p(a), int(n_blocks), _p(counts))
    return counts


def join_per_block(ids, table, fill: int = -1) -> np.ndarray:
    """Per-point join: table[id] for ids in [0, len(table)), else fill."""
    a, t = _c(ids, np.int32), _c(table, np.int64)
    out = np.empty(a.shape[0], np.int64)
    _L().orc_join_per_block(a.shape[0], _p(a), t.shape[0], _p(t), int(fill), _p(out))
    return out


class Hier:
    """The paper's hierarchy route (Sec. III): group boxes level by level, then
    the crossing-number test on every surviving block."""

    def __init__(self, vert_off, verts, n_groups, parents):
        self._vo = _c(vert_off, np.int64)
        self._vv = _c(verts, np.int32)
        self._ng = np.asarray(n_groups, np.int64)
        self._par = [_c(p, np.int32) for p in parents]
        arr = (C.c_void_p * max(len(self._par), 1))(*[p.ctypes.data for p in self._par])
        self._arr = arr
        self._lib = _L()  # the library that made it also maps and frees it
        self._h = self._lib.orc_hier_create(self._vo.shape[0] - 1, _p(self._vo), _p(self._vv),
                                       len(self._par), _p(self._ng) if len(self._ng) else None, arr)

    @classmethod
    def from_geometry(cls, g):
        return cls(g.vert_off, g.verts, g.n_groups, g.parents)

    def map(self, xy, with_counts: bool = False):
        pts = _c(xy, np.int32)
        out = np.empty(pts.shape[0], np.int32)
        cnt = Counts()
        self._lib.orc_hier_map(self._h, pts.shape[0], _p(pts), _p(out), C.byref(cnt))
        return (out, cnt.as_dict()) if with_counts else out

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        lib = getattr(self, "_lib", None)
        if h and lib is not None:
            lib.orc_hier_destroy(h)
