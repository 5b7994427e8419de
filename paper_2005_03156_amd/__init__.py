"""Python binding of libblockmap (argument marshalling only).

Every step of the mapping runs in the HIP kernels of ``libblockmap.so``; this
module only turns numpy arrays and torch tensors into the pointers, sizes and
HIP streams of the C interface (``include/blockmap.h``). Torch provides device
memory and streams. If the library is missing the import fails: there is no
other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libblockmap.so")

BM_OK, BM_EINVAL, BM_ERANGE, BM_ENOMEM, BM_EHIP, BM_EBUSY, BM_ETIMEDOUT, BM_EIO = range(8)
_NAMES = {0: "BM_OK", 1: "BM_EINVAL", 2: "BM_ERANGE", 3: "BM_ENOMEM", 4: "BM_EHIP", 5: "BM_EBUSY",
          6: "BM_ETIMEDOUT", 7: "BM_EIO"}


class BlockmapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


if not os.path.exists(LIB_PATH):
    raise ImportError("libblockmap.so is not built (run python paper_2005_03156_amd/build.py)")

lib = C.CDLL(LIB_PATH)


class IndexDesc(C.Structure):
    _fields_ = [("n_blocks", C.c_int64), ("vert_off", C.c_void_p), ("verts_xy", C.c_void_p),
                ("n_levels", C.c_int32), ("n_groups", C.c_void_p), ("parent", C.c_void_p),
                ("keep_all_levels", C.c_int32)]


class IndexInfo(C.Structure):
    _fields_ = [("n_blocks", C.c_int64), ("n_vertices", C.c_int64), ("n_nodes", C.c_int64),
                ("device_bytes", C.c_int64), ("n_levels", C.c_int32), ("device", C.c_int32),
                ("top_groups", C.c_int64), ("sort_bins", C.c_int32), ("sort_adaptive", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("edge_chunk", C.c_int32), ("blocks_per_cu", C.c_int32), ("tile_points", C.c_int32),
                ("presort", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class CoverCfg(C.Structure):
    _fields_ = [("cell_log2", C.c_int32), ("threads", C.c_int32)]


class CoverInfo(C.Structure):
    _fields_ = [("origin_x", C.c_int32), ("origin_y", C.c_int32), ("log2_side", C.c_int32),
                ("trie_levels", C.c_int32), ("last_level_bits", C.c_int32), ("cell_log2", C.c_int32),
                ("trie_entries", C.c_int64), ("interior_entries", C.c_int64), ("node_entries", C.c_int64),
                ("boundary_cells", C.c_int64), ("empty_entries", C.c_int64), ("cell_leaves", C.c_int64),
                ("device_bytes", C.c_int64), ("build_seconds", C.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if k == "build_seconds" else int(getattr(self, k)))
                for k, _ in self._fields_}


class LaunchTimes(C.Structure):
    _fields_ = [("map_ms", C.c_double), ("sort_ms", C.c_double), ("map_launches", C.c_int32),
                ("sort_launches", C.c_int32), ("unsort_ms", C.c_double), ("unsort_launches", C.c_int32)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class Batch(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("out_ids", C.c_void_p), ("n", C.c_int64)]


class ServerCfg(C.Structure):
    _fields_ = [("mem_budget_bytes", C.c_int64), ("max_batch_points", C.c_int64), ("max_slots", C.c_int32),
                ("n_streams", C.c_int32), ("coalesce_us", C.c_int32), ("queue_capacity", C.c_int32),
                ("flags", C.c_int32), ("tuning", Tuning), ("copy_threads", C.c_int32),
                ("direct_min_points", C.c_int64)]


class ServerStats(C.Structure):
    _fields_ = [("completed", C.c_int64), ("points", C.c_int64), ("batches", C.c_int64),
                ("rejected", C.c_int64), ("mean_requests_per_batch", C.c_double), ("p50_us", C.c_double),
                ("p99_us", C.c_double), ("mean_us", C.c_double), ("max_us", C.c_double),
                ("points_per_s", C.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class Request(C.Structure):
    _fields_ = [("xy", C.c_void_p), ("out_ids", C.c_void_p), ("n", C.c_int64)]


BM_SERVER_FAIL_ALLOC = 1
BM_SERVER_ONE_PER_BATCH = 2

_P, _I64, _I32 = C.c_void_p, C.c_int64, C.c_int32
_SIGS = {
    "bm_index_create": (C.c_int, [C.POINTER(IndexDesc), C.POINTER(C.c_void_p)]),
    "bm_index_destroy": (None, [_P]),
    "bm_index_get_info": (C.c_int, [_P, C.POINTER(IndexInfo)]),
    "bm_index_save": (C.c_int, [_P, C.c_char_p]),
    "bm_index_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_void_p)]),
    "bm_index_build_file": (C.c_int, [C.POINTER(IndexDesc), C.c_char_p]),
    "map_points": (C.c_int, [_P, _P, _I64, _P, _P]),
    "map_points_tuned": (C.c_int, [_P, _P, _I64, _P, C.POINTER(Tuning), _P]),
    "map_points_noalloc": (C.c_int, [_P, _P, _I64, _P, _P]),
    "bm_quantize_lonlat": (C.c_int, [_P, _I64, _P, _P]),
    "map_points_timed": (C.c_int, [_P, _P, _I64, _P, C.POINTER(Tuning), _P, C.POINTER(LaunchTimes)]),
    "bm_tuning_default": (C.c_int, [C.POINTER(Tuning)]),
    "bm_autotune": (C.c_int, [_P, _P, _I64, C.POINTER(Tuning), _P]),
    "bm_map_batches": (C.c_int, [_P, _P, _P, _I64, _P, C.POINTER(Tuning), _P]),
    "bm_map_batch_table": (C.c_int, [_P, _P, _I64, C.POINTER(Tuning), _P]),
    "bm_batch_plan_create": (C.c_int, [_P, _I64, _I64, C.POINTER(Tuning), C.POINTER(C.c_void_p)]),
    "bm_batch_plan_run": (C.c_int, [_P, _P, _P, _I64, _P, _P]),
    "bm_batch_plan_run_table": (C.c_int, [_P, C.POINTER(Batch), _I64, _P]),
    "bm_batch_plan_destroy": (None, [_P]),
    "bm_server_cfg_default": (C.c_int, [C.POINTER(ServerCfg)]),
    "bm_server_create": (C.c_int, [_P, C.POINTER(ServerCfg), C.POINTER(C.c_void_p)]),
    "bm_server_submit": (C.c_int, [_P, _P, _I64, _P, C.POINTER(C.c_uint64)]),
    "bm_server_wait": (C.c_int, [_P, C.c_uint64, _I64]),
    "bm_server_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "bm_server_get_stats": (C.c_int, [_P, C.POINTER(ServerStats)]),
    "bm_server_reset_stats": (C.c_int, [_P]),
    "bm_server_run_trace": (C.c_int, [_P, C.POINTER(Request), _I64, _P]),
    "bm_server_destroy": (None, [_P]),
    "bm_cover_create": (C.c_int, [_P, C.POINTER(IndexDesc), C.POINTER(CoverCfg), C.POINTER(C.c_void_p)]),
    "bm_cover_destroy": (None, [_P]),
    "bm_cover_get_info": (C.c_int, [_P, C.POINTER(CoverInfo)]),
    "bm_cover_build_file": (C.c_int, [C.POINTER(IndexDesc), C.POINTER(CoverCfg), C.c_char_p]),
    "map_points_cover": (C.c_int, [_P, _P, _I64, _P, C.c_int32, _P]),
    "bm_count_per_block": (C.c_int, [_P, _I64, _I64, _P, _P]),
    "bm_join_per_block": (C.c_int, [_P, _I64, _P, _I64, _I64, _P, _P]),
    "bm_last_error": (C.c_char_p, []),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc: int) -> None:
    if rc != BM_OK:
        raise BlockmapError(rc, (lib.bm_last_error() or b"").decode())


def _stream_handle(stream):
    """torch stream / raw handle / None -> hipStream_t value."""
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _dev_ptr(t, dtype_name: str, shape_tail=()):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if str(t.dtype) != "torch." + dtype_name:
        raise TypeError("expected dtype %s, got %s" % (dtype_name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError("bad tensor shape %s" % (tuple(t.shape),))
    return C.c_void_p(t.data_ptr()) if t.numel() else C.c_void_p(0)


def tuning_default() -> Tuning:
    t = Tuning()
    _check(lib.bm_tuning_default(C.byref(t)))
    return t


def _desc(vert_off, verts, n_groups, parents, keep_all_levels=False):
    vo = np.ascontiguousarray(vert_off, np.int64)
    vv = np.ascontiguousarray(verts, np.int32)
    ng = np.ascontiguousarray(n_groups, np.int64)
    pars = [np.ascontiguousarray(p, np.int32) for p in parents]
    parr = (C.c_void_p * max(len(pars), 1))(*[p.ctypes.data for p in pars])
    d = IndexDesc(vo.shape[0] - 1, vo.ctypes.data, vv.ctypes.data, len(pars),
                  ng.ctypes.data if len(pars) else None, C.cast(parr, C.c_void_p), int(bool(keep_all_levels)))
    return d, (vo, vv, ng, pars, parr)


def build_index_file(path: str, vert_off, verts, n_groups=(), parents=(), *, keep_all_levels=False) -> None:
    """Build an index on the host only and write it to a file (no GPU needed)."""
    d, keep = _desc(vert_off, verts, n_groups, parents, keep_all_levels)
    _check(lib.bm_index_build_file(C.byref(d), os.fsencode(path)))
    del keep


class Index:
    """A block partition and its hierarchy, resident in device memory."""

    def __init__(self, vert_off, verts, n_groups=(), parents=(), *, keep_all_levels=False, _handle=None):
        self._h = None
        if _handle is not None:
            self._h = _handle
            return
        d, keep = _desc(vert_off, verts, n_groups, parents, keep_all_levels)
        h = C.c_void_p()
        _check(lib.bm_index_create(C.byref(d), C.byref(h)))
        del keep
        self._h = h

    @classmethod
    def from_geometry(cls, g, *, keep_all_levels=False) -> "Index":
        return cls(g.vert_off, g.verts, g.n_groups, g.parents, keep_all_levels=keep_all_levels)

    @classmethod
    def load(cls, path: str) -> "Index":
        h = C.c_void_p()
        _check(lib.bm_index_load(os.fsencode(path), C.byref(h)))
        return cls(None, None, _handle=h)

    def save(self, path: str) -> None:
        _check(lib.bm_index_save(self._h, os.fsencode(path)))

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = IndexInfo()
        _check(lib.bm_index_get_info(self._h, C.byref(i)))
        return {k: int(getattr(i, k)) for k, _ in IndexInfo._fields_}

    def close(self) -> None:
        h, self._h = self._h, None
        if h:
            lib.bm_index_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def map_points(index: Index, xy, out=None, stream=None, tuning: Tuning | None = None):
    """Block id (or -1) of every point: xy is an int32 CUDA tensor [n, 2]."""
    import torch
    n = xy.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=xy.device)
    pxy = _dev_ptr(xy, "int32", (2,))
    pout = _dev_ptr(out, "int32")
    if out.shape[0] != n:
        raise ValueError("out has the wrong length")
    s = _stream_handle(stream)
    if tuning is None:
        _check(lib.map_points(index.handle, pxy, n, pout, s))
    else:
        _check(lib.map_points_tuned(index.handle, pxy, n, pout, C.byref(tuning), s))
    return out


def map_points_noalloc(index: Index, xy, out, stream=None):
    """map_points through the entry point that allocates nothing (at most
    2^22 points per call; out is a caller-allocated int32 CUDA tensor [n])."""
    n = xy.shape[0]
    pxy = _dev_ptr(xy, "int32", (2,))
    pout = _dev_ptr(out, "int32")
    if out.shape[0] != n:
        raise ValueError("out has the wrong length")
    _check(lib.map_points_noalloc(index.handle, pxy, n, pout, _stream_handle(stream)))
    return out


def build_cover_file(path: str, vert_off, verts, n_groups=(), parents=(), cell_log2: int = 0,
                     threads: int = 0) -> None:
    """Build an index and its cell cover on the host only and write the cover
    to a file (no GPU needed)."""
    d, keep = _desc(vert_off, verts, n_groups, parents)
    cfg = CoverCfg(cell_log2, threads)
    _check(lib.bm_cover_build_file(C.byref(d), C.byref(cfg), os.fsencode(path)))
    del keep


class Cover:
    """The cell cover (fast approach) of a resident index, built from the same
    rings the index was built from; keeps the index alive."""

    def __init__(self, index: Index, vert_off, verts, cell_log2: int = 0, threads: int = 0):
        self._h = None
        self.index = index
        d, keep = _desc(vert_off, verts, (), ())
        cfg = CoverCfg(cell_log2, threads)
        h = C.c_void_p()
        _check(lib.bm_cover_create(index.handle, C.byref(d), C.byref(cfg), C.byref(h)))
        del keep
        self._h = h

    @classmethod
    def from_geometry(cls, index: Index, g, cell_log2: int = 0, threads: int = 0) -> "Cover":
        return cls(index, g.vert_off, g.verts, cell_log2, threads)

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = CoverInfo()
        _check(lib.bm_cover_get_info(self._h, C.byref(i)))
        return i.as_dict()

    def close(self) -> None:
        h, self._h = self._h, None
        if h:
            lib.bm_cover_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def map_points_cover(cover: Cover, xy, out=None, approx: bool = False, stream=None):
    """Block id (or -1) of every point through the cell cover; approx=True
    answers boundary cells with their centre's block."""
    import torch
    n = xy.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int32, device=xy.device)
    if out.shape[0] != n:
        raise ValueError("out has the wrong length")
    _check(lib.map_points_cover(cover.handle, _dev_ptr(xy, "int32", (2,)), n, _dev_ptr(out, "int32"),
                                1 if approx else 0, _stream_handle(stream)))
    return out


def count_per_block(ids, n_blocks: int, counts=None, stream=None):
    """Points per block from a CUDA int32 id tensor: a uint64 tensor (as int64)
    of n_blocks + 1 counts, the last one for ids outside [0, n_blocks).
    Accumulates into `counts` when one is given."""
    import torch
    if counts is None:
        counts = torch.zeros(n_blocks + 1, dtype=torch.int64, device=ids.device)
    if counts.shape[0] != n_blocks + 1:
        raise ValueError("counts must hold n_blocks + 1 entries")
    _check(lib.bm_count_per_block(_dev_ptr(ids, "int32"), ids.shape[0], n_blocks, _dev_ptr(counts, "int64"),
                                  _stream_handle(stream)))
    return counts


def join_per_block(ids, table, out=None, fill: int = -1, stream=None):
    """Per-point join on the device: out[i] = table[ids[i]] for ids in
    [0, len(table)), else fill. `ids` is a CUDA int32 tensor, `table` a CUDA
    int64 tensor of per-block attributes (e.g. numeric FIPS codes); returns
    (or fills) a CUDA int64 tensor of len(ids)."""
    import torch
    if out is None:
        out = torch.empty(ids.shape[0], dtype=torch.int64, device=ids.device)
    if out.shape[0] != ids.shape[0]:
        raise ValueError("out must hold one entry per id")
    _check(lib.bm_join_per_block(_dev_ptr(ids, "int32"), ids.shape[0], _dev_ptr(table, "int64"), table.shape[0],
                                 int(fill), _dev_ptr(out, "int64"), _stream_handle(stream)))
    return out


def map_points_timed(index: Index, xy, out, stream=None, tuning: Tuning | None = None) -> dict:
    """map_points with event timing of the mapping-kernel launches and of the
    spatial-sort phases (waits for the stream)."""
    t = LaunchTimes()
    _check(lib.map_points_timed(index.handle, _dev_ptr(xy, "int32", (2,)), xy.shape[0], _dev_ptr(out, "int32"),
                                C.byref(tuning) if tuning is not None else None, _stream_handle(stream),
                                C.byref(t)))
    return t.as_dict()


def quantize_lonlat(lonlat, out=None, stream=None):
    """float64 CUDA tensor [n, 2] of (lon, lat) -> int32 [n, 2] fixed point."""
    import torch
    n = lonlat.shape[0]
    if out is None:
        out = torch.empty((n, 2), dtype=torch.int32, device=lonlat.device)
    _check(lib.bm_quantize_lonlat(_dev_ptr(lonlat, "float64", (2,)), n, _dev_ptr(out, "int32", (2,)),
                                  _stream_handle(stream)))
    return out


def autotune(index: Index, sample_xy, stream=None) -> Tuning:
    """Launch shape picked by timing on a sample (int32 CUDA tensor [n, 2])."""
    t = Tuning()
    _check(lib.bm_autotune(index.handle, _dev_ptr(sample_xy, "int32", (2,)), sample_xy.shape[0],
                           C.byref(t), _stream_handle(stream)))
    return t


def _batch_rows(xys, outs):
    if len(xys) != len(outs):
        raise ValueError("xys and outs differ in length")
    rows = []
    for xy, out in zip(xys, outs):
        n = xy.shape[0]
        if out.shape[0] != n:
            raise ValueError("an output has the wrong length")
        rows.append((_dev_ptr(xy, "int32", (2,)).value or 0, _dev_ptr(out, "int32").value or 0, n))
    return rows


def make_rows(rows):
    """ctypes Batch array from (xy pointer, out pointer, n) triples."""
    return (Batch * max(len(rows), 1))(*[Batch(a, b, n) for a, b, n in rows])


def batch_table(xys, outs, device=None):
    """Device table of (xy, out, n) descriptors for map_batches (int64 [nb, 3])."""
    import torch
    rows = _batch_rows(xys, outs)
    dev = device if device is not None else (xys[0].device if xys else "cuda")
    return torch.tensor(rows if rows else [[0, 0, 0]], dtype=torch.int64)[: len(rows)].to(dev)


def map_batch_table(index: Index, table, stream=None, tuning: Tuning | None = None) -> None:
    """Map every batch of a device table built by batch_table() in one launch."""
    import torch
    if not (isinstance(table, torch.Tensor) and table.is_cuda and table.dtype == torch.int64
            and table.dim() == 2 and table.shape[1] == 3 and table.is_contiguous()):
        raise TypeError("table must be a contiguous int64 CUDA tensor [nb, 3]")
    nb = table.shape[0]
    _check(lib.bm_map_batch_table(index.handle, C.c_void_p(table.data_ptr()) if nb else None, nb,
                                  C.byref(tuning) if tuning is not None else None, _stream_handle(stream)))


def map_batches(index: Index, xy, batch_off, out, stream=None, tuning: Tuning | None = None) -> None:
    """Map nb = len(batch_off) - 1 batches lying back to back in xy (int32
    CUDA [n, 2]); batch_off is an int64 CUDA tensor of nb + 1 offsets, out an
    int32 CUDA tensor [n]. One persistent launch."""
    nb = batch_off.shape[0] - 1
    if nb < 0:
        raise ValueError("batch_off needs at least one entry")
    if out.shape[0] != xy.shape[0]:
        raise ValueError("out has the wrong length")
    _check(lib.bm_map_batches(index.handle, _dev_ptr(xy, "int32", (2,)), _dev_ptr(batch_off, "int64"), nb,
                              _dev_ptr(out, "int32"), C.byref(tuning) if tuning is not None else None,
                              _stream_handle(stream)))


class BatchPlan:
    """Batched form as captured HIP graphs, replayed with new batches: offsets
    into one concatenated array (run_offsets), or a host table of
    descriptors (run, run_rows)."""

    def __init__(self, index: Index, max_batches: int, tuning: Tuning | None = None, max_points: int = 0):
        self._index = index  # keep alive
        h = C.c_void_p()
        _check(lib.bm_batch_plan_create(index.handle, max_points, max_batches,
                                        C.byref(tuning) if tuning is not None else None, C.byref(h)))
        self._h = h
        self.max_batches = max_batches
        self.max_points = max_points

    def run_offsets(self, xy, batch_off, out, stream=None) -> None:
        """Replay over batches back to back in xy (int32 CUDA [n, 2]) with
        device offsets batch_off (int64 CUDA [nb + 1]) into out (int32 CUDA
        [n]); batches ending beyond max_points are skipped."""
        nb = batch_off.shape[0] - 1
        if nb < 0:
            raise ValueError("batch_off needs at least one entry")
        if out.shape[0] != xy.shape[0]:
            raise ValueError("out has the wrong length")
        _check(lib.bm_batch_plan_run(self._h, _dev_ptr(xy, "int32", (2,)), _dev_ptr(batch_off, "int64"), nb,
                                     _dev_ptr(out, "int32"), _stream_handle(stream)))

    def run(self, xys, outs, stream=None) -> None:
        rows = _batch_rows(xys, outs)
        self.run_rows(make_rows(rows), len(rows), stream)

    def run_rows(self, rows, nb: int, stream=None) -> None:
        """Replay with a prebuilt ctypes Batch array (see make_rows)."""
        _check(lib.bm_batch_plan_run_table(self._h, rows, nb, _stream_handle(stream)))

    def close(self) -> None:
        h, self._h = getattr(self, "_h", None), None
        if h:
            lib.bm_batch_plan_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def server_cfg(**kw) -> ServerCfg:
    c = ServerCfg()
    _check(lib.bm_server_cfg_default(C.byref(c)))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class Server:
    """Continuous-batching request loop over a resident index (host buffers)."""

    def __init__(self, index: Index, cfg: ServerCfg | None = None):
        self._index = index
        h = C.c_void_p()
        _check(lib.bm_server_create(index.handle, C.byref(cfg) if cfg is not None else None, C.byref(h)))
        self._h = h

    def submit(self, xy: np.ndarray, out: np.ndarray) -> int:
        """Queue int32 [n, 2] points; results land in int32 [n] `out` (both
        numpy arrays, kept alive by the caller until wait())."""
        assert xy.dtype == np.int32 and xy.flags.c_contiguous and xy.ndim == 2 and xy.shape[1] == 2
        assert out.dtype == np.int32 and out.flags.c_contiguous and out.shape == (xy.shape[0],)
        t = C.c_uint64()
        _check(lib.bm_server_submit(self._h, xy.ctypes.data if xy.size else None, xy.shape[0],
                                    out.ctypes.data if out.size else None, C.byref(t)))
        return t.value

    def try_submit(self, xy, out):
        try:
            return self.submit(xy, out)
        except BlockmapError as e:
            if e.code == BM_EBUSY:
                return None
            raise

    def wait(self, ticket: int, timeout_us: int = -1) -> None:
        _check(lib.bm_server_wait(self._h, ticket, timeout_us))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib.bm_server_stats(self._h, C.byref(st)))
        return st.as_dict()

    def reset_stats(self) -> None:
        _check(lib.bm_server_reset_stats(self._h))

    def run_trace(self, reqs, arrival_us) -> None:
        """reqs: list of (xy, out) numpy pairs; arrival_us: float64 offsets."""
        arr = (Request * max(len(reqs), 1))(*[Request(x.ctypes.data, o.ctypes.data, x.shape[0]) for x, o in reqs])
        at = np.ascontiguousarray(arrival_us, np.float64)
        _check(lib.bm_server_run_trace(self._h, arr, len(reqs), at.ctypes.data))

    def close(self) -> None:
        h, self._h = getattr(self, "_h", None), None
        if h:
            lib.bm_server_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def exported_symbols():
    return sorted(_SIGS)
