"""The C interface without a GPU: the library loads, exports every declared
entry point, and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", txt, flags=re.M):
            name = m.group(1)
            if name not in ("if", "while", "for", "return", "sizeof"):
                names.add(name)
    return names


def test_library_exports_every_declared_symbol():
    import paper_2005_03156_amd as bm
    declared = _declared()
    assert {"map_points", "bm_index_create", "bm_quantize_lonlat", "bm_last_error"} <= declared
    lib = C.CDLL(bm.LIB_PATH)
    missing = [n for n in sorted(declared) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(bm.exported_symbols()) <= declared


def test_library_is_built_for_gfx950():
    import paper_2005_03156_amd as bm
    data = open(bm.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _square_desc(bm, verts, off, n_groups=None, parents=None):
    vo = np.ascontiguousarray(off, np.int64)
    vv = np.ascontiguousarray(verts, np.int32)
    keep = [vo, vv]
    if parents is None:
        d = bm.IndexDesc(vo.shape[0] - 1, vo.ctypes.data, vv.ctypes.data, 0, None, None)
    else:
        ng = np.ascontiguousarray(n_groups, np.int64)
        ps = [np.ascontiguousarray(p, np.int32) for p in parents]
        arr = (C.c_void_p * len(ps))(*[p.ctypes.data for p in ps])
        keep += [ng, ps, arr]
        d = bm.IndexDesc(vo.shape[0] - 1, vo.ctypes.data, vv.ctypes.data, len(ps), ng.ctypes.data,
                         C.cast(arr, C.c_void_p))
    return d, keep


def _create(bm, d):
    h = C.c_void_p()
    rc = bm.lib.bm_index_create(C.byref(d), C.byref(h))
    return rc, bm.lib.bm_last_error().decode()


def test_descriptor_validation_without_gpu():
    import paper_2005_03156_amd as bm
    sq = [[0, 0], [10, 0], [10, 10], [0, 10]]
    # negative coordinate
    d, keep = _square_desc(bm, [[0, 0], [10, -1], [10, 10], [0, 10]], [0, 4])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_ERANGE and "coordinate" in msg
    # ring with two vertices
    d, keep = _square_desc(bm, [[0, 0], [10, 0]], [0, 2])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_EINVAL and "fewer than 3" in msg
    # ring above 2^24 vertices (the buffer is as long as declared)
    d, keep = _square_desc(bm, np.zeros(((1 << 24) + 1, 2), np.int32), [0, (1 << 24) + 1])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_EINVAL and "2^24" in msg
    # vert_off[0] != 0
    d, keep = _square_desc(bm, sq, [1, 4])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_EINVAL
    # parent out of range
    d, keep = _square_desc(bm, sq, [0, 4], [2], [np.array([2], np.int32)])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_EINVAL and "parent" in msg
    # zero groups on a level
    d, keep = _square_desc(bm, sq, [0, 4], [0], [np.array([0], np.int32)])
    rc, msg = _create(bm, d)
    assert rc == bm.BM_EINVAL
    # null descriptor / output
    assert bm.lib.bm_index_create(None, None) == bm.BM_EINVAL
    del keep


def test_map_points_argument_errors_without_gpu():
    import paper_2005_03156_amd as bm
    assert bm.lib.map_points(None, None, 10, None, None) == bm.BM_EINVAL
    assert "null index" in bm.lib.bm_last_error().decode()
    assert bm.lib.bm_quantize_lonlat(None, -1, None, None) == bm.BM_EINVAL
    assert bm.lib.bm_quantize_lonlat(None, 0, None, None) == bm.BM_OK
    t = bm.tuning_default()
    assert t.edge_chunk in (4, 8, 16) and 1 <= t.blocks_per_cu <= 8


def test_product_package_does_not_reference_the_oracle():
    """The product path (package sources) never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2005_03156_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert "oracle" not in txt.lower().replace("oracle-free", ""), fn


def test_count_and_cover_argument_checks():
    """Bad sizes and null buffers are refused before any device work."""
    import paper_2005_03156_amd as bm
    lib = bm.lib
    assert lib.bm_count_per_block(None, -1, 10, None, None) == bm.BM_EINVAL
    assert lib.bm_count_per_block(None, 5, 10, None, None) == bm.BM_EINVAL
    assert lib.bm_count_per_block(None, 0, -3, None, None) == bm.BM_EINVAL
    assert lib.map_points_cover(None, None, 10, None, 0, None) == bm.BM_EINVAL
    assert lib.bm_cover_create(None, None, None, None) == bm.BM_EINVAL
    assert lib.bm_cover_get_info(None, None) == bm.BM_EINVAL
    lib.bm_cover_destroy(None)
    assert b"cover" in lib.bm_last_error()
