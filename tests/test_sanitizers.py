"""Host code under sanitizers (nothing here touches a GPU): the CPU oracle
and the host-side index and cell-cover builders built with AddressSanitizer
and UndefinedBehaviorSanitizer, each giving exactly what the ordinary builds
give (the oracle's three routes per point; the index and cover files byte
for byte); and the served form's host copy pool under ThreadSanitizer and
AddressSanitizer. Any sanitizer report aborts the program, so each run must
exit cleanly."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2005_03156_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    probe = d / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    if subprocess.run(["gcc", *SAN, str(probe), "-o", str(d / "probe")], capture_output=True).returncode:
        pytest.skip("no sanitizer runtime for gcc here")
    od = str(d / "oracle_driver")
    subprocess.check_call(["gcc", "-std=gnu11", "-fopenmp", *SAN, os.path.join(HERE, "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "oracle.c"), "-o", od])
    idr = str(d / "index_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + CSRC,
                           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "sanitize", "index_driver.cpp"),
                           os.path.join(CSRC, "index.cpp"), os.path.join(CSRC, "cover.cpp"), "-L/opt/rocm/lib",
                           "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread", "-o", idr])
    return d, od, idr


def _comb(T=300, H=5000, o=1000):
    v = [(0, 0), (20 * (T - 1) + 10, 0)]
    for i in range(T - 1, -1, -1):
        v += [(20 * i + 10, H), (20 * i, H)]
        if i > 0:
            v += [(20 * i, 100), (20 * (i - 1) + 10, 100)]
    return np.array(v, np.int32) + o


def _cases():
    """(name, vert_off, verts, n_groups, parents, points)"""
    g = synth.geometry("grid1k")
    rng = np.random.default_rng(21)
    v = g.verts[rng.choice(g.verts.shape[0], 400, replace=False)]
    pts = np.concatenate([synth.points("grid1k", 3000), v, v - 1, v + 1]).astype(np.int32)
    out = [("grid1k", g.vert_off, g.verts, g.n_groups, g.parents, pts)]
    # a random two-level grouping with empty groups
    mid = rng.integers(0, 300, g.n_blocks).astype(np.int32)
    top = rng.integers(0, 7, 300).astype(np.int32)
    out.append(("grid1k random groups", g.vert_off, g.verts, [7, 300], [top, mid], pts))
    # overlapping rectangles and a comb (long slab lists), no hierarchy
    rects = [np.array([[x, y], [x + w, y], [x + w, y + h], [x, y + h]], np.int32)
             for x, y, w, h in rng.integers(0, 4000, (40, 4)) // [1, 1, 2, 2] + [0, 0, 1, 1]]
    rings = rects + [_comb()]
    off = np.concatenate([[0], np.cumsum([len(r) for r in rings])]).astype(np.int64)
    verts = np.concatenate(rings).astype(np.int32)
    p2 = np.stack([rng.integers(-10, 8000, 4000), rng.integers(-10, 6200, 4000)], 1).astype(np.int32)
    out.append(("rectangles and comb", off, verts, [], [], np.concatenate([p2, verts, verts - 1]).astype(np.int32)))
    return out


def _write_groups(f, n_groups, parents):
    f.write(np.asarray(n_groups, np.int64).tobytes())
    for p in parents:
        p = np.ascontiguousarray(p, np.int32)
        f.write(np.int64(p.shape[0]).tobytes())
        f.write(p.tobytes())


@pytest.mark.parametrize("case", range(3))
def test_oracle_under_sanitizers(drivers, case):
    d, od, _ = drivers
    name, vo, vv, ng, par, pts = _cases()[case]
    vo, vv = np.ascontiguousarray(vo, np.int64), np.ascontiguousarray(vv, np.int32)
    inp, outp = str(d / ("o%d.in" % case)), str(d / ("o%d.out" % case))
    with open(inp, "wb") as f:
        f.write(np.array([vo.shape[0] - 1, vv.shape[0], len(ng), pts.shape[0]], np.int64).tobytes())
        f.write(vo.tobytes())
        f.write(vv.tobytes())
        _write_groups(f, ng, par)
        f.write(np.ascontiguousarray(pts, np.int32).tobytes())
    r = subprocess.run([od, inp, outp], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (name, r.returncode, r.stderr[-3000:])
    got = np.fromfile(outp, np.int32).reshape(3, -1)
    want = oracle.brute(vo, vv, pts)
    assert np.array_equal(got[0], want), name
    assert np.array_equal(got[1], want), name
    if len(ng):
        assert np.array_equal(got[2], oracle.Hier(vo, vv, ng, par).map(pts)), name
    else:
        assert np.array_equal(got[2], want), name


@pytest.mark.parametrize("case, keep", [(0, 0), (0, 1), (1, 0), (2, 0)])
def test_index_and_cover_builders_under_sanitizers(drivers, case, keep):
    import paper_2005_03156_amd as bm
    d, _, idr = drivers
    name, vo, vv, ng, par, _ = _cases()[case]
    vo, vv = np.ascontiguousarray(vo, np.int64), np.ascontiguousarray(vv, np.int32)
    inp = str(d / ("i%d%d.in" % (case, keep)))
    got_ix, got_cv = str(d / ("i%d%d.bmi" % (case, keep))), str(d / ("c%d%d.bmc" % (case, keep)))
    with open(inp, "wb") as f:
        f.write(np.array([vo.shape[0] - 1, vv.shape[0], len(ng)], np.int64).tobytes())
        f.write(np.array([keep, 0], np.int32).tobytes())
        f.write(vo.tobytes())
        f.write(vv.tobytes())
        _write_groups(f, ng, par)
    r = subprocess.run([idr, inp, got_ix, got_cv], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (name, r.returncode, r.stderr[-3000:])
    want_ix, want_cv = str(d / "want.bmi"), str(d / "want.bmc")
    bm.build_index_file(want_ix, vo, vv, ng, par, keep_all_levels=bool(keep))
    assert open(got_ix, "rb").read() == open(want_ix, "rb").read(), name
    if not keep:  # the cover builds its own index with the default levels
        bm.build_cover_file(want_cv, vo, vv, ng, par, 0, 4)
        assert open(got_cv, "rb").read() == open(want_cv, "rb").read(), name


@pytest.mark.parametrize("san", ["thread", "address"])
def test_copy_pool_under_sanitizers(tmp_path, san):
    """The served form's host copy pool (several callers at once, long copies
    cut and shared out over the workers) under ThreadSanitizer and
    AddressSanitizer: every destination byte right, no report."""
    exe = str(tmp_path / ("copy_pool_" + san))
    flags = ["-fsanitize=" + san, "-fno-omit-frame-pointer", "-g", "-O1"]
    r = subprocess.run(["g++", "-std=c++17", *flags, "-I" + CSRC, os.path.join(HERE, "sanitize", "copy_pool_driver.cpp"),
                        "-o", exe, "-lpthread"], capture_output=True, text=True)
    if r.returncode:
        pytest.skip("no %s sanitizer runtime for g++ here" % san)
    for threads, callers, rounds in ((6, 4, 40), (1, 3, 10), (3, 8, 20)):
        r = subprocess.run([exe, str(threads), str(callers), str(rounds)], env=ENV, capture_output=True, text=True,
                           timeout=600)
        assert r.returncode == 0, (san, threads, callers, r.stdout[-500:], r.stderr[-3000:])
        assert " 0 wrong copies" in r.stdout
