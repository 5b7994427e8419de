"""The entry point that allocates nothing (map_points_noalloc): called through
the C-ABI, its ids equal those of map_points, the entry point it varies, on two
calls in a row (the second smaller, so it runs over the first call's leftover
scratch), on an unsorted small call, on an empty call, and over both index
kinds (2^22-point and 2^26-point sort chunks); a call above its limit is
refused without touching the GPU."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[gpu]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    import paper_2005_03156_amd as bm
    return torch, bm


@pytest.mark.parametrize("workload", ["grid221k", "quadtree8m"])
def test_noalloc_equals_map_points(env, workload):
    torch, bm = env
    g = synth.geometry(workload)
    ix = bm.Index.from_geometry(g)
    s = torch.cuda.current_stream()
    for k, n in enumerate([1 << 22, 1_500_001, 4_097, 0, (1 << 20) + 3]):
        _say("noalloc", workload, "call", k, "n =", n)
        xy = torch.from_numpy(synth.points(workload, n, i0=3_000_000 * k)).cuda()
        a = torch.full((n,), -7, dtype=torch.int32, device="cuda")
        b = torch.full((n,), -9, dtype=torch.int32, device="cuda")
        bm.map_points_noalloc(ix, xy, a, s)
        bm.map_points(ix, xy, b, s)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (workload, k, n)
    xy = torch.zeros(((1 << 22) + 1, 2), dtype=torch.int32, device="cuda")
    out = torch.empty((1 << 22) + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(bm.BlockmapError) as e:
        bm.map_points_noalloc(ix, xy, out, s)
    assert e.value.code == bm.BM_ERANGE
    ix.close()
