"""GPU parity of the per-block aggregation that the mapping feeds (paper
Sec. I-II: merging census data by block; App. A: each point's block FIPS code):
points per block and the per-point join of a block table, against the CPU
oracle's plain loops, element by element."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_map import boundary_points, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    return torch


@pytest.fixture(scope="module")
def bm():
    import paper_2005_03156_amd as bm
    return bm


def _odd_ids(nb, n, seed):
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, -7, nb, nb - 1, 2**31 - 1, -2**31, 0, 5], np.int32), n)


def test_join_per_block_vs_oracle(torch_cuda, bm):
    """Codes joined per point on the device equal the oracle's join, for the
    mapped ids of grid221k points (with boundary points), for ids outside the
    table, ragged and empty calls, and pointers not 16-byte aligned (the
    one-id-per-thread form)."""
    torch = torch_cuda
    g = synth.geometry("grid221k")
    ix = bm.Index.from_geometry(g)
    table = synth.block_codes(g)
    dtab = torch.from_numpy(table).cuda()
    pts = np.concatenate([synth.points("grid221k", 1_000_003, i0=77_000_000), boundary_points(g, 5000, seed=9)])
    ids = bm.map_points(ix, torch.from_numpy(pts).cuda())
    odd = torch.from_numpy(_odd_ids(g.n_blocks, 10_001, 1)).cuda()
    for name, t in [("mapped", ids), ("odd", odd), ("ragged", ids[:4097]), ("one", ids[:1]), ("empty", ids[:0]),
                    ("offset by one id", ids[1:100_001])]:
        for fill in (-1, 123456789012):
            say("join", name, fill)
            got = bm.join_per_block(t, dtab, fill=fill).cpu().numpy()
            want = oracle.join_per_block(t.cpu().numpy(), table, fill=fill)
            assert np.array_equal(got, want), (name, fill)
    # an output that starts 8 bytes into its allocation (not 16-byte aligned)
    big = torch.full((ids.shape[0] + 1,), -5, dtype=torch.int64, device="cuda")
    bm.join_per_block(ids, dtab, out=big[1:])
    want = oracle.join_per_block(ids.cpu().numpy(), table)
    got = big.cpu().numpy()
    assert got[0] == -5 and np.array_equal(got[1:], want)
    # an empty table: every id takes the fill value
    e = bm.join_per_block(ids[:1000], dtab[:0], fill=3).cpu().numpy()
    assert (e == 3).all()


def test_count_per_block_vs_oracle(torch_cuda, bm):
    """Points per block on the device (atomic form below 2^20 ids, bucketed
    above) equal the oracle's count, for mapped ids and ids outside [0, nb)."""
    torch = torch_cuda
    g = synth.geometry("grid221k")
    ix = bm.Index.from_geometry(g)
    ids = bm.map_points(ix, torch.from_numpy(synth.points("grid221k", 3_000_000, i0=60_000_000)).cuda())
    odd = torch.from_numpy(_odd_ids(g.n_blocks, 2_000_000, 2)).cuda()
    for name, t in [("mapped", ids), ("mapped, small call", ids[:300_001]), ("odd", odd),
                    ("odd, small call", odd[:5000])]:
        say("count", name)
        got = bm.count_per_block(t, g.n_blocks).cpu().numpy().view(np.uint64)
        assert np.array_equal(got, oracle.count_per_block(t.cpu().numpy(), g.n_blocks)), name


def test_aggregation_at_full_size(torch_cuda, bm):
    """The census-scale workload's 100M mapped ids: per-block counts and the
    per-point code join equal the oracle's over every element."""
    torch = torch_cuda
    g = synth.geometry("grid221k")
    ix = bm.Index.from_geometry(g)
    n = synth.n_points("grid221k")
    say("aggregation full size: mapping", n)
    ids = bm.map_points(ix, torch.from_numpy(synth.points("grid221k", n)).cuda())
    host = ids.cpu().numpy()
    counts = bm.count_per_block(ids, g.n_blocks).cpu().numpy().view(np.uint64)
    assert np.array_equal(counts, oracle.count_per_block(host, g.n_blocks))
    table = synth.block_codes(g)
    codes = bm.join_per_block(ids, torch.from_numpy(table).cuda())
    say("aggregation full size: join")
    assert np.array_equal(codes.cpu().numpy(), oracle.join_per_block(host, table))
