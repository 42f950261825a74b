"""Parity of the persistent tile-selection kernel (wm_select_tile) with the
FP64 oracle: the selected local index is bit-exact; near-ties (runner-up
within 1e-6) are reported separately and accepted when the GPU picks any
member of the near-tie set."""
import numpy as np
import pytest
import torch

from paper_2605_04178_amd import synth
from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def wmb():
    need_gpu()
    from paper_2605_04178_amd import wavemodel
    wavemodel.lib()
    return wavemodel


def _check(wmb, orc, p, sh, tag):
    say("select_tile parity", tag, "shapes =", sh.n)
    dsh = wmb.DeviceShapes.from_host(sh)
    best, cost, tie = (x.cpu().numpy() for x in wmb.select_tile(dsh, p))
    bo, co, to = orc.select_tile(p, sh)
    clean = to == 0
    assert np.array_equal(best[clean], bo[clean]), (tag, np.nonzero(best[clean] != bo[clean])[0][:5])
    assert np.array_equal(tie, to), tag
    fin = np.isfinite(co)
    assert np.array_equal(np.isfinite(cost), fin)
    assert np.all(np.abs(cost[fin] - co[fin]) <= 1e-12 * co[fin])
    # near-ties: the GPU's pick lies in the set within 1e-6 of the minimum
    if (~clean).any():
        allc = orc.tile_costs(p, sh)
        for i in np.nonzero(~clean)[0]:
            a, b = sh.cand_off[i], sh.cand_off[i + 1]
            c = allc[a:b]
            members = np.nonzero(np.isfinite(c) & (c <= co[i] * (1 + 1e-6)))[0]
            assert best[i] in members
    return best, cost, tie, bo, to


@pytest.mark.parametrize("dt_seed", [102, 5])
def test_select_tile_full_size(wmb, orc, dt_seed):
    """2^16 shapes, 8-96 candidates each, every output checked."""
    p = synth.param_set(0)
    sh = synth.shapes(1 << 16, dt_seed)
    best, cost, tie, bo, to = _check(wmb, orc, p, sh, f"seed {dt_seed}")
    assert (best >= 0).mean() > 0.9
    say("near ties:", int(to.sum()), "of", sh.n)


@pytest.mark.parametrize("which", ["mi300a", "L3", "eta"])
def test_select_tile_other_parameter_sets(wmb, orc, which):
    p = {"mi300a": synth.mi300a_like(), "L3": synth.param_set(0, n_levels=3),
         "eta": synth.param_set(0, combine=1)}[which]
    _check(wmb, orc, p, synth.shapes(8192, 7), which)


def test_select_tile_edge_cases(wmb, orc):
    p = synth.param_set(0)
    codes = synth.all_tile_codes()
    big = [int(synth.tile_code(3, 3, 2, 1))]                  # 256x256x64 fp64: infeasible
    lists = [
        [],                                                   # no candidates
        big,                                                  # nothing feasible
        [int(codes[10]), int(codes[10]), int(codes[3])],      # exact duplicate -> tie, lowest index
        [int(codes[5]) | (1 << 9), int(codes[7])],            # reserved bit -> invalid candidate
        [int(synth.tile_code(0, 0, 3, 1)), int(codes[0])],    # kd code 3 -> invalid
        list(int(c) for c in codes),                          # the full 384-tile sweep
        list(int(c) for c in codes[::-1]),
        [int(codes[20])],
    ]
    M = np.array([512, 16384, 1000, 300, 128, 16384, 4096, 1], np.int32)
    N = np.array([512, 16384, 1000, 5000, 128, 16384, 128, 1], np.int32)
    K = np.array([512, 16384, 77, 300, 128, 16384, 16384, 1], np.int32)
    dt = np.array([0, 0, 1, 2, 3, 0, 3, 1], np.int32)
    off = np.zeros(len(lists) + 1, np.int32)
    off[1:] = np.cumsum([len(x) for x in lists])
    code = np.array([c for x in lists for c in x], np.uint32)
    sh = synth.Shapes(M, N, K, dt, off, code)
    best, cost, tie, bo, to = _check(wmb, orc, p, sh, "edge")
    assert best[0] == -1 and np.isinf(cost[0])
    assert best[1] == -1 and np.isinf(cost[1])
    if bo[2] in (0, 1):
        assert best[2] == 0 and tie[2] == 1
    assert best[3] == 1 and best[4] == 1


@pytest.mark.parametrize("n", [1, 2, 7, 9, 13, 1001])
def test_select_tile_ragged_shape_counts(wmb, orc, n):
    """Shape counts that leave the last batch of eight partly empty."""
    _check(wmb, orc, synth.param_set(0), synth.shapes(n, 40 + n), f"n={n}")


def test_select_tile_int32_limit_shapes(wmb, orc):
    """Sides up to 2^31 - 1 with the full 384-tile sweep: flops and bytes past
    2^63, tiles whose grid exceeds 2^31 - 1 workgroups (infeasible)."""
    p = synth.param_set(0)
    big = 2 ** 31 - 1
    dims = [(big, big, big, 0), (big, big, big, 3), (big, 1, big, 0), (1 << 20, 1 << 20, big, 1),
            (big, 64, big, 3), (65536, 65536, 65536, 2), (1 << 21, 1 << 21, 7, 2), (1, big, 1, 1)]
    codes = synth.all_tile_codes().astype(np.uint32)
    M, N, K, dt = (np.array(c, np.int32) for c in zip(*dims))
    off = (np.arange(len(dims) + 1) * len(codes)).astype(np.int32)
    sh = synth.Shapes(M, N, K, dt, off, np.tile(codes, len(dims)))
    best, cost, tie, bo, to = _check(wmb, orc, p, sh, "int32 limits")
    assert best[0] == -1 and best[1] == -1          # every grid too large
    assert (best[2:] >= 0).all()


def test_select_tile_list_lengths_and_duplicates(wmb, orc):
    """List lengths around one and two wavefronts (63..129, 200) and lists
    built from two or three distinct codes repeated, so that a shape puts up
    to its whole list into the float64 window; several thousand shapes so
    that every wave handles many of them.  Exact duplicates cost the same,
    so the pick must be the first occurrence of the winning code."""
    p = synth.param_set(0)
    rng = np.random.Generator(np.random.PCG64(31))
    tiles = synth.all_tile_codes()
    lens = np.array([1, 2, 63, 64, 65, 127, 128, 129, 200, 40])
    n = 6000
    cnt = lens[rng.integers(0, len(lens), n)]
    lists = []
    for i in range(n):
        if i % 3 == 0:
            pool = tiles[rng.permutation(len(tiles))[:int(rng.integers(2, 4))]]
            lists.append(pool[rng.integers(0, len(pool), cnt[i])])
        else:
            lists.append(tiles[rng.integers(0, len(tiles), cnt[i])])
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum(cnt)
    M = np.round(np.exp(rng.uniform(np.log(128), np.log(16384), n))).astype(np.int32)
    N = np.round(np.exp(rng.uniform(np.log(128), np.log(16384), n))).astype(np.int32)
    K = np.round(np.exp(rng.uniform(np.log(128), np.log(16384), n))).astype(np.int32)
    dt = rng.integers(0, 4, n).astype(np.int32)
    sh = synth.Shapes(M, N, K, dt, off, np.concatenate(lists).astype(np.uint32))
    best, cost, tie, bo, to = _check(wmb, orc, p, sh, "lengths/duplicates")
    for i in np.nonzero(best >= 0)[0]:
        L = lists[i]
        assert best[i] == int(np.nonzero(L == L[best[i]])[0][0]), i
    say("near ties:", int(to.sum()), "of", n)


def test_select_tile_graph_replay(wmb, orc):
    """The launch captured in a HIP graph and replayed, with eager work and
    syncs between replays; every replay must equal the eager result."""
    p = synth.param_set(0)
    sh = synth.shapes(20000, 9)
    dsh = wmb.DeviceShapes.from_host(sh)
    eager = [x.clone() for x in wmb.select_tile(dsh, p)]
    out = tuple(torch.full_like(x, 0) for x in eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        wmb.select_tile(dsh, p, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        wmb.select_tile(dsh, p, out=out)
    for r in range(4):
        for x in out:
            x.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(out, eager):
            assert torch.equal(a, b), r
        _ = torch.randn(1000, device="cuda").sum().item()   # eager work between replays


@pytest.mark.parametrize("pset", ["seed0", "seed1", "L3", "mi300a_like"])
def test_float32_cost_error_is_inside_the_window(wmb, orc, pset):
    """The selection re-evaluates in float64 every candidate within delta =
    3e-5 of the float32 minimum; that is sound if delta >= 4 x the float32
    cost error.  Every candidate of the 2^16-shape sweep (about 3.4 million)
    through wm_tile_costs (the selection's own first pass) against the
    oracle's float64 costs: infeasibility identical, largest relative error
    at most delta / 4."""
    p = {"seed0": synth.param_set(0), "seed1": synth.param_set(1), "L3": synth.param_set(2, n_levels=3),
         "mi300a_like": synth.mi300a_like()}[pset]
    sh = synth.shapes(1 << 16, 102)
    c32 = wmb.tile_costs(wmb.DeviceShapes.from_host(sh), p).cpu().numpy().astype(np.float64)
    c64 = orc.tile_costs(p, sh)
    fin = np.isfinite(c64)
    assert np.array_equal(np.isfinite(c32), fin)
    assert np.all(np.isposinf(c32[~fin]))
    err = np.abs(c32[fin] / c64[fin] - 1.0)
    say(f"tile costs ({pset}): {int(fin.sum())} feasible of {c64.size}, float32 error max {err.max():.2e}, "
        f"99.9th percentile {np.quantile(err, 0.999):.2e}; window 3e-5 / 4 = 7.5e-6")
    assert 4.0 * err.max() <= 3e-5
