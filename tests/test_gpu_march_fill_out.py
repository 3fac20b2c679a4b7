"""The march fill's output contract through the C-ABI: every packed sample
lands at its row's start plus its index, bit for bit the oracle's, whatever
the output arrays' alignment; nothing is written outside the rows (gaps
between rows), at or beyond a row's count or at or beyond the capacity."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, grid_spec, host

pytestmark = pytest.mark.gpu

SENTINEL = np.float32(-7.25)


@pytest.fixture(scope="module")
def case(gpu_lib):
    w = scenes.tiny()
    ref = oracle.march(w.rays_o, w.rays_d, w.bits, w.res, n_levels=w.n_levels,
                       half_extent0=w.half_extent0, dt0=w.dt0)
    return w, ref


def fill_raw(txs, w, info, capacity, t0, t1, rid, grid=None):
    from paper_2305_04966_amd import ops
    g = grid if grid is not None else grid_spec(txs, w.bits, w.res, w.n_levels, w.half_extent0)
    o, d = dev(w.rays_o), dev(w.rays_d)
    p = ops._params(0.0, float("inf"), w.dt0, 0)
    st = txs.load().txs_march_fill(C.byref(g.struct()), C.byref(p), ops._ptr(o), ops._ptr(d),
                                   o.shape[0], ops._ptr(info), capacity, ops._ptr(t0),
                                   ops._ptr(t1), ops._ptr(rid), ops._stream())
    ops.check(st, "txs_march_fill")
    torch.cuda.synchronize()


def out_arrays(n, offsets, want_rid=True):
    """Sentinel-filled outputs whose data starts `offsets` elements into
    their allocation (so 4, 8 or 12 bytes off 16-byte alignment)."""
    def one(off, dtype, fill):
        buf = torch.full((n + off + 8,), fill, dtype=dtype, device="cuda")
        return buf[off:off + n]
    t0 = one(offsets[0], torch.float32, float(SENTINEL))
    t1 = one(offsets[1], torch.float32, float(SENTINEL))
    rid = one(offsets[2], torch.int32, -3) if want_rid else None
    return t0, t1, rid


@pytest.mark.parametrize("offsets,want_rid", [((0, 0, 0), True), ((1, 0, 0), True),
                                              ((0, 3, 2), True), ((2, 2, 1), False),
                                              ((0, 0, 0), False)])
def test_fill_any_alignment(gpu_lib, case, offsets, want_rid):
    w, ref = case
    S = int(ref["total"])
    t0, t1, rid = out_arrays(S, offsets, want_rid)
    fill_raw(gpu_lib, w, dev(ref["packed_info"]), S, t0, t1, rid)
    assert np.array_equal(host(t0), ref["t0"])
    assert np.array_equal(host(t1), ref["t1"])
    if want_rid:
        assert np.array_equal(host(rid), ref["ray_id"])


@pytest.mark.parametrize("offsets", [(0, 0, 0), (3, 1, 2)])
def test_fill_rows_with_gaps_and_short_counts(gpu_lib, case, offsets):
    # rows placed with gaps of 0..9 positions between them, and every 5th
    # row's count cut short: the fill writes exactly each row's first `count`
    # samples at its start and leaves every other position untouched
    w, ref = case
    counts = ref["counts"].astype(np.int64)
    g = scenes.rng(17)
    gaps = g.integers(0, 10, counts.size)
    cut = counts.copy()
    cut[::5] = counts[::5] // 3
    starts = np.concatenate([[0], np.cumsum(counts + gaps)[:-1]]) + gaps[0]
    S = int(starts[-1] + counts[-1] + 5)
    info = np.stack([starts, cut], 1).astype(np.int32)
    t0, t1, rid = out_arrays(S, offsets)
    fill_raw(gpu_lib, w, dev(info), S, t0, t1, rid)
    e0 = np.full(S, SENTINEL, np.float32)
    e1 = np.full(S, SENTINEL, np.float32)
    er = np.full(S, -3, np.int32)
    rs = ref["packed_info"][:, 0]
    for r in range(counts.size):
        a, c = starts[r], cut[r]
        e0[a:a + c] = ref["t0"][rs[r]:rs[r] + c]
        e1[a:a + c] = ref["t1"][rs[r]:rs[r] + c]
        er[a:a + c] = r
    assert np.array_equal(host(t0), e0)
    assert np.array_equal(host(t1), e1)
    assert np.array_equal(host(rid), er)


@pytest.mark.parametrize("frac", [0.0, 0.01, 0.5, 0.999])
def test_fill_capacity_bound(gpu_lib, case, frac):
    # a capacity below the total: positions below it are the oracle's, the
    # rest of the (larger) buffer is untouched
    w, ref = case
    S = int(ref["total"])
    cap = int(S * frac) + 3
    t0, t1, rid = out_arrays(S, (1, 0, 0))
    fill_raw(gpu_lib, w, dev(ref["packed_info"]), cap, t0, t1, rid)
    for got, exp, fill in ((t0, ref["t0"], SENTINEL), (t1, ref["t1"], SENTINEL),
                           (rid, ref["ray_id"], -3)):
        got = host(got)
        assert np.array_equal(got[:cap], exp[:cap])
        assert (got[cap:] == fill).all()


def test_fill_skipping_kernel_gaps(gpu_lib, case):
    # the skipping kernels write their samples under the same contract
    w, ref = case
    g = gpu_lib.GridSpec(dev(np.asarray(w.bits, np.uint32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                         w.half_extent0, skip=True)
    counts = ref["counts"].astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(counts + 3)[:-1]]) + 1
    S = int(starts[-1] + counts[-1] + 2)
    info = np.stack([starts, counts], 1).astype(np.int32)
    t0, t1, rid = out_arrays(S, (0, 2, 0))
    fill_raw(gpu_lib, w, dev(info), S, t0, t1, rid, grid=g)
    sel = np.concatenate([np.arange(s, s + c) for s, c in zip(starts, counts)])
    got0, got1, gotr = host(t0), host(t1), host(rid)
    assert np.array_equal(got0[sel], ref["t0"]) and np.array_equal(got1[sel], ref["t1"])
    assert np.array_equal(gotr[sel], ref["ray_id"])
    rest = np.ones(S, bool)
    rest[sel] = False
    assert (got0[rest] == SENTINEL).all() and (gotr[rest] == -3).all()
