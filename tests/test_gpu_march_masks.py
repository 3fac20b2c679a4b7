"""Masked lattice march: txs_march_count_masked records the occupancy ballot of
every 64-point group a ray walks and txs_march_fill_masked replays it instead
of testing the cells again.  The packed samples must equal the oracle's and
the unmasked march's bit for bit whether every row replays, some rows run
past their mask budget (the fill then tests their points), none records
(groups_per_ray 0) or the skipping kernels march (rows marked not
replayable)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, grid_spec, host

pytestmark = pytest.mark.gpu


def run(txs, w, groups=None, rays=None, grid=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    o, d = dev(o), dev(d)
    g = grid if grid is not None else grid_spec(txs, w.bits, w.res, w.n_levels, w.half_extent0)
    if groups is None:
        groups = txs.MarchMasks.groups_for(g, w.dt0)
    m = txs.MarchMasks(o.shape[0], groups, o.device)
    p = txs.march(g, o, d, dt0=w.dt0, masks=m, **kw)
    plain = txs.march(g, o, d, dt0=w.dt0, **kw)
    torch.cuda.synchronize()
    rows = host(m.words).reshape(o.shape[0], groups + 1)
    return p, plain, rows


def oracle_march(w, rays=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    return oracle.march(o, d, w.bits, w.res, n_levels=w.n_levels, half_extent0=w.half_extent0,
                        dt0=w.dt0, **kw)


def assert_same(p, q):
    for name in ("packed_info", "t0", "t1", "ray_id"):
        assert np.array_equal(host(getattr(p, name)), host(getattr(q, name))), name


def assert_oracle(p, ref):
    assert np.array_equal(host(p.packed_info), ref["packed_info"])
    assert np.array_equal(host(p.t0), ref["t0"])
    assert np.array_equal(host(p.t1), ref["t1"])
    assert np.array_equal(host(p.ray_id), ref["ray_id"])


def popcounts(rows):
    """Per ray: occupied points over the recorded groups (words 1 .. word 0)."""
    g = rows.shape[1] - 1
    walked = rows[:, 0].astype(np.int64)
    keep = np.arange(g)[None, :] < np.minimum(walked, g)[:, None]
    bits = np.unpackbits(np.ascontiguousarray(rows[:, 1:]).view(np.uint8), axis=1)
    per_word = bits.reshape(rows.shape[0], g, 64).sum(axis=2)
    return (per_word * keep).sum(axis=1)


@pytest.fixture(scope="module")
def tiny():
    return scenes.tiny()


def test_masked_tiny_every_row_replays(gpu_lib, tiny):
    p, plain, rows = run(gpu_lib, tiny)
    g = rows.shape[1] - 1
    ref = oracle_march(tiny)
    assert ref["total"] > 10000
    assert_oracle(p, ref)
    assert_same(p, plain)
    # the bound on groups per ray holds: every row was recorded whole
    assert (rows[:, 0] <= g).all() and (rows[:, 0] > 0).any()
    # the recorded ballots hold exactly the samples the count found
    assert np.array_equal(popcounts(rows), ref["counts"])


def test_masked_image_full_size(gpu_lib):
    # 1024x1024 camera rays in the benchmark's launch: the masked march equals
    # the unmasked one everywhere and the oracle on every 37th ray
    w = scenes.image()
    p, plain, rows = run(gpu_lib, w)
    assert_same(p, plain)
    assert (rows[:, 0] <= rows.shape[1] - 1).all()
    idx = np.arange(0, w.n_rays, 37)
    ref = oracle_march(w, rays=(w.rays_o[idx], w.rays_d[idx]))
    info = host(p.packed_info)
    assert np.array_equal(info[idx, 1], ref["counts"])
    sel = np.concatenate([np.arange(info[r, 0], info[r, 0] + info[r, 1]) for r in idx])
    assert np.array_equal(host(p.t0)[sel], ref["t0"])
    assert np.array_equal(host(p.t1)[sel], ref["t1"])


def test_masked_cascade(gpu_lib):
    w = scenes.unbounded(128, 64, n_cams=8, res=64)
    p, plain, rows = run(gpu_lib, w)
    ref = oracle_march(w)
    assert ref["total"] > 0
    assert_oracle(p, ref)
    assert_same(p, plain)
    assert (rows[:, 0] <= rows.shape[1] - 1).all()
    assert np.array_equal(popcounts(rows), ref["counts"])


@pytest.mark.parametrize("groups", [0, 3, 10, 12])
def test_masked_budget_overflow(gpu_lib, tiny, groups):
    # rows that walk more groups than the budget are not replayed: the fill
    # tests their points; rows within it replay
    p, plain, rows = run(gpu_lib, tiny, groups=groups)
    ref = oracle_march(tiny)
    assert_oracle(p, ref)
    assert_same(p, plain)
    over = rows[:, 0] > groups
    assert over.any()
    if groups >= 10:
        # the tiny workload's rays walk 10 to 16 groups: rows of exactly the
        # budget and below replay
        assert (~over & (ref["counts"] > 0)).any()


@pytest.mark.parametrize("kw", [dict(max_per_ray=11), dict(near=2.5, far=3.4), dict(near=0.5)])
def test_masked_options(gpu_lib, tiny, kw):
    p, plain, rows = run(gpu_lib, tiny, **kw)
    assert_oracle(p, oracle_march(tiny, **kw))
    assert_same(p, plain)


def test_masked_with_brick_occupancy(gpu_lib, tiny):
    # a grid descriptor carrying brick occupancy selects the skipping
    # kernels, which record nothing: every row is marked not replayable
    g = gpu_lib.GridSpec(dev(np.asarray(tiny.bits, np.uint32)), tiny.res, tiny.n_levels,
                         (0.0, 0.0, 0.0), tiny.half_extent0, skip=True)
    p, plain, rows = run(gpu_lib, tiny, grid=g)
    assert_oracle(p, oracle_march(tiny))
    assert_same(p, plain)
    assert (rows[:, 0] == rows.shape[1]).all()


def test_masked_degenerate(gpu_lib, tiny):
    # no rays; rays that all miss (rows of zero groups replay trivially)
    w0 = scenes.Workload("x", tiny.fld, tiny.bits, 64, 1, 1.5, tiny.rays_o[:0],
                         tiny.rays_d[:0], 0.01)
    p, _, _ = run(gpu_lib, w0, groups=4)
    assert p.n_samples == 0 and p.packed_info.shape == (0, 2)
    miss_o = np.tile(np.float32([[0, 0, 5.0]]), (100, 1))
    miss_d = np.tile(np.float32([[0, 0, 1.0]]), (100, 1))
    p, _, rows = run(gpu_lib, tiny, rays=(miss_o, miss_d))
    assert p.n_samples == 0 and (rows[:, 0] == 0).all()


def test_masked_rejects_budget_above_limit(gpu_lib, tiny):
    g = grid_spec(gpu_lib, tiny.bits, tiny.res)
    o, d = dev(tiny.rays_o[:64]), dev(tiny.rays_d[:64])
    m = gpu_lib.MarchMasks(64, 1, o.device)
    m.groups = (1 << 14) + 1  # words sized for the check below to pass first
    m.words = torch.empty(int(gpu_lib.load().txs_march_mask_words(64, m.groups)),
                          dtype=torch.int64, device=o.device)
    with pytest.raises(gpu_lib.TxsError, match="groups_per_ray"):
        gpu_lib.march_count(g, o, d, dt0=tiny.dt0, masks=m)
