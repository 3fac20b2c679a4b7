"""Empty-space skipping in the march (Section 3.1, "Spatial Skipping"; Table 1,
occupancy-grid row): the brick occupancy the march skips with, and the march
with it against the oracle's dense march (every lattice point tested), bit
for bit.  Sparse grids put their occupied cells on brick faces and the rays
run along and across brick planes (the cases where a bound that ignored the
recipe's rounding would skip an occupied point)."""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, grid_spec, host

pytestmark = pytest.mark.gpu


def brick_rays(res, n, seed, h=1.5):
    """Axis-parallel rays on brick planes (exactly, or a few binary32 steps
    off), rays tilted slightly or strongly off those planes, and diagonals
    through brick corners."""
    g = scenes.rng(seed)
    cell = 2 * h / res
    o = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for i in range(n):
        ax = g.integers(0, 3)
        oo = g.integers(0, res // 8 + 1, 3) * 8 * cell - h
        if g.random() < 0.5:
            oo = oo + g.integers(-2, 3, 3) * 1e-7
        oo[ax] = -2 * h if g.random() < 0.5 else 2 * h
        dd = np.zeros(3)
        dd[ax] = -np.sign(oo[ax])
        if g.random() < 0.5:
            dd = dd + g.standard_normal(3) * [1e-7, 1e-3, 1e-2, 0.3][g.integers(0, 4)]
        o[i], d[i] = oo, dd / np.linalg.norm(dd)
    diag = g.choice([-1.0, 1.0], (n // 4, 3))
    diag /= np.linalg.norm(diag, axis=1, keepdims=True)
    od = -2 * h * diag + g.integers(-2, 3, (n // 4, 3)) * 8 * cell
    return (np.concatenate([o, od]).astype(np.float32),
            np.concatenate([d, diag]).astype(np.float32))


def face_cells(res, n_cells, seed):
    """A sparse grid whose occupied cells sit on brick faces (first or last
    cell of a brick along a random axis)."""
    g = scenes.rng(seed)
    idx = g.integers(0, res, (n_cells, 3))
    ax = g.integers(0, 3, n_cells)
    side = g.random(n_cells) < 0.5
    r = np.arange(n_cells)
    idx[r, ax] = np.where(side, (idx[r, ax] // 8) * 8, (idx[r, ax] // 8) * 8 + 7)
    occ = np.zeros(res ** 3, bool)
    occ[idx[:, 0] + res * (idx[:, 1] + res * idx[:, 2])] = True
    return occ


@pytest.mark.parametrize("res,L,p", [(8, 1, 0.01), (16, 2, 0.002), (64, 1, 0.0005),
                                     (128, 4, 0.0001), (128, 1, 0.3)])
def test_grid_coarsen(gpu_lib, res, L, p):
    bits = np.concatenate([scenes.random_bits(res, p, 80 + l) for l in range(L)])
    g = grid_spec(gpu_lib, bits, res, n_levels=L)
    assert g.coarse is not None
    got = host(g.coarse).view(np.uint32)
    ref = oracle.grid_bricks(bits, res, n_levels=L)
    nb3 = (res // 8) ** 3
    half = max(1, (nb3 + 31) // 32)
    got = got.reshape(L, 2 * half + 1)
    for l in range(L):
        for a in range(2):
            bitsl = scenes.unpack_bits(got[l, a * half:(a + 1) * half], 32 * half)[:nb3]
            assert np.array_equal(bitsl, ref[l, a]), (l, a)
        assert got[l, 2 * half] == ref[l, 0].sum()  # occupied bricks of the level


def march_both(gpu_lib, w, **kw):
    # skip=True: the descriptor always carries the brick occupancy, so the
    # library's own per-level and per-segment rules choose where to skip
    g = gpu_lib.GridSpec(dev(np.asarray(w.bits, np.uint32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                         w.half_extent0, skip=True)
    o, d = dev(w.rays_o), dev(w.rays_d)
    p = gpu_lib.march(g, o, d, dt0=w.dt0, **kw)
    ref = oracle.march(w.rays_o, w.rays_d, w.bits, w.res, n_levels=w.n_levels,
                       half_extent0=w.half_extent0, dt0=w.dt0, **kw)
    return g, p, ref


def assert_same(p, ref):
    assert np.array_equal(host(p.packed_info), ref["packed_info"])
    assert np.array_equal(host(p.t0), ref["t0"])
    assert np.array_equal(host(p.t1), ref["t1"])
    assert np.array_equal(host(p.ray_id), ref["ray_id"])


@pytest.mark.parametrize("res,n_cells,dt,skips", [(32, 20, 0.0123, True), (32, 20, 0.003, True),
                                                  (64, 120, 0.005, True), (64, 120, 0.011, True),
                                                  (16, 3, 0.0021, True), (32, 60, 0.0123, False)])
def test_march_sparse_grid_brick_faces(gpu_lib, res, n_cells, dt, skips):
    occ = face_cells(res, n_cells, res + n_cells)
    assert occ.mean() <= 0.05
    # the march skips on levels with at most 5/16 of their bricks occupied
    assert (oracle.grid_bricks(scenes.pack_bits(occ), res)[0, 0].mean() <= 5 / 16) == skips
    o, d = brick_rays(res, 3000, res)
    w = scenes.Workload("sparse", scenes.blob_field(8), scenes.pack_bits(occ), res, 1, 1.5,
                        o, d, dt)
    g, p, ref = march_both(gpu_lib, w)
    assert ref["total"] > 200  # the rays do meet the occupied cells
    assert_same(p, ref)
    # spans too
    span, hit = gpu_lib.march_span(g, dev(o), dev(d), dt0=dt)
    rs, rh = oracle.march_span(o, d, w.bits, res, dt0=dt)
    assert np.array_equal(host(hit), rh) and np.array_equal(host(span), rs)


def test_march_sparse_cascade_and_cap(gpu_lib):
    """A 4-level cascade of sparse face-cell grids (distance-doubling steps) and
    a per-ray cap, against the oracle."""
    res, L = 32, 4
    # level 0 dense enough to test every point, the others skipping
    occ = np.concatenate([face_cells(res, 80 if l == 0 else 20, 90 + l) for l in range(L)])
    frac = oracle.grid_bricks(scenes.pack_bits(occ), res, n_levels=L)[:, 0].mean(axis=1)
    assert frac[0] > 5 / 16 and np.all(frac[1:] <= 5 / 16)
    g0 = scenes.rng(91)
    eyes = 3.0 * g0.standard_normal((3000, 3))
    tgt = g0.uniform(-1.0, 1.0, (3000, 3))
    d = tgt - eyes
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o2, d2 = brick_rays(res, 2000, 92, h=1.5 * 2 ** (L - 1))
    o = np.concatenate([eyes, o2]).astype(np.float32)
    d = np.concatenate([d, d2]).astype(np.float32)
    # steps small enough that segments of every level run past the 256 lattice
    # points from which the march skips
    w = scenes.Workload("sparse4", scenes.blob_field(8), scenes.pack_bits(occ), res, L, 1.5,
                        o, d, 0.001)
    _, p, ref = march_both(gpu_lib, w)
    assert ref["total"] > 500
    assert_same(p, ref)
    _, p, ref = march_both(gpu_lib, w, max_per_ray=3)
    assert_same(p, ref)


def test_skip_equals_dense_at_full_size(gpu_lib):
    """The benchmark workload (2^20 rays, 128^3 grid; its bricks are dense
    enough that every point is tested), the same camera on an 8-blob field (19%
    of the bricks occupied: skipping) and the unbounded workload (4 x 128^3
    cascade, two of its levels sparse): the march with brick occupancy gives
    the same packed samples as the march that tests every lattice point."""
    f8 = scenes.blob_field(8)
    o8, d8 = scenes.pinhole_rays()
    sparse = scenes.Workload("sparse", f8, scenes.occupancy_bits(f8, 128), 128, 1, 1.5, o8, d8,
                             scenes.IMAGE_STEP)
    for w in (scenes.image(), sparse, scenes.unbounded()):
        o, d = dev(w.rays_o), dev(w.rays_d)
        outs = []
        for skip in (True, "auto", False):
            g = gpu_lib.GridSpec(dev(w.bits.view(np.int32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                                 w.half_extent0, skip=skip)
            assert (g.coarse is not None) == (skip is not False)
            p = gpu_lib.march(g, o, d, dt0=w.dt0)
            outs.append([host(t) for t in (p.packed_info, p.t0, p.t1, p.ray_id)])
            del p
            torch.cuda.empty_cache()
        for other in outs[1:]:
            for a, b in zip(outs[0], other):
                assert np.array_equal(a, b)


def test_large_grid_marches_without_bricks(gpu_lib):
    """Brick occupancy too large for a block's LDS (4 levels of 256^3) is not
    used; the march still tests every point and matches the oracle."""
    res, L = 256, 4
    occ = np.concatenate([scenes.unpack_bits(scenes.random_bits(res, 0.01, 95 + l), res ** 3)
                          for l in range(L)])
    o, d = scenes.sphere_rays(300, radius=20.0)
    w = scenes.Workload("big", scenes.blob_field(8), scenes.pack_bits(occ), res, L, 1.5, o, d,
                        0.02)
    g, p, ref = march_both(gpu_lib, w)
    assert g.coarse is not None and ref["total"] > 100
    assert_same(p, ref)


def test_grid_update_refreshes_bricks(gpu_lib):
    """After the estimator's update changes the bits, the march sees the new
    occupancy (the brick occupancy is rebuilt with them)."""
    from paper_2305_04966_amd.pipeline import OccupancyGrid
    res = 32
    bits = torch.zeros(res ** 3 // 32, dtype=torch.int32, device="cuda")
    grid = gpu_lib.GridSpec(bits, res, skip=True)
    assert grid.coarse is not None and int(grid.coarse.abs().sum()) == 0
    est = OccupancyGrid(grid)
    occ = face_cells(res, 15, 96)  # sparse enough for the march to skip
    assert oracle.grid_bricks(scenes.pack_bits(occ), res)[0, 0].mean() <= 5 / 16
    sig = dev(np.where(occ, 1.0, 0.0).astype(np.float32))
    est.update(lambda pts: sig, gamma=0.0, tau=0.5)
    assert np.array_equal(scenes.unpack_bits(host(bits).view(np.uint32), res ** 3), occ)
    o, d = brick_rays(res, 1000, 97)
    p = gpu_lib.march(grid, dev(o), dev(d), dt0=0.004)
    ref = oracle.march(o, d, scenes.pack_bits(occ), res, dt0=0.004)
    assert ref["total"] > 50
    assert_same(p, ref)
