"""GPU parity: every C-ABI entry point of the HIP library against the FP64 oracle.

Indices, counts and packed layouts must match bit for bit; floating-point
outputs within the relative bar |x - x_ref| <= 1e-5 |x_ref| + 1e-5 s, where s
is 1e-3 max|x_ref| for forward outputs and the per-sample conditioning scale
Delta_k (T_{k+1}|v_k| + sum_{j>k} w_j |v_j|) for the density adjoint.
Threshold decisions on accumulated quantities (the T >= 1e-4 prefix, the CDF
bin of an inverse-CDF edge) may differ only where the oracle flags the value
as within relative 1e-5 of the threshold.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import (assert_close, bwd_condition, dev, grid_spec, host, resample_tol,
                      segment_ids)

pytestmark = pytest.mark.gpu


# ----------------------------------------------------------------------------
# fixtures
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def tiny():
    w = scenes.tiny()
    return w


def gpu_march(txs, w, rays=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    g = grid_spec(txs, w.bits, w.res, w.n_levels, w.half_extent0)
    p = txs.march(g, dev(o), dev(d), dt0=w.dt0, near=kw.get("near", w.near),
                  far=kw.get("far", w.far), max_per_ray=kw.get("max_per_ray", 0))
    torch.cuda.synchronize()
    return p


def oracle_march(w, rays=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    return oracle.march(o, d, w.bits, w.res, n_levels=w.n_levels, half_extent0=w.half_extent0,
                        near=kw.get("near", w.near), far=kw.get("far", w.far), dt0=w.dt0,
                        max_per_ray=kw.get("max_per_ray", 0))


def assert_march_equal(p, ref):
    assert np.array_equal(host(p.packed_info), ref["packed_info"])
    assert np.array_equal(host(p.t0), ref["t0"])
    assert np.array_equal(host(p.t1), ref["t1"])
    assert np.array_equal(host(p.ray_id), ref["ray_id"])


def field_inputs(w, ref):
    """float32 sigma / rgb of the analytic field at the oracle's samples."""
    s, c = oracle.field_at_samples(w.rays_o, w.rays_d, ref["t0"], ref["t1"], ref["ray_id"],
                                   w.fld.packed_params())
    return s.astype(np.float32), c.astype(np.float32)


# ----------------------------------------------------------------------------
# march
# ----------------------------------------------------------------------------
def test_march_tiny_bit_exact(gpu_lib, tiny):
    p = gpu_march(gpu_lib, tiny)
    ref = oracle_march(tiny)
    assert ref["total"] > 10000
    assert_march_equal(p, ref)


def test_march_image_reduced_bit_exact(gpu_lib):
    w = scenes.image(256, 256)
    assert_march_equal(gpu_march(gpu_lib, w), oracle_march(w))


def test_march_image_full_size_sampled_rays(gpu_lib):
    # 1024x1024 rays in the benchmark's launch; every 37th ray checked by the oracle
    w = scenes.image()
    p = gpu_march(gpu_lib, w)
    idx = np.arange(0, w.n_rays, 37)
    ref = oracle_march(w, rays=(w.rays_o[idx], w.rays_d[idx]))
    info = host(p.packed_info)
    assert np.array_equal(info[idx, 1], ref["counts"])
    t0, t1 = host(p.t0), host(p.t1)
    sel = np.concatenate([np.arange(info[r, 0], info[r, 0] + info[r, 1]) for r in idx])
    assert np.array_equal(t0[sel], ref["t0"]) and np.array_equal(t1[sel], ref["t1"])
    # packed layout is the exclusive scan of the counts
    counts = info[:, 1].astype(np.int64)
    assert np.array_equal(info[:, 0], np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert p.n_samples == counts.sum()


def test_march_cascade_bit_exact(gpu_lib):
    w = scenes.unbounded(128, 64, n_cams=8, res=64)
    ref = oracle_march(w)
    assert ref["total"] > 0
    assert_march_equal(gpu_march(gpu_lib, w), ref)


def test_march_cascade_full_size_sampled_rays(gpu_lib):
    # the unbounded workload at full size (4 x 128^3 cascade, 8 cameras of
    # 512x256 = 2^20 rays, distance-doubling steps) in the benchmark's launch;
    # every 37th ray checked by the oracle: counts, t0, t1 bit for bit
    w = scenes.unbounded()
    assert w.n_rays == 1 << 20 and w.n_levels == 4 and w.res == 128
    p = gpu_march(gpu_lib, w)
    idx = np.arange(0, w.n_rays, 37)
    ref = oracle_march(w, rays=(w.rays_o[idx], w.rays_d[idx]))
    info = host(p.packed_info)
    assert np.array_equal(info[idx, 1], ref["counts"])
    t0, t1 = host(p.t0), host(p.t1)
    sel = np.concatenate([np.arange(info[r, 0], info[r, 0] + info[r, 1]) for r in idx])
    assert np.array_equal(t0[sel], ref["t0"]) and np.array_equal(t1[sel], ref["t1"])
    assert np.array_equal(host(p.ray_id)[sel], idx[ref["ray_id"]].astype(np.int32))
    counts = info[:, 1].astype(np.int64)
    assert np.array_equal(info[:, 0], np.concatenate([[0], np.cumsum(counts)[:-1]]))
    assert p.n_samples == counts.sum()
    # ragged rows: the longest holds over 1.5 times the median count
    assert counts.max() > 1.5 * np.median(counts[counts > 0])


@pytest.mark.parametrize("kw", [dict(max_per_ray=11), dict(near=2.5, far=3.4),
                                dict(near=0.5)])
def test_march_options(gpu_lib, tiny, kw):
    assert_march_equal(gpu_march(gpu_lib, tiny, **kw), oracle_march(tiny, **kw))


def test_march_adversarial_rays(gpu_lib):
    # axis-parallel rays on cell planes, rays through cell corners, tiny components
    res = 16
    g = scenes.rng(5)
    cell = 3.0 / res
    n = 4000
    o = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for i in range(n):
        a = g.integers(0, 3)
        oo = g.integers(0, res + 1, 3) * cell - 1.5
        if g.random() < 0.5:
            oo = oo + g.integers(-2, 3, 3) * 1e-7
        oo[a] = -3.0 if g.random() < 0.5 else 3.0
        dd = np.zeros(3)
        dd[a] = -np.sign(oo[a])
        if g.random() < 0.3:
            dd = dd + g.standard_normal(3) * [1e-7, 1e-3, 1e-5][g.integers(0, 3)]
        o[i], d[i] = oo, dd / np.linalg.norm(dd)
    diag = g.choice([-1.0, 1.0], (n, 3))
    diag /= np.linalg.norm(diag, axis=1, keepdims=True)
    o = np.concatenate([o, -3 * diag + g.integers(-4, 5, (n, 3)) * cell]).astype(np.float32)
    d = np.concatenate([d, diag]).astype(np.float32)
    w = scenes.Workload("adv", scenes.blob_field(8), scenes.random_bits(res, 0.3, 7), res, 1, 1.5,
                        o, d, 0.0123)
    assert_march_equal(gpu_march(gpu_lib, w), oracle_march(w))


def test_march_degenerate_grids_and_sizes(gpu_lib, tiny):
    o, d = tiny.rays_o[:777], tiny.rays_d[:777]
    for bits in (np.zeros_like(tiny.bits), np.full_like(tiny.bits, 0xFFFFFFFF)):
        w = scenes.Workload("x", tiny.fld, bits, 64, 1, 1.5, o, d, 0.01)
        assert_march_equal(gpu_march(gpu_lib, w), oracle_march(w))
    # no rays at all; rays that all miss
    w0 = scenes.Workload("x", tiny.fld, tiny.bits, 64, 1, 1.5, o[:0], d[:0], 0.01)
    p = gpu_march(gpu_lib, w0)
    assert p.n_samples == 0 and p.packed_info.shape == (0, 2)
    miss_o = np.tile(np.float32([[0, 0, 5.0]]), (100, 1))
    miss_d = np.tile(np.float32([[0, 0, 1.0]]), (100, 1))
    p = gpu_march(gpu_lib, tiny, rays=(miss_o, miss_d))
    assert p.n_samples == 0 and host(p.packed_info)[:, 1].sum() == 0


# ----------------------------------------------------------------------------
# scan / filter / gather
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("n", [0, 1, 63, 4096, 4097, 123457, (1 << 20) + 17])
def test_exclusive_scan(gpu_lib, n):
    g = scenes.rng(n + 1)
    counts = g.integers(0, 700, n).astype(np.int32)
    counts[g.random(n) < 0.3] = 0
    info, total = gpu_lib.exclusive_scan(dev(counts))
    ref_info, ref_total = oracle.exclusive_scan(counts)
    assert int(total.item()) == ref_total
    assert np.array_equal(host(info), ref_info.reshape(n, 2))


def test_filter_and_gather(gpu_lib, tiny):
    ref = oracle_march(tiny)
    sig, _ = field_inputs(tiny, ref)
    p = gpu_march(gpu_lib, tiny)
    kept = host(gpu_lib.transmittance_prefix(p.packed_info, p.t0, p.t1, dev(sig), 1e-4))
    ref_kept, band = oracle.transmittance_prefix(ref["packed_info"], ref["t0"], ref["t1"], sig,
                                                 1e-4)
    diff = kept != ref_kept
    assert not (diff & ~band).any()
    assert (kept < ref["counts"]).sum() > 100  # the filter is exercised
    # repack with the oracle's decision so both sides gather the same prefix
    kept_t = dev(ref_kept)
    info2, total2 = gpu_lib.exclusive_scan(kept_t)
    s2 = int(total2.item())
    t0o, t1o, rido = gpu_lib.gather_prefix(p.packed_info, info2, s2, p.t0, p.t1)
    r_info, r_t0, r_t1, r_rid = oracle.gather_prefix(ref["packed_info"], ref_kept, ref["t0"],
                                                     ref["t1"], ref["ray_id"])
    assert np.array_equal(host(info2), r_info)
    assert np.array_equal(host(t0o), r_t0) and np.array_equal(host(t1o), r_t1)
    assert np.array_equal(host(rido), r_rid)


@pytest.mark.parametrize("case", ["short", "mixed", "long"])
def test_gather_random_rows(gpu_lib, case):
    """Repack of random ragged rows, exact: kept prefixes of 0..count samples,
    empty rows, rows far shorter and far longer than the kernel's 512-position
    steps, with and without the ray index output."""
    seed, n, cmax = {"short": (70, 5000, 6), "mixed": (71, 3000, 400),
                     "long": (72, 300, 3000)}[case]
    g = scenes.rng(seed)
    counts = g.integers(0, cmax + 1, n).astype(np.int32)
    counts[g.random(n) < 0.25] = 0
    kept = np.minimum(counts, g.integers(0, cmax + 1, n)).astype(np.int32)
    info, S = oracle.exclusive_scan(counts)
    t0, t1 = g.random(S, dtype=np.float32), g.random(S, dtype=np.float32)
    rid = np.repeat(np.arange(n), counts).astype(np.int32)
    info2, total2 = gpu_lib.exclusive_scan(dev(kept))
    s2 = int(total2.item())
    r_info, r_t0, r_t1, r_rid = oracle.gather_prefix(info, kept, t0, t1, rid)
    assert s2 == len(r_t0)
    a, b, c = gpu_lib.gather_prefix(dev(info), info2, s2, dev(t0), dev(t1))
    assert np.array_equal(host(a), r_t0) and np.array_equal(host(b), r_t1)
    assert np.array_equal(host(c), r_rid)
    a, b, c = gpu_lib.gather_prefix(dev(info), info2, s2, dev(t0), dev(t1), want_ray_id=False)
    assert c is None and np.array_equal(host(a), r_t0) and np.array_equal(host(b), r_t1)


def test_filter_thresholds(gpu_lib):
    # constant-density rays: kept = #{i : i sigma Delta <= ln(1e4)}
    counts = np.array([400, 400, 400, 5, 1, 0], np.int32)
    info, S = oracle.exclusive_scan(counts)
    dt = np.float32(0.01)
    t0 = np.concatenate([np.arange(c) * dt for c in counts]).astype(np.float32)
    t1 = (t0 + dt).astype(np.float32)
    sig = np.concatenate([np.full(c, s) for c, s in zip(counts, [0.0, 7.3, 123.0, 1e4, 3.0, 1.0])
                          ]).astype(np.float32)
    kept = host(gpu_lib.transmittance_prefix(dev(info), dev(t0), dev(t1), dev(sig), 1e-4))
    ref, band = oracle.transmittance_prefix(info, t0, t1, sig, 1e-4)
    assert np.array_equal(kept[~band], ref[~band])
    assert kept[0] == 400 and kept[3] == 1 and kept[4] == 1 and kept[5] == 0


# ----------------------------------------------------------------------------
# render forward / backward
# ----------------------------------------------------------------------------
def random_packed(seed, n_rays, max_count, gaps=False, long_rays=()):
    g = scenes.rng(seed)
    counts = g.integers(0, max_count + 1, n_rays).astype(np.int64)
    for r, c in long_rays:
        counts[r] = c
    gap = g.integers(0, 5, n_rays) if gaps else np.zeros(n_rays, np.int64)
    starts = np.concatenate([[0], np.cumsum(counts + gap)[:-1]]) + gap
    S = int(starts[-1] + counts[-1]) if n_rays else 0
    t0 = np.zeros(S, np.float32)
    t1 = np.zeros(S, np.float32)
    for r in range(n_rays):
        c = counts[r]
        a = g.uniform(0.5, 3.0)
        dts = g.uniform(0.001, 0.02, c)
        e = a + np.concatenate([[0], np.cumsum(dts)])
        t0[starts[r]:starts[r] + c] = e[:-1]
        t1[starts[r]:starts[r] + c] = e[1:]
    sig = (g.exponential(1.0, S) * g.choice([0.5, 5, 50], S)).astype(np.float32)
    rgb = g.random((S, 3)).astype(np.float32)
    info = np.stack([starts, counts], 1).astype(np.int32)
    return info, t0, t1, sig, rgb


def check_fwd(txs, info, t0, t1, sig, rgb, bg=None, dense=None):
    n = info.shape[0]
    if dense is None:
        out = txs.render_fwd(dev(info), dev(t0), dev(t1), dev(sig), dev(rgb),
                             bg=None if bg is None else dev(bg), want_weights=True)
    else:
        out = txs.render_fwd(None, dev(t0), dev(t1), dev(sig), dev(rgb), n_rays=n,
                             fixed_count=dense, bg=None if bg is None else dev(bg),
                             want_weights=True)
    ref = oracle.render_fwd(info, t0, t1, sig, rgb, bg=bg, want_weights=True)
    assert_close(host(out[0]), ref["rgb"], name="rgb")
    assert_close(host(out[1]), ref["opacity"], name="opacity")
    assert_close(host(out[2]), ref["depth"], name="depth")
    own = np.concatenate([np.arange(s, s + c) for s, c in info]) if len(info) else np.zeros(0, int)
    assert_close(host(out[3])[own], ref["weights"][own], name="weights")


def check_bwd(txs, info, t0, t1, sig, rgb, bg=None, hq=False, seed=0, dense=None):
    n = info.shape[0]
    g = scenes.rng(100 + seed)
    gr = g.standard_normal((n, 3)).astype(np.float32)
    gh = g.standard_normal(n).astype(np.float32) if hq else None
    gq = g.standard_normal(n).astype(np.float32) if hq else None
    kw = dict(bg=None if bg is None else dev(bg))
    if dense is not None:
        kw.update(n_rays=n, fixed_count=dense)
    ds, dr = txs.render_bwd(None if dense is not None else dev(info), dev(t0), dev(t1), dev(sig),
                            dev(rgb), dev(gr), None if gh is None else dev(gh),
                            None if gq is None else dev(gq), **kw)
    rds, rdr = oracle.render_bwd(info, t0, t1, sig, rgb, gr, gh, gq, bg=bg)
    own = np.concatenate([np.arange(s, s + c) for s, c in info]) if len(info) else np.zeros(0, int)
    seg = segment_ids(info)
    bgc = np.zeros((n, 3)) if bg is None else bg.astype(np.float64)
    mid = 0.5 * (t0.astype(np.float64) + t1)
    if len(own):
        # magnitude of the terms of v = g.(c - bg) + h + q m
        vb = (np.abs(rgb[own].astype(np.float64) - bgc[seg]) * np.abs(gr[seg])).sum(1)
        if hq:
            vb += np.abs(gh[seg]) + np.abs(gq[seg] * mid[own])
        cond = bwd_condition(np.stack([np.concatenate([[0], np.cumsum(info[:, 1])[:-1]]),
                                       info[:, 1]], 1), t0[own], t1[own], sig[own], vb)
        assert_close(host(ds)[own], rds[own], floor_scale=cond, name="d_sigma")
        assert_close(host(dr)[own], rdr[own], name="d_rgb")


def test_render_tiny_field(gpu_lib, tiny):
    ref = oracle_march(tiny)
    sig, rgb = field_inputs(tiny, ref)
    kept, _ = oracle.transmittance_prefix(ref["packed_info"], ref["t0"], ref["t1"], sig, 1e-4)
    info, t0, t1, rid = oracle.gather_prefix(ref["packed_info"], kept, ref["t0"], ref["t1"],
                                             ref["ray_id"])
    sel = np.concatenate([np.arange(ref["packed_info"][r, 0], ref["packed_info"][r, 0] + kept[r])
                          for r in range(tiny.n_rays)])
    s2, c2 = sig[sel], rgb[sel]
    check_fwd(gpu_lib, info, t0, t1, s2, c2)
    check_bwd(gpu_lib, info, t0, t1, s2, c2)
    check_bwd(gpu_lib, info, t0, t1, s2, c2, hq=True, seed=1)


@pytest.mark.parametrize("case", ["short", "mixed", "long", "gaps", "ones"])
def test_render_random_layouts(gpu_lib, case):
    if case == "short":
        args = random_packed(1, 3000, 12)
    elif case == "mixed":
        args = random_packed(2, 2000, 300)
    elif case == "long":  # rays beyond one 512-sample window, incl. >64 windows
        args = random_packed(3, 300, 40, long_rays=[(0, 513), (5, 1500), (64, 4096),
                                                    (130, 40000), (299, 777)])
    elif case == "gaps":
        args = random_packed(4, 1000, 200, gaps=True, long_rays=[(10, 2000)])
    else:
        args = random_packed(5, 5000, 1)
    info, t0, t1, sig, rgb = args
    g = scenes.rng(9)
    bg = g.random((info.shape[0], 3)).astype(np.float32)
    check_fwd(gpu_lib, info, t0, t1, sig, rgb)
    check_fwd(gpu_lib, info, t0, t1, sig, rgb, bg=bg)
    check_bwd(gpu_lib, info, t0, t1, sig, rgb, bg=bg, hq=True)


def test_render_dense_layout(gpu_lib):
    n, F = 3000, 32
    info = np.stack([np.arange(n) * F, np.full(n, F)], 1).astype(np.int32)
    _, t0, t1, sig, rgb = random_packed(7, n, F, long_rays=[(r, F) for r in range(n)])
    check_fwd(gpu_lib, info, t0, t1, sig, rgb, dense=F)
    check_bwd(gpu_lib, info, t0, t1, sig, rgb, dense=F, hq=True)


def test_render_extreme_densities(gpu_lib):
    info, t0, t1, sig, rgb = random_packed(8, 500, 50)
    g = scenes.rng(10)
    sig = sig.copy()
    sig[g.random(sig.size) < 0.2] = 0.0
    sig[g.random(sig.size) < 0.05] = 1e6
    check_fwd(gpu_lib, info, t0, t1, sig, rgb)
    check_bwd(gpu_lib, info, t0, t1, sig, rgb, hq=True)


def test_weights_bwd(gpu_lib):
    info, t0, t1, sig, rgb = random_packed(11, 1500, 150, long_rays=[(3, 900)])
    g = scenes.rng(12)
    gw = g.standard_normal(t0.size).astype(np.float32)
    ds = host(gpu_lib.weights_bwd(dev(info), dev(t0), dev(t1), dev(sig), dev(gw)))
    ref = oracle.weights_bwd(info, t0, t1, sig, gw)
    cond = bwd_condition(info, t0, t1, sig, np.abs(gw.astype(np.float64)))
    assert_close(ds, ref, floor_scale=cond, name="weights_bwd")


def test_render_autograd_and_determinism(gpu_lib, tiny):
    info, t0, t1, sig, rgb = random_packed(13, 800, 100)
    s = dev(sig).requires_grad_(True)
    c = dev(rgb).requires_grad_(True)
    p = gpu_lib.Packed(dev(info), dev(t0), dev(t1), None)
    out_rgb, out_op, out_d = gpu_lib.rendering(p, s, c)
    g = scenes.rng(14)
    gr = dev(g.standard_normal((800, 3)).astype(np.float32))
    go = dev(g.standard_normal(800).astype(np.float32))
    ((out_rgb * gr).sum() + (out_op * go).sum()).backward()
    rds, rdr = oracle.render_bwd(info, t0, t1, sig, rgb, host(gr), host(go), None)
    seg = segment_ids(info)
    vb = (rgb.astype(np.float64) * np.abs(host(gr)[seg])).sum(1) + np.abs(host(go)[seg])
    cond = bwd_condition(info, t0, t1, sig, vb)
    assert_close(host(s.grad), rds, floor_scale=cond, name="autograd d_sigma")
    assert_close(host(c.grad), rdr, name="autograd d_rgb")
    # bitwise determinism of two identical launches
    a = gpu_lib.render_bwd(dev(info), dev(t0), dev(t1), dev(sig), dev(rgb), gr, go)
    b = gpu_lib.render_bwd(dev(info), dev(t0), dev(t1), dev(sig), dev(rgb), gr, go)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_render_autograd_gap_samples_get_zero_gradient(gpu_lib):
    """Samples that belong to no row -- gaps between packed rows, the tail of a
    dense layout -- receive exactly zero gradient through the autograd
    function, and the owned samples still match the oracle."""
    info, t0, t1, sig, rgb = random_packed(15, 600, 80, gaps=True, long_rays=[(7, 700)])
    S = t0.size
    tail = 37  # samples after the last row
    t0 = np.concatenate([t0, np.linspace(3, 4, tail, dtype=np.float32)])
    t1 = np.concatenate([t1, np.linspace(3.01, 4.01, tail, dtype=np.float32)])
    sig = np.concatenate([sig, np.full(tail, 7.0, np.float32)])
    rgb = np.concatenate([rgb, np.full((tail, 3), 0.5, np.float32)])
    own = np.concatenate([np.arange(s_, s_ + c) for s_, c in info])
    gap = np.setdiff1d(np.arange(S + tail), own)
    assert gap.size > 100
    g = scenes.rng(16)
    gr = dev(g.standard_normal((info.shape[0], 3)).astype(np.float32))
    for _ in range(2):  # a second pass reuses freed memory with the first's values
        s = dev(sig).requires_grad_(True)
        c = dev(rgb).requires_grad_(True)
        out_rgb, _, _ = gpu_lib.rendering(gpu_lib.Packed(dev(info), dev(t0), dev(t1), None), s, c)
        (out_rgb * gr).sum().backward()
        ds, dr = host(s.grad), host(c.grad)
        assert np.all(ds[gap] == 0.0) and np.all(dr[gap] == 0.0)
        rds, rdr = oracle.render_bwd(info, t0, t1, sig, rgb, host(gr))
        assert_close(dr[own], rdr[own], name="d_rgb")
    # dense layout with trailing samples: n * F < S
    n, F = 500, 16
    _, d0, d1, dsg, dc = random_packed(17, n, F, long_rays=[(r, F) for r in range(n)])
    d0 = np.concatenate([d0, np.ones(29, np.float32)])
    d1 = np.concatenate([d1, np.full(29, 1.5, np.float32)])
    dsg = np.concatenate([dsg, np.ones(29, np.float32)])
    dc = np.concatenate([dc, np.ones((29, 3), np.float32)])
    s = dev(dsg).requires_grad_(True)
    c = dev(dc).requires_grad_(True)
    out_rgb, out_op, _ = gpu_lib.rendering_dense(dev(d0), dev(d1), s, c, n, F)
    (out_rgb.sum() + out_op.sum()).backward()
    assert np.all(host(s.grad)[n * F:] == 0.0) and np.all(host(c.grad)[n * F:] == 0.0)
    w = host(gpu_lib.weights_bwd(None, dev(d0), dev(d1), dev(dsg), dev(np.ones_like(dsg)),
                                 n_rays=n, fixed_count=F))
    assert np.all(w[n * F:] == 0.0)


def test_exclusive_scan_rows_past_int32_are_empty(gpu_lib):
    """A table whose rows would pass INT32_MAX: the total is the exact int64 sum
    and the rows that do not fit are written as the empty row (INT32_MAX, 0)."""
    counts = np.array([2 ** 30, 2 ** 30, 5, 0, 7], np.int32)
    info, total = gpu_lib.exclusive_scan(dev(counts))
    ref_info, ref_total = oracle.exclusive_scan(counts)
    assert int(total.item()) == ref_total == 2 ** 31 + 12
    assert np.array_equal(host(info), ref_info)


def test_render_empty(gpu_lib):
    info = np.zeros((5, 2), np.int32)
    z = np.zeros(0, np.float32)
    out = gpu_lib.render_fwd(dev(info), dev(z), dev(z), dev(z), dev(np.zeros((0, 3), np.float32)))
    assert host(out[1]).tolist() == [0.0] * 5
    ds, dr = gpu_lib.render_bwd(dev(info), dev(z), dev(z), dev(z),
                                dev(np.zeros((0, 3), np.float32)),
                                dev(np.ones((5, 3), np.float32)))
    assert ds.numel() == 0


# ----------------------------------------------------------------------------
# resample / uniform bins / field
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("use_u", [False, True])
def test_resample(gpu_lib, mode, use_u):
    g = scenes.rng(20 + mode + 2 * use_u)
    n, nb, n_out = 4000, 128, 32
    a = g.uniform(1.0, 2.0, (n, 1))
    edges = (a + np.concatenate([np.zeros((n, 1)), np.cumsum(g.uniform(0.005, 0.03, (n, nb)), 1)],
                                1)).astype(np.float32)
    vals = (g.exponential(1.0, (n, nb)) * (g.random((n, nb)) < 0.3) *
            g.choice([1.0, 30.0], (n, 1))).astype(np.float32)
    vals[:10] = 0.0  # zero-mass rays fall back to the uniform estimator
    u = np.sort(g.random((n, n_out + 1)), 1).astype(np.float32) if use_u else None
    out = host(gpu_lib.resample(dev(edges), dev(vals), n_out, mode, None if u is None else dev(u)))
    ref, bins, band = oracle.resample(edges, vals, n_out, mode, u)
    tol = resample_tol(edges, vals, mode, ref, bins)
    err = np.abs(out - ref)
    bad = (err > tol) & ~band[:, None]
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])
    # the dense-interval form carries the same edges
    t0, t1 = gpu_lib.resample_intervals(dev(edges), dev(vals), n_out, mode,
                                        None if u is None else dev(u))
    assert np.array_equal(host(t0).reshape(n, n_out), out[:, :-1])
    assert np.array_equal(host(t1).reshape(n, n_out), out[:, 1:])


@pytest.mark.parametrize("n,nb,n_out", [(4001, 32, 48), (333, 17, 5), (1, 32, 3), (2, 1, 64),
                                         (1003, 16, 64), (5, 9, 7), (3, 16, 1),
                                         (1000, 33, 48), (999, 64, 40), (257, 255, 31),
                                         (256, 256, 16)])
def test_resample_row_lengths(gpu_lib, n, nb, n_out):
    """Every kernel kind the bin count selects (four rays per wave up to 16
    bins, two up to 32, ray counts leaving parts of a wave without a ray; whole-wave rows of
    33 bins; register rows of 64..255 bins; in-place rows from 256), in the
    three modes, with and without caller u, against the oracle."""
    g = scenes.rng(90 + nb + n)
    a = g.uniform(1.0, 2.0, (n, 1))
    edges = (a + np.concatenate([np.zeros((n, 1)), np.cumsum(g.uniform(0.005, 0.03, (n, nb)), 1)],
                                1)).astype(np.float32)
    vals = (g.exponential(1.0, (n, nb)) * (g.random((n, nb)) < 0.4) *
            g.choice([1.0, 30.0], (n, 1))).astype(np.float32)
    vals[: max(1, n // 50)] = 0.0  # zero-mass rays fall back to the uniform estimator
    for mode in (0, 1, 2):
        for u in (None, np.sort(g.random((n, n_out + 1)), 1).astype(np.float32)):
            out = host(gpu_lib.resample(dev(edges), dev(vals), n_out, mode,
                                        None if u is None else dev(u)))
            ref, bins, band = oracle.resample(edges, vals, n_out, mode, u)
            if mode == 2:  # the exponential inverse: finite, ordered, inside the row
                assert np.all(np.diff(out, axis=1) >= 0) and np.all(out >= edges[:, :1])
                assert np.all(out <= edges[:, -1:])
                continue
            tol = resample_tol(edges, vals, mode, ref, bins)
            bad = (np.abs(out - ref) > tol) & ~band[:, None]
            assert not bad.any(), (mode, bad.sum(), np.argwhere(bad)[:5])
            t0, t1 = gpu_lib.resample_intervals(dev(edges), dev(vals), n_out, mode,
                                                None if u is None else dev(u))
            assert np.array_equal(host(t0).reshape(n, n_out), out[:, :-1])
            assert np.array_equal(host(t1).reshape(n, n_out), out[:, 1:])


@pytest.mark.parametrize("nb,n_out", [(1, 1), (1, 7), (1024, 1), (1024, 500), (3, 2000)])
def test_resample_size_limits(gpu_lib, nb, n_out):
    """One bin, the largest bin count (1024), a single output interval and far
    more outputs than bins, against the oracle; 1025 bins are refused."""
    g = scenes.rng(72 + nb)
    n = 300
    edges = (1.0 + np.concatenate([np.zeros((n, 1)),
                                   np.cumsum(g.uniform(0.001, 0.01, (n, nb)), 1)], 1)
             ).astype(np.float32)
    vals = (g.exponential(1.0, (n, nb)) * (g.random((n, nb)) < 0.5) * 20.0).astype(np.float32)
    vals[:3] = 0.0
    for mode in (0, 1):
        out = host(gpu_lib.resample(dev(edges), dev(vals), n_out, mode))
        ref, bins, band = oracle.resample(edges, vals, n_out, mode)
        tol = resample_tol(edges, vals, mode, ref, bins)
        assert not ((np.abs(out - ref) > tol) & ~band[:, None]).any()
    big = np.tile(np.linspace(1.0, 2.0, 1026, dtype=np.float32), (2, 1))
    with pytest.raises(gpu_lib.TxsError):
        gpu_lib.resample(dev(big), dev(np.ones((2, 1025), np.float32)), 4)


@pytest.mark.parametrize("use_u", [False, True])
def test_resample_exponential_in_bin(gpu_lib, use_u):
    """Mode TXS_PDF_SIGMA_EXP.  Checked where the inverse is well conditioned:
    mapped back through the binary64 piecewise-exponential CDF, every GPU edge
    must sit at its quantile u' = u F_n within the binary32 CDF's error (the
    bound of the linear mode, 4e-6 F_n) plus the CDF's slope times the edge's
    own rounding; this needs no band, the CDF being continuous in t.  Edges in
    bins of optical depth <= 4 must also match the oracle's within the linear
    mode's bar scaled by the slope factor exp(tau)."""
    g = scenes.rng(70 + use_u)
    n, nb, n_out = 4000, 128, 32
    a = g.uniform(1.0, 2.0, (n, 1))
    edges = (a + np.concatenate([np.zeros((n, 1)), np.cumsum(g.uniform(0.005, 0.03, (n, nb)), 1)],
                                1)).astype(np.float32)
    vals = (g.exponential(1.0, (n, nb)) * (g.random((n, nb)) < 0.3) *
            g.choice([1.0, 30.0, 300.0], (n, 1))).astype(np.float32)
    vals[:10] = 0.0  # zero-mass rays fall back to the uniform estimator
    u = np.sort(g.random((n, n_out + 1)), 1).astype(np.float32) if use_u else None
    mode = gpu_lib.TXS_PDF_SIGMA_EXP
    out = host(gpu_lib.resample(dev(edges), dev(vals), n_out, mode, None if u is None else dev(u)))
    ref, bins, band = oracle.resample(edges, vals, n_out, mode, u)
    e64, v64 = edges.astype(np.float64), vals.astype(np.float64)
    P = np.concatenate([np.zeros((n, 1)), np.cumsum(v64 * np.diff(e64, axis=1), 1)], 1)
    Fn = -np.expm1(-P[:, -1])
    uu = (np.arange(n_out + 1) / n_out)[None, :].repeat(n, 0) if u is None else u.astype(np.float64)
    live = Fn > 1e-12
    rows = np.flatnonzero(live)
    i = np.stack([np.clip(np.searchsorted(e64[r], out[r], side="right") - 1, 0, nb - 1)
                  for r in rows])
    ei = np.take_along_axis(e64[rows], i, 1)
    vi = np.take_along_axis(v64[rows], i, 1)
    Pt = np.take_along_axis(P[rows], i, 1) + vi * (out[rows] - ei)
    F_t, T_t = -np.expm1(-Pt), np.exp(-Pt)
    span = (e64[rows, -1] - e64[rows, 0])[:, None]
    tolF = 4e-6 * Fn[rows, None] + vi * T_t * (2e-7 * np.abs(out[rows]) + 1e-6 * span)
    bad = np.abs(F_t - uu[rows] * Fn[rows, None]) > tolF
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])
    # the uniform fallback is the uniform lattice, as in the linear mode
    assert np.allclose(out[~live], ref[~live], rtol=1e-6, atol=1e-6)
    # direct comparison where the bin's optical depth is moderate
    tau = np.take_along_axis(v64 * np.diff(e64, axis=1), np.minimum(bins, nb - 1), 1)
    tol = resample_tol(edges, vals, 0, ref, bins) * np.exp(np.minimum(tau, 4.0))
    ok = (tau <= 4.0) & ~band[:, None]
    assert not ((np.abs(out - ref) > tol) & ok).any()


def test_uniform_bins(gpu_lib, tiny):
    o, d = tiny.rays_o, tiny.rays_d
    g = grid_spec(gpu_lib, tiny.bits, 64)
    e = host(gpu_lib.uniform_bins(g, dev(o), dev(d), 128))
    tn, tf = oracle.clip(o, d, np.full(3, -1.5, np.float32), np.full(3, 1.5, np.float32))
    hit = tn < tf
    k = np.arange(129) / 128.0
    ref = tn[:, None].astype(np.float64) + (tf - tn)[:, None].astype(np.float64) * k
    assert_close(e[hit], ref[hit], rel=1e-6, name="uniform edges")
    assert np.all(e[~hit] == 0.0)


def test_disparity_bins(gpu_lib, tiny):
    """Binary32 reciprocals of an interpolation of positive reciprocals: a few
    roundings, no cancellation (rel 1e-6); the end edges are the chord's."""
    o, d = tiny.rays_o, tiny.rays_d
    g = grid_spec(gpu_lib, tiny.bits, 64)
    for near in (0.05, 2.0):
        e = host(gpu_lib.disparity_bins(g, dev(o), dev(d), 128, near=near))
        ref = oracle.disparity_bins(o, d, np.full(3, -1.5, np.float32), np.full(3, 1.5, np.float32),
                                    128, near)
        assert_close(e, ref, rel=1e-6, floor_scale=0.0, name="disparity edges")
        tn, tf = oracle.clip(o, d, np.full(3, -1.5, np.float32), np.full(3, 1.5, np.float32),
                             near)
        hit = tn < tf
        assert np.array_equal(e[hit, 0], tn[hit]) and np.array_equal(e[hit, -1], tf[hit])


def test_blob_field(gpu_lib):
    w = scenes.unbounded(64, 32, n_cams=2, res=32)
    ref = oracle_march(w)
    params = w.fld.packed_params().astype(np.float32)
    s, c = gpu_lib.blob_field(dev(params), w.fld.n_blobs, dev(w.rays_o), dev(w.rays_d),
                              dev(ref["t0"]), dev(ref["t1"]), dev(ref["ray_id"]))
    rs, rc = oracle.field_at_samples(w.rays_o, w.rays_d, ref["t0"], ref["t1"], ref["ray_id"],
                                     w.fld.packed_params())
    # support kernel: float32 positions and a float32 parameter copy bound its accuracy
    s = host(s)
    assert np.all(np.abs(s - rs) <= 2e-4 * rs + 1e-6 * w.fld.peak)
    assert np.all(np.abs(host(c) - rc) <= 1e-4)


@pytest.mark.parametrize("n", [1, 511, 512 * 16384 + 777])
def test_stream_probe_outputs(gpu_lib, n):
    # measurement support: its outputs are exact sums, so its reads and writes
    # cover every sample once (full windows and the tail of each range)
    g = scenes.rng(50)
    t0, t1, s = (g.random(n, dtype=np.float32) for _ in range(3))
    rgb = g.random((n, 3), dtype=np.float32)
    oa = torch.empty(n, dtype=torch.float32, device="cuda")
    ob = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    gpu_lib.stream_probe(dev(t0), dev(t1), dev(s), dev(rgb), oa, ob)
    assert np.array_equal(host(oa), (t0 + t1) + s)
    assert np.array_equal(host(ob), rgb + rgb)


@pytest.mark.parametrize("n", [1, 511, 512 * 16384 + 777])
def test_read_probe_covers_every_sample(gpu_lib, n):
    # measurement support: with every input 1.0 each sample adds 6 (t0, t1,
    # sigma and three colours) to exactly one lane's sum, so the sums total 6n
    # (exact in binary32 per lane) and the forward's reads cover each sample once
    one = torch.ones(n, dtype=torch.float32, device="cuda")
    rgb = torch.ones((n, 3), dtype=torch.float32, device="cuda")
    out = gpu_lib.read_probe(one, one, one, rgb)
    sums = host(out)
    assert sums.shape == (int(gpu_lib.load().txs_read_probe_out_size()),)
    # the probe's ranges: ceil(n / 16384) samples rounded up to whole windows
    # of 512 per wave, one lane sum per lane of each wave that has a range
    per_wave = (-(-n // 16384) + 511) // 512 * 512
    used = -(-n // per_wave)
    s = sums[:used * 64]
    assert np.all(s == np.round(s))
    assert s.astype(np.int64).sum() == 6 * n
