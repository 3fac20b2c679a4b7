"""The combined estimator (occupancy grid, then the proposal network inside
each ray's occupied span) on the GPU against the oracle.

* the span march is bit-exact: its ends are the first sample's t0 and the last
  sample's t1 of the dense march, on single grids, cascades, near/far planes,
  degenerate grids and adversarial rays;
* compaction and expansion of per-ray rows are exact (they move words);
* span bins follow the binary32 recipe of the uniform bins (rel 1e-6);
* the whole combined forward with a network of constant density (the
  composition of span, compaction, bins, proposal, inverse CDF, field, render
  and expansion) matches the oracle's chain to the field's binary32 bar.
Inputs come from seeded generators or the oracle, never from the library.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, grid_spec, host
from gpu_util import resample_tol

pytestmark = pytest.mark.gpu


def gpu_span(txs, w, rays=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    g = grid_spec(txs, w.bits, w.res, w.n_levels, w.half_extent0)
    span, hit = txs.march_span(g, dev(o), dev(d), dt0=w.dt0, near=kw.get("near", w.near),
                               far=kw.get("far", w.far))
    return host(span), host(hit)


def oracle_span(w, rays=None, **kw):
    o, d = (w.rays_o, w.rays_d) if rays is None else rays
    return oracle.march_span(o, d, w.bits, w.res, n_levels=w.n_levels,
                             half_extent0=w.half_extent0, near=kw.get("near", w.near),
                             far=kw.get("far", w.far), dt0=w.dt0)


def assert_span_equal(got, ref):
    assert np.array_equal(got[1], ref[1])
    assert np.array_equal(got[0], ref[0])


@pytest.mark.parametrize("kw", [{}, dict(near=2.5, far=3.4), dict(near=0.5)])
def test_march_span_tiny(gpu_lib, kw):
    w = scenes.tiny()
    ref = oracle_span(w, **kw)
    assert 0 < ref[1].sum() < w.n_rays
    assert_span_equal(gpu_span(gpu_lib, w, **kw), ref)


def test_march_span_cascade_and_image_rays(gpu_lib):
    w = scenes.unbounded(128, 64, n_cams=8, res=64)
    assert_span_equal(gpu_span(gpu_lib, w), oracle_span(w))
    img = scenes.image()
    sel = np.arange(0, img.n_rays, 97)
    rays = (img.rays_o[sel], img.rays_d[sel])
    ref = oracle_span(img, rays)
    assert 0 < ref[1].sum() < len(sel)
    assert_span_equal(gpu_span(gpu_lib, img, rays), ref)


def test_march_span_degenerate_grids_and_rays(gpu_lib):
    tiny = scenes.tiny(777)
    for bits in (np.zeros_like(tiny.bits), np.full_like(tiny.bits, 0xFFFFFFFF)):
        w = scenes.Workload("x", tiny.fld, bits, 64, 1, 1.5, tiny.rays_o, tiny.rays_d, 0.01)
        assert_span_equal(gpu_span(gpu_lib, w), oracle_span(w))
    # axis-parallel rays on cell planes and through corners, near-zero components
    res, g, cell = 16, scenes.rng(64), 3.0 / 16
    n = 2000
    a = g.integers(0, 3, n)
    o = g.integers(0, res + 1, (n, 3)) * cell - 1.5
    o[np.arange(n), a] = -3.0
    d = np.zeros((n, 3))
    d[np.arange(n), a] = 1.0
    d += (g.random((n, 1)) < 0.3) * g.standard_normal((n, 3)) * 1e-6
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    w = scenes.Workload("adv", scenes.blob_field(8), scenes.random_bits(res, 0.2, 9), res, 1,
                        1.5, o.astype(np.float32), d.astype(np.float32), 0.0123)
    assert_span_equal(gpu_span(gpu_lib, w), oracle_span(w))
    # no rays at all
    w0 = scenes.Workload("x", tiny.fld, tiny.bits, 64, 1, 1.5, tiny.rays_o[:0], tiny.rays_d[:0],
                         0.01)
    s, h = gpu_span(gpu_lib, w0)
    assert s.shape == (0, 2) and h.shape == (0,)


def test_march_span_requires_uncapped_march(gpu_lib):
    """The span is that of every sample: a per-ray cap is refused on the host."""
    from paper_2305_04966_amd._lib import MarchParams, TXS_EINVAL
    w = scenes.tiny(64)
    g = grid_spec(gpu_lib, w.bits, w.res).struct()
    p = MarchParams()
    p.near_plane, p.far_plane, p.dt0, p.max_per_ray = 0.0, float("inf"), w.dt0, 5
    o, d = dev(w.rays_o), dev(w.rays_d)
    span = torch.empty((64, 2), dtype=torch.float32, device="cuda")
    hit = torch.empty(64, dtype=torch.int32, device="cuda")
    rc = gpu_lib.load().txs_march_span(C.byref(g), C.byref(p), C.c_void_p(o.data_ptr()),
                                      C.c_void_p(d.data_ptr()), 64,
                                      C.c_void_p(span.data_ptr()), C.c_void_p(hit.data_ptr()),
                                      None)
    assert rc == TXS_EINVAL


@pytest.mark.parametrize("n", [0, 1, 1000, (1 << 20) + 3])
def test_compact_and_expand_rows(gpu_lib, n):
    g = scenes.rng(65)
    hit = (g.random(n) < 0.4).astype(np.int32)
    table, total = gpu_lib.exclusive_scan(dev(hit))
    m = int(host(total)[0])
    assert m == hit.sum()
    alive = hit.astype(bool)
    for src in (g.standard_normal((n, 3)).astype(np.float32),
                g.integers(-5, 1 << 30, (n, 2)).astype(np.int32),
                g.random(n).astype(np.float32)):
        got = host(gpu_lib.compact_rows(table, m, dev(src)))
        assert np.array_equal(got, src[alive])
    rows = g.standard_normal((m, 3)).astype(np.float32)
    full = host(gpu_lib.expand_rows(table, dev(rows), fill=-2.5))
    ref = np.full((n, 3), -2.5, np.float32)
    ref[alive] = rows
    assert np.array_equal(full, ref)


def test_span_bins(gpu_lib):
    w = scenes.tiny()
    span, hit = oracle_span(w)
    e = host(gpu_lib.span_bins(dev(span), 128))
    ref = oracle.span_bins(span, 128)
    # two roundings (difference, product) and one of the sum, as the uniform bins
    assert np.all(np.abs(e - ref) <= 1e-6 * np.abs(ref) + 1e-7)
    assert np.all(e[~hit.astype(bool)] == 0.0)


def test_combined_forward_constant_density_network(gpu_lib):
    """A proposal network of constant density softplus(3) (all weights zero)
    makes the whole combined forward depend on the grid, the span bins, the
    inverse CDF, the field and the renderer only: it must match the oracle's
    chain to the field's binary32 bar (1e-4 in colour), give exact zeros on
    the rays the grid drops and positive opacity on the others."""
    from paper_2305_04966_amd.learned import ProposalEstimator, combined_render, occupied_span
    w = scenes.tiny()
    H, nb, n_out = 64, 61, 24  # co-prime, so that few quantiles fall on a bin edge
    params = np.zeros(oracle.mlp_param_count(H), np.float32)
    params[-1] = 3.0
    fp = w.fld.packed_params()
    fpd = dev(fp.astype(np.float32))
    field = lambda o, d, t0, t1, n: gpu_lib.blob_field(fpd, w.fld.n_blobs, o, d, t0, t1,
                                                      fixed_count=n)
    g = grid_spec(gpu_lib, w.bits, w.res)
    est = ProposalEstimator(dev(params), H, scale=1.5)
    sp = occupied_span(g, dev(w.rays_o), dev(w.rays_d), dt0=w.dt0)
    rgb, opa, dep = (host(t) for t in combined_render(est, sp, nb, n_out, field))

    span, hit = oracle_span(w)
    alive = hit.astype(bool)
    M = int(alive.sum())
    assert sp.n_alive == M
    o, d = w.rays_o[alive], w.rays_d[alive]
    edges = oracle.span_bins(span[alive], nb).astype(np.float32)
    sig = oracle.mlp_fwd(oracle.bin_midpoints(o, d, edges), params, H, scale=1.5,
                         emulate_bf16=True).astype(np.float32).reshape(M, nb)
    out_e, bins, band = oracle.resample(edges, sig, n_out, oracle.MODE_SIGMA)
    t0 = out_e[:, :-1].astype(np.float32).reshape(-1)
    t1 = out_e[:, 1:].astype(np.float32).reshape(-1)
    rid = np.repeat(np.arange(M), n_out)
    s, c = oracle.field_at_samples(o, d, t0, t1, rid, fp)
    info = np.stack([np.arange(M) * n_out, np.full(M, n_out)], 1).astype(np.int32)
    ref = oracle.render_fwd(info, t0, t1, s.astype(np.float32), c.astype(np.float32))

    assert not rgb[~alive].any() and not opa[~alive].any() and not dep[~alive].any()
    # rays with a quantile within relative 1e-5 of a bin edge of the oracle's CDF
    # may take the other bin: compared through the edges below, not the colours
    ok = ~band
    assert ok.mean() > 0.95
    err = np.abs(rgb[alive][ok] - ref["rgb"][ok])
    assert err.max() <= 1e-4, err.max()
    assert np.abs(opa[alive][ok] - ref["opacity"][ok]).max() <= 1e-4
    assert (opa[alive] > 0).all()
    # the inverse-CDF edges themselves, within the resampler's conditioning bar
    a, b = est.sample_intervals(sp.rays_o, sp.rays_d, sp.bins(nb), n_out)
    got_e = np.concatenate([host(a).reshape(M, n_out), host(b).reshape(M, n_out)[:, -1:]], 1)
    tol = resample_tol(edges, sig, 0, out_e, bins)
    bad = (np.abs(got_e - out_e) > tol) & ~band[:, None]
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])
