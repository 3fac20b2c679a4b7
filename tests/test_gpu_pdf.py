"""The coarse-to-fine PDF estimator (Table 1, third row, as vanilla NeRF runs
it) on the GPU against the oracle.

* merging two sorted edge rows is exact (it moves values), ties included;
* the whole estimator (uniform coarse bins, the field's density on them,
  inverse CDF, merged edges, field, render) against the oracle's chain.  The
  GPU field is binary32 (2e-4 relative in density at worst, its own test), so
  the GPU's coarse CDF is within 2e-4 F_n of the oracle's.  A quantile farther
  than that from every CDF knot falls in the same bin on both sides; its edge
  then moves by dF / slope, and the colour by about slope times that, i.e.
  by about 2e-4 per edge.  Rays with every quantile outside that band (4e-4
  F_n, twice the bound) must agree to 2e-4 in colour for 99% of them and to
  2e-3 (ten edges' worth) for all; a quantile inside the band may take the
  neighbouring bin, and across a run of bins of negligible mass its edge may
  jump the whole run.  The edge of u = 0 sits at the end of the leading run
  of zero-density bins, and a density below the binary32 normal range may be
  zero on the GPU (flushed) and not in the oracle, so rays whose first
  non-zero coarse density is that small count as in the band too.  Rays in
  the band are held only to the mean: the mean colour error over all rays
  must stay below 2e-5.
Inputs come from seeded generators or the oracle, never from the library.
"""
import numpy as np
import pytest

import oracle
import scenes
from gpu_util import assert_close, dev, host, resample_tol

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,na,nb", [(0, 3, 4), (1, 1, 1), (1000, 129, 33), (257, 65, 64),
                                     ((1 << 18) + 5, 129, 33), (40, 4096, 4096)])
def test_merge_edges(gpu_lib, n, na, nb):
    g = scenes.rng(67)
    # quantised values: many ties inside and across the rows
    a = np.sort(g.integers(0, 200, (n, na)), 1).astype(np.float32) * np.float32(0.25)
    b = np.sort(g.integers(0, 200, (n, nb)), 1).astype(np.float32) * np.float32(0.25)
    got = host(gpu_lib.merge_edges(dev(a), dev(b)))
    assert np.array_equal(got, oracle.merge_edges(a, b))


def oracle_pdf(w, n_coarse, n_fine, union):
    o, d = w.rays_o, w.rays_d
    fp = w.fld.packed_params()
    tn, tf = oracle.clip(o, d, np.full(3, -1.5, np.float32), np.full(3, 1.5, np.float32))
    hit = tn < tf
    tn, tf = np.where(hit, tn, 0.0), np.where(hit, tf, 0.0)
    k = np.arange(n_coarse + 1) / n_coarse
    edges = (tn[:, None].astype(np.float64) + (tf - tn)[:, None] * k).astype(np.float32)
    n = o.shape[0]
    rid = np.repeat(np.arange(n), n_coarse)
    sc, _ = oracle.field_at_samples(o, d, edges[:, :-1].reshape(-1), edges[:, 1:].reshape(-1),
                                    rid, fp)
    fine, _, _ = oracle.resample(edges, sc.astype(np.float32).reshape(n, n_coarse), n_fine,
                                 oracle.MODE_SIGMA)
    e = oracle.merge_edges(edges, fine.astype(np.float32)) if union else fine.astype(np.float32)
    m = e.shape[1] - 1
    t0, t1 = e[:, :-1].reshape(-1), e[:, 1:].reshape(-1)
    s, c = oracle.field_at_samples(o, d, t0, t1, np.repeat(np.arange(n), m), fp)
    info = np.stack([np.arange(n) * m, np.full(n, m)], 1).astype(np.int32)
    ref = oracle.render_fwd(info, t0, t1, s.astype(np.float32), c.astype(np.float32))
    # rays with an interior quantile within 4e-4 F_n of an interior knot of the
    # coarse CDF (u = 0 and u = 1 map to the end edges on both sides)
    P = np.cumsum(sc.reshape(n, n_coarse) * np.diff(edges.astype(np.float64), axis=1), 1)
    F = np.concatenate([np.zeros((n, 1)), -np.expm1(-P)], 1)
    Fn = F[:, -1:]
    up = (np.arange(1, n_fine) / n_fine)[None, :] * Fn
    near_knot = np.abs(up[:, :, None] - F[:, None, 1:-1]) <= 4e-4 * Fn[:, :, None]
    # u = 0 maps to the end of the leading run of zero-density bins; a density
    # below twice the smallest normal binary32 value may be flushed to zero by
    # the GPU, moving that edge by whole bins
    s32 = sc.reshape(n, n_coarse).astype(np.float32)
    tiny = (s32 > 0) & (sc.reshape(n, n_coarse) < 2 * np.finfo(np.float32).tiny)
    first_pos = np.argmax(s32 > 0, axis=1)
    lead_tiny = tiny[np.arange(n), first_pos]
    ref["wide_band"] = (near_knot.any(axis=(1, 2)) | lead_tiny) & (Fn[:, 0] > 1e-12)
    return ref


@pytest.mark.parametrize("union", [True, False])
def test_pdf_estimator_matches_oracle_chain(gpu_lib, union):
    w = scenes.tiny()
    nc, nf = 64, 32
    fpd = dev(w.fld.packed_params().astype(np.float32))
    nbl = w.fld.n_blobs
    dens = lambda o, d, t0, t1, n: gpu_lib.blob_field(fpd, nbl, o, d, t0, t1, fixed_count=n,
                                                     want_rgb=False)[0]
    field = lambda o, d, t0, t1, n: gpu_lib.blob_field(fpd, nbl, o, d, t0, t1, fixed_count=n)
    g = gpu_lib.GridSpec(dev(w.bits), w.res)
    o, d = dev(w.rays_o), dev(w.rays_d)
    edges = gpu_lib.uniform_bins(g, o, d, nc)
    rgb, opa, _ = (host(t) for t in gpu_lib.pdf_render(dens, field, o, d, edges, nf,
                                                       union=union))
    ref = oracle_pdf(w, nc, nf, union)
    err = np.abs(rgb - ref["rgb"]).max(1)
    assert ref["opacity"].mean() > 0.2  # the rays do see the scene
    out = ~ref["wide_band"]
    assert out.mean() > 0.5, out.mean()
    assert np.quantile(err[out], 0.99) <= 2e-4, np.quantile(err[out], 0.99)
    assert err[out].max() <= 2e-3, err[out].max()
    assert err.mean() <= 2e-5, err.mean()


@pytest.mark.parametrize("union", [True, False])
def test_pdf_estimator_steps_on_oracle_densities(gpu_lib, union):
    """The estimator's own steps held to the 1e-5 bar on identical inputs: the
    oracle's coarse edges and float32 coarse densities feed the GPU inverse
    CDF (edges within the resample bar, only quantiles the oracle flags as
    within 1e-5 of a CDF knot excused); the sorted merge of the coarse edges
    with those fine edges (sorting moves no value by more than the largest
    input difference, so the merged rows keep the fine edges' bound); and the
    render on the oracle's merged intervals and float32 field values within
    1e-5.  The field itself is checked in its own test."""
    w = scenes.tiny()
    nc, nf = 64, 32
    o, d = w.rays_o, w.rays_d
    n = o.shape[0]
    fp = w.fld.packed_params()
    tn, tf = oracle.clip(o, d, np.full(3, -1.5, np.float32), np.full(3, 1.5, np.float32))
    hit = tn < tf
    span = np.stack([np.where(hit, tn, 0.0), np.where(hit, tf, 0.0)], 1)
    edges = oracle.span_bins(span, nc).astype(np.float32)
    sc, _ = oracle.field_at_samples(o, d, edges[:, :-1].reshape(-1), edges[:, 1:].reshape(-1),
                                    np.repeat(np.arange(n), nc), fp)
    sc32 = sc.astype(np.float32).reshape(n, nc)
    assert (sc32.sum(1) > 0).mean() > 0.3  # most rays cross the blobs
    # inverse CDF
    fine = host(gpu_lib.resample(dev(edges), dev(sc32), nf, mode=gpu_lib.TXS_PDF_SIGMA))
    ref, bins, _ = oracle.resample(edges, sc32, nf, oracle.MODE_SIGMA)
    tol = resample_tol(edges, sc32, 0, ref, bins)
    # an interior quantile within 1e-5 F_n of a non-zero interior knot may take
    # the neighbouring bin (the two sides sum the same binary32 inputs in
    # different orders); runs of empty bins have exactly zero mass on both
    # sides, so the first edge is never excused
    P = np.cumsum(sc32.astype(np.float64) * np.diff(edges.astype(np.float64), axis=1), 1)
    F = -np.expm1(-P)
    Fn = F[:, -1:]
    up = (np.arange(nf + 1) / nf)[None, :] * Fn
    knots = np.where(F[:, :-1] > 0, F[:, :-1], -1.0)
    near = (np.abs(up[:, :, None] - knots[:, None, :]) <= 1e-5 * Fn[:, :, None]).any(axis=2)
    near[:, 0] = near[:, -1] = False
    err = np.abs(fine - ref)
    bad = (err > tol) & ~near
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])
    assert near.mean() < 0.01, near.mean()
    band = near.any(axis=1)
    # merge (exact on its own inputs: test_merge_edges): within the fine edges'
    # bound of the oracle's merge of its own rows
    ref32 = ref.astype(np.float32)
    if union:
        m_gpu = host(gpu_lib.merge_edges(dev(edges), dev(fine)))
        m_ref = oracle.merge_edges(edges, ref32)
        ok = ~band
        assert np.all(np.abs(m_gpu - m_ref)[ok].max(1) <= tol[ok].max(1)
                      + np.spacing(np.abs(m_ref[ok]).max(1)))
    else:
        m_ref = ref32
    # render on the oracle's intervals and field values
    m = m_ref.shape[1] - 1
    t0, t1 = m_ref[:, :-1].reshape(-1), m_ref[:, 1:].reshape(-1)
    s, c = oracle.field_at_samples(o, d, t0, t1, np.repeat(np.arange(n), m), fp)
    s32, c32 = s.astype(np.float32), c.astype(np.float32)
    out = gpu_lib.render_fwd(None, dev(t0), dev(t1), dev(s32), dev(c32), n_rays=n,
                             fixed_count=m)
    info = np.stack([np.arange(n) * m, np.full(n, m)], 1).astype(np.int32)
    r = oracle.render_fwd(info, t0, t1, s32, c32)
    assert_close(host(out[0]), r["rgb"], name="rgb")
    assert_close(host(out[1]), r["opacity"], name="opacity")
    assert_close(host(out[2]), r["depth"], name="depth")
