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
from gpu_util import dev, host

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
