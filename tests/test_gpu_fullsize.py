"""Parity at the full workload sizes, in the launch configurations the benchmark
and the training driver use, on outputs the oracle can compute one by one.

* render forward / adjoint / filter: 2^20 rays with a ragged seeded layout of
  the image workload's size (~2.6e8 samples), every 4099th ray checked;
* repack of kept prefixes at that size: every element;
* inverse CDF: the proposal configuration, 2^18 rays x 128 bins -> 32, every ray;
* proposal MLP forward: the training shape, 2^20 rays x 128 bins, hidden 128,
  contracted encoding, 4096 sampled points;
* MLP adjoint at that shape: the gradient is linear in the upstream gradient,
  so an upstream gradient that is non-zero at 8192 sampled points only gives
  exactly the oracle's sum over those points (the other 1.3e8 contribute exact
  zeros);
* histogram loss: 2^20 rays x 128 bins with ~2e7 ragged targets, every 4099th
  ray.
Inputs come from seeded generators (or the oracle), never from the library.
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import assert_close, bwd_condition, dev, host
from test_gpu_learned import assert_bf16_close, assert_grad_close, bf16_ulp  # noqa: F401
from gpu_util import resample_tol

pytestmark = pytest.mark.gpu

N_FULL = 1 << 20
STRIDE = 4099


def ragged_layout(seed, n, lo, hi):
    """Per-ray lattice intervals a_r + k dt_r, k < count_r (contiguous rows)."""
    g = scenes.rng(seed)
    counts = g.integers(lo, hi, n).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    S = int(counts.sum())
    a = g.uniform(0.5, 2.0, n).astype(np.float32)
    dt = g.uniform(0.004, 0.006, n).astype(np.float32)
    t0 = np.empty(S, np.float32)
    t1 = np.empty(S, np.float32)
    CH = 1 << 16
    for r0 in range(0, n, CH):
        r1 = min(n, r0 + CH)
        c = counts[r0:r1]
        ray = np.repeat(np.arange(r0, r1), c)
        k = (np.arange(starts[r0], starts[r0] + c.sum()) - starts[ray]).astype(np.float32)
        sl = slice(starts[r0], starts[r0] + c.sum())
        t0[sl] = a[ray] + k * dt[ray]
        t1[sl] = a[ray] + (k + 1.0) * dt[ray]
    info = np.stack([starts, counts], 1).astype(np.int32)
    return info, t0, t1


def rows(info, sel):
    """Sample indices of the selected rays, and their packed table rebased to 0."""
    idx = np.concatenate([np.arange(s, s + c) for s, c in info[sel]])
    cnt = info[sel, 1].astype(np.int64)
    sub = np.stack([np.concatenate([[0], np.cumsum(cnt)[:-1]]), cnt], 1).astype(np.int32)
    return idx, sub


def test_render_and_filter_full_size(gpu_lib):
    info, t0, t1 = ragged_layout(41, N_FULL, 150, 352)
    S = t0.shape[0]
    assert S > 2.5e8
    g = scenes.rng(42)
    sig = (g.exponential(1.0, S).astype(np.float32) * np.float32(8.0))
    rgb = g.random((S, 3), dtype=np.float32)
    gr = g.standard_normal((N_FULL, 3)).astype(np.float32)
    D = {k: dev(v) for k, v in dict(info=info, t0=t0, t1=t1, sig=sig, rgb=rgb, gr=gr).items()}
    kept = host(gpu_lib.transmittance_prefix(D["info"], D["t0"], D["t1"], D["sig"], 1e-4))
    out = gpu_lib.render_fwd(D["info"], D["t0"], D["t1"], D["sig"], D["rgb"],
                             want_optical_depth=True)
    ds, dr = gpu_lib.render_bwd(D["info"], D["t0"], D["t1"], D["sig"], D["rgb"], D["gr"],
                                optical_depth=out[4])
    torch.cuda.synchronize()
    sel = np.arange(0, N_FULL, STRIDE)
    idx, sub = rows(info, sel)
    st0, st1, ssig, srgb = t0[idx], t1[idx], sig[idx], rgb[idx]
    rk, band = oracle.transmittance_prefix(sub, st0, st1, ssig, 1e-4)
    assert np.array_equal(kept[sel][~band], rk[~band])
    ref = oracle.render_fwd(sub, st0, st1, ssig, srgb)
    assert_close(host(out[0])[sel], ref["rgb"], name="rgb")
    assert_close(host(out[1])[sel], ref["opacity"], name="opacity")
    assert_close(host(out[2])[sel], ref["depth"], name="depth")
    rds, rdr = oracle.render_bwd(sub, st0, st1, ssig, srgb, gr[sel])
    seg = np.repeat(np.arange(len(sel)), sub[:, 1])
    vb = (np.abs(srgb.astype(np.float64)) * np.abs(gr[sel][seg])).sum(1)
    cond = bwd_condition(sub, st0, st1, ssig, vb)
    assert_close(host(ds)[idx], rds, floor_scale=cond, name="d_sigma")
    assert_close(host(dr)[idx], rdr, name="d_rgb")


def test_gather_full_size(gpu_lib):
    """The repack in the benchmark's launch: 2^20 ragged rows of the image
    workload's size, seeded kept prefixes (0..count, a fifth of them whole),
    every output element compared (data movement: exact)."""
    info, t0, t1 = ragged_layout(44, N_FULL, 150, 352)
    g = scenes.rng(45)
    counts = info[:, 1]
    kept = np.where(g.random(N_FULL) < 0.2, counts,
                    g.integers(0, counts + 1)).astype(np.int32)
    rid = np.repeat(np.arange(N_FULL), counts).astype(np.int32)
    info2, total2 = gpu_lib.exclusive_scan(dev(kept))
    s2 = int(total2.item())
    a, b, c = gpu_lib.gather_prefix(dev(info), info2, s2, dev(t0), dev(t1))
    r_info, r_t0, r_t1, r_rid = oracle.gather_prefix(info, kept, t0, t1, rid)
    assert s2 == len(r_t0) > 1e8
    assert np.array_equal(host(info2), r_info)
    assert np.array_equal(host(a), r_t0) and np.array_equal(host(b), r_t1)
    assert np.array_equal(host(c), r_rid)


def test_resample_proposal_configuration(gpu_lib):
    n, nb, n_out = 1 << 18, 128, 32
    g = scenes.rng(43)
    a = g.uniform(1.0, 2.0, (n, 1))
    edges = (a + np.concatenate([np.zeros((n, 1)), np.cumsum(g.uniform(0.005, 0.03, (n, nb)), 1)],
                                1)).astype(np.float32)
    vals = (g.exponential(1.0, (n, nb)) * (g.random((n, nb)) < 0.3) *
            g.choice([1.0, 30.0], (n, 1))).astype(np.float32)
    out = host(gpu_lib.resample(dev(edges), dev(vals), n_out, 0))
    ref, bins, band = oracle.resample(edges, vals, n_out, 0)
    tol = resample_tol(edges, vals, 0, ref, bins)
    bad = (np.abs(out - ref) > tol) & ~band[:, None]
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])


@pytest.fixture(scope="module")
def training_shape():
    w = scenes.unbounded()
    h = w.half_extent0 * 2.0 ** (w.n_levels - 1)
    tn, tf = oracle.clip(w.rays_o, w.rays_d, np.full(3, -h, np.float32), np.full(3, h, np.float32))
    k = np.arange(129) / 128.0
    edges = (tn[:, None].astype(np.float64) + (tf - tn)[:, None] * k).astype(np.float32)
    params = scenes.mlp_init(128)
    g = scenes.rng(44)
    params[39 * 128:40 * 128] = g.normal(0, 0.3, 128)
    params[40 * 128 + 128 * 128:41 * 128 + 128 * 128] = g.normal(0, 0.3, 128)
    return w, edges, params


def test_mlp_forward_training_shape(gpu_lib, training_shape):
    w, edges, params = training_shape
    spec = gpu_lib.MlpSpec(dev(params), 128, 1.5, True).repack()
    sig = host(gpu_lib.prop_mlp_fwd(spec, dev(w.rays_o), dev(w.rays_d), dev(edges)))
    g = scenes.rng(45)
    pts = g.choice(sig.size, 4096, replace=False)
    r, j = pts // 128, pts % 128
    x = oracle.bin_midpoints(w.rays_o[r], w.rays_d[r], np.stack([edges[r, j], edges[r, j + 1]], 1))
    ref = oracle.mlp_fwd(x, params, 128, contract=True, emulate_bf16=True)
    assert_bf16_close(sig.reshape(-1)[pts], ref, "training shape")


def test_mlp_adjoint_training_shape(gpu_lib, training_shape):
    w, edges, params = training_shape
    spec = gpu_lib.MlpSpec(dev(params), 128, 1.5, True).repack()
    g = scenes.rng(46)
    pts = np.sort(g.choice(N_FULL * 128, 8192, replace=False))
    vals = g.standard_normal(pts.size).astype(np.float32)
    ds = torch.zeros(N_FULL * 128, dtype=torch.float32, device="cuda")
    ds[torch.from_numpy(pts).cuda()] = torch.from_numpy(vals).cuda()
    got = host(gpu_lib.prop_mlp_bwd(spec, dev(w.rays_o), dev(w.rays_d), dev(edges),
                                    ds.view(N_FULL, 128)))
    r, j = pts // 128, pts % 128
    x = oracle.bin_midpoints(w.rays_o[r], w.rays_d[r], np.stack([edges[r, j], edges[r, j + 1]], 1))
    ref, mag = oracle.mlp_bwd(x, params, 128, vals, contract=True, emulate_bf16=True,
                              want_abs=True)
    assert_grad_close(got, ref, mag, "training shape, sampled points")


def test_hist_loss_full_size(gpu_lib):
    n, nb = N_FULL, 128
    g = scenes.rng(47)
    counts = g.integers(0, 40, n).astype(np.int64)
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    S = int(counts.sum())
    ray = np.repeat(np.arange(n), counts)
    k = np.arange(S) - starts[ray]
    # disjoint sorted target intervals: slot k of [1.5, 4.5] split into 40 slots
    lo = 1.5 + 3.0 * k / 40.0
    t0 = (lo + g.uniform(0.0, 0.03, S)).astype(np.float32)
    t1 = (lo + g.uniform(0.04, 0.07, S)).astype(np.float32)
    tw = (g.exponential(0.05, S) * (g.random(S) < 0.8)).astype(np.float32)
    info = np.stack([starts, counts], 1).astype(np.int32)
    edges = (1.5 + np.concatenate([np.zeros((n, 1), np.float32),
                                   np.cumsum(g.uniform(0, 1, (n, nb)).astype(np.float32), 1)], 1)
             * np.float32(3.0 / nb)).astype(np.float32)
    pw = (g.exponential(1.0, (n, nb)).astype(np.float32) / nb)
    loss, d = gpu_lib.hist_loss(dev(info), dev(t0), dev(t1), dev(tw), dev(edges), dev(pw))
    sel = np.arange(0, n, STRIDE)
    idx, sub = rows(info, sel)
    rl, rd = oracle.hist_loss(sub, t0[idx], t1[idx], tw[idx], edges[sel], pw[sel])
    # the oracle normalises by its own ray count: rescale to the full mean
    rd = rd * (len(sel) / n)
    np.testing.assert_allclose(host(loss)[sel], rl, rtol=2e-5, atol=1e-7)
    np.testing.assert_allclose(host(d)[sel], rd, rtol=2e-5, atol=1e-12)
