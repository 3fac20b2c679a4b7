"""The learned estimator's update step, end to end, against the oracle.

Per-step gradient parity (proposal forward -> weights -> PDF-matching loss ->
weights adjoint -> MLP adjoint): at every step both sides start from the same
parameters, which follow the oracle's own binary64 Adam trajectory, so no
oracle input comes from the GPU.  Edges and targets are the oracle's too.
The GPU density differs from the bf16-emulated oracle by at most a couple of
bf16 ulps at a few points (test_gpu_learned); that difference travels through
the loss, so the bar here is a relative gradient error of 1e-2, far below what
a layout or normalisation mistake produces (order one).
"""
import numpy as np
import pytest
import torch

import oracle
import scenes
from gpu_util import dev, host

pytestmark = pytest.mark.gpu

SCALE, CONTRACT = 1.5, True


@pytest.fixture(scope="module")
def scene():
    # 2 cameras x 32x16 = 1024 rays of the unbounded scene, 4 cascade levels
    w = scenes.unbounded(32, 16, n_cams=2, res=64)
    return w


def oracle_edges(w, nb):
    h = w.half_extent0 * 2.0 ** (w.n_levels - 1)
    tn, tf = oracle.clip(w.rays_o, w.rays_d, np.full(3, -h, np.float32), np.full(3, h, np.float32))
    k = np.arange(nb + 1) / nb
    return (tn[:, None].astype(np.float64) + (tf - tn)[:, None] * k).astype(np.float32)


def oracle_targets(w):
    m = oracle.march(w.rays_o, w.rays_d, w.bits, w.res, n_levels=w.n_levels,
                     half_extent0=w.half_extent0, dt0=w.dt0)
    p = w.fld.packed_params()
    s_ng, _ = oracle.field_at_samples(w.rays_o, w.rays_d, m["t0"], m["t1"], m["ray_id"], p)
    kept, _ = oracle.transmittance_prefix(m["packed_info"], m["t0"], m["t1"],
                                          s_ng.astype(np.float32), w.t_min)
    info, t0, t1, rid = oracle.gather_prefix(m["packed_info"], kept, m["t0"], m["t1"],
                                             m["ray_id"])
    s, c = oracle.field_at_samples(w.rays_o, w.rays_d, t0, t1, rid, p)
    r = oracle.render_fwd(info, t0, t1, s.astype(np.float32), c.astype(np.float32),
                          want_weights=True)
    return info, t0, t1, r["weights"].astype(np.float32)


def oracle_step(w, edges, tgt, params, H):
    """Loss and gradient of the proposal update in the oracle (bf16-emulated MLP)."""
    n, nb = edges.shape[0], edges.shape[1] - 1
    x = oracle.bin_midpoints(w.rays_o, w.rays_d, edges)
    sig = oracle.mlp_fwd(x, params, H, scale=SCALE, contract=CONTRACT,
                         emulate_bf16=True).astype(np.float32)
    info = np.stack([np.arange(n) * nb, np.full(n, nb)], 1).astype(np.int32)
    t0, t1 = edges[:, :-1].ravel(), edges[:, 1:].ravel()
    wh = oracle.render_fwd(info, t0, t1, sig, np.zeros((n * nb, 3), np.float32),
                           want_weights=True)["weights"].astype(np.float32)
    loss, d_prop = oracle.hist_loss(*tgt, edges, wh.reshape(n, nb))
    ds = oracle.weights_bwd(info, t0, t1, sig, d_prop.astype(np.float32).ravel())
    g = oracle.mlp_bwd(x, params, H, ds.astype(np.float32), scale=SCALE, contract=CONTRACT,
                       emulate_bf16=True)
    return loss, g


@pytest.mark.parametrize("H,nb,steps", [(64, 32, 20), (128, 32, 2)])
def test_update_gradient_parity_along_oracle_trajectory(gpu_lib, scene, H, nb, steps):
    from paper_2305_04966_amd.learned import GridRender, ProposalEstimator, cosine_lr
    w = scene
    edges = oracle_edges(w, nb)
    tgt = oracle_targets(w)
    assert tgt[0][:, 1].sum() > 10 * w.n_rays  # targets are not trivial
    info, t0, t1, tw = (dev(a) for a in tgt)
    target = GridRender(gpu_lib.Packed(info, t0, t1, None), tw, None, None)
    o, d, e = dev(w.rays_o), dev(w.rays_d), dev(edges)
    p = scenes.mlp_init(H).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    est = ProposalEstimator(dev(p.astype(np.float32)), H, scale=SCALE, contract=CONTRACT)
    for step in range(1, steps + 1):
        p32 = p.astype(np.float32)
        est.params.copy_(torch.from_numpy(p32))
        est.spec.repack()
        loss_gpu, g_gpu = est.loss_and_grad(o, d, e, target)
        loss_ref, g_ref = oracle_step(w, edges, tgt, p32, H)
        lg, gg = host(loss_gpu).astype(np.float64), host(g_gpu).astype(np.float64)
        lrel = abs(lg.mean() - loss_ref.mean()) / loss_ref.mean()
        grel = np.linalg.norm(gg - g_ref) / np.linalg.norm(g_ref)
        cos = gg @ g_ref / (np.linalg.norm(gg) * np.linalg.norm(g_ref))
        assert lrel <= 1e-3, (step, lrel)
        assert grel <= 1e-2 and cos >= 0.9999, (step, grel, cos)
        p, m, v = oracle.adam(p32, m, v, g_ref, lr=cosine_lr(step, 20), step=step)


def test_training_beats_untrained_network(gpu_lib):
    """What the trained estimator gains: at equal final samples, its inverse-CDF
    intervals render the field much closer to the grid renderer's colours than
    the untrained network's, and the PDF-matching loss falls by orders of
    magnitude (every 64th ray of the 2^20-ray unbounded rig, 250 steps)."""
    from paper_2305_04966_amd.learned import ProposalEstimator, cosine_lr, grid_render
    w = scenes.unbounded()
    idx = np.arange(0, w.n_rays, 64)
    o, d = dev(w.rays_o[idx]), dev(w.rays_d[idx])
    grid = gpu_lib.GridSpec(dev(w.bits.view(np.int32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                            w.half_extent0)
    fp = dev(w.fld.packed_params().astype(np.float32))
    nb = w.fld.n_blobs
    judge = grid_render(grid, o, d, fp, nb, dt0=w.dt0, t_min=w.t_min)
    edges = gpu_lib.uniform_bins(grid, o, d, 128)
    est = ProposalEstimator(dev(scenes.mlp_init(128)), 128, scale=1.5, contract=True)

    def err(n_out):
        e = est.sample(o, d, edges, n_out)
        a, b = est.dense_intervals(e)
        sig, rgb = gpu_lib.blob_field(fp, nb, o, d, a, b, fixed_count=n_out)
        out = gpu_lib.render_fwd(None, a, b, sig, rgb, n_rays=len(idx), fixed_count=n_out)
        return float((out[0] - judge.rgb).abs().mean())

    before = err(64)
    t0, t1 = est.dense_intervals(edges)
    first = None
    for step in range(1, 251):
        loss = est.train_step(o, d, edges, judge, cosine_lr(step, 250), t0, t1)
        if step == 1:
            first = float(loss.mean())
    last = float(loss.mean())
    after = err(64)
    assert np.isfinite(host(est.params)).all()
    assert last < 1e-2 * first, (first, last)
    assert after < 0.2 * before, (before, after)


def test_grid_judge_matches_oracle(gpu_lib):
    """The learned sampler's quality judge is the GPU grid renderer; on every
    256th ray of the 2^20-ray unbounded rig it equals the oracle's own full grid
    path (binary32 march recipe, binary64 field and compositing) to 1e-4 in
    colour: the GPU field is binary32 (its own test bounds it at 2e-4 relative
    in density), everything after it is held to 1e-5 by the render tests."""
    from paper_2305_04966_amd.learned import grid_render
    w = scenes.unbounded()
    idx = np.arange(0, w.n_rays, 256)
    o, d = w.rays_o[idx], w.rays_d[idx]
    grid = gpu_lib.GridSpec(dev(w.bits.view(np.int32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                            w.half_extent0)
    fp = dev(w.fld.packed_params().astype(np.float32))
    judge = grid_render(grid, dev(o), dev(d), fp, w.fld.n_blobs, dt0=w.dt0, t_min=w.t_min)
    p = w.fld.packed_params()
    m = oracle.march(o, d, w.bits, w.res, n_levels=w.n_levels, half_extent0=w.half_extent0,
                     dt0=w.dt0)
    s_ng, _ = oracle.field_at_samples(o, d, m["t0"], m["t1"], m["ray_id"], p)
    kept, _ = oracle.transmittance_prefix(m["packed_info"], m["t0"], m["t1"],
                                          s_ng.astype(np.float32), w.t_min)
    info, t0, t1, rid = oracle.gather_prefix(m["packed_info"], kept, m["t0"], m["t1"],
                                             m["ray_id"])
    s, c = oracle.field_at_samples(o, d, t0, t1, rid, p)
    ref = oracle.render_fwd(info, t0, t1, s.astype(np.float32), c.astype(np.float32))
    err = np.abs(host(judge.rgb) - ref["rgb"])
    assert err.max() <= 1e-4, err.max()
    assert ref["opacity"].mean() > 0.5  # the rays do see the scene


def test_two_proposal_rounds_train(gpu_lib):
    """Two rounds: the second network, trained on the intervals the first one
    draws, fits the same targets (its loss falls by 10x in 150 steps), and the
    trained two-round sampler renders far closer to the grid renderer than the
    untrained one at equal final samples (every 64th ray of the 2^20-ray
    unbounded rig)."""
    from paper_2305_04966_amd.learned import (ProposalEstimator, cosine_lr, grid_render,
                                              train_two_rounds, two_round_intervals)
    w = scenes.unbounded()
    idx = np.arange(0, w.n_rays, 64)
    o, d = dev(w.rays_o[idx]), dev(w.rays_d[idx])
    grid = gpu_lib.GridSpec(dev(w.bits.view(np.int32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                            w.half_extent0)
    fp = dev(w.fld.packed_params().astype(np.float32))
    nb = w.fld.n_blobs
    judge = grid_render(grid, o, d, fp, nb, dt0=w.dt0, t_min=w.t_min)
    edges = gpu_lib.disparity_bins(grid, o, d, 64, near=1.0)
    est1 = ProposalEstimator(dev(scenes.mlp_init(64)), 64, scale=1.5, contract=True)
    est2 = ProposalEstimator(dev(scenes.mlp_init(64, seed=scenes.SEED_MLP + 16)), 64, scale=1.5,
                             contract=True)
    t0, t1 = est1.dense_intervals(edges)

    def err(a, b, n):
        sig, rgb = gpu_lib.blob_field(fp, nb, o, d, a, b, fixed_count=n)
        out = gpu_lib.render_fwd(None, a, b, sig, rgb, n_rays=len(idx), fixed_count=n)
        return float((out[0] - judge.rgb).abs().mean())

    before = err(*two_round_intervals(est1, est2, o, d, edges, 32, 32), 32)
    first = None
    for step in range(1, 151):
        l1, l2 = train_two_rounds(est1, est2, o, d, edges, judge, cosine_lr(step, 150), 32, t0, t1)
        if step == 1:
            first = float(l2.mean())
    assert float(l2.mean()) < 0.1 * first, (first, float(l2.mean()))
    after = err(*two_round_intervals(est1, est2, o, d, edges, 32, 32), 32)
    assert after < 0.2 * before, (before, after)
