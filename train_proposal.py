"""Learned transmittance estimator versus the occupancy grid, on one MI355X.

The unbounded scene (64 blobs and a background shell, 4 nested 128^3 grids,
8 cameras of 512x256 = 2^20 rays).  Steps:

1. Judge and targets: the plain grid renderer (march, no-gradient filter at
   T < 1e-4, field, render with weights).  Its colours judge the learned
   sampler; its weights are the PDF-matching targets.
2. Train the proposal network (hidden 128, contracted Fourier encoding) for
   `steps` Adam steps, full batch over the training rays (every
   `train_stride`-th ray), lr cosine 1e-2 -> 1e-4, on 128 uniform bins per ray
   over the chord through the outermost grid cube.
3. Sweep the number of final samples drawn from the proposal by inverse CDF;
   render the field on them; mean |rgb - judge| over all evaluation rays and
   channels, for the trained and the untrained network.
4. Time both samplers end to end (fwd + bwd, field stand-in included on both
   sides) at the smallest sample count within the error bar.

`run_combined` repeats steps 1-4 on the bounded image scene (32 blobs, one
128^3 grid, 1024x1024 pinhole camera) for the proposal network alone and for
the combined estimator (Section 4.4, "Combined Sampling"): the grid first drops
the rays that cross no occupied cell and narrows every other ray to its
occupied span, and the proposal network bins only that span.

`run_pdf` runs the coarse-to-fine PDF estimator of vanilla NeRF (Table 1,
third row) on the image scene: the field's density on coarse uniform bins,
inverse CDF, the field on the coarse and fine edges together.

`python train_proposal.py` prints one JSON line (`--combined`, `--pdf` for the
other experiments); --save writes the trained parameters (.npy).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _timed(torch, fn, reps):
    """Mean ms of fn over reps calls (HIP events on the current stream)."""
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


class _Scene:
    """A workload's rays, grid and field stand-in on the device."""

    def __init__(self, torch, txs, w):
        import numpy as np_
        self.w = w
        self.dev = lambda a: torch.from_numpy(np_.ascontiguousarray(a)).cuda()
        self.grid = txs.GridSpec(self.dev(w.bits.view(np_.int32)), w.res, w.n_levels,
                                 (0.0, 0.0, 0.0), w.half_extent0)
        self.fp = self.dev(w.fld.packed_params().astype(np_.float32))
        nb = w.fld.n_blobs
        fp = self.fp
        self.field = lambda o, d, t0, t1, n: txs.blob_field(fp, nb, o, d, t0, t1,
                                                             fixed_count=n)


def _train(est, steps, lr0, lr1, log_every, log, step_fn):
    """Cosine-decayed Adam steps; -> (seconds, [(step, mean loss)])."""
    import torch
    from paper_2305_04966_amd.learned import cosine_lr
    losses = []
    torch.cuda.synchronize()
    t = time.perf_counter()
    for step in range(1, steps + 1):
        loss = step_fn(cosine_lr(step, steps, lr0, lr1))
        if step == 1 or step % log_every == 0 or step == steps:
            lm = float(loss.mean())
            losses.append((step, lm))
            log(f"[train] step {step} loss {lm:.6g} {time.perf_counter() - t:.1f} s")
    torch.cuda.synchronize()
    return time.perf_counter() - t, losses


def mlp_flops(hidden, adjoint=False):
    """Algorithmic FLOP per point of the proposal network.  Forward:
    2 (39 H + H^2 + H).  Adjoint: twice the forward (the usual backward count,
    one product for the activation gradients and one for the weight gradients
    per layer), which is the training step's accounting of 2^27 points at
    H = 128 = 1.73e13 FLOP for forward and backward together.  The forward the
    adjoint kernel recomputes is not counted in it (see mlp_recompute_flops)."""
    f = 2 * (39 * hidden + hidden * hidden + hidden)
    return 2 * f if adjoint else f


def mlp_recompute_flops(hidden):
    """FLOP per point of the forward the adjoint kernel recomputes instead of
    reading stored activations (work done, not counted as algorithmic)."""
    return mlp_flops(hidden)


def run(*, steps=1000, hidden=128, bins=128, ray_stride=1, train_stride=1,
        sweep=(32, 48, 64, 96, 128, 192, 256), err_bar=1e-3, lr0=1e-2, lr1=1e-4,
        log_every=50, time_reps=5, untrained=True, spacing="linear", near=1.0, rounds=1,
        n_mid=64, in_bin="linear", heldout=None, log=print):
    """The learned-versus-grid experiment.  With heldout = (i, j), cameras i
    and j of the rig's seeded eye sequence (cameras the 8 of the workload
    never include) are two held-out views: the number of final samples is
    chosen on view i (the fewest within err_bar of the grid renderer there)
    and the error is reported on view j, which neither training nor the
    choice has seen.  Returns (record, estimator, extras); extras holds view
    j's rays and renders for a comparison against an independent judge."""
    import torch

    import paper_2305_04966_amd as txs
    import scenes
    from paper_2305_04966_amd.learned import (ProposalEstimator, cosine_lr, grid_render,
                                              train_two_rounds, two_round_intervals)

    txs.load()
    w = scenes.unbounded()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    grid = txs.GridSpec(dev(w.bits.view(np.int32)), w.res, w.n_levels, (0.0, 0.0, 0.0),
                        w.half_extent0)
    fp = dev(w.fld.packed_params().astype(np.float32))
    nb = w.fld.n_blobs
    field = lambda o, d, t0, t1, n: txs.blob_field(fp, nb, o, d, t0, t1, fixed_count=n)

    ev = np.arange(0, w.n_rays, ray_stride)
    tr = np.arange(0, w.n_rays, train_stride)
    o, d = dev(w.rays_o[ev]), dev(w.rays_d[ev])
    ot, dt = dev(w.rays_o[tr]), dev(w.rays_d[tr])
    N = len(ev)
    rec = {"workload": f"unbounded: 64 blobs + shell, 4x128^3 cascade, 8 cameras; "
                       f"{N} evaluation rays, {len(tr)} training rays",
           "hidden": hidden, "bins": bins, "train_steps": steps, "err_bar": err_bar,
           "training_rays": len(tr),
           "spacing": spacing if spacing == "linear" else f"disparity from t = {near}"}

    def bins_of(ro, rd):
        """The proposal's bins over the chord through the outermost cube:
        equal in t, or equal in disparity 1/t from `near`."""
        if spacing == "disparity":
            return txs.disparity_bins(grid, ro, rd, bins, near=near)
        return txs.uniform_bins(grid, ro, rd, bins)

    # 1. judge (evaluation rays) and targets (training rays)
    judge = grid_render(grid, o, d, fp, nb, dt0=w.dt0, t_min=w.t_min)
    target = judge if train_stride == ray_stride else grid_render(grid, ot, dt, fp, nb,
                                                                  dt0=w.dt0, t_min=w.t_min)
    torch.cuda.synchronize()
    rec["grid_samples"] = judge.samples.n_samples
    log(f"[judge] {N} rays, {judge.samples.n_samples} grid samples")

    # 2. train
    edges = bins_of(o, d)
    edges_t = edges if train_stride == ray_stride else bins_of(ot, dt)
    est = ProposalEstimator(dev(scenes.mlp_init(hidden)), hidden, scale=1.5, contract=True,
                            sample_mode=txs.TXS_PDF_SIGMA_EXP if in_bin == "exp" else txs.TXS_PDF_SIGMA)
    # a second round: its own network, drawn from a second seed
    est2 = (ProposalEstimator(dev(scenes.mlp_init(hidden, seed=scenes.SEED_MLP + 16)), hidden,
                              scale=1.5, contract=True) if rounds == 2 else None)
    if rounds == 2:
        rec["rounds"] = f"2 ({bins} bins, then {n_mid} intervals)"
    rec["in_bin"] = in_bin

    def intervals(ro, rd, e, n_out):
        if rounds == 2:
            return two_round_intervals(est, est2, ro, rd, e, n_mid, n_out)
        return est.sample_intervals(ro, rd, e, n_out)

    def render_learned(ro, rd, e, n_out, keep=False):
        a, b = intervals(ro, rd, e, n_out)
        sg, rgb = field(ro, rd, a, b, n_out)
        out = txs.render_fwd(None, a, b, sg, rgb, n_rays=e.shape[0], fixed_count=n_out,
                             want_optical_depth=keep)
        return (a, b, sg, rgb, out[4]) if keep else out[0]

    def err(n_out):
        return float((render_learned(o, d, edges, n_out) - judge.rgb).abs().mean())

    # held-out views: judges from the same grid renderer
    views = {}
    if heldout is not None:
        for role, cam in zip(("select", "report"), heldout):
            ho, hd = scenes.rig_camera(cam)
            ho_t, hd_t = dev(ho), dev(hd)
            views[role] = (ho, hd, ho_t, hd_t, bins_of(ho_t, hd_t),
                           grid_render(grid, ho_t, hd_t, fp, nb, dt0=w.dt0, t_min=w.t_min))
        rec["heldout_cameras"] = {"select": int(heldout[0]), "report": int(heldout[1]),
                                  "rays_each": int(views["select"][0].shape[0])}

    def view_err(role, n_out, mask=None):
        _, _, ho_t, hd_t, e_h, jdg = views[role]
        diff = (render_learned(ho_t, hd_t, e_h, n_out) - jdg.rgb).abs()
        return float((diff if mask is None else diff[mask]).mean())

    if untrained:
        rec["untrained_err"] = {n: err(n) for n in sweep}
    t0d, t1d = est.dense_intervals(edges_t)
    losses = []
    torch.cuda.synchronize()
    t_train = time.perf_counter()
    for step in range(1, steps + 1):
        lr = cosine_lr(step, steps, lr0, lr1)
        if rounds == 2:
            loss = train_two_rounds(est, est2, ot, dt, edges_t, target, lr, n_mid, t0d, t1d)[1]
        else:
            loss = est.train_step(ot, dt, edges_t, target, lr, t0d, t1d)
        if step == 1 or step % log_every == 0 or step == steps:
            lm = float(loss.mean())
            losses.append((step, lm))
            log(f"[train] step {step} loss {lm:.6g} {time.perf_counter() - t_train:.1f} s")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t_train
    rec["train_s"] = train_s
    rec["ms_per_train_step"] = 1000.0 * train_s / max(steps, 1)
    rec["loss"] = losses
    rec["trained_err"] = {n: err(n) for n in sweep}
    log(f"[eval] trained {rec['trained_err']}")
    if heldout is not None:
        rec["select_err"] = {n: view_err("select", n) for n in sweep}
        log(f"[eval] held-out selection view {rec['select_err']}")
        choose = rec["select_err"]
    else:
        choose = rec["trained_err"]
    ok = [n for n in sweep if choose[n] <= err_bar]
    n_star = min(ok) if ok else max(sweep)
    rec["n_final"] = n_star
    rec["within_err_bar"] = bool(ok)
    seen = judge.opacity > 0.01  # the rays where the judge sees the scene
    rec["trained_err_seen"] = float((render_learned(o, d, edges, n_star)[seen] -
                                     judge.rgb[seen]).abs().mean())
    rec["rays_seen"] = int(seen.sum())
    extras = {}
    if heldout is not None:
        rec["heldout_err"] = view_err("report", n_star)
        rec["heldout_within_err_bar"] = rec["heldout_err"] <= err_bar
        ho, hd, ho_t, hd_t, e_h, jdg = views["report"]
        extras = {"rays_o": ho, "rays_d": hd,
                  "learned_rgb": render_learned(ho_t, hd_t, e_h, n_star).cpu().numpy(),
                  "judge_rgb": jdg.rgb.cpu().numpy()}
        log(f"[eval] held-out report view at {n_star} samples: {rec['heldout_err']:.3g}")

    # 4. timing, fwd + bwd, field included on both sides
    g_rgb = dev(w.grads[ev])

    def grid_step():
        p = txs.march(grid, o, d, dt0=w.dt0)
        sg, _ = txs.blob_field(fp, nb, o, d, p.t0, p.t1, p.ray_id, want_rgb=False)
        q = txs.filter_transmittance(p, sg, w.t_min)
        sg, rgb = txs.blob_field(fp, nb, o, d, q.t0, q.t1, q.ray_id)
        out = txs.render_fwd(q.packed_info, q.t0, q.t1, sg, rgb, want_optical_depth=True)
        txs.render_bwd(q.packed_info, q.t0, q.t1, sg, rgb, g_rgb, optical_depth=out[4],
                       tight=q.tight)

    def learned_step():
        a, b, sg, rgb, od = render_learned(o, d, bins_of(o, d), n_star, keep=True)
        txs.render_bwd(None, a, b, sg, rgb, g_rgb, n_rays=N, fixed_count=n_star,
                       optical_depth=od)

    for name, fn in (("grid", grid_step), ("learned", learned_step)):
        ms = _timed(torch, fn, time_reps)
        rec[f"{name}_ms"] = ms
        rec[f"{name}_rays_per_s"] = N / (ms * 1e-3)
    rec["learned_over_grid"] = rec["learned_rays_per_s"] / rec["grid_rays_per_s"]

    # the proposal network's kernels alone: the forward on every evaluation
    # ray's bins (as in the learned step), the adjoint on the training batch
    e_ev = bins_of(o, d)
    ds = torch.ones((edges_t.shape[0], bins), dtype=torch.float32, device=e_ev.device)
    rec["mlp_fwd_points"] = N * bins
    rec["mlp_fwd_ms"] = _timed(torch, lambda: est.density(o, d, e_ev), time_reps)
    rec["mlp_bwd_points"] = edges_t.shape[0] * bins
    rec["mlp_bwd_ms"] = _timed(torch, lambda: txs.prop_mlp_bwd(est.spec, ot, dt, edges_t, ds,
                                                               workspace=est.workspace),
                               time_reps)
    rec["mlp_fwd_flop_per_point"] = mlp_flops(hidden)
    rec["mlp_bwd_flop_per_point"] = mlp_flops(hidden, adjoint=True)
    rec["mlp_bwd_recompute_flop_per_point"] = mlp_recompute_flops(hidden)
    return rec, est, extras


def run_proposal_config(*, n_rays=1 << 18, hidden=64, bins=128, n_out=32, time_reps=5, log=print):
    """The proposal round at its own configuration, timed end to end: 2^18 rays
    from a radius-3 sphere into the [-1.5, 1.5]^3 box, 128 uniform bins, the
    hidden-64 network (seeded initialisation: timing does not depend on the
    weights), inverse CDF to 32 intervals, the 64-blob field without the
    background shell, render fwd + bwd.  Parity of each step at this size is
    in the test-suite."""
    import torch

    import paper_2305_04966_amd as txs
    import scenes
    from paper_2305_04966_amd.learned import ProposalEstimator

    txs.load()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    o_np, d_np = scenes.sphere_rays(n_rays)
    o, d = dev(o_np), dev(d_np)
    fld = scenes.blob_field(64)
    fp = dev(fld.packed_params().astype(np.float32))
    grid = txs.GridSpec(torch.zeros(max(1, 64 ** 3 // 32), dtype=torch.int32, device="cuda"), 64)
    est = ProposalEstimator(dev(scenes.mlp_init(hidden)), hidden, scale=1.5)
    g_rgb = dev(scenes.upstream_grads(n_rays))

    def step():
        e = txs.uniform_bins(grid, o, d, bins)
        a, b = est.sample_intervals(o, d, e, n_out)
        sg, rgb = txs.blob_field(fp, fld.n_blobs, o, d, a, b, fixed_count=n_out)
        out = txs.render_fwd(None, a, b, sg, rgb, n_rays=n_rays, fixed_count=n_out,
                             want_optical_depth=True)
        txs.render_bwd(None, a, b, sg, rgb, g_rgb, n_rays=n_rays, fixed_count=n_out,
                       optical_depth=out[4])

    e0 = txs.uniform_bins(grid, o, d, bins)
    ms = _timed(torch, step, time_reps)
    fwd_ms = _timed(torch, lambda: est.density(o, d, e0), time_reps)
    rec = {"workload": f"proposal round: {n_rays} sphere rays, {bins} uniform bins, hidden "
                       f"{hidden}, inverse CDF to {n_out} intervals, 64-blob field, render "
                       f"fwd + bwd", "ms": ms, "rays_per_s": n_rays / (ms * 1e-3),
           "mlp_fwd_points": n_rays * bins, "mlp_fwd_ms": fwd_ms,
           "mlp_fwd_flop_per_point": mlp_flops(hidden)}
    log(f"[proposal config] {rec}")
    return rec


def run_combined(*, steps=300, hidden=128, bins=128, eval_bins=(16, 32, 64, 128), ray_stride=1,
                 train_stride=4, sweep=(32, 48, 64, 96, 128, 192, 256), err_bar=1e-3, lr0=1e-2,
                 lr1=1e-4, log_every=50, time_reps=5, log=print):
    """Proposal network alone versus the combined estimator on the image scene.

    Both train the same network from the same initialisation with the same
    recipe on `bins` bins per ray; the proposal alone bins each ray's chord
    through the grid cube, the combined estimator bins the occupied span of
    the rays the grid keeps.  Each is then evaluated with every proposal bin
    count in `eval_bins` and final sample count in `sweep`; for each bin count
    the fewest final samples within `err_bar` of the grid renderer's colours
    is timed end to end (fwd + bwd, field stand-in included), and the fastest
    such configuration is each estimator's result."""
    import torch

    import paper_2305_04966_amd as txs
    import scenes
    from paper_2305_04966_amd.learned import (ProposalEstimator, combined_render, grid_render,
                                              occupied_span, proposal_render)

    txs.load()
    sc = _Scene(torch, txs, scenes.image())
    w, dev, grid = sc.w, sc.dev, sc.grid
    ev = np.arange(0, w.n_rays, ray_stride)
    tr = np.arange(0, w.n_rays, train_stride)
    o, d = dev(w.rays_o[ev]), dev(w.rays_d[ev])
    ot, dt = dev(w.rays_o[tr]), dev(w.rays_d[tr])
    N = len(ev)
    rec = {"workload": f"image: 32 blobs, 128^3 grid over [-1.5,1.5]^3, 1024x1024 pinhole; "
                       f"{N} evaluation rays, {len(tr)} training rays",
           "hidden": hidden, "train_bins": bins, "train_steps": steps, "err_bar": err_bar}

    judge = grid_render(grid, o, d, sc.fp, w.fld.n_blobs, dt0=w.dt0, t_min=w.t_min)
    target = judge if train_stride == ray_stride else grid_render(
        grid, ot, dt, sc.fp, w.fld.n_blobs, dt0=w.dt0, t_min=w.t_min)
    g_rgb = dev(w.grads[ev])
    sp = occupied_span(grid, o, d, dt0=w.dt0)
    chord = txs.uniform_bins(grid, o, d, bins)
    chord_len = (chord[:, -1] - chord[:, 0]).double().sum()
    span_len = (sp.span[:, 1] - sp.span[:, 0]).double().sum()
    rec["rays_hit"] = sp.n_alive
    rec["span_over_chord"] = float(span_len / chord_len)

    # training: the proposal alone on chord bins, the combined estimator on span bins
    chord_t = chord if train_stride == ray_stride else txs.uniform_bins(grid, ot, dt, bins)
    est_p = ProposalEstimator(dev(scenes.mlp_init(hidden)), hidden, scale=1.5)
    a_t, b_t = est_p.dense_intervals(chord_t)
    secs_p, loss_p = _train(est_p, steps, lr0, lr1, log_every, log,
                            lambda lr: est_p.train_step(ot, dt, chord_t, target, lr, a_t, b_t))
    sp_t = sp if train_stride == ray_stride else occupied_span(grid, ot, dt, dt0=w.dt0)
    span_t = sp_t.bins(bins)
    tgt_c = sp_t.target(target)
    est_c = ProposalEstimator(dev(scenes.mlp_init(hidden)), hidden, scale=1.5)
    c_t0, c_t1 = est_c.dense_intervals(span_t)
    secs_c, loss_c = _train(est_c, steps, lr0, lr1, log_every, log,
                            lambda lr: est_c.train_step(sp_t.rays_o, sp_t.rays_d, span_t, tgt_c,
                                                        lr, c_t0, c_t1))

    def render_p(nb, n):
        return proposal_render(est_p, o, d, txs.uniform_bins(grid, o, d, nb), n, sc.field)[0]

    def render_c(nb, n):
        return combined_render(est_c, sp, nb, n, sc.field)[0]

    def step_p(nb, n):
        e0 = txs.uniform_bins(grid, o, d, nb)
        a, b, sg, rgb, od = proposal_render(est_p, o, d, e0, n, sc.field, keep=True)
        txs.render_bwd(None, a, b, sg, rgb, g_rgb, n_rays=N, fixed_count=n, optical_depth=od)

    def step_c(nb, n):
        s = occupied_span(grid, o, d, dt0=w.dt0)
        _, (a, b, sg, rgb, od) = combined_render(est_c, s, nb, n, sc.field, keep=True)
        txs.render_bwd(None, a, b, sg, rgb, s.compact(g_rgb), n_rays=s.n_alive, fixed_count=n,
                       optical_depth=od)

    for name, render, step, secs, losses in (("proposal", render_p, step_p, secs_p, loss_p),
                                             ("combined", render_c, step_c, secs_c, loss_c)):
        err = {nb: {n: float((render(nb, n) - judge.rgb).abs().mean()) for n in sweep}
               for nb in eval_bins}
        log(f"[eval] {name} {err}")
        timed = {}
        for nb in eval_bins:
            ok = [n for n in sweep if err[nb][n] <= err_bar]
            if ok:
                timed[(nb, min(ok))] = _timed(torch, lambda: step(nb, min(ok)), time_reps)
        best = min(timed, key=timed.get) if timed else None
        rec[name] = {"err": {str(nb): {str(n): e for n, e in err[nb].items()} for nb in err},
                     "timed_ms": {f"{nb}x{n}": ms for (nb, n), ms in timed.items()},
                     "bins": best[0] if best else None, "n_final": best[1] if best else None,
                     "ms": timed[best] if best else None,
                     "rays_per_s": N / (timed[best] * 1e-3) if best else None,
                     "final_loss": losses[-1][1] if losses else None,
                     "ms_per_train_step": 1000.0 * secs / max(steps, 1)}

    def grid_step():
        p = txs.march(grid, o, d, dt0=w.dt0)
        sg, _ = txs.blob_field(sc.fp, w.fld.n_blobs, o, d, p.t0, p.t1, p.ray_id, want_rgb=False)
        q = txs.filter_transmittance(p, sg, w.t_min)
        sg, rgb = txs.blob_field(sc.fp, w.fld.n_blobs, o, d, q.t0, q.t1, q.ray_id)
        out = txs.render_fwd(q.packed_info, q.t0, q.t1, sg, rgb, want_optical_depth=True)
        txs.render_bwd(q.packed_info, q.t0, q.t1, sg, rgb, g_rgb, optical_depth=out[4],
                       tight=q.tight)

    rec["grid_ms"] = _timed(torch, grid_step, time_reps)
    rec["grid_rays_per_s"] = N / (rec["grid_ms"] * 1e-3)
    if rec["proposal"]["ms"] and rec["combined"]["ms"]:
        rec["combined_over_proposal"] = rec["proposal"]["ms"] / rec["combined"]["ms"]
    return rec


def run_pdf(*, coarse=(32, 64, 128), fine=(16, 32, 64, 128), ray_stride=1, err_bar=1e-3,
            time_reps=5, log=print):
    """The coarse-to-fine PDF estimator (Table 1, third row, as vanilla NeRF
    runs it) on the image scene: the field's own density on n_c uniform bins
    over each ray's chord through the grid cube, inverse CDF to n_f intervals,
    the field rendered on the coarse and fine edges together.  For each n_c
    the fewest n_f within `err_bar` of the grid renderer's colours is timed end
    to end (coarse density, fine field, render fwd + bwd); the fastest such
    configuration is the estimator's result.  Nothing is trained: the coarse
    density is the field itself (the ideal coarse network)."""
    import torch

    import paper_2305_04966_amd as txs
    import scenes
    from paper_2305_04966_amd.learned import grid_render

    txs.load()
    sc = _Scene(torch, txs, scenes.image())
    w, dev, grid = sc.w, sc.dev, sc.grid
    ev = np.arange(0, w.n_rays, ray_stride)
    o, d = dev(w.rays_o[ev]), dev(w.rays_d[ev])
    N = len(ev)
    nb = w.fld.n_blobs
    dens = lambda o_, d_, t0, t1, n: txs.blob_field(sc.fp, nb, o_, d_, t0, t1, fixed_count=n,
                                                    want_rgb=False)[0]
    judge = grid_render(grid, o, d, sc.fp, nb, dt0=w.dt0, t_min=w.t_min)
    g_rgb = dev(w.grads[ev])
    rec = {"workload": f"image: 32 blobs, 128^3 grid over [-1.5,1.5]^3, 1024x1024 pinhole; "
                       f"{N} evaluation rays", "err_bar": err_bar}

    def render(nc, nf):
        e = txs.uniform_bins(grid, o, d, nc)
        return txs.pdf_render(dens, sc.field, o, d, e, nf)[0]

    def step(nc, nf):
        e = txs.uniform_bins(grid, o, d, nc)
        a, b, sg, rgb, od, m = txs.pdf_render(dens, sc.field, o, d, e, nf, keep=True)
        txs.render_bwd(None, a, b, sg, rgb, g_rgb, n_rays=N, fixed_count=m, optical_depth=od)

    err = {nc: {nf: float((render(nc, nf) - judge.rgb).abs().mean()) for nf in fine}
           for nc in coarse}
    log(f"[eval] pdf {err}")
    timed = {}
    for nc in coarse:
        ok = [nf for nf in fine if err[nc][nf] <= err_bar]
        if ok:
            timed[(nc, min(ok))] = _timed(torch, lambda: step(nc, min(ok)), time_reps)
    best = min(timed, key=timed.get) if timed else None
    rec.update({"err": {str(nc): {str(nf): e for nf, e in err[nc].items()} for nc in err},
                "timed_ms": {f"{nc}+{nf}": ms for (nc, nf), ms in timed.items()},
                "n_coarse": best[0] if best else None, "n_fine": best[1] if best else None,
                "ms": timed[best] if best else None,
                "rays_per_s": N / (timed[best] * 1e-3) if best else None})
    return rec


def run_contracted(*, res=128, scale=1.5, tau=0.01, time_reps=5, log=print):
    """The grid estimator over contracted space on the unbounded scene: one
    res^3 grid over Mip-NeRF 360's contracted cube, built by the EMA update
    (gamma = 0) from the field's density at the cells' centre points, marched
    on the cascade's lattice; its renders against the cascade grid renderer
    (the judge of the learned experiment), and both paths timed end to end
    (march, field, filter, field, render fwd + bwd)."""
    import torch

    import paper_2305_04966_amd as txs
    import scenes
    from paper_2305_04966_amd.learned import grid_render
    from paper_2305_04966_amd.pipeline import OccupancyGrid, march_contracted

    txs.load()
    sc = _Scene(torch, txs, scenes.unbounded())
    w, dev, grid = sc.w, sc.dev, sc.grid
    o, d = dev(w.rays_o), dev(w.rays_d)
    N = w.n_rays
    nb = w.fld.n_blobs
    judge = grid_render(grid, o, d, sc.fp, nb, dt0=w.dt0, t_min=w.t_min)
    cg = txs.GridSpec(torch.zeros(res ** 3 // 32, dtype=torch.int32, device="cuda"), res,
                      w.n_levels, (0.0, 0.0, 0.0), w.half_extent0)
    est = OccupancyGrid(cg, contract_scale=scale)
    zero = torch.zeros((res ** 3, 3), dtype=torch.float32, device="cuda")
    t0z = torch.zeros(res ** 3, dtype=torch.float32, device="cuda")
    est.update(lambda pts: txs.blob_field(sc.fp, nb, pts, zero, t0z, t0z, fixed_count=1,
                                          want_rgb=False)[0], gamma=0.0, tau=tau)
    g_rgb = dev(w.grads)

    def render(contracted):
        if contracted:
            p = march_contracted(cg, o, d, scale, dt0=w.dt0)
        else:
            p = txs.march(grid, o, d, dt0=w.dt0)
        sg, _ = txs.blob_field(sc.fp, nb, o, d, p.t0, p.t1, p.ray_id, want_rgb=False)
        q = txs.filter_transmittance(p, sg, w.t_min)
        sg, rgb = txs.blob_field(sc.fp, nb, o, d, q.t0, q.t1, q.ray_id)
        out = txs.render_fwd(q.packed_info, q.t0, q.t1, sg, rgb, want_optical_depth=True)
        return p, q, sg, rgb, out

    p, q, _, _, out = render(True)
    rec = {"workload": f"unbounded: 64 blobs + shell, 8 cameras, {N} rays; contracted grid "
                       f"{res}^3 (scale {scale}) vs 4 x 128^3 cascade",
           "occupied_fraction": float(scenes.unpack_bits(cg.bits.cpu().numpy().view(np.uint32),
                                                         res ** 3).mean()),
           "marched_samples": p.n_samples, "kept_samples": q.n_samples,
           "cascade_marched_samples": None,
           "err_vs_cascade": float((out[0] - judge.rgb).abs().mean())}
    pc = txs.march(grid, o, d, dt0=w.dt0)
    rec["cascade_marched_samples"] = pc.n_samples

    def step(contracted):
        _, q_, sg, rgb, out_ = render(contracted)
        txs.render_bwd(q_.packed_info, q_.t0, q_.t1, sg, rgb, g_rgb, optical_depth=out_[4],
                       tight=q_.tight)

    for name, c in (("cascade", False), ("contracted", True)):
        ms = _timed(torch, lambda: step(c), time_reps)
        rec[f"{name}_ms"] = ms
        rec[f"{name}_rays_per_s"] = N / (ms * 1e-3)
    log(f"[contracted] {rec}")
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--bins", type=int, default=128)
    ap.add_argument("--ray-stride", type=int, default=1, help="evaluate every k-th ray")
    ap.add_argument("--train-stride", type=int, default=1, help="train on every k-th ray")
    ap.add_argument("--sweep", default="32,48,64,96,128,192,256")
    ap.add_argument("--err-bar", type=float, default=1e-3)
    ap.add_argument("--lr0", type=float, default=1e-2)
    ap.add_argument("--lr1", type=float, default=1e-4)
    ap.add_argument("--log-every", type=int, default=50)
    ap.add_argument("--time-reps", type=int, default=5)
    ap.add_argument("--save", default="")
    ap.add_argument("--combined", action="store_true",
                    help="proposal alone vs combined grid + proposal on the image scene")
    ap.add_argument("--spacing", default="linear", choices=["linear", "disparity"],
                    help="proposal bins equal in t or in 1/t over the chord")
    ap.add_argument("--near", type=float, default=1.0, help="near plane of disparity bins")
    ap.add_argument("--rounds", type=int, default=1, choices=[1, 2],
                    help="proposal rounds (2: a second network on the first one's intervals)")
    ap.add_argument("--n-mid", type=int, default=64, help="intervals the first round draws")
    ap.add_argument("--in-bin", default="linear", choices=["linear", "exp"],
                    help="inverse CDF inside a proposal bin: linear or exponential")
    ap.add_argument("--heldout", default="",
                    help="two rig camera indices i,j (>= 8): choose the final sample count "
                         "on view i, report the error on view j")
    ap.add_argument("--contracted", action="store_true",
                    help="the grid over contracted space against the cascade (unbounded)")
    ap.add_argument("--pdf", action="store_true",
                    help="the coarse-to-fine PDF estimator on the image scene")
    args = ap.parse_args()
    if args.contracted:
        print(json.dumps(run_contracted(time_reps=args.time_reps,
                                        log=lambda s: print(s, flush=True))), flush=True)
        return
    if args.pdf:
        rec = run_pdf(ray_stride=args.ray_stride, err_bar=args.err_bar,
                      time_reps=args.time_reps, log=lambda s: print(s, flush=True))
        print(json.dumps(rec), flush=True)
        return
    if args.combined:
        rec = run_combined(steps=args.steps, hidden=args.hidden, bins=args.bins,
                           ray_stride=args.ray_stride, train_stride=args.train_stride,
                           sweep=[int(s) for s in args.sweep.split(",")], err_bar=args.err_bar,
                           lr0=args.lr0, lr1=args.lr1, log_every=args.log_every,
                           time_reps=args.time_reps, log=lambda s: print(s, flush=True))
        print(json.dumps(rec), flush=True)
        return
    rec, est, _ = run(steps=args.steps, hidden=args.hidden, bins=args.bins,
                   ray_stride=args.ray_stride, train_stride=args.train_stride,
                   sweep=[int(s) for s in args.sweep.split(",")], err_bar=args.err_bar,
                   lr0=args.lr0, lr1=args.lr1, log_every=args.log_every,
                   time_reps=args.time_reps, spacing=args.spacing, near=args.near,
                   rounds=args.rounds, n_mid=args.n_mid, in_bin=args.in_bin,
                   heldout=(tuple(int(c) for c in args.heldout.split(",")) if args.heldout
                            else None),
                   log=lambda s: print(s, flush=True))
    if args.save:
        np.save(args.save, est.params.cpu().numpy())
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
