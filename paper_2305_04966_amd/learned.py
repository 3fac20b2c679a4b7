"""Learned transmittance estimator: the proposal network and its update.

Section 3.1 ("PDF Approaches"), Table 1 third row and Eq. 4: a small network
predicts density along each ray; its rendering weights on uniform bins are
fitted by gradient descent to the weights the radiance field renders (a
PDF-matching loss), and sampling draws the final intervals from its
transmittance by inverse CDF (Eq. 3).  One update step, all in the HIP
library:

    uniform bins (fixed per ray set) -> prop_mlp_fwd -> render_fwd (weights
    only, dense bins) -> hist_loss -> weights_bwd -> prop_mlp_bwd -> adam_step
    -> mlp_pack

Targets come from the plain occupancy-grid renderer (march, filter, field,
render with weights), computed by `grid_render`.

The combined estimator (Section 3.3, "Insights from Unified Formulation";
Section 4.4, "Combined Sampling") stacks the occupancy grid on the proposal
network: `occupied_span` marches the grid for each ray's occupied span and
compacts the rays that have one, and `combined_render` bins only that span
for the proposal network.  Only argument plumbing lives here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import torch

from . import ops
from .pipeline import Packed, march, filter_transmittance


@dataclass
class GridRender:
    """Plain grid renderer output on a ray set: samples, weights, colours."""
    samples: Packed
    weights: torch.Tensor   # float32 [S]
    rgb: torch.Tensor       # float32 [N, 3]
    opacity: torch.Tensor   # float32 [N]


def grid_render(grid: ops.GridSpec, rays_o, rays_d, field_params, n_blobs, *, dt0,
                t_min=1e-4, near=0.0, far=float("inf")) -> GridRender:
    """Occupancy-grid sampling + filter + field + render (no gradient)."""
    p = march(grid, rays_o, rays_d, dt0=dt0, near=near, far=far)
    sig, _ = ops.blob_field(field_params, n_blobs, rays_o, rays_d, p.t0, p.t1, p.ray_id,
                            want_rgb=False)
    q = filter_transmittance(p, sig, t_min)
    sig, rgb = ops.blob_field(field_params, n_blobs, rays_o, rays_d, q.t0, q.t1, q.ray_id)
    out = ops.render_fwd(q.packed_info, q.t0, q.t1, sig, rgb, want_weights=True)
    return GridRender(q, out[3], out[0], out[1])


def cosine_lr(step, total, lr0=1e-2, lr1=1e-4):
    """Cosine decay from lr0 (step 1) to lr1 (step total)."""
    if total <= 1:
        return lr0
    c = 0.5 * (1.0 + math.cos(math.pi * (step - 1) / (total - 1)))
    return lr1 + (lr0 - lr1) * c


@dataclass
class ProposalEstimator:
    """Proposal network with fp32 master weights, bf16 operand tiles and Adam state."""
    params: torch.Tensor            # float32 [param count]
    hidden: int
    scale: float = 1.5
    contract: bool = False
    betas: tuple = (0.9, 0.99)
    eps: float = 1e-15
    step_count: int = 0
    spec: Optional[ops.MlpSpec] = None
    m: Optional[torch.Tensor] = None
    v: Optional[torch.Tensor] = None
    workspace: Optional[torch.Tensor] = None
    # inverse CDF inside a bin: linear (TXS_PDF_SIGMA) or exponential (TXS_PDF_SIGMA_EXP)
    sample_mode: int = ops.TXS_PDF_SIGMA

    def __post_init__(self):
        self.spec = ops.MlpSpec(self.params, self.hidden, self.scale, self.contract).repack()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        nbytes = int(ops.load().txs_mlp_bwd_workspace_size(self.hidden))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.params.device)

    # ------------------------------------------------------------ sampling
    def density(self, rays_o, rays_d, edges):
        """Proposal density at the bin midpoints -> float32 [N, n_bins]."""
        return ops.prop_mlp_fwd(self.spec, rays_o, rays_d, edges)

    def density_at(self, points):
        """Proposal density at arbitrary points [n, 3] -> float32 [n]: each point
        is a one-bin row whose midpoint is t = 0 (so x = o exactly).  This is
        the density an occupancy grid can cache when the network stands for a
        field with learnable parameters (the grid update of Section 3.1)."""
        n = points.shape[0]
        d = torch.zeros_like(points)
        d[:, 0] = 1.0
        e = torch.zeros((n, 2), dtype=torch.float32, device=points.device)
        return ops.prop_mlp_fwd(self.spec, points.contiguous(), d, e).view(-1)

    def sample(self, rays_o, rays_d, edges, n_out, u=None):
        """Inverse-CDF intervals from the proposal transmittance -> edges [N, n_out+1]."""
        sig = self.density(rays_o, rays_d, edges)
        return ops.resample(edges, sig, n_out, mode=self.sample_mode, u=u)

    def sample_intervals(self, rays_o, rays_d, edges, n_out, u=None):
        """The same intervals in the dense layout -> (t0, t1) [N*n_out]."""
        sig = self.density(rays_o, rays_d, edges)
        return ops.resample_intervals(edges, sig, n_out, mode=self.sample_mode, u=u)

    # ------------------------------------------------------------ update
    @staticmethod
    def dense_intervals(edges):
        """(t0, t1) [N*n_bins] of dense bins."""
        return ops.edges_to_intervals(edges)

    def loss_and_grad(self, rays_o, rays_d, edges, target: GridRender, t0=None, t1=None):
        """Mean PDF-matching loss and its gradient w.r.t. the parameters."""
        n, nb = edges.shape[0], edges.shape[1] - 1
        if t0 is None:
            t0, t1 = self.dense_intervals(edges)
        sig = self.density(rays_o, rays_d, edges).view(-1)
        out = ops.render_fwd(None, t0, t1, sig, None, n_rays=n, fixed_count=nb,
                             want_weights=True, want_optical_depth=True)
        w_hat = out[3].view(n, nb)
        q = target.samples
        loss, d_prop = ops.hist_loss(q.packed_info, q.t0, q.t1, target.weights, edges, w_hat)
        d_sig = ops.weights_bwd(None, t0, t1, sig, d_prop.view(-1), n_rays=n, fixed_count=nb,
                                optical_depth=out[4])
        grad = ops.prop_mlp_bwd(self.spec, rays_o, rays_d, edges, d_sig.view(n, nb),
                                workspace=self.workspace)
        return loss, grad

    def apply(self, grad, lr):
        """One Adam step on the fp32 master weights, then refresh the bf16 tiles."""
        self.step_count += 1
        ops.adam_step(self.params, self.m, self.v, grad, lr=lr, beta1=self.betas[0],
                      beta2=self.betas[1], eps=self.eps, step=self.step_count)
        self.spec.repack()

    def train_step(self, rays_o, rays_d, edges, target: GridRender, lr, t0=None, t1=None):
        loss, grad = self.loss_and_grad(rays_o, rays_d, edges, target, t0, t1)
        self.apply(grad, lr)
        return loss

    def update_every_n_steps(self, step, rays_o, rays_d, edges, target: GridRender, lr, n=1,
                             t0=None, t1=None):
        """The estimator update of Algorithm 1: a train step on every n-th
        training step of the radiance field (returns its loss), else None."""
        if step % n != 0:
            return None
        return self.train_step(rays_o, rays_d, edges, target, lr, t0, t1)


def proposal_render(est: ProposalEstimator, rays_o, rays_d, edges, n_out, field_fn, keep=False):
    """Render with the learned sampler: proposal density on `edges` -> inverse
    CDF to n_out intervals -> field_fn(rays_o, rays_d, t0, t1, n_out) ->
    (sigma, rgb) -> render forward.  Returns (rgb, opacity, depth), or with
    keep=True (t0, t1, sigma, rgb, optical_depth) for a backward."""
    n = edges.shape[0]
    t0, t1 = est.sample_intervals(rays_o, rays_d, edges, n_out)
    sig, rgb = field_fn(rays_o, rays_d, t0, t1, n_out)
    out = ops.render_fwd(None, t0, t1, sig, rgb, n_rays=n, fixed_count=n_out,
                         want_optical_depth=keep)
    if keep:
        return t0, t1, sig, rgb, out[4]
    return out[0], out[1], out[2]


# ---------------------------------------------------------------- two rounds
def two_round_intervals(est1: ProposalEstimator, est2: ProposalEstimator, rays_o, rays_d, edges,
                        n_mid, n_out):
    """Two proposal rounds (as Mip-NeRF 360 stacks them): est1 on `edges` ->
    inverse CDF to n_mid intervals -> est2 on those -> inverse CDF to n_out
    dense intervals (t0, t1)."""
    e1 = est1.sample(rays_o, rays_d, edges, n_mid)
    return est2.sample_intervals(rays_o, rays_d, e1, n_out)


def train_two_rounds(est1: ProposalEstimator, est2: ProposalEstimator, rays_o, rays_d, edges,
                     target: GridRender, lr, n_mid, t0=None, t1=None):
    """One update of both rounds against the same target weights: est1 on the
    fixed `edges`, then est2 on the n_mid intervals est1 now draws (no
    gradient flows through the resampling).  Returns both losses."""
    l1 = est1.train_step(rays_o, rays_d, edges, target, lr, t0, t1)
    e1 = est1.sample(rays_o, rays_d, edges, n_mid)
    l2 = est2.train_step(rays_o, rays_d, e1, target, lr)
    return l1, l2


# ---------------------------------------------------------------- combined
@dataclass
class OccupiedSpan:
    """The occupancy grid's part of the combined estimator: the rays that
    cross occupied space, compacted in ray order, with their occupied spans."""
    table: torch.Tensor     # int32 [N, 2]: (slot, hit) per ray
    n_alive: int
    rays_o: torch.Tensor    # float32 [M, 3]
    rays_d: torch.Tensor    # float32 [M, 3]
    span: torch.Tensor      # float32 [M, 2]

    def bins(self, n_bins):
        """Uniform proposal bins over every occupied span -> edges [M, n_bins+1]."""
        return ops.span_bins(self.span, n_bins)

    def compact(self, rows):
        """Rows of every ray -> rows of the rays that hit."""
        return ops.compact_rows(self.table, self.n_alive, rows)

    def expand(self, rows, fill=0.0):
        """Rows of the rays that hit -> rows of every ray (`fill` elsewhere)."""
        return ops.expand_rows(self.table, rows, fill)

    def target(self, judge: GridRender) -> GridRender:
        """A grid renderer's output restricted to the rays that hit (its packed
        rows re-indexed; the samples themselves are shared)."""
        q = judge.samples
        info = self.compact(q.packed_info)
        return GridRender(Packed(info, q.t0, q.t1, None), judge.weights,
                          self.compact(judge.rgb), self.compact(judge.opacity))


def occupied_span(grid: ops.GridSpec, rays_o, rays_d, *, dt0, near=0.0,
                  far=float("inf")) -> OccupiedSpan:
    """March the grid for every ray's occupied span, drop the rays without
    one and compact the rest (one device -> host read: their number)."""
    span, hit = ops.march_span(grid, rays_o, rays_d, dt0=dt0, near=near, far=far)
    table, total = ops.exclusive_scan(hit)
    m = int(total.item())
    return OccupiedSpan(table, m, ops.compact_rows(table, m, rays_o),
                        ops.compact_rows(table, m, rays_d), ops.compact_rows(table, m, span))


def combined_render(est: ProposalEstimator, sp: OccupiedSpan, n_bins, n_out, field_fn,
                    keep=False):
    """Render with the combined estimator: uniform bins over each occupied span
    -> proposal density -> inverse CDF to n_out intervals -> field -> render.
    Returns (rgb, opacity, depth) of every ray (zero where a ray found no
    occupied cell); with keep=True also the compacted (t0, t1, sigma, rgb,
    optical_depth) for a backward over the rays that hit."""
    edges = sp.bins(n_bins)
    t0, t1 = est.sample_intervals(sp.rays_o, sp.rays_d, edges, n_out)
    sig, rgb = field_fn(sp.rays_o, sp.rays_d, t0, t1, n_out)
    out = ops.render_fwd(None, t0, t1, sig, rgb, n_rays=sp.n_alive, fixed_count=n_out,
                         want_optical_depth=keep)
    full = (sp.expand(out[0]), sp.expand(out[1]), sp.expand(out[2]))
    if keep:
        return full, (t0, t1, sig, rgb, out[4])
    return full
