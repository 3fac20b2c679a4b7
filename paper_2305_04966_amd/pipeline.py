"""Composition of the C-ABI calls into the paper's rendering pipeline (Algorithm 1).

sampling:  march_count -> exclusive_scan -> (one host read of the total) ->
           march_fill -> density (no grad) -> transmittance_prefix ->
           exclusive_scan -> gather_prefix
rendering: render_fwd, with render_bwd as the autograd backward.
pdf_render: the coarse-to-fine PDF estimator (uniform bins -> field density ->
           resample -> merge_edges -> field -> render_fwd).
Only argument plumbing lives here; every step runs in the HIP library.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import torch

from . import ops
from ._lib import TXS_EOVERFLOW, TxsError

INT32_LIMIT = 2 ** 31


@dataclass
class Packed:
    """Packed interval samples (Section 4.2): per-ray (start, count) + samples."""
    packed_info: torch.Tensor  # int32 [N, 2]
    t0: torch.Tensor           # float32 [S]
    t1: torch.Tensor           # float32 [S]
    ray_id: Optional[torch.Tensor]  # int32 [S]
    tight: bool = False  # rows tile [0, S) exactly (a table scanned from counts)

    @property
    def n_samples(self) -> int:
        return int(self.t0.shape[0])


def _host_total(total: torch.Tensor) -> int:
    s = int(total.item())  # the one device -> host read of a sampling pass
    if s >= INT32_LIMIT:
        raise TxsError(TXS_EOVERFLOW, f"{s} samples do not fit the int32 packed layout")
    return s


def march(grid: ops.GridSpec, rays_o, rays_d, *, dt0, near=0.0, far=float("inf"),
          max_per_ray=0) -> Packed:
    counts = ops.march_count(grid, rays_o, rays_d, near=near, far=far, dt0=dt0,
                             max_per_ray=max_per_ray)
    info, total = ops.exclusive_scan(counts)
    s = _host_total(total)
    t0, t1, rid = ops.march_fill(grid, rays_o, rays_d, info, s, near=near, far=far, dt0=dt0,
                                 max_per_ray=max_per_ray)
    return Packed(info, t0, t1, rid, tight=True)


def march_contracted(grid: ops.GridSpec, rays_o, rays_d, contract_scale, *, dt0, near=0.0,
                     far=float("inf"), max_per_ray=0) -> Packed:
    """The lattice march with occupancy from a grid over contracted space."""
    counts = ops.march_count_contracted(grid, rays_o, rays_d, contract_scale, near=near,
                                        far=far, dt0=dt0, max_per_ray=max_per_ray)
    info, total = ops.exclusive_scan(counts)
    s = _host_total(total)
    t0, t1, rid = ops.march_fill_contracted(grid, rays_o, rays_d, contract_scale, info, s,
                                            near=near, far=far, dt0=dt0,
                                            max_per_ray=max_per_ray)
    return Packed(info, t0, t1, rid, tight=True)


def filter_transmittance(p: Packed, sigma, t_min=1e-4) -> Packed:
    """No-gradient filtering: keep each ray's prefix with T >= t_min."""
    kept = ops.transmittance_prefix(p.packed_info, p.t0, p.t1, sigma, t_min)
    info, total = ops.exclusive_scan(kept)
    s = _host_total(total)
    t0, t1, rid = ops.gather_prefix(p.packed_info, info, s, p.t0, p.t1)
    return Packed(info, t0, t1, rid, tight=True)


def sampling(grid: ops.GridSpec, rays_o, rays_d, density_fn: Callable, *, dt0,
             near=0.0, far=float("inf"), t_min=1e-4) -> Packed:
    """Occupancy-grid sampling followed by no-gradient filtering (Algorithm 1)."""
    p = march(grid, rays_o, rays_d, dt0=dt0, near=near, far=far)
    with torch.no_grad():
        sigma = density_fn(p.t0, p.t1, p.ray_id)
    return filter_transmittance(p, sigma, t_min)


class RenderFn(torch.autograd.Function):
    """Differentiable packed compositing.

    The backward recomputes T and w from the inputs; the only forward state it
    keeps is the per-ray total optical depth (binary64, 8 bytes per ray).
    """

    @staticmethod
    def forward(ctx, sigma, rgb, packed_info, t0, t1, bg, n_rays, fixed_count, tight=False):
        out_rgb, out_op, out_d, _, od = ops.render_fwd(packed_info, t0, t1, sigma.contiguous(),
                                                       rgb.contiguous(), n_rays=n_rays,
                                                       fixed_count=fixed_count, bg=bg,
                                                       want_optical_depth=True)
        ctx.save_for_backward(sigma, rgb, packed_info, t0, t1, bg, od)
        ctx.n_rays, ctx.fixed_count, ctx.tight = n_rays, fixed_count, tight
        return out_rgb, out_op, out_d

    @staticmethod
    def backward(ctx, g_rgb, g_op, g_d):
        sigma, rgb, packed_info, t0, t1, bg, od = ctx.saved_tensors
        n = ctx.n_rays
        dev = t0.device
        g_rgb = g_rgb.contiguous() if g_rgb is not None else torch.zeros((n, 3), device=dev)
        g_op = g_op.contiguous() if g_op is not None else None
        g_d = g_d.contiguous() if g_d is not None else None
        ds, dr = ops.render_bwd(packed_info, t0, t1, sigma.contiguous(), rgb.contiguous(),
                                g_rgb, g_op, g_d, n_rays=n, fixed_count=ctx.fixed_count, bg=bg,
                                optical_depth=od, want_d_rgb=ctx.needs_input_grad[1],
                                tight=ctx.tight)
        return ds, dr, None, None, None, None, None, None, None


def rendering(p: Packed, sigma, rgb, bg=None):
    """-> (rgb [N,3], opacity [N], depth [N]); differentiable in sigma and rgb."""
    n = p.packed_info.shape[0]
    return RenderFn.apply(sigma, rgb, p.packed_info, p.t0, p.t1, bg, n, None, p.tight)


def rendering_dense(t0, t1, sigma, rgb, n_rays, fixed_count, bg=None):
    return RenderFn.apply(sigma, rgb, None, t0, t1, bg, n_rays, fixed_count, False)


def pdf_render(density_fn: Callable, field_fn: Callable, rays_o, rays_d, edges, n_fine, *,
               union=True, keep=False):
    """Coarse-to-fine PDF estimator (Table 1, third row, as vanilla NeRF runs it):
    the radiance field's own density on the coarse bins `edges` [N, n_c+1]
    (no gradient) -> inverse CDF of its transmittance to n_fine intervals ->
    with union=True the coarse and fine edges together -> field -> render.
    density_fn(rays_o, rays_d, t0, t1, n) -> sigma and field_fn(...) ->
    (sigma, rgb) evaluate the field on n dense intervals per ray.  Returns
    (rgb, opacity, depth), or with keep=True (t0, t1, sigma, rgb,
    optical_depth, n) for a backward."""
    n, nc = edges.shape[0], edges.shape[1] - 1
    t0c, t1c = ops.edges_to_intervals(edges)
    sig_c = density_fn(rays_o, rays_d, t0c, t1c, nc)
    fine = ops.resample(edges, sig_c.view(n, nc), n_fine, mode=ops.TXS_PDF_SIGMA)
    e = ops.merge_edges(edges, fine) if union else fine
    m = e.shape[1] - 1
    t0, t1 = ops.edges_to_intervals(e)
    sig, rgb = field_fn(rays_o, rays_d, t0, t1, m)
    out = ops.render_fwd(None, t0, t1, sig, rgb, n_rays=n, fixed_count=m,
                         want_optical_depth=keep)
    if keep:
        return t0, t1, sig, rgb, out[4], m
    return out[0], out[1], out[2]


class OccupancyGrid:
    """The occupancy-grid transmittance estimator with its EMA update.

    density: float32 [n_levels res^3] cached density; grid: the GridSpec whose
    bits the marcher reads (updated in place).  update() evaluates
    density_fn(points [n, 3]) -> sigma [n] at one point per cell and blends
    it in (Section 3.1, Spatial Skipping; Table 1, occupancy-grid row).
    """

    def __init__(self, grid: ops.GridSpec, density: Optional[torch.Tensor] = None,
                 contract_scale: Optional[float] = None):
        """contract_scale: the grid is one res^3 level over contracted space (read
        by march_contracted) instead of the cascade of cubes."""
        n = (1 if contract_scale else grid.n_levels) * grid.res ** 3
        self.grid = grid
        self.contract_scale = contract_scale
        self.density = (density if density is not None else
                        torch.zeros(n, dtype=torch.float32, device=grid.bits.device))

    def points(self, u=None):
        """The cell points the update evaluates the field at."""
        if self.contract_scale:
            return ops.grid_points_contracted(self.grid, self.contract_scale, u)
        return ops.grid_points(self.grid, u)

    def update(self, density_fn: Callable, gamma=0.95, tau=0.01, u=None):
        sigma = density_fn(self.points(u))
        n = self.density.shape[0]
        ops.grid_ema(self.density, sigma, gamma, tau, self.grid.bits[:n // 32])
        self.grid.refresh()  # the brick occupancy follows the new bits

    def update_every_n_steps(self, step, density_fn: Callable, n=16, gamma=0.95, tau=0.01,
                             u=None):
        """Algorithm 1's estimator update for the grid: every n-th training step."""
        if step % n == 0:
            self.update(density_fn, gamma, tau, u)

