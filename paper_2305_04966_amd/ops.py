"""Thin Python binding of the txs C ABI: one function per entry point, same names.

Every function takes CUDA (HIP) torch tensors, checks dtype / layout / device,
allocates the outputs with torch (device memory only) and calls the library on
torch's current stream.  No computation of the method happens here.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from ._lib import TXS_PDF_SIGMA, TXS_PDF_SIGMA_EXP, TXS_PDF_WEIGHTS, Grid, MarchParams, check, load

__all__ = ["GridSpec", "march_count", "exclusive_scan", "exclusive_scan_noalloc",
           "exclusive_scan_noalloc_max_rays", "march_fill", "transmittance_prefix",
           "gather_prefix", "render_fwd", "render_bwd", "weights_bwd", "resample",
           "uniform_bins", "edges_to_intervals", "resample_intervals", "blob_field",
           "march_span", "compact_rows", "expand_rows", "span_bins", "merge_edges", "disparity_bins", "march_count_contracted",
           "march_fill_contracted", "grid_points_contracted",
           "TXS_PDF_SIGMA",
           "TXS_PDF_WEIGHTS", "TXS_PDF_SIGMA_EXP"]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch.Tensor")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def _opt(t, name, dtype, shape=None):
    return None if t is None else _need(t, name, dtype, shape)


@dataclass
class GridSpec:
    """Occupancy grid: bits (uint32-in-int32 tensor), res, levels, box.

    Unless skip is False (and for res >= 8) the grid keeps its brick
    occupancy (`coarse`, built by txs_grid_coarsen when the spec is made) for
    the march's empty-space skipping: with skip="auto" the descriptor passes
    it when every level is sparse (see refresh), with skip=True always (the
    library still skips only where its per-level and per-segment rules
    allow).  After changing `bits` in place, call refresh() so that the brick
    occupancy describes the new bits."""
    bits: torch.Tensor
    res: int
    n_levels: int = 1
    center: tuple = (0.0, 0.0, 0.0)
    half_extent0: float = 1.5
    skip: object = "auto"
    coarse: torch.Tensor = None

    def __post_init__(self):
        if self.skip is not False and self.coarse is None:
            w = int(load().txs_grid_coarse_words(self.res))
            if w > 0 and self.bits.numel() * 32 >= self.n_levels * self.res ** 3:
                self.coarse = torch.empty(w * self.n_levels, dtype=torch.int32,
                                          device=self.bits.device)
                self.refresh()

    def refresh(self):
        """Rebuilds the brick occupancy from the current bits (no-op without it).

        The march skips only on levels with at most 5/16 of their bricks
        occupied, and skipping pays only on sparse grids (measured on MI355X:
        one 128^3 level with 19% of its bricks occupied, the count pass 10%
        faster; a 4-level cascade with two of its levels that sparse, 18%
        slower, the dense levels paying for the skipping kernel); so the
        descriptor carries the brick occupancy only when every level is that
        sparse (one small device-to-host read of the per-level counts, once
        per grid update)."""
        self._skip_levels = False
        if self.coarse is not None:
            g = self._fill(Grid())
            g.coarse = None
            check(load().txs_grid_coarsen(C.byref(g), _ptr(self.coarse), _stream()),
                  "txs_grid_coarsen")
            per_level = self.coarse.numel() // self.n_levels
            counts = self.coarse.view(self.n_levels, per_level)[:, -1].cpu()
            bricks = (self.res // 8) ** 3
            self._skip_levels = (self.skip is True or
                                 bool((16 * counts.to(torch.int64) <= 5 * bricks).all()))
        return self

    def struct_contracted(self) -> Grid:
        """The descriptor of a grid over contracted space (one res^3 level of bits)."""
        _need(self.bits, "grid.bits", torch.int32)
        if self.bits.numel() * 32 < self.res ** 3:
            raise ValueError("grid.bits holds fewer than res^3 bits")
        g = self._fill(Grid())
        g.coarse = None
        return g

    def struct(self) -> Grid:
        _need(self.bits, "grid.bits", torch.int32)
        if self.bits.numel() * 32 < self.n_levels * self.res ** 3:
            raise ValueError("grid.bits holds fewer than n_levels*res^3 bits")
        return self._fill(Grid())

    def _fill(self, g: Grid) -> Grid:
        g.bits = self.bits.data_ptr()
        g.res = self.res
        g.n_levels = self.n_levels
        g.center = (C.c_float * 3)(*self.center)
        g.half_extent0 = self.half_extent0
        use = self.coarse is not None and getattr(self, "_skip_levels", False)
        g.coarse = self.coarse.data_ptr() if use else None
        return g


def _params(near, far, dt0, max_per_ray):
    p = MarchParams()
    p.near_plane, p.far_plane, p.dt0, p.max_per_ray = near, far, dt0, max_per_ray
    return p


def _rays(rays_o, rays_d):
    n = rays_o.shape[0]
    _need(rays_o, "rays_o", torch.float32, (n, 3))
    _need(rays_d, "rays_d", torch.float32, (n, 3))
    return n


def march_count(grid: GridSpec, rays_o, rays_d, *, near=0.0, far=float("inf"), dt0,
                max_per_ray=0, counts=None):
    n = _rays(rays_o, rays_d)
    counts = counts if counts is not None else torch.empty(n, dtype=torch.int32,
                                                           device=rays_o.device)
    _need(counts, "counts", torch.int32, (n,))
    g, p = grid.struct(), _params(near, far, dt0, max_per_ray)
    check(load().txs_march_count(C.byref(g), C.byref(p), _ptr(rays_o), _ptr(rays_d), n,
                                 _ptr(counts), _stream()), "txs_march_count")
    return counts


def exclusive_scan(counts, packed_info=None, total=None):
    """-> (packed_info int32 [N,2], total int64 [1] on the device)."""
    n = counts.shape[0]
    _need(counts, "counts", torch.int32, (n,))
    dev = counts.device
    packed_info = packed_info if packed_info is not None else torch.empty(
        (n, 2), dtype=torch.int32, device=dev)
    total = total if total is not None else torch.empty(1, dtype=torch.int64, device=dev)
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    _need(total, "total", torch.int64, (1,))
    L = load()
    ws_bytes = int(L.txs_scan_workspace_size(n))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    check(L.txs_exclusive_scan(_ptr(counts), n, _ptr(packed_info), _ptr(total), _ptr(ws),
                               ws_bytes, _stream()), "txs_exclusive_scan")
    return packed_info, total


def exclusive_scan_noalloc(counts, packed_info, total):
    """txs_exclusive_scan without a workspace: the caller passes the outputs
    (packed_info int32 [N,2], total int64 [1]) and nothing is allocated."""
    n = counts.shape[0]
    _need(counts, "counts", torch.int32, (n,))
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    _need(total, "total", torch.int64, (1,))
    check(load().txs_exclusive_scan_noalloc(_ptr(counts), n, _ptr(packed_info), _ptr(total),
                                            _stream()), "txs_exclusive_scan_noalloc")
    return packed_info, total


def exclusive_scan_noalloc_max_rays():
    return int(load().txs_exclusive_scan_noalloc_max_rays())


def march_fill(grid: GridSpec, rays_o, rays_d, packed_info, n_samples, *, near=0.0,
               far=float("inf"), dt0, max_per_ray=0, want_ray_id=True):
    n = _rays(rays_o, rays_d)
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    dev = rays_o.device
    t0 = torch.empty(n_samples, dtype=torch.float32, device=dev)
    t1 = torch.empty(n_samples, dtype=torch.float32, device=dev)
    rid = torch.empty(n_samples, dtype=torch.int32, device=dev) if want_ray_id else None
    g, p = grid.struct(), _params(near, far, dt0, max_per_ray)
    check(load().txs_march_fill(C.byref(g), C.byref(p), _ptr(rays_o), _ptr(rays_d), n,
                                _ptr(packed_info), n_samples, _ptr(t0), _ptr(t1), _ptr(rid),
                                _stream()), "txs_march_fill")
    return t0, t1, rid


def march_count_contracted(grid: GridSpec, rays_o, rays_d, contract_scale, *, near=0.0,
                           far=float("inf"), dt0, max_per_ray=0):
    """Counts of the lattice march with occupancy from a grid over contracted space."""
    n = _rays(rays_o, rays_d)
    counts = torch.empty(n, dtype=torch.int32, device=rays_o.device)
    g, p = grid.struct_contracted(), _params(near, far, dt0, max_per_ray)
    check(load().txs_march_count_contracted(C.byref(g), C.byref(p), float(contract_scale),
                                            _ptr(rays_o), _ptr(rays_d), n, _ptr(counts),
                                            _stream()), "txs_march_count_contracted")
    return counts


def march_fill_contracted(grid: GridSpec, rays_o, rays_d, contract_scale, packed_info,
                          n_samples, *, near=0.0, far=float("inf"), dt0, max_per_ray=0,
                          want_ray_id=True):
    n = _rays(rays_o, rays_d)
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    dev = rays_o.device
    t0 = torch.empty(n_samples, dtype=torch.float32, device=dev)
    t1 = torch.empty(n_samples, dtype=torch.float32, device=dev)
    rid = torch.empty(n_samples, dtype=torch.int32, device=dev) if want_ray_id else None
    g, p = grid.struct_contracted(), _params(near, far, dt0, max_per_ray)
    check(load().txs_march_fill_contracted(C.byref(g), C.byref(p), float(contract_scale),
                                           _ptr(rays_o), _ptr(rays_d), n, _ptr(packed_info),
                                           n_samples, _ptr(t0), _ptr(t1), _ptr(rid), _stream()),
          "txs_march_fill_contracted")
    return t0, t1, rid


def transmittance_prefix(packed_info, t0, t1, sigma, t_min=1e-4):
    n = packed_info.shape[0]
    s = t0.shape[0]
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma)):
        _need(t, name, torch.float32, (s,))
    kept = torch.empty(n, dtype=torch.int32, device=t0.device)
    check(load().txs_transmittance_prefix(_ptr(packed_info), n, s, _ptr(t0), _ptr(t1),
                                          _ptr(sigma), float(t_min), _ptr(kept), _stream()),
          "txs_transmittance_prefix")
    return kept


def gather_prefix(packed_info_in, packed_info_out, n_out, t0, t1, want_ray_id=True):
    n = packed_info_in.shape[0]
    s = t0.shape[0]
    _need(packed_info_in, "packed_info_in", torch.int32, (n, 2))
    _need(packed_info_out, "packed_info_out", torch.int32, (n, 2))
    _need(t0, "t0", torch.float32, (s,))
    _need(t1, "t1", torch.float32, (s,))
    dev = t0.device
    t0o = torch.empty(n_out, dtype=torch.float32, device=dev)
    t1o = torch.empty(n_out, dtype=torch.float32, device=dev)
    rido = torch.empty(n_out, dtype=torch.int32, device=dev) if want_ray_id else None
    check(load().txs_gather_prefix(_ptr(packed_info_in), _ptr(packed_info_out), n, s, _ptr(t0),
                                   _ptr(t1), n_out, _ptr(t0o), _ptr(t1o), _ptr(rido),
                                   _stream()), "txs_gather_prefix")
    return t0o, t1o, rido


def _layout(packed_info, fixed_count, n_rays):
    if packed_info is not None:
        _need(packed_info, "packed_info", torch.int32, (n_rays, 2))
        return 0
    if fixed_count is None or fixed_count < 0:
        raise ValueError("dense layout needs fixed_count >= 0")
    return int(fixed_count)


def render_fwd(packed_info, t0, t1, sigma, rgb, *, n_rays=None, fixed_count=None, bg=None,
               want_weights=False, want_optical_depth=False):
    """-> (rgb [N,3], opacity [N], depth [N], weights [S] or None[, optical depth f64 [N]])."""
    n = packed_info.shape[0] if packed_info is not None else int(n_rays)
    fc = _layout(packed_info, fixed_count, n)
    s = t0.shape[0]
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma)):
        _need(t, name, torch.float32, (s,))
    _opt(rgb, "rgb", torch.float32, (s, 3))  # None: weights / opacity / depth only
    _opt(bg, "bg", torch.float32, (n, 3))
    dev = t0.device
    out_rgb = torch.empty((n, 3), dtype=torch.float32, device=dev)
    out_op = torch.empty(n, dtype=torch.float32, device=dev)
    out_d = torch.empty(n, dtype=torch.float32, device=dev)
    w = torch.empty(s, dtype=torch.float32, device=dev) if want_weights else None
    od = torch.empty(n, dtype=torch.float64, device=dev) if want_optical_depth else None
    check(load().txs_render_fwd(_ptr(packed_info), fc, n, s, _ptr(t0), _ptr(t1), _ptr(sigma),
                                _ptr(rgb), _ptr(bg), _ptr(out_rgb), _ptr(out_op), _ptr(out_d),
                                _ptr(w), _ptr(od), _stream()), "txs_render_fwd")
    if want_optical_depth:
        return out_rgb, out_op, out_d, w, od
    return out_rgb, out_op, out_d, w


def _covers(packed_info, fc, n, s, tight):
    """True when the rows are known to tile [0, s): the adjoint then writes
    every output sample and the outputs need no clearing.  A dense layout
    tiles it iff n * fixed_count == s; a packed table only when the caller
    says so (a table from the scan of its own counts, with s = the total)."""
    return (n * fc == s) if packed_info is None else bool(tight)


def _grad_out(shape, covered, dev):
    # the adjoint leaves samples outside every row unchanged: those are zero
    return (torch.empty if covered else torch.zeros)(shape, dtype=torch.float32, device=dev)


def render_bwd(packed_info, t0, t1, sigma, rgb, g_rgb, g_opacity=None, g_depth=None, *,
               n_rays=None, fixed_count=None, bg=None, optical_depth=None, want_d_rgb=True,
               tight=False):
    """-> (d_sigma [S], d_rgb [S,3] or None).  optical_depth: the forward's, or None.

    Samples that belong to no row get zero gradient.  tight=True states that
    packed_info's rows tile [0, S) (e.g. a table scanned from counts summing to
    S), which spares clearing the outputs first."""
    n = packed_info.shape[0] if packed_info is not None else int(n_rays)
    fc = _layout(packed_info, fixed_count, n)
    s = t0.shape[0]
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma)):
        _need(t, name, torch.float32, (s,))
    _need(rgb, "rgb", torch.float32, (s, 3))
    _need(g_rgb, "g_rgb", torch.float32, (n, 3))
    _opt(g_opacity, "g_opacity", torch.float32, (n,))
    _opt(g_depth, "g_depth", torch.float32, (n,))
    _opt(bg, "bg", torch.float32, (n, 3))
    _opt(optical_depth, "optical_depth", torch.float64, (n,))
    dev = t0.device
    covered = _covers(packed_info, fc, n, s, tight)
    ds = _grad_out(s, covered, dev)
    dr = _grad_out((s, 3), covered, dev) if want_d_rgb else None
    check(load().txs_render_bwd(_ptr(packed_info), fc, n, s, _ptr(t0), _ptr(t1), _ptr(sigma),
                                _ptr(rgb), _ptr(bg), _ptr(optical_depth), _ptr(g_rgb),
                                _ptr(g_opacity), _ptr(g_depth), _ptr(ds), _ptr(dr), _stream()),
          "txs_render_bwd")
    return ds, dr


def weights_bwd(packed_info, t0, t1, sigma, g_w, *, n_rays=None, fixed_count=None,
                optical_depth=None, tight=False):
    """dL/dsigma from dL/dw; zero for samples that belong to no row (tight as
    for render_bwd)."""
    n = packed_info.shape[0] if packed_info is not None else int(n_rays)
    fc = _layout(packed_info, fixed_count, n)
    s = t0.shape[0]
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma), ("g_w", g_w)):
        _need(t, name, torch.float32, (s,))
    _opt(optical_depth, "optical_depth", torch.float64, (n,))
    ds = _grad_out(s, _covers(packed_info, fc, n, s, tight), t0.device)
    check(load().txs_weights_bwd(_ptr(packed_info), fc, n, s, _ptr(t0), _ptr(t1), _ptr(sigma),
                                 _ptr(optical_depth), _ptr(g_w), _ptr(ds), _stream()),
          "txs_weights_bwd")
    return ds


def resample(edges, vals, n_out, mode=TXS_PDF_SIGMA, u=None):
    n, nb1 = edges.shape
    _need(edges, "edges", torch.float32, (n, nb1))
    _need(vals, "vals", torch.float32, (n, nb1 - 1))
    _opt(u, "u", torch.float32, (n, n_out + 1))
    out = torch.empty((n, n_out + 1), dtype=torch.float32, device=edges.device)
    check(load().txs_resample(n, nb1 - 1, _ptr(edges), _ptr(vals), mode, n_out, _ptr(u),
                              _ptr(out), _stream()), "txs_resample")
    return out


def resample_intervals(edges, vals, n_out, mode=TXS_PDF_SIGMA, u=None):
    """Inverse CDF straight to dense intervals -> (t0, t1) float32 [N*n_out]."""
    n, nb1 = edges.shape
    _need(edges, "edges", torch.float32, (n, nb1))
    _need(vals, "vals", torch.float32, (n, nb1 - 1))
    _opt(u, "u", torch.float32, (n, n_out + 1))
    t0 = torch.empty(n * n_out, dtype=torch.float32, device=edges.device)
    t1 = torch.empty_like(t0)
    check(load().txs_resample_intervals(n, nb1 - 1, _ptr(edges), _ptr(vals), mode, n_out,
                                        _ptr(u), _ptr(t0), _ptr(t1), _stream()),
          "txs_resample_intervals")
    return t0, t1


def edges_to_intervals(edges):
    """Dense (t0, t1) [N*n] of per-ray edges [N, n+1]."""
    n, nb1 = edges.shape
    _need(edges, "edges", torch.float32, (n, nb1))
    t0 = torch.empty(n * (nb1 - 1), dtype=torch.float32, device=edges.device)
    t1 = torch.empty_like(t0)
    check(load().txs_edges_to_intervals(_ptr(edges), n, nb1 - 1, _ptr(t0), _ptr(t1), _stream()),
          "txs_edges_to_intervals")
    return t0, t1


def uniform_bins(grid: GridSpec, rays_o, rays_d, n_bins, *, near=0.0, far=float("inf")):
    n = _rays(rays_o, rays_d)
    out = torch.empty((n, n_bins + 1), dtype=torch.float32, device=rays_o.device)
    g = grid.struct()
    check(load().txs_uniform_bins(C.byref(g), float(near), float(far), _ptr(rays_o),
                                  _ptr(rays_d), n, n_bins, _ptr(out), _stream()),
          "txs_uniform_bins")
    return out


def disparity_bins(grid: GridSpec, rays_o, rays_d, n_bins, *, near, far=float("inf")):
    """Chord bins of equal width in 1/t (near > 0) -> edges [N, n_bins+1]."""
    n = _rays(rays_o, rays_d)
    out = torch.empty((n, n_bins + 1), dtype=torch.float32, device=rays_o.device)
    g = grid.struct()
    check(load().txs_disparity_bins(C.byref(g), float(near), float(far), _ptr(rays_o),
                                    _ptr(rays_d), n, n_bins, _ptr(out), _stream()),
          "txs_disparity_bins")
    return out


def blob_field(params, n_blobs, rays_o, rays_d, t0, t1, ray_id=None, fixed_count=0,
               want_rgb=True):
    """Support: analytic stand-in radiance field at interval midpoints."""
    n_rays = _rays(rays_o, rays_d)
    s = t0.shape[0]
    _need(params, "params", torch.float32, (32 + 3 * n_blobs,))
    _need(t0, "t0", torch.float32, (s,))
    _need(t1, "t1", torch.float32, (s,))
    _opt(ray_id, "ray_id", torch.int32, (s,))
    dev = t0.device
    sigma = torch.empty(s, dtype=torch.float32, device=dev)
    rgb = torch.empty((s, 3), dtype=torch.float32, device=dev) if want_rgb else None
    check(load().txs_blob_field(_ptr(params), n_blobs, _ptr(rays_o), _ptr(rays_d), n_rays, _ptr(t0),
                                _ptr(t1), _ptr(ray_id), int(fixed_count), s, _ptr(sigma),
                                _ptr(rgb), _stream()), "txs_blob_field")
    return sigma, rgb


# ---------------------------------------------------------------- proposal MLP
@dataclass
class MlpSpec:
    """Proposal network: fp32 parameter vector + its packed bf16 operand tiles."""
    params: torch.Tensor  # float32 [txs_mlp_param_count(hidden)]
    hidden: int
    scale: float = 1.5
    contract: bool = False
    packed: torch.Tensor = None  # uint8 [txs_mlp_packed_bytes(hidden)]

    def repack(self):
        """Refresh the bf16 operand tiles from the fp32 parameters (after an update)."""
        L = load()
        n = int(L.txs_mlp_param_count(self.hidden))
        _need(self.params, "mlp.params", torch.float32, (n,))
        nbytes = int(L.txs_mlp_packed_bytes(self.hidden))
        if self.packed is None or self.packed.numel() != nbytes:
            self.packed = torch.empty(nbytes, dtype=torch.uint8, device=self.params.device)
        check(L.txs_mlp_pack(_ptr(self.params), self.hidden, _ptr(self.packed), _stream()),
              "txs_mlp_pack")
        return self

    def struct(self):
        from ._lib import Mlp
        if self.packed is None:
            self.repack()
        m = Mlp()
        m.packed, m.params = self.packed.data_ptr(), self.params.data_ptr()
        m.hidden, m.scale, m.contract = self.hidden, float(self.scale), int(self.contract)
        return m


def mlp_param_count(hidden):
    return int(load().txs_mlp_param_count(hidden))


def prop_mlp_bwd(mlp: MlpSpec, rays_o, rays_d, edges, d_sigma, workspace=None):
    """dL/dparams (float32 [param count]) given dL/dsigma at the bin midpoints.

    workspace: optional uint8 device tensor of txs_mlp_bwd_workspace_size bytes,
    reused across calls; allocated here when None.
    """
    n = _rays(rays_o, rays_d)
    nb1 = edges.shape[1]
    _need(edges, "edges", torch.float32, (n, nb1))
    _need(d_sigma, "d_sigma", torch.float32, (n, nb1 - 1))
    L = load()
    need = int(L.txs_mlp_bwd_workspace_size(mlp.hidden))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=edges.device)
    grad = torch.empty(mlp.params.numel(), dtype=torch.float32, device=edges.device)
    m = mlp.struct()
    check(L.txs_prop_mlp_bwd(C.byref(m), _ptr(rays_o), _ptr(rays_d), n, nb1 - 1, _ptr(edges),
                             _ptr(d_sigma), _ptr(grad), _ptr(workspace),
                             workspace.numel() * workspace.element_size(), _stream()),
          "txs_prop_mlp_bwd")
    return grad


def hist_loss(packed_info, t0, t1, w, edges, prop_w, eps=1e-7, want_grad=True):
    """Proposal loss per ray and d(mean loss)/d prop_w ([N, n_bins] or None)."""
    n = packed_info.shape[0]
    s = t0.shape[0]
    _need(packed_info, "packed_info", torch.int32, (n, 2))
    for name, t in (("t0", t0), ("t1", t1), ("w", w)):
        _need(t, name, torch.float32, (s,))
    nb1 = edges.shape[1]
    _need(edges, "edges", torch.float32, (n, nb1))
    _need(prop_w, "prop_w", torch.float32, (n, nb1 - 1))
    loss = torch.empty(n, dtype=torch.float32, device=edges.device)
    d = torch.empty((n, nb1 - 1), dtype=torch.float32, device=edges.device) if want_grad else None
    check(load().txs_hist_loss(_ptr(packed_info), n, s, _ptr(t0), _ptr(t1), _ptr(w), nb1 - 1,
                               _ptr(edges), _ptr(prop_w), float(eps), _ptr(loss), _ptr(d),
                               _stream()), "txs_hist_loss")
    return loss, d


def adam_step(params, m, v, grad, lr, step, beta1=0.9, beta2=0.99, eps=1e-15):
    """In-place Adam step on fp32 parameter / moment tensors."""
    n = params.numel()
    for name, t in (("params", params), ("m", m), ("v", v), ("grad", grad)):
        _need(t, name, torch.float32, (n,))
    check(load().txs_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), n, float(lr),
                               float(beta1), float(beta2), float(eps), int(step), _stream()),
          "txs_adam_step")


def prop_mlp_fwd(mlp: MlpSpec, rays_o, rays_d, edges):
    """Proposal density at bin midpoints -> float32 [N, n_bins]."""
    n = _rays(rays_o, rays_d)
    nb1 = edges.shape[1]
    _need(edges, "edges", torch.float32, (n, nb1))
    out = torch.empty((n, nb1 - 1), dtype=torch.float32, device=edges.device)
    m = mlp.struct()
    check(load().txs_prop_mlp_fwd(C.byref(m), _ptr(rays_o), _ptr(rays_d), n, nb1 - 1,
                                  _ptr(edges), _ptr(out), _stream()), "txs_prop_mlp_fwd")
    return out


def grid_points(grid: GridSpec, u=None):
    """One point per grid cell (centres, or jittered by u [n_cells, 3]) -> [n_cells, 3]."""
    n = grid.n_levels * grid.res ** 3
    g = grid.struct()
    _opt(u, "u", torch.float32, (n, 3))
    out = torch.empty((n, 3), dtype=torch.float32, device=grid.bits.device)
    check(load().txs_grid_points(C.byref(g), _ptr(u), _ptr(out), _stream()), "txs_grid_points")
    return out


def grid_points_contracted(grid: GridSpec, contract_scale, u=None):
    """One point per cell of a grid over contracted space -> [res^3, 3]."""
    n = grid.res ** 3
    g = grid.struct_contracted()
    _opt(u, "u", torch.float32, (n, 3))
    out = torch.empty((n, 3), dtype=torch.float32, device=grid.bits.device)
    check(load().txs_grid_points_contracted(C.byref(g), float(contract_scale), _ptr(u), _ptr(out),
                                            _stream()), "txs_grid_points_contracted")
    return out


def grid_ema(density, sigma, gamma, tau, bits):
    """In place: density <- gamma density + (1 - gamma) sigma; bits <- density > tau."""
    n = density.shape[0]
    _need(density, "density", torch.float32, (n,))
    _need(sigma, "sigma", torch.float32, (n,))
    _need(bits, "bits", torch.int32, (n // 32,))
    check(load().txs_grid_ema(n, _ptr(density), _ptr(sigma), float(gamma), float(tau),
                              _ptr(bits), _stream()), "txs_grid_ema")


def stream_probe(t0, t1, sigma, rgb, out_a, out_b):
    """Measurement support: the render adjoint's traffic with trivial arithmetic."""
    n = t0.shape[0]
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma), ("out_a", out_a)):
        _need(t, name, torch.float32, (n,))
    _need(rgb, "rgb", torch.float32, (n, 3))
    _need(out_b, "out_b", torch.float32, (n, 3))
    check(load().txs_stream_probe(n, _ptr(t0), _ptr(t1), _ptr(sigma), _ptr(rgb), _ptr(out_a),
                                  _ptr(out_b), _stream()), "txs_stream_probe")


def read_probe(t0, t1, sigma, rgb, out=None):
    """Measurement support: the forward render's reads with trivial arithmetic."""
    n = t0.shape[0]
    for name, t in (("t0", t0), ("t1", t1), ("sigma", sigma)):
        _need(t, name, torch.float32, (n,))
    _need(rgb, "rgb", torch.float32, (n, 3))
    size = int(load().txs_read_probe_out_size())
    out = out if out is not None else torch.empty(size, dtype=torch.float32, device=t0.device)
    _need(out, "out", torch.float32, (size,))
    check(load().txs_read_probe(n, _ptr(t0), _ptr(t1), _ptr(sigma), _ptr(rgb), _ptr(out),
                                _stream()), "txs_read_probe")
    return out


def march_span(grid: GridSpec, rays_o, rays_d, *, near=0.0, far=float("inf"), dt0):
    """Occupied span of every ray -> (span float32 [N, 2], hit int32 [N])."""
    n = _rays(rays_o, rays_d)
    dev = rays_o.device
    span = torch.empty((n, 2), dtype=torch.float32, device=dev)
    hit = torch.empty(n, dtype=torch.int32, device=dev)
    g, p = grid.struct(), _params(near, far, dt0, 0)
    check(load().txs_march_span(C.byref(g), C.byref(p), _ptr(rays_o), _ptr(rays_d), n,
                                _ptr(span), _ptr(hit), _stream()), "txs_march_span")
    return span, hit


def compact_rows(table, n_alive, src):
    """Rows of src [N, ...] of the rays whose table flag is 1 -> [n_alive, ...]."""
    n = table.shape[0]
    _need(table, "table", torch.int32, (n, 2))
    if src.shape[0] != n or src.element_size() != 4:
        raise ValueError("compact_rows: src must be [n_rays, ...] of 32-bit words")
    if not src.is_cuda or not src.is_contiguous():
        raise ValueError("compact_rows: src must be a contiguous GPU tensor")
    width = max(1, src[0].numel()) if n else 1
    dst = torch.empty((n_alive,) + tuple(src.shape[1:]), dtype=src.dtype, device=src.device)
    check(load().txs_compact_rows(n, _ptr(table), width, _ptr(src), _ptr(dst), _stream()),
          "txs_compact_rows")
    return dst


def expand_rows(table, src, fill=0.0):
    """Compacted rows src [n_alive, ...] back to every ray, `fill` where a ray missed."""
    n = table.shape[0]
    _need(table, "table", torch.int32, (n, 2))
    _need(src, "src", torch.float32)
    width = 1
    for s in src.shape[1:]:
        width *= s
    dst = torch.empty((n,) + tuple(src.shape[1:]), dtype=torch.float32, device=table.device)
    check(load().txs_expand_rows(n, _ptr(table), width, _ptr(src) if src.numel() else None,
                                 float(fill), _ptr(dst), _stream()), "txs_expand_rows")
    return dst


def span_bins(span, n_bins):
    """n_bins+1 equally spaced edges over each span [N, 2] -> [N, n_bins+1]."""
    n = span.shape[0]
    _need(span, "span", torch.float32, (n, 2))
    out = torch.empty((n, n_bins + 1), dtype=torch.float32, device=span.device)
    check(load().txs_span_bins(n, _ptr(span), n_bins, _ptr(out), _stream()), "txs_span_bins")
    return out


def merge_edges(a, b):
    """Sorted union of two ascending edge rows per ray: [N, na] + [N, nb] -> [N, na+nb]."""
    n = a.shape[0]
    _need(a, "a", torch.float32, (n, a.shape[1]))
    _need(b, "b", torch.float32, (n, b.shape[1]))
    out = torch.empty((n, a.shape[1] + b.shape[1]), dtype=torch.float32, device=a.device)
    check(load().txs_merge_edges(n, a.shape[1], _ptr(a), b.shape[1], _ptr(b), _ptr(out),
                                 _stream()), "txs_merge_edges")
    return out
