"""FP64 CPU oracle of the sampling / rendering path -- TEST INFRASTRUCTURE.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2305_04966_amd``) and imports nothing from it; both sides receive the
same seeded inputs from the ``scenes`` module.

The numerical work lives in ``txs_oracle.c`` (plain C loops, binary32 for the
geometric decisions, binary64 for everything continuous).  This module only
builds it with gcc and marshals numpy arrays.  The proposal-MLP, histogram
loss and optimiser references live in ``oracle.learned``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "txs_oracle.c"), os.path.join(_HERE, "learned.c")]
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
          "-std=c11", "-Wall"]


def build(force: bool = True) -> str:
    """Compile txs_oracle.c into liboracle.so next to it (gcc)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or (os.path.getmtime(_LIB_PATH)
                                                 < max(map(os.path.getmtime, _SRCS))):
                build(force=True)
            _lib = C.CDLL(_LIB_PATH)
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def num_threads() -> int:
    L = lib()
    L.oracle_num_threads.restype = C.c_int32
    return int(L.oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's loops over rays (timing only; results do not
    depend on it)."""
    lib().oracle_set_num_threads(C.c_int32(int(n)))


# ----------------------------------------------------------------------------
def clip(o, d, bmin, bmax, near=0.0, far=float("inf")):
    """Slab clip in the binary32 recipe -> (t_near, t_far) float32 arrays."""
    o, d = _f32(o), _f32(d)
    n = o.shape[0]
    tn = np.empty(n, np.float32)
    tf = np.empty(n, np.float32)
    lib().oracle_clip(C.c_int32(n), _p(o), _p(d), _p(_f32(bmin)), _p(_f32(bmax)),
                      C.c_float(near), C.c_float(far), _p(tn), _p(tf))
    return tn, tf


def march(o, d, bits, res, *, n_levels=1, center=(0.0, 0.0, 0.0), half_extent0=1.5,
          near=0.0, far=float("inf"), dt0=0.005, max_per_ray=0, want_level=False,
          contract_scale=0.0):
    """Dense-definition occupancy march.  contract_scale > 0: the occupancy of
    every sample comes from one res^3 grid over contracted space (the lattice
    is still that of the n_levels cubes).

    Returns dict(packed_info [N,2] int32, t0, t1 float32 [S], ray_id int32 [S],
    counts [N], total, level (optional)).
    """
    o, d = _f32(o), _f32(d)
    bits = np.ascontiguousarray(bits, dtype=np.uint32)
    n = o.shape[0]
    assert bits.size * 32 >= (1 if contract_scale > 0 else n_levels) * res ** 3
    cen = _f32(center)
    args_head = (C.c_int32(n), _p(o), _p(d), _p(bits), C.c_int32(res), C.c_int32(n_levels),
                 _p(cen), C.c_float(half_extent0), C.c_float(near), C.c_float(far),
                 C.c_float(dt0), C.c_int32(max_per_ray), C.c_float(contract_scale))
    counts = np.zeros(n, np.int32)
    L = lib()
    L.oracle_march(*args_head, _p(counts), None, None, None, None, None)
    offsets = np.zeros(n, np.int64)
    if n:
        offsets[1:] = np.cumsum(counts.astype(np.int64))[:-1]
    total = int(counts.astype(np.int64).sum())
    t0 = np.empty(total, np.float32)
    t1 = np.empty(total, np.float32)
    rid = np.empty(total, np.int32)
    lvl = np.empty(total, np.int32) if want_level else None
    counts2 = np.zeros(n, np.int32)
    L.oracle_march(*args_head, _p(counts2), _p(offsets), _p(t0), _p(t1), _p(rid), _p(lvl))
    assert np.array_equal(counts, counts2)
    info = np.stack([offsets.astype(np.int32), counts], axis=1)
    out = dict(packed_info=np.ascontiguousarray(info), t0=t0, t1=t1, ray_id=rid,
               counts=counts, total=total)
    if want_level:
        out["level"] = lvl
    return out


def render_fwd(packed_info, t0, t1, sigma, rgb, bg=None, want_weights=False):
    """FP64 compositing of packed samples -> dict(rgb [N,3], opacity, depth, weights)."""
    info = _i32(packed_info)
    n = info.shape[0]
    t0, t1, sigma, rgb = _f32(t0), _f32(t1), _f32(sigma), _f32(rgb)
    bg = None if bg is None else _f32(bg)
    out_rgb = np.zeros((n, 3), np.float64)
    out_op = np.zeros(n, np.float64)
    out_dep = np.zeros(n, np.float64)
    w = np.zeros(t0.shape[0], np.float64) if want_weights else None
    lib().oracle_render_fwd(C.c_int32(n), _p(info), _p(t0), _p(t1), _p(sigma), _p(rgb), _p(bg),
                            _p(out_rgb), _p(out_op), _p(out_dep), _p(w))
    return dict(rgb=out_rgb, opacity=out_op, depth=out_dep, weights=w)


def render_bwd(packed_info, t0, t1, sigma, rgb, g_rgb, g_opacity=None, g_depth=None, bg=None):
    """FP64 adjoint -> (d_sigma [S], d_rgb [S,3])."""
    info = _i32(packed_info)
    n = info.shape[0]
    t0, t1, sigma, rgb = _f32(t0), _f32(t1), _f32(sigma), _f32(rgb)
    g_rgb = _f32(g_rgb)
    g_opacity = None if g_opacity is None else _f32(g_opacity)
    g_depth = None if g_depth is None else _f32(g_depth)
    bg = None if bg is None else _f32(bg)
    ds = np.zeros(t0.shape[0], np.float64)
    dr = np.zeros((t0.shape[0], 3), np.float64)
    lib().oracle_render_bwd(C.c_int32(n), _p(info), _p(t0), _p(t1), _p(sigma), _p(rgb), _p(bg),
                            _p(g_rgb), _p(g_opacity), _p(g_depth), _p(ds), _p(dr))
    return ds, dr


def weights_bwd(packed_info, t0, t1, sigma, g_w):
    info = _i32(packed_info)
    t0, t1, sigma, g_w = _f32(t0), _f32(t1), _f32(sigma), _f32(g_w)
    ds = np.zeros(t0.shape[0], np.float64)
    lib().oracle_weights_bwd(C.c_int32(info.shape[0]), _p(info), _p(t0), _p(t1), _p(sigma),
                             _p(g_w), _p(ds))
    return ds


def transmittance_prefix(packed_info, t0, t1, sigma, t_min=1e-4):
    """kept[r] = #samples with T_i >= t_min; band[r] flags near-threshold rays."""
    info = _i32(packed_info)
    n = info.shape[0]
    kept = np.zeros(n, np.int32)
    band = np.zeros(n, np.int32)
    lib().oracle_transmittance_prefix(C.c_int32(n), _p(info), _p(_f32(t0)), _p(_f32(t1)),
                                      _p(_f32(sigma)), C.c_double(t_min), _p(kept), _p(band))
    return kept, band.astype(bool)


def gather_prefix(packed_info, kept, t0, t1, ray_id):
    """Repack the first kept[r] samples of each ray -> (packed_info_out, t0, t1, ray_id)."""
    info = _i32(packed_info)
    kept = _i32(kept)
    n = info.shape[0]
    starts = np.zeros(n, np.int64)
    if n:
        starts[1:] = np.cumsum(kept.astype(np.int64))[:-1]
    total = int(kept.astype(np.int64).sum())
    idx = (np.repeat(info[:, 0].astype(np.int64) - starts, kept)
           + np.arange(total, dtype=np.int64))
    info_out = np.stack([starts.astype(np.int32), kept], axis=1)
    return np.ascontiguousarray(info_out), t0[idx], t1[idx], ray_id[idx]


INT32_MAX = 2 ** 31 - 1


def exclusive_scan(counts):
    """Packed table of per-ray counts (Section 4.2, "Packed Tensor"): row r =
    (sum of the counts before r, count r); returns (table int32 [N, 2], the
    exact total).  Starts are int32, so a row that does not end by INT32_MAX
    cannot be addressed and is the empty row (INT32_MAX, 0)."""
    counts = np.asarray(counts, np.int64)
    total = int(counts.sum())
    starts = np.zeros_like(counts)
    if counts.size:
        starts[1:] = np.cumsum(counts)[:-1]
    fits = starts + counts <= INT32_MAX
    info = np.stack([np.where(fits, starts, INT32_MAX), np.where(fits, counts, 0)],
                    axis=1).astype(np.int32)
    return info, total


MODE_SIGMA, MODE_WEIGHTS, MODE_SIGMA_EXP = 0, 1, 2


def resample(edges, vals, n_out, mode=MODE_SIGMA, u=None):
    """Inverse-CDF resampling -> (edges_out float64 [N,n_out+1], bin int32, band bool [N])."""
    edges, vals = _f32(edges), _f32(vals)
    n, nb = vals.shape
    assert edges.shape == (n, nb + 1)
    out = np.zeros((n, n_out + 1), np.float64)
    bins = np.zeros((n, n_out + 1), np.int32)
    band = np.zeros(n, np.int32)
    uu = None if u is None else _f32(u)
    lib().oracle_resample(C.c_int32(n), C.c_int32(nb), _p(edges), _p(vals), C.c_int32(mode),
                          C.c_int32(n_out), _p(uu), _p(out), _p(bins), _p(band))
    return out, bins, band.astype(bool)


def field(x, params):
    """FP64 analytic field at points x [n,3] -> (sigma [n], rgb [n,3])."""
    x = _f64(x).reshape(-1, 3)
    p = _f64(params)
    n = x.shape[0]
    s = np.zeros(n, np.float64)
    c = np.zeros((n, 3), np.float64)
    lib().oracle_field(C.c_int64(n), _p(x), _p(p), _p(s), _p(c))
    return s, c


def field_at_samples(o, d, t0, t1, ray_id, params):
    """Field at interval midpoints x = o + (t0+t1)/2 d (FP64)."""
    o = np.asarray(o, np.float64)
    d = np.asarray(d, np.float64)
    tm = 0.5 * (np.asarray(t0, np.float64) + np.asarray(t1, np.float64))
    rid = np.asarray(ray_id, np.int64)
    x = o[rid] + tm[:, None] * d[rid]
    return field(x, params)


# ----------------------------------------------------------------------------
# learned estimator (learned.c)
# ----------------------------------------------------------------------------
def mlp_param_count(H: int) -> int:
    """W1 [H,39], b1 [H], W2 [H,H], b2 [H], w3 [H], b3."""
    return H * H + 42 * H + 1


def bin_midpoints(o, d, edges):
    """FP64 points x = o + (e_j + e_{j+1})/2 d for dense bins -> [N*n_bins, 3]."""
    e = np.asarray(edges, np.float64)
    tm = 0.5 * (e[:, :-1] + e[:, 1:])
    x = np.asarray(o, np.float64)[:, None, :] + tm[..., None] * np.asarray(d, np.float64)[:, None, :]
    return x.reshape(-1, 3)


def mlp_fwd(x, params, H, scale=1.5, contract=False, emulate_bf16=False, want_z=False):
    """Proposal MLP at points x [n,3] -> sigma [n] (FP64 or bf16-emulated)."""
    x = _f64(x).reshape(-1, 3)
    p = _f32(params)
    assert p.size == mlp_param_count(H)
    n = x.shape[0]
    s = np.zeros(n, np.float64)
    z = np.zeros(n, np.float64) if want_z else None
    lib().oracle_mlp_fwd(C.c_int64(n), _p(x), _p(p), C.c_int32(H), C.c_double(scale),
                         C.c_int32(int(contract)), C.c_int32(int(emulate_bf16)), _p(s), _p(z))
    return (s, z) if want_z else s


def mlp_bwd(x, params, H, d_sigma, scale=1.5, contract=False, emulate_bf16=False,
            want_abs=False):
    """Gradient of sum_i d_sigma_i sigma(x_i) w.r.t. the parameter vector (FP64).

    With want_abs, returns (grad, grad_abs): grad_abs sums |term| instead of term.
    """
    x = _f64(x).reshape(-1, 3)
    p = _f32(params)
    g = np.zeros(mlp_param_count(H), np.float64)
    ga = np.zeros_like(g) if want_abs else None
    lib().oracle_mlp_bwd(C.c_int64(x.shape[0]), _p(x), _p(p), C.c_int32(H), C.c_double(scale),
                         C.c_int32(int(contract)), C.c_int32(int(emulate_bf16)),
                         _p(_f64(d_sigma)), _p(g), _p(ga))
    return (g, ga) if want_abs else g


def hist_loss(packed_info, t0, t1, w, edges, wp, eps=1e-7, want_grad=True):
    """Per-ray proposal loss and d(mean loss)/d(proposal weights)."""
    info = _i32(packed_info)
    n = info.shape[0]
    edges, wp = _f32(edges), _f32(wp)
    nb = wp.shape[1]
    loss = np.zeros(n, np.float64)
    d = np.zeros((n, nb), np.float64) if want_grad else None
    lib().oracle_hist_loss(C.c_int32(n), _p(info), _p(_f32(t0)), _p(_f32(t1)), _p(_f32(w)),
                           C.c_int32(nb), _p(edges), _p(wp), C.c_double(eps), _p(loss), _p(d))
    return loss, d


def adam(p, m, v, g, lr, b1=0.9, b2=0.99, eps=1e-15, step=1):
    """One Adam step in FP64, in place on copies -> (p, m, v)."""
    p, m, v = _f64(p).copy(), _f64(m).copy(), _f64(v).copy()
    lib().oracle_adam(C.c_int64(p.size), _p(p), _p(m), _p(v), _p(_f64(g)), C.c_double(lr),
                      C.c_double(b1), C.c_double(b2), C.c_double(eps), C.c_int32(step))
    return p, m, v


def grid_points(res, n_levels=1, center=(0.0, 0.0, 0.0), half_extent0=1.5, u=None):
    """One point per cell, level-major, cell index x + res (y + res z) -> [L res^3, 3]."""
    n = n_levels * res ** 3
    out = np.zeros((n, 3), np.float64)
    lib().oracle_grid_points(C.c_int32(res), C.c_int32(n_levels), _p(_f32(center)),
                             C.c_double(half_extent0), _p(None if u is None else _f32(u)),
                             _p(out))
    return out


def grid_points_contracted(res, contract_scale, center=(0.0, 0.0, 0.0), u=None):
    """One point per cell of a grid over contracted space -> [res^3, 3] (binary64)."""
    out = np.zeros((res ** 3, 3), np.float64)
    lib().oracle_grid_points_contracted(C.c_int32(res), _p(_f32(center)),
                                        C.c_double(contract_scale),
                                        _p(None if u is None else _f32(u)), _p(out))
    return out


def grid_ema(density, sigma, gamma, tau):
    """D <- gamma D + (1 - gamma) sigma; occupied = D > tau -> (D, occupied bool)."""
    d = _f64(density).copy()
    occ = np.zeros(d.shape[0], np.uint8)
    lib().oracle_grid_ema(C.c_int64(d.shape[0]), _p(d), _p(_f64(sigma)), C.c_double(gamma),
                          C.c_double(tau), _p(occ))
    return d, occ.astype(bool)


def grid_bricks(bits, res, n_levels=1):
    """Brick occupancy of a grid (the spatial-skipping estimator's coarse level,
    Section 3.1): bricks of 8^3 cells, per level (plain [b^3], block [b^3]) with
    b = res/8, brick (bx, by, bz) at index bx + b (by + b bz); plain = some cell
    of the brick occupied, block = some cell of the bricks (bx..bx+1, by..by+1,
    bz..bz+1) occupied (clipped at the far faces).  -> bool [n_levels, 2, b^3]."""
    b = res // 8
    words = np.asarray(bits, np.uint32).reshape(-1)
    occ = ((words[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(bool).reshape(-1)
    out = np.zeros((n_levels, 2, b ** 3), bool)
    for l in range(n_levels):
        cells = occ[l * res ** 3:(l + 1) * res ** 3].reshape(res, res, res)  # [z, y, x]
        plain = np.zeros((b, b, b), bool)
        for bz in range(b):
            for by in range(b):
                for bx in range(b):
                    plain[bz, by, bx] = cells[8 * bz:8 * bz + 8, 8 * by:8 * by + 8,
                                              8 * bx:8 * bx + 8].any()
        block = np.zeros_like(plain)
        for bz in range(b):
            for by in range(b):
                for bx in range(b):
                    block[bz, by, bx] = plain[bz:bz + 2, by:by + 2, bx:bx + 2].any()
        out[l, 0] = plain.reshape(-1)
        out[l, 1] = block.reshape(-1)
    return out


def march_span(o, d, bits, res, **march_kw):
    """Occupied span of every ray (Section 4.4, "Combined Sampling": the grid
    shrinks each ray's near-far interval to where it found occupied space):
    (t0 of the first sample, t1 of the last) of the dense march, (0, 0) for a
    ray with none -> (span float32 [N, 2], hit int32 [N])."""
    m = march(o, d, bits, res, **march_kw)
    start, cnt = m["packed_info"][:, 0].astype(np.int64), m["counts"].astype(np.int64)
    hit = cnt > 0
    span = np.zeros((cnt.shape[0], 2), np.float32)
    span[hit, 0] = m["t0"][start[hit]]
    span[hit, 1] = m["t1"][start[hit] + cnt[hit] - 1]
    return span, hit.astype(np.int32)


def span_bins(span, n_bins):
    """n_bins+1 equally spaced edges over each span, in binary64 -> [N, n_bins+1]."""
    s = _f64(span)
    k = np.arange(n_bins + 1, dtype=np.float64) / n_bins
    return s[:, :1] + (s[:, 1:2] - s[:, :1]) * k


def merge_edges(a, b):
    """Sorted union of two edge rows per ray (the fine pass of the coarse-to-fine
    PDF estimator renders coarse and fine edges together) -> [N, na+nb]."""
    return np.sort(np.concatenate([_f32(a), _f32(b)], axis=1), axis=1, kind="stable")


def disparity_bins(o, d, bmin, bmax, n_bins, near, far=float("inf")):
    """Chord bins of equal width in 1/t (binary64 from the binary32 clip);
    a ray that misses gets all edges at `near` -> [N, n_bins+1]."""
    tn, tf = clip(o, d, bmin, bmax, near, far)
    hit = tn < tf
    lo = np.where(hit, tn, near).astype(np.float64)
    hi = np.where(hit, tf, near).astype(np.float64)
    k = np.arange(n_bins + 1, dtype=np.float64) / n_bins
    return 1.0 / (1.0 / lo[:, None] + (1.0 / hi[:, None] - 1.0 / lo[:, None]) * k)
