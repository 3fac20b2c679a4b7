"""Helpers shared by the GPU parity tests: device transfer, tolerance metrics."""
import numpy as np
import torch


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    return t.detach().cpu().numpy()


def grid_spec(txs, bits, res, n_levels=1, half_extent0=1.5):
    return txs.GridSpec(dev(np.asarray(bits, np.uint32)), res, n_levels, (0.0, 0.0, 0.0),
                        half_extent0)


FLT_MIN = float(np.finfo(np.float32).tiny)  # 2^-126: binary32 has no relative precision below


def assert_close(x, ref, *, rel=1e-5, floor_scale=None, name=""):
    """|x - ref| <= rel |ref| + rel * s + FLT_MIN, s = 1e-3 max|ref| unless given."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    assert x.shape == ref.shape, (name, x.shape, ref.shape)
    if ref.size == 0:
        return
    s = 1e-3 * np.max(np.abs(ref)) if floor_scale is None else floor_scale
    err = np.abs(x - ref)
    tol = rel * np.abs(ref) + rel * s + FLT_MIN
    bad = ~(err <= tol)
    if bad.any():
        i = np.flatnonzero(bad.reshape(-1))[:5]
        raise AssertionError(
            f"{name}: {bad.sum()} / {bad.size} outside tolerance; worst rel "
            f"{np.max(err / (np.abs(ref) + 1e-300)):.3e}; first idx {i.tolist()} "
            f"x={x.reshape(-1)[i].tolist()} ref={ref.reshape(-1)[i].tolist()}")
    l2 = np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300)
    return float(l2)


def segment_ids(packed_info):
    info = np.asarray(packed_info)
    return np.repeat(np.arange(info.shape[0]), info[:, 1])


def bwd_condition(packed_info, t0, t1, sigma, v):
    """Per-sample scale Delta_k (T_{k+1} vb_k + sum_{j>k} w_j vb_j) of the adjoint (FP64).

    vb is the magnitude of the terms that make up v = dL/dw (pass it already
    made non-negative): the adjoint subtracts those terms, so binary32 carries
    an error relative to this scale, not to the cancelled result.
    """
    info = np.asarray(packed_info)
    seg = segment_ids(info)
    delta = np.asarray(t1, np.float64) - np.asarray(t0, np.float64)
    tau = np.asarray(sigma, np.float64) * delta
    starts = info[:, 0].astype(np.int64)
    S = tau.shape[0]
    if S == 0:
        return np.zeros(0)
    # samples are contiguous per ray here (starts = cumsum of counts)
    c = np.cumsum(tau)
    base = np.concatenate([[0.0], c])[starts][seg]
    P_incl = c - base
    T_next = np.exp(-P_incl)
    w = np.exp(-(P_incl - tau)) * -np.expm1(-tau)
    a = w * np.abs(v)
    ca = np.cumsum(a)
    ends = starts + info[:, 1]
    tot = np.concatenate([[0.0], ca])[ends][seg]
    suffix = tot - ca
    return delta * (T_next * np.abs(v) + np.maximum(suffix, 0.0))


def resample_tol(edges, vals, mode, out_ref, bins_ref):
    """Inverse-CDF conditioning: a CDF error eps moves t by eps/(F_{i+1}-F_i) of the bin."""
    e = edges.astype(np.float64)
    v = vals.astype(np.float64)
    if mode == 0:
        F = -np.expm1(-np.cumsum(v * np.diff(e, axis=1), axis=1))
    else:
        F = np.cumsum(v, axis=1)
    F = np.concatenate([np.zeros((F.shape[0], 1)), F], 1)
    Fn = F[:, -1:]
    uni = Fn[:, 0] <= 1e-12
    F[uni] = np.linspace(0, 1, F.shape[1])
    Fn = F[:, -1:]
    i = np.minimum(bins_ref, e.shape[1] - 2)
    dF = np.take_along_axis(F, i + 1, 1) - np.take_along_axis(F, i, 1)
    width = np.take_along_axis(e, i + 1, 1) - np.take_along_axis(e, i, 1)
    span = e[:, -1:] - e[:, :1]
    return (1e-5 * np.abs(out_ref) + 1e-6 * span
            + width * np.minimum(1.0, 4e-6 * Fn / np.maximum(dF, 1e-300)))
