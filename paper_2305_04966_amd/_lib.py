"""ctypes loader of libtxs.so: declares every entry point of include/*.h."""
from __future__ import annotations

import ctypes as C
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtxs.so")

TXS_OK, TXS_EINVAL, TXS_ECAPACITY, TXS_EHIP, TXS_EOVERFLOW = 0, -1, -2, -3, -4
TXS_PDF_SIGMA, TXS_PDF_WEIGHTS, TXS_PDF_SIGMA_EXP = 0, 1, 2

_STATUS = {TXS_EINVAL: "EINVAL", TXS_ECAPACITY: "ECAPACITY", TXS_EHIP: "EHIP",
           TXS_EOVERFLOW: "EOVERFLOW"}


class TxsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"txs {_STATUS.get(status, status)}: {message}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("bits", C.c_void_p), ("res", C.c_int32), ("n_levels", C.c_int32),
                ("center", C.c_float * 3), ("half_extent0", C.c_float),
                ("coarse", C.c_void_p)]


class MarchParams(C.Structure):
    _fields_ = [("near_plane", C.c_float), ("far_plane", C.c_float), ("dt0", C.c_float),
                ("max_per_ray", C.c_int32)]


class Mlp(C.Structure):
    _fields_ = [("packed", C.c_void_p), ("params", C.c_void_p), ("hidden", C.c_int32),
                ("scale", C.c_float), ("contract", C.c_int32)]


P, I32, I64, F32, SZ = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_size_t
GP, MP, MLP = C.POINTER(Grid), C.POINTER(MarchParams), C.POINTER(Mlp)

SIGNATURES = {
    "txs_last_error": (C.c_char_p, []),
    "txs_abi_version": (I32, []),
    "txs_grid_coarse_words": (I64, [I32]),
    "txs_grid_coarsen": (I32, [GP, P, P]),
    "txs_march_count": (I32, [GP, MP, P, P, I32, P, P]),
    "txs_scan_workspace_size": (SZ, [I32]),
    "txs_exclusive_scan": (I32, [P, I32, P, P, P, SZ, P]),
    "txs_exclusive_scan_noalloc_max_rays": (I32, []),
    "txs_exclusive_scan_noalloc": (I32, [P, I32, P, P, P]),
    "txs_march_fill": (I32, [GP, MP, P, P, I32, P, I64, P, P, P, P]),
    "txs_transmittance_prefix": (I32, [P, I32, I64, P, P, P, F32, P, P]),
    "txs_gather_prefix": (I32, [P, P, I32, I64, P, P, I64, P, P, P, P]),
    "txs_render_fwd": (I32, [P, I32, I32, I64, P, P, P, P, P, P, P, P, P, P, P]),
    "txs_render_bwd": (I32, [P, I32, I32, I64, P, P, P, P, P, P, P, P, P, P, P, P]),
    "txs_weights_bwd": (I32, [P, I32, I32, I64, P, P, P, P, P, P, P]),
    "txs_resample": (I32, [I32, I32, P, P, I32, I32, P, P, P]),
    "txs_resample_intervals": (I32, [I32, I32, P, P, I32, I32, P, P, P, P]),
    "txs_uniform_bins": (I32, [GP, F32, F32, P, P, I32, I32, P, P]),
    "txs_edges_to_intervals": (I32, [P, I32, I32, P, P, P]),
    "txs_blob_field": (I32, [P, I32, P, P, I32, P, P, P, I32, I64, P, P, P]),
    "txs_mlp_param_count": (SZ, [I32]),
    "txs_mlp_packed_bytes": (SZ, [I32]),
    "txs_mlp_pack": (I32, [P, I32, P, P]),
    "txs_prop_mlp_fwd": (I32, [MLP, P, P, I32, I32, P, P, P]),
    "txs_mlp_bwd_workspace_size": (SZ, [I32]),
    "txs_prop_mlp_bwd": (I32, [MLP, P, P, I32, I32, P, P, P, P, SZ, P]),
    "txs_hist_loss": (I32, [P, I32, I64, P, P, P, I32, P, P, F32, P, P, P]),
    "txs_adam_step": (I32, [P, P, P, P, I64, F32, F32, F32, F32, I32, P]),
    "txs_stream_probe": (I32, [I64, P, P, P, P, P, P, P]),
    "txs_read_probe_out_size": (I64, []),
    "txs_read_probe": (I32, [I64, P, P, P, P, P, P]),
    "txs_grid_points": (I32, [GP, P, P, P]),
    "txs_grid_ema": (I32, [I64, P, P, F32, F32, P, P]),
    "txs_march_span": (I32, [GP, MP, P, P, I32, P, P, P]),
    "txs_compact_rows": (I32, [I32, P, I32, P, P, P]),
    "txs_expand_rows": (I32, [I32, P, I32, P, F32, P, P]),
    "txs_span_bins": (I32, [I32, P, I32, P, P]),
    "txs_merge_edges": (I32, [I32, I32, P, I32, P, P, P]),
    "txs_disparity_bins": (I32, [GP, F32, F32, P, P, I32, I32, P, P]),
    "txs_march_count_contracted": (I32, [GP, MP, F32, P, P, I32, P, P]),
    "txs_march_fill_contracted": (I32, [GP, MP, F32, P, P, I32, P, I64, P, P, P, P]),
    "txs_grid_points_contracted": (I32, [GP, F32, P, P, P]),
}

_lock = threading.Lock()
_lib = None


def load():
    """Loads libtxs.so from the package directory; raises if it was not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with "
                    "`python -m paper_2305_04966_amd.build` (hipcc, gfx950)")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def exported_symbols():
    return list(SIGNATURES)


def check(status: int, name: str):
    if status != TXS_OK:
        msg = load().txs_last_error()
        raise TxsError(status, f"{name}: {msg.decode() if msg else ''}")
