"""MI355X (gfx950) transmittance-estimator sampling and packed volume rendering.

The compute runs in libtxs.so (hand-written HIP kernels behind the C ABI of
include/txs.h); this package only marshals torch tensors into that ABI.
Importing it does not touch the GPU; `load()` raises if the library is absent.
"""
from ._lib import (TXS_EHIP, TXS_EINVAL, TXS_ECAPACITY, TXS_EOVERFLOW, TXS_OK,
                   TXS_PDF_SIGMA, TXS_PDF_SIGMA_EXP, TXS_PDF_WEIGHTS, LIB_PATH, TxsError,
                   exported_symbols, load)
from .ops import (GridSpec, MlpSpec, adam_step, blob_field, compact_rows, disparity_bins,
                  edges_to_intervals,
                  exclusive_scan, exclusive_scan_noalloc, exclusive_scan_noalloc_max_rays,
                  expand_rows, gather_prefix, grid_ema, grid_points,
                  grid_points_contracted, hist_loss,
                  march_count, march_count_contracted, march_fill, march_fill_contracted,
                  march_span, merge_edges, mlp_param_count, prop_mlp_bwd,
                  prop_mlp_fwd, render_bwd, render_fwd, resample, resample_intervals,
                  read_probe, span_bins, stream_probe, transmittance_prefix, uniform_bins,
                  weights_bwd)
from .pipeline import (OccupancyGrid, Packed, RenderFn, filter_transmittance, march,
                       march_contracted, pdf_render, rendering, rendering_dense, sampling)

__all__ = [n for n in dir() if not n.startswith("_")]
