"""MI355X-native fast spin spherical-harmonic transform (McEwen, arXiv:0807.4494).

The transform runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/sht.h`` (``libsht.so``); this package is its thin Python binding.
"""

from .sht import (PRECISIONS, Graph, error_metrics, forward, forward_lstsq, forward_real,
                  forward_triangular, forward_multi, inverse, inverse_multi, inverse_noalloc,
                  inverse_real, io_dtype, plan_tables, plan_warmup,
                  real_dtype, release_all, spin_pair, tile_set, trace_enable, trace_read, tune,
                  version, workspace_bytes)

__all__ = ["PRECISIONS", "Graph", "error_metrics", "forward", "forward_lstsq", "forward_real",
           "forward_triangular", "forward_multi", "inverse", "inverse_multi", "inverse_noalloc",
           "inverse_real", "io_dtype", "plan_tables", "plan_warmup",
           "real_dtype", "release_all", "spin_pair", "tile_set", "trace_enable", "trace_read", "tune",
           "version", "workspace_bytes"]
