"""MI355X-native union-find connected-components labeling (three phases:
tile-local merge, boundary analysis on tile-edge cells, link).

The arithmetic runs in hand-written HIP kernels for gfx950 inside
``libccl.so``; this package only marshals arguments to its C ABI.  The
library is loaded on first use; a missing or unbuilt library raises
``RuntimeError`` -- there is no CPU fallback.
"""
from .binding import (  # noqa: F401
    BatchContext,
    CclError,
    autotune,
    label,
    label_batch,
    component_stats,
    label_equal,
    label3d,
    label_plain,
    library_path,
    load_library,
    tuning_clear,
    tuning_get,
    tuning_load,
    tuning_save,
)
