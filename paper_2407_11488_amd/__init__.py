"""Auto-tuned FP32 direct 2D convolution (and hotspot thermal stencil) for
MI355X (gfx950).

``out[y][x] = sum_{i,j} in[y+i][x+j] * f[i][j]`` (valid cross-correlation),
hand-written HIP behind a C ABI (``include/conv2d.h``); this package is the
thin binding. PyTorch is used only for device memory and streams.

    import torch, paper_2407_11488_amd as C
    plan = C.Plan(4096, 4096, 17, 17)            # tuned winner if cached
    out = plan(inp_cuda, filt_cuda)               # enqueued on the current stream
"""
from __future__ import annotations

from ._binding import (CONV2D_EBUSY, CONV2D_ECOMPILE, CONV2D_EHIP, CONV2D_EINVAL, CONV2D_ELAUNCH,  # noqa: F401
                       CONV2D_ENOMEM, CONV2D_ENOTUNED, CONV2D_EVERIFY, CONV2D_OK, LIB_PATH, Config,
                       Conv2dError, Shape, TuneOpts, TuneResult, config, conv2d_cache_lookup,
                       conv2d_benchmark, conv2d_cache_store, conv2d_compile, conv2d_config_check, conv2d_default_config,
                       conv2d_destroy, conv2d_fill_uniform, conv2d_geometry, conv2d_kernel_hash, conv2d_last_error,
                       conv2d_lds_bytes, conv2d_plan, conv2d_plan_config, conv2d_reference, conv2d_run,
                       conv2d_space, conv2d_tune, conv2d_tune_defaults, conv2d_tune_synthetic,
                       conv2d_version, lib, shape)
from ._binding import (CONV2D_BATCH_BY_SIZE, CONV2D_BATCH_NO_GRAPH, CONV2D_BATCH_NO_PTR_CHECK, conv2d_batch_destroy,  # noqa: F401
                       conv2d_batch_info, conv2d_batch_plan, conv2d_batch_run, conv2d_batch_tune,
                       conv2d_batch_tune_defaults, conv2d_compile_batch, conv2d_size_bucket, conv2d_warm_cache)
from ._binding import (REQUEST_DTYPE, ServeOpts, ServeReport, conv2d_serve, conv2d_serve_defaults,  # noqa: F401
                       conv2d_serve_free, requests_array)
from ._binding import (HotspotCoeffs, HotspotConfig, HotspotShape, HotspotTuneOpts,  # noqa: F401
                       HotspotTuneResult, hotspot_coeffs, hotspot_compile, hotspot_config,
                       hotspot_config_check, hotspot_default_config, hotspot_destroy, hotspot_lds_bytes,
                       hotspot_plan, hotspot_plan_config, hotspot_reference, hotspot_run, hotspot_shape,
                       hotspot_kernel_hash, hotspot_space, hotspot_tune, hotspot_tune_defaults)
from .api import Batch, Hotspot, Plan, conv2d, reference, reference_hotspot  # noqa: F401
