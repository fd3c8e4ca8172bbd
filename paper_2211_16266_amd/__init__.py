"""MI355X (gfx950) equirectangular PatchMatch-Stereo densification.

Surmann, Thurow, Slomma, "PatchMatch-Stereo-Panorama, a fast dense
reconstruction from 360 degree video images", Sec. III: a keyframe is
densified against its neighbouring keyframes with slanted-plane PatchMatch
on equirectangular images (random initialisation, red-black propagation,
random refinement) and filtered by geometric consistency.

The work runs in the HIP kernels of ``libpms.so`` behind the C ABI of
``include/pms.h``; this package only marshals torch device tensors to it.
"""
import torch  # noqa: F401  (load torch's HIP runtime before libpms)

from ._binding import (LIB_PATH, coverage, fuse, MAX_BATCH, MAX_MAPS, MAX_VIEWS, Batch, Context,  # noqa: F401
                       JobDesc, PmsError, Server, consistency, default_context, default_params, densify,
                       densify_batch, densify_job, densify_noalloc, eval_cost, halfsweep, job, lib,
                       philox_stream, view_filter, warp_planes)
