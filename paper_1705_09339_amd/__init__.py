"""MI355X (gfx950) Cascade-of-Gaussians background subtractor.

The method runs in the HIP library ``libcog.so`` (C ABI in include/cog.h);
``paper_1705_09339_amd.cog`` is its ctypes binding.  Importing the package
fails if the library has not been built.
"""
from . import cog  # noqa: F401
from .cog import (  # noqa: F401
    CogError, CogStream, cog_params, cog_step_info,
    cog_default_params, cog_state_bytes, cog_canonical_bytes, cog_create, cog_train_prior,
    cog_step, cog_step_frames, cog_reset, cog_destroy, cog_export_state, cog_import_state,
    cog_kde_weights, cog_last_error,
    COG_U8, COG_F32, COG_STAGE_FD, COG_STAGE_RGA, COG_STAGE_KDE, COG_STAGE_ALL,
    COG_PATH_CASCADE, COG_PATH_GMM,
)
