"""MI355X (gfx950) implementation of one optimizer iteration of 3DGS^2-TR.

The compute path is the HIP library ``libgs3tr.so`` (C ABI in
``include/gs3tr.h``); this package only marshals arguments to it.  Importing
the package does not load the library; ``Scene`` does, and fails loudly if it
has not been built.
"""
from .api import (ADAM_GROUP_ORDER, TR_MEAN_EXACT, TR_SECOND_ORDER, TR_SH_JOINT, Scene,  # noqa: F401
                  n_params, profile_count, profile_enable, profile_read, profile_reset, scene_bytes)
