"""MI355X (gfx950) implementation of one optimizer iteration of 3DGS^2-TR.

The compute path is the HIP library ``libgs3tr.so`` (C ABI in
``include/gs3tr.h``); this package only marshals arguments to it.  Importing
the package does not load the library; ``Scene`` does, and fails loudly if it
has not been built.
"""
from .api import (ADAM_GROUP_ORDER, Scene, n_params, profile_enable, profile_read,  # noqa: F401
                  profile_reset, scene_bytes)
