"""MI355X-native device-memory checkpoint drain/refill (libckpt).

The C ABI is include/ckpt.h; `ckpt` is its Python binding.  Build the HIP
library with `python -m paper_2008_10596_amd.build`.
"""
from . import ckpt  # noqa: F401
from .ckpt import (Context, Image, CkptError, checkpoint_batch,  # noqa: F401
                   CKPT_DEVICE, CKPT_MANAGED, CKPT_FULL, CKPT_INCREMENTAL)
