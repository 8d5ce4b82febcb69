"""MI355X-native XTRG: the beta-doubling hot path as a HIP library (libxtrg.so)
with a thin ctypes binding.  See include/xtrg.h for the C ABI."""
from .xtrg import XTRG_BF16X3, XTRG_FP32, XTRG_FP64, Context, MPO, XtrgError, load_library, run  # noqa: F401
