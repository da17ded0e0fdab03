"""MI355X-native w-projection kernel generation (Lucas, Skipper & Scaife 2019).

The compute path is the HIP library ``libwkern.so`` (C ABI in
``include/wkern.h``); ``wkern`` is its Python binding and ``autograd`` wraps
it in a ``torch.autograd.Function``.
"""
from .wkern import (ABI_VERSION, EXPORTS, FFT2DPlan, Plan, WkernError,  # noqa: F401
                    layout_desc, load_library, store_ceiling, wpartition, wpartition_noalloc,
                    wpartition_workspace)
