"""MI355X-native w-projection kernel generation (Lucas, Skipper & Scaife 2019).

The compute path is the HIP library ``libwkern.so`` (C ABI in
``include/wkern.h``); ``wkern`` is its Python binding and ``autograd`` wraps
it in a ``torch.autograd.Function``.
"""
from .wkern import (ABI_VERSION, EXPORTS, Plan, WkernError, layout_desc,  # noqa: F401
                    load_library)
