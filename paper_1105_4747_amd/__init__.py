"""MI355X-native Lyman-alpha optical depths (Greig, Bolton & Wyithe 2011, Sec. 2.3).

The product is liblyaf.so (HIP, gfx950) behind the C ABI of include/lyaf.h;
``paper_1105_4747_amd.lyaf`` is its ctypes binding and autograd wrapper.
"""
from . import lyaf  # noqa: F401

__all__ = ["lyaf"]
