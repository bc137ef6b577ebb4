"""MI355X-native GOCP ADAPT-VQE hot path (HIP kernels for gfx950 behind a C ABI).

The computation lives in libgocp.so (``csrc/``, declared in ``include/gocp.h``);
this package is its ctypes binding.  Importing the package loads the library
and fails loudly if it has not been built.
"""

from ._lib import load as _load, GocpError

_load()

from .api import *  # noqa: E402,F401,F403
from .api import __all__ as _api_all  # noqa: E402

__all__ = list(_api_all) + ["GocpError"]
