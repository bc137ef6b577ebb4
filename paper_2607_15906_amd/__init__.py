"""MI355X-native GOCP ADAPT-VQE hot path (HIP kernels for gfx950 behind a C ABI).

The computation lives in libgocp.so (``csrc/``, declared in ``include/gocp.h``);
this package is its ctypes binding.  Importing the package loads the library
and fails loudly if it has not been built.
"""

# torch first: libgocp then binds to the HIP runtime torch has loaded, the one
# that owns the streams and device buffers handed to the library.
try:
    import torch as _torch  # noqa: F401
except ImportError:          # host-only use (Hamiltonians, pools, partitions)
    _torch = None

from ._lib import load as _load, GocpError  # noqa: E402

_load()

from .api import *  # noqa: E402,F401,F403
from .api import __all__ as _api_all  # noqa: E402

__all__ = list(_api_all) + ["GocpError"]
