"""MI355X (gfx950) data-parallel primitives for accelerated expressions.

``abi`` is the thin binding of the C ABI (include/mx.h) with the same names as
the C entry points; ``api`` adds output allocation, cached workspaces and
autograd wrappers.  Importing the package loads libmx.so and fails if it has not
been built: there is no CPU fallback.
"""
from . import _lib

_lib.load()

from . import abi  # noqa: E402
from .abi import *  # noqa: E402,F401,F403
from . import api  # noqa: E402

__all__ = ["abi", "api"]
