"""MI355X (gfx950) pc-ePIE reconstruction: Python binding of libptycho.so.

The HIP library does all of the reconstruction arithmetic; this package only
marshals arguments (numpy host arrays or torch device tensors) to the C ABI of
``include/ptycho.h``.  Importing it fails loudly if the library is not built.
"""

from .ptycho import *  # noqa: F401,F403
from . import learned  # noqa: F401
