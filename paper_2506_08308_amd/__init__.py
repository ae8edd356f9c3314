"""MI355X (gfx950) spin-1 Bogoliubov-de Gennes excitation solver.

The compute path is the HIP library ``libbdg.so`` (C ABI in ``include/bdg.h``); this
package only marshals torch device tensors into it.  Importing works without a GPU;
creating a :class:`BdgContext` needs the built library and a gfx950 device.
"""
from .api import BdgContext, BdgError, Precision, Form  # noqa: F401
from ._lib import LIB_PATH  # noqa: F401
