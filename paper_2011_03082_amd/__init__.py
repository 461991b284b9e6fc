"""libmsst: MI355X (gfx950) learned sphere tracing of volumetric subsurface
scattering (arXiv 2011.03082).  All computation runs in the HIP library
libmsst.so; this package is its Python binding."""
from . import _abi
from ._abi import MsError, lib
from .binding import *  # noqa: F401,F403
