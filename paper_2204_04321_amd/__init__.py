"""MI355X (gfx950) first-order Stokes finite-element assembly library.

The compute path lives in libfo_stokes.so (HIP kernels behind the C ABI of
include/fo_stokes.h); this package only marshals arguments.
"""
from ._lib import FoError  # noqa: F401


def __getattr__(name):
    if name in ("Mesh", "Ensemble", "Mdsc", "aggregate_graph"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
