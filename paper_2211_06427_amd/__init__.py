"""Weighted-quadrature row assembly for cut tensor-product B-spline meshes on MI355X (gfx950).

Importing the package does not load the HIP library; `Rules` (and everything that computes)
loads libwqfd.so and raises if it is missing.
"""
from ._lib import WQ_F32, WQ_F64, WQ_MASS, WQ_STIFF, WqError  # noqa: F401


def __getattr__(name):
    if name in ("Rules", "WQAssemble"):
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
