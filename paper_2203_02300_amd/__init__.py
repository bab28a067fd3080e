"""MI355X (gfx950) two-stage adaptive AD-census stereo matcher.

The sparse-disparity front end of the depth contour occlusion method
(arXiv 2203.02300, Sec. 4): census transform, cross-support arms, the
adaptive AD-census cost (Eq. 1), two-stage aggregation over the adaptive
region (Eq. 2), winner-take-all (Eq. 3) with sub-pixel refinement and a
left-right check, as hand-written HIP kernels behind a C ABI
(include/dco_stereo.h).  The torch objects are imported lazily so that the
scene generator can be used without a GPU.
"""

__all__ = ["StereoMatcher", "BatchMatcher", "DcoSoftArgmin", "soft_argmin_disparity",
           "default_params", "Densifier", "ContourFilter"]


import importlib

_LAZY = {"StereoMatcher": "api", "default_params": "api", "BatchMatcher": "batch",
         "DcoSoftArgmin": "soft", "soft_argmin_disparity": "soft", "Densifier": "densify",
         "ContourFilter": "contour"}


def __getattr__(name):
    if name in _LAZY:
        mod = importlib.import_module(f"{__name__}.{_LAZY[name]}")
        return getattr(mod, name)
    raise AttributeError(name)
