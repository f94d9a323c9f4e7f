"""MI355X-native Riemannian ray tracer (hand-written HIP for gfx950).

Traces geodesics of metrics built from graphs of functions (g = I + grad f
grad f^T, f a sum of Gaussian bumps) and from diffeomorphism pull-backs
(g = J^T J) per pixel until they hit a scene of spheres, planes and tori.
The engine is the C-ABI library ``librt.so`` (include/rt.h); ``rt`` is its
Python binding.  Build with ``paper_2005_05386_amd.build.build()``.
"""

__all__ = ["rt", "build"]


def __getattr__(name):
    if name in ("rt", "build"):
        import importlib
        return importlib.import_module(__name__ + "." + name)
    raise AttributeError(name)
