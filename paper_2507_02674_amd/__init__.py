"""MI355X (gfx950) hot path of real-time image-based glint lighting.

``glint`` binds the C ABI of ``libglint.so`` (HIP kernels, built in-tree by
``build.py``); ``pipeline`` manages device buffers for one environment and one
frame.  Importing the package loads nothing; the library is loaded on the
first call and there is no CPU fallback.
"""
__all__ = ["glint", "pipeline", "build"]
