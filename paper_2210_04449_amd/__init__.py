"""RTSDF signed-distance-field generation on MI355X (gfx950).

The HIP library (``librtsdf.so``, C ABI in include/rtsdf.h) is loaded by
:mod:`paper_2210_04449_amd.rtsdf`; :class:`paper_2210_04449_amd.pipeline.Pipeline`
runs the per-frame update.  Submodules are imported on demand so that
``paper_2210_04449_amd.build`` works on a machine without the built library.
"""
__all__ = ["rtsdf", "pipeline", "build"]
