"""Uniform H-matrix matrix-vector products on MI355X (gfx950).

The package is import-light: importing it loads no native library.  ``binding`` loads
the HIP library ``libuhm.so`` on first use and raises if it is missing; ``builder``
loads the host builder library ``libuhm_builder.so``.
"""
__all__ = ["inputs", "builder", "binding"]
