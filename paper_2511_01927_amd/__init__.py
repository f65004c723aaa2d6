"""MI355X (gfx950) contour-integral eigensolver for sparse symmetric-definite pencils.

The compute path is the HIP library ``libgepci.so`` built from ``csrc/``;
``gep_ci`` is a thin ctypes binding with the same entry-point names.
"""
