"""Shrink-and-expand block eigensolvers (arXiv 2409.05572) on MI355X.

The solver runs in the HIP library ``libse.so`` (C ABI in ``include/se.h``);
this package is its thin Python binding. Importing the package loads nothing;
``paper_2409_05572_amd.api`` loads the library on first use and raises if it is
missing (there is no CPU fallback).
"""
__all__ = ["api"]
