"""MI355X-native cross-spectrum FRB search (Liu et al. 2018, arXiv:1801.02391).

The search runs in the HIP library ``libfrbx.so`` (C ABI declared in
``include/frbx.h``); :mod:`paper_1801_02391_amd.frbx` is its Python binding
and :mod:`paper_1801_02391_amd.workloads` draws seeded synthetic inputs.
Importing the package loads nothing native; the binding loads the library on
first use and raises if it is missing.
"""
__all__ = ["workloads", "frbx"]
