"""MI355X-native RLFC decode-and-render.

The compute path lives in the HIP library ``liblfc.so`` (C ABI declared in
``include/lfc.h``); ``paper_1805_06019_amd.lfc`` is its Python binding.
Importing the package loads nothing; the binding loads the library on first
use and raises if it is missing.
"""
