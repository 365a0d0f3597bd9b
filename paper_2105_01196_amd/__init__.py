"""MI355X-native EBIC fitness evaluation (arXiv 2105.01196).

The HIP library ``libebic.so`` (C ABI: include/ebic.h) does the work; the
``ebic`` module is its Python binding. Import ``paper_2105_01196_amd.ebic``
to load the library (it raises when the library has not been built).
"""
__all__ = ["ebic", "build"]
