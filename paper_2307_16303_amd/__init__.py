"""MI355X-native HODLR3D matrix-vector product (arXiv 2307.16303).

The compute path is the HIP library ``libhodlr3d.so`` built from ``csrc/``;
the Python layer in ``hodlr3d.py`` only marshals arguments through its C ABI.
Importing this package loads nothing; the library is loaded on first use.
"""
