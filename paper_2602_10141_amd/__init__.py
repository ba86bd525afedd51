"""MI355X-native Gray-code Glynn permanents over C, R and F_p with CRT lifting.

The compute path is the C-ABI library ``libperm.so`` (HIP kernels for
gfx950, declared in ``include/perm.h``); ``perm`` is its Python binding and
``ensembles`` the seeded input generators.  Importing the package loads
nothing; ``paper_2602_10141_amd.perm`` loads the library on first use and
raises if it has not been built.
"""
__all__ = ["ensembles", "perm"]
