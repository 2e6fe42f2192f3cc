"""MI355X-native local affine-body Newton solve of the consensus-ADMM
method (distributed ABD, Eq. 5): C-ABI library libabd (include/abd.h) with
hand-written gfx950 HIP kernels, a thin ctypes binding (abd.py) and the
seeded scene generators (scenes.py).  Importing the package does not load
the library; abd.lib() does, and raises if it was not built."""
__all__ = ["abd", "scenes", "build"]
