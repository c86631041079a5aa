"""MI355X-native weakly-compressible SPH step (arXiv:2207.11328).

The compute path is libsph.so: hand-written HIP for gfx950 behind the C ABI
declared in include/sph.h.  `abi` binds it with ctypes (argument marshalling
only) and `sim` drives the step sequence over it.  Importing `abi` fails if
the library is not built: there is no CPU fallback.
"""
__all__ = ["abi", "sim", "build"]
