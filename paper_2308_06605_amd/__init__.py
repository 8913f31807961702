"""MI355X-native flux-reconstruction residual and Runge-Kutta stage library.

The compute path lives in libfr.so (HIP kernels for gfx950 behind the C ABI declared in
include/fr.h); `paper_2308_06605_amd.fr` is a thin ctypes binding with the same names.
`paper_2308_06605_amd.inputs` builds synthetic meshes and closed-form states.
"""
__all__ = ["fr", "inputs"]
