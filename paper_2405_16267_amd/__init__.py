"""MI355X (gfx950) implementation of the Bi-cADMM hot path: HIP kernels behind the
C ABI in include/bca.h (libbca.so), with a thin ctypes binding (``bca.py``).

The binding is loaded on first use of any of its names; it raises ImportError
when libbca.so has not been built (there is no CPU fallback).  The build step
(``paper_2405_16267_amd.build``) imports without the library.
"""
_BINDING_NAMES = {"BcaError", "Problem", "topk", "lib", "LIB_PATH", "EXPORTS", "VEC_X", "VEC_U",
                  "VEC_Z", "VEC_S", "VEC_OMEGA", "VEC_NU", "VEC_TV", "KC_STREAM", "KC_SOLVE",
                  "KC_GLOBAL", "KC_GRAM", "KC_FACTOR", "Params", "batch_step", "batch_step_noalloc",
                  "batch_solve", "batch_autotune", "batch_set_tracing", "batch_get_tracing",
                  "BATCH_PHASES", "Server", "REQ_QUEUED", "REQ_RUNNING",
                  "REQ_DONE", "REQ_FAILED", "REQ_CANCELLED"}

__all__ = sorted(_BINDING_NAMES)


def __getattr__(name):
    if name in _BINDING_NAMES:
        from . import bca as _b
        return getattr(_b, name)
    raise AttributeError(name)
