"""MI355X (gfx950) implementation of the Bi-cADMM hot path: HIP kernels behind the
C ABI in include/bca.h (libbca.so), with a thin ctypes binding."""
from .bca import (BcaError, Problem, topk, lib, LIB_PATH, EXPORTS, VEC_X, VEC_U, VEC_Z, VEC_S,
                  VEC_OMEGA, VEC_NU, VEC_TV, KC_STREAM, KC_SOLVE, KC_GLOBAL, KC_GRAM, KC_FACTOR)

__all__ = ["BcaError", "Problem", "topk", "lib", "LIB_PATH", "EXPORTS"]
