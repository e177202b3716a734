"""Thin ctypes binding of libbca.so (include/bca.h).

Only argument marshalling happens here: every step of the solver runs in the
library's HIP kernels.  Importing this module fails loudly when the library has
not been built; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbca.so")

BCA_OK = 0
ERRORS = {-1: "BCA_E_INVALID", -2: "BCA_E_OOM", -3: "BCA_E_STATE", -4: "BCA_E_NONFINITE",
          -5: "BCA_E_DEVICE", -6: "BCA_E_BUDGET", -7: "BCA_E_NOTFOUND", -8: "BCA_E_CANCELLED"}
LOSS = {"squared": 0, "logistic": 1, "softmax": 2, "hinge": 3}
FLAG_EXACT_X = 1
FLAG_WOODBURY = 2
DTYPE = {"f64": 0, "f32": 1, "bf16": 2}
MEM_HOST, MEM_DEVICE = 0, 1
VEC_X, VEC_U, VEC_Z, VEC_S, VEC_OMEGA, VEC_NU, VEC_TV = range(7)
KC_STREAM, KC_SOLVE, KC_GLOBAL, KC_GRAM, KC_FACTOR = range(5)

EXPORTS = ["bca_create", "bca_set_data", "bca_finalize", "bca_step", "bca_solve",
           "bca_get_support", "bca_get_coef", "bca_get_residuals", "bca_get_history",
           "bca_get_objective", "bca_get_vector", "bca_set_vector", "bca_get_state",
           "bca_set_state", "bca_get_inverse", "bca_set_timing", "bca_get_timing", "bca_destroy",
           "bca_last_error", "bca_topk", "bca_batch_step", "bca_batch_step_noalloc", "bca_batch_solve",
           "bca_batch_autotune", "bca_batch_set_shape", "bca_batch_get_shape",
           "bca_batch_set_tracing", "bca_batch_get_tracing",
           "bca_server_create", "bca_server_submit", "bca_server_poll", "bca_server_fetch",
           "bca_server_cancel", "bca_server_stats", "bca_server_timing", "bca_server_destroy"]


class BcaError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "BCA_E_?"), code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("n_classes", ctypes.c_int32), ("n_partitions", ctypes.c_int32),
                ("n_blocks", ctypes.c_int32), ("kappa", ctypes.c_int32),
                ("rows", ctypes.POINTER(ctypes.c_int64)),
                ("gamma", ctypes.c_double), ("rho_c", ctypes.c_double),
                ("rho_b", ctypes.c_double), ("rho_l", ctypes.c_double),
                ("inner_iters", ctypes.c_int32), ("max_iters", ctypes.c_int32),
                ("tol_p", ctypes.c_double), ("tol_d", ctypes.c_double), ("tol_b", ctypes.c_double),
                ("a_dtype", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libbca.so is not built (%s); run `python -m paper_2405_16267_amd.build`"
                          % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    pi32, pdbl, psz = ctypes.POINTER(i32), ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "bca_create": [ctypes.POINTER(Params), P, ctypes.POINTER(P)],
        "bca_set_data": [P, i32, P, i64, P, i32],
        "bca_finalize": [P],
        "bca_step": [P, i32, pi32],
        "bca_solve": [P, pi32, pi32],
        "bca_get_support": [P, P, pi32],
        "bca_get_coef": [P, P],
        "bca_get_residuals": [P, pdbl, pdbl, pdbl, pi32],
        "bca_get_history": [P, P, i32, pi32],
        "bca_get_objective": [P, pdbl],
        "bca_get_vector": [P, i32, i32, P],
        "bca_set_vector": [P, i32, i32, P],
        "bca_get_state": [P, P, psz],
        "bca_set_state": [P, P, ctypes.c_size_t],
        "bca_get_inverse": [P, i32, i32, P],
        "bca_set_timing": [P, i32],
        "bca_get_timing": [P, i32, pi32, pdbl],
        "bca_destroy": [P],
        "bca_topk": [P, i32, i64, i32, P, P],
        "bca_batch_step": [P, i32, i32, P],
        "bca_batch_step_noalloc": [P, i32, i32, P],
        "bca_batch_solve": [P, i32, P],
        "bca_batch_autotune": [P, i32, P],
        "bca_batch_set_shape": [P, i32, i32],
        "bca_batch_get_shape": [P, pi32, pi32],
        "bca_batch_set_tracing": [i32],
        "bca_batch_get_tracing": [pdbl, i32, ctypes.POINTER(i64)],
        "bca_server_create": [ctypes.c_size_t, i32, i32, P, ctypes.POINTER(P)],
        "bca_server_submit": [P, ctypes.POINTER(Params), P, P, ctypes.POINTER(ctypes.c_uint64)],
        "bca_server_poll": [P, ctypes.c_uint64, pi32],
        "bca_server_fetch": [P, ctypes.c_uint64, P, P, pdbl, pdbl],
        "bca_server_cancel": [P, ctypes.c_uint64],
        "bca_server_stats": [P, pi32, pi32, pdbl, ctypes.POINTER(ctypes.c_int64)],
        "bca_server_timing": [P, pdbl, i32],
        "bca_server_destroy": [P],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.bca_last_error.argtypes = []
    lib.bca_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()

# Handles still open when the interpreter exits are released by an exit hook that
# runs before module teardown, while the HIP runtime (and any profiler attached to
# it) is still up: Problem.__del__ / Server.__del__ during interpreter finalisation
# would otherwise call into the runtime in an unspecified order with its own exit
# handlers (the server's scheduler thread would still be running).
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def lib():
    return _lib


def _check(code: int):
    if code != BCA_OK:
        raise BcaError(code, _lib.bca_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(None)


_NP_DTYPE = {"f64": np.float64, "f32": np.float32, "bf16": np.uint16}


class Problem:
    """One Bi-cADMM problem: N sample partitions x M feature blocks on the GPU."""

    def __init__(self, loss: str, n: int, rows: Sequence[int], n_blocks: int, kappa: int,
                 gamma: float = 10.0, rho_c: float = 1.0, rho_b: float = 0.5,
                 rho_l: float = 1.0, inner_iters: int = 5, max_iters: int = 100,
                 dtype: str = "f32", n_classes: int = 1, tol=(1e-6, 1e-6, 1e-6),
                 check_every: int = 10, stream=None, exact_x: bool = False,
                 woodbury: bool = False):
        self.loss, self.n, self.dtype = loss, n, dtype
        self.rows = [int(r) for r in rows]
        # the exact x-update factors all n features as one block
        self.N, self.M, self.kappa, self.C = len(self.rows), 1 if exact_x else n_blocks, kappa, n_classes
        self.max_iters = max_iters
        self._rows = (ctypes.c_int64 * self.N)(*self.rows)
        p = Params(loss=LOSS[loss], n_features=n, n_classes=n_classes, n_partitions=self.N,
                   n_blocks=n_blocks, kappa=kappa, rows=self._rows, gamma=gamma, rho_c=rho_c,
                   rho_b=rho_b, rho_l=rho_l, inner_iters=inner_iters, max_iters=max_iters,
                   tol_p=tol[0], tol_d=tol[1], tol_b=tol[2], a_dtype=DTYPE[dtype],
                   check_every=check_every,
                   flags=(FLAG_EXACT_X if exact_x else 0) | (FLAG_WOODBURY if woodbury else 0))
        self._stream = _current_stream() if stream is None else ctypes.c_void_p(stream)
        h = ctypes.c_void_p()
        _check(_lib.bca_create(ctypes.byref(p), self._stream, ctypes.byref(h)))
        self._h = h
        _LIVE.add(self)

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.bca_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- data
    def set_data(self, part: int, A, b):
        """A: m_i x n (numpy in the storage dtype, or a contiguous torch CUDA tensor);
        b: float64 targets/labels (int32 class ids for softmax), same placement."""
        try:
            import torch
            is_t = isinstance(A, torch.Tensor)
        except Exception:
            is_t = False
        if is_t:
            assert A.is_cuda and b.is_cuda, "device tensors expected"
            A = A.contiguous()
            b = b.contiguous()
            _check(_lib.bca_set_data(self._h, part, ctypes.c_void_p(A.data_ptr()), A.shape[1],
                                     ctypes.c_void_p(b.data_ptr()), MEM_DEVICE))
            return
        A = np.ascontiguousarray(A, dtype=_NP_DTYPE[self.dtype])
        b = np.ascontiguousarray(b, dtype=np.int32 if self.loss == "softmax" else np.float64)
        if A.shape != (self.rows[part], self.n):
            raise ValueError("partition %d: A has shape %s, expected %s"
                             % (part, A.shape, (self.rows[part], self.n)))
        _check(_lib.bca_set_data(self._h, part, _ptr(A), A.shape[1], _ptr(b), MEM_HOST))

    def finalize(self):
        _check(_lib.bca_finalize(self._h))

    # -- iterations
    def step(self, outer_iters: int = 1) -> int:
        k = ctypes.c_int32()
        _check(_lib.bca_step(self._h, outer_iters, ctypes.byref(k)))
        return k.value

    def solve(self):
        k, c = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.bca_solve(self._h, ctypes.byref(k), ctypes.byref(c)))
        return k.value, bool(c.value)

    # -- queries
    def support(self) -> np.ndarray:
        idx = np.zeros(self.kappa, dtype=np.int32)
        _check(_lib.bca_get_support(self._h, _ptr(idx), None))
        return idx

    def coef(self) -> np.ndarray:
        x = np.zeros(self.n * self.C)
        _check(_lib.bca_get_coef(self._h, _ptr(x)))
        return x if self.C == 1 else x.reshape(self.n, self.C)

    def residuals(self):
        pr, dr, br, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        _check(_lib.bca_get_residuals(self._h, ctypes.byref(pr), ctypes.byref(dr),
                                      ctypes.byref(br), ctypes.byref(it)))
        return pr.value, dr.value, br.value, it.value

    def history(self) -> np.ndarray:
        h = np.zeros((self.max_iters, 3))
        k = ctypes.c_int32()
        _check(_lib.bca_get_history(self._h, _ptr(h), self.max_iters, ctypes.byref(k)))
        return h[:k.value]

    def objective(self) -> float:
        f = ctypes.c_double()
        _check(_lib.bca_get_objective(self._h, ctypes.byref(f)))
        return f.value

    def _vlen(self, which, part):
        if which in (VEC_X, VEC_U, VEC_Z):
            return self.n * self.C
        if which == VEC_S:
            return self.n
        if which in (VEC_OMEGA, VEC_NU):
            return self.rows[part] * self.C
        return 2

    def get_vector(self, which: int, part: int = 0) -> np.ndarray:
        out = np.zeros(self._vlen(which, part))
        _check(_lib.bca_get_vector(self._h, which, part, _ptr(out)))
        return out

    def set_vector(self, which: int, part: int, values) -> None:
        v = np.ascontiguousarray(values, dtype=np.float64).ravel()
        if v.size != self._vlen(which, part):
            raise ValueError("wrong length")
        _check(_lib.bca_set_vector(self._h, which, part, _ptr(v)))

    def get_state(self) -> bytes:
        n = ctypes.c_size_t()
        _check(_lib.bca_get_state(self._h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(_lib.bca_get_state(self._h, buf, ctypes.byref(n)))
        return buf.raw

    def set_state(self, blob: bytes) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(_lib.bca_set_state(self._h, buf, len(blob)))

    def inverse(self, part: int, block: int) -> np.ndarray:
        """The cached K_ij^-1 of block (part, block), dense n_j x n_j."""
        q, r = divmod(self.n, self.M)
        nj = q + (1 if block < r else 0)
        K = np.zeros((nj, nj))
        _check(_lib.bca_get_inverse(self._h, part, block, _ptr(K)))
        return K

    def batch_shape(self):
        t, i = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.bca_batch_get_shape(self._h, ctypes.byref(t), ctypes.byref(i)))
        return t.value, i.value

    def set_batch_shape(self, rows_per_tile: int, rows_per_item: int):
        _check(_lib.bca_batch_set_shape(self._h, rows_per_tile, rows_per_item))

    def set_timing(self, on: bool = True):
        _check(_lib.bca_set_timing(self._h, 1 if on else 0))

    def timing(self, kernel_class: int):
        n, ms = ctypes.c_int32(), ctypes.c_double()
        _check(_lib.bca_get_timing(self._h, kernel_class, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value


def topk(z, kappa: int):
    """Top-kappa indices (ascending) of |z| for a CUDA tensor z (float64/float32)."""
    import torch
    assert z.is_cuda and z.dim() == 1
    z = z.contiguous()
    dt = {torch.float64: 0, torch.float32: 1}[z.dtype]
    idx = torch.empty(kappa, dtype=torch.int32, device=z.device)
    _check(_lib.bca_topk(ctypes.c_void_p(z.data_ptr()), dt, z.numel(), kappa,
                         ctypes.c_void_p(idx.data_ptr()), _current_stream()))
    return idx


def _handles(problems):
    arr = (ctypes.c_void_p * len(problems))(*[p._h.value for p in problems])
    return arr


def batch_step(problems, outer_iters: int, stream=None):
    """Advance every problem by up to outer_iters outer iterations in one persistent launch."""
    st = _current_stream() if stream is None else ctypes.c_void_p(stream)
    _check(_lib.bca_batch_step(_handles(problems), len(problems), outer_iters, st))


def batch_step_noalloc(problems, outer_iters: int, stream=None):
    """batch_step without device allocation (the library's fixed 16 MiB scratch)."""
    st = _current_stream() if stream is None else ctypes.c_void_p(stream)
    _check(_lib.bca_batch_step_noalloc(_handles(problems), len(problems), outer_iters, st))


def batch_solve(problems, stream=None):
    st = _current_stream() if stream is None else ctypes.c_void_p(stream)
    _check(_lib.bca_batch_solve(_handles(problems), len(problems), st))


def batch_autotune(problems, stream=None):
    st = _current_stream() if stream is None else ctypes.c_void_p(stream)
    _check(_lib.bca_batch_autotune(_handles(problems), len(problems), st))


BATCH_PHASES = ("prime", "rhs", "symv", "xupd", "stream", "global")


def batch_set_tracing(on: bool):
    """Phase tracing of the batched launches (bca_batch_set_tracing)."""
    _check(_lib.bca_batch_set_tracing(1 if on else 0))


def batch_get_tracing():
    """Summed microseconds per batched phase kind, and the traced launch count."""
    us = (ctypes.c_double * len(BATCH_PHASES))()
    n = ctypes.c_int64()
    _check(_lib.bca_batch_get_tracing(us, len(BATCH_PHASES), ctypes.byref(n)))
    return dict(zip(BATCH_PHASES, list(us))), n.value


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED, REQ_CANCELLED = range(5)


class Server:
    """Continuous-batching request loop (bca_server_*)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 256, round_iters: int = 5,
                 stream=None):
        st = _current_stream() if stream is None else ctypes.c_void_p(stream)
        h = ctypes.c_void_p()
        _check(_lib.bca_server_create(hbm_budget_bytes, max_slots, round_iters, st, ctypes.byref(h)))
        self._h = h
        self._meta = {}
        _LIVE.add(self)

    def submit(self, loss: str, A_parts, b_parts, n_blocks: int, kappa: int, gamma=10.0,
               rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5, max_iters=100, dtype="f32",
               n_classes=1) -> int:
        N = len(A_parts)
        rows = (ctypes.c_int64 * N)(*[a.shape[0] for a in A_parts])
        n = A_parts[0].shape[1]
        p = Params(loss=LOSS[loss], n_features=n, n_classes=n_classes, n_partitions=N,
                   n_blocks=n_blocks, kappa=kappa, rows=rows, gamma=gamma, rho_c=rho_c,
                   rho_b=rho_b, rho_l=rho_l, inner_iters=inner_iters, max_iters=max_iters,
                   tol_p=0.0, tol_d=0.0, tol_b=0.0, a_dtype=DTYPE[dtype], check_every=0, flags=0)
        As = [np.ascontiguousarray(a, dtype=_NP_DTYPE[dtype]) for a in A_parts]
        bs = [np.ascontiguousarray(b, dtype=np.int32 if loss == "softmax" else np.float64)
              for b in b_parts]
        pa = (ctypes.c_void_p * N)(*[a.ctypes.data for a in As])
        pb = (ctypes.c_void_p * N)(*[b.ctypes.data for b in bs])
        t = ctypes.c_uint64()
        _check(_lib.bca_server_submit(self._h, ctypes.byref(p), pa, pb, ctypes.byref(t)))
        self._meta[t.value] = (n, kappa, n_classes)
        return t.value

    def poll(self, ticket: int) -> int:
        s = ctypes.c_int32()
        _check(_lib.bca_server_poll(self._h, ticket, ctypes.byref(s)))
        return s.value

    def fetch(self, ticket: int):
        n, kappa, C = self._meta[ticket]
        idx = np.zeros(kappa, dtype=np.int32)
        x = np.zeros(n * C)
        f, lat = ctypes.c_double(), ctypes.c_double()
        _check(_lib.bca_server_fetch(self._h, ticket, _ptr(idx), _ptr(x), ctypes.byref(f),
                                     ctypes.byref(lat)))
        return idx, (x if C == 1 else x.reshape(n, C)), f.value, lat.value

    def cancel(self, ticket: int):
        _check(_lib.bca_server_cancel(self._h, ticket))

    def stats(self):
        q, r, u, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()
        _check(_lib.bca_server_stats(self._h, ctypes.byref(q), ctypes.byref(r), ctypes.byref(u),
                                     ctypes.byref(k)))
        return dict(queued=q.value, running=r.value, used_bytes=u.value, rounds=k.value)

    def timing(self):
        """Seconds per server activity (bca_server_timing)."""
        t = (ctypes.c_double * 7)()
        _check(_lib.bca_server_timing(self._h, t, 7))
        return dict(zip(("softmax", "batched", "retire", "materialise", "materialiser_wait",
                         "scheduler_wait", "release"), list(t)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.bca_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
