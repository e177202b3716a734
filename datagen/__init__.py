"""Seeded synthetic workloads for sparse learning over sample partitions.

This module only produces inputs: data blocks A_i, targets or labels b_i, the
planted model and the solver parameters of each workload.  It contains none of
the fitting method's arithmetic, so the FP64 reference implementation and the
GPU library can both be fed from it without sharing any code.

Recipes follow the experimental section of the paper (dense Gaussian feature
matrices with per-node unit-norm columns, a planted sparse ground truth, noisy
linear targets); the logistic, softmax and batched recipes are synthetic
workloads of the same kind (AR(1) rows with Toeplitz covariance 0.3^|i-j|,
Bernoulli-logit labels, argmax-plus-Gumbel class labels).

Random numbers are Philox4x32-10 (Salmon et al., SC 2011) addressed by
(seed, stream, row, column); the C part lives in ``bcdata.c``.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bcdata.c")
_LIB = os.path.join(_HERE, "libbcdata.so")

# Stream tags: each kind of draw has its own Philox stream.
S_A = 0x1000          # + partition: feature matrix entries
S_NOISE = 0x2000      # + partition: target noise
S_LABEL = 0x3000      # + partition: label uniforms / Gumbel noise
S_SUPPORT = 0x10      # planted support keys
S_VALUES = 0x11       # planted values
S_SIGNS = 0x12        # planted signs
S_SIZES = 0x20        # instance sizes (batched / serving)
S_ARRIVAL = 0x21      # serving arrival times
S_KIND = 0x22         # serving request kinds

LOSS_SQUARED, LOSS_LOGISTIC, LOSS_SOFTMAX, LOSS_HINGE = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C generator (gcc, OpenMP) next to this file."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, u64, u32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double
        _lib.bcd_philox4x32_10.argtypes = [P, P, P]
        _lib.bcd_normal_matrix.argtypes = [u64, u32, i64, i64, i64, P, i64]
        _lib.bcd_uniform_vector.argtypes = [u64, u32, u64, i64, i64, P]
        _lib.bcd_normal_vector.argtypes = [u64, u32, u64, i64, i64, P]
        _lib.bcd_ar1_rows.argtypes = [P, i64, i64, i64, dbl]
        _lib.bcd_normalize_columns.argtypes = [P, i64, i64, i64]
        _lib.bcd_to_f32.argtypes = [P, i64, i64, i64, P, i64]
        _lib.bcd_gaussian_block.argtypes = [u64, u32, i64, i64, i64, ctypes.c_int, P, P, i64]
        _lib.bcd_f32_to_bf16.argtypes = [P, i64, i64, i64, P, i64]
        _lib.bcd_bf16_to_f64.argtypes = [P, i64, i64, i64, P, i64]
        _lib.bcd_sparse_predict_f32.argtypes = [P, i64, i64, P, P, i64, P]
        _lib.bcd_sparse_predict_f64.argtypes = [P, i64, i64, P, P, i64, P]
        for f in ("bcd_philox4x32_10", "bcd_normal_matrix", "bcd_uniform_vector",
                  "bcd_normal_vector", "bcd_ar1_rows", "bcd_normalize_columns", "bcd_to_f32", "bcd_gaussian_block",
                  "bcd_f32_to_bf16", "bcd_bf16_to_f64", "bcd_sparse_predict_f32",
                  "bcd_sparse_predict_f64"):
            getattr(_lib, f).restype = None
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# ---------------------------------------------------------------- primitives
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().bcd_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def normal_matrix(seed: int, stream: int, m: int, n: int, row0: int = 0) -> np.ndarray:
    out = np.empty((m, n), dtype=np.float64)
    lib().bcd_normal_matrix(seed, stream, m, n, row0, _p(out), n)
    return out


def uniform_vector(seed: int, stream: int, n: int, row: int = 0, k0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().bcd_uniform_vector(seed, stream, row, k0, n, _p(out))
    return out


def normal_vector(seed: int, stream: int, n: int, row: int = 0, k0: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    lib().bcd_normal_vector(seed, stream, row, k0, n, _p(out))
    return out


def to_f32(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty(a.shape, dtype=np.float32)
    lib().bcd_to_f32(_p(a), a.shape[0], a.shape[1], a.shape[1], _p(out), a.shape[1])
    return out


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (uint16), round to nearest even."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    out = np.empty(a.shape, dtype=np.uint16)
    lib().bcd_f32_to_bf16(_p(a), a.shape[0], a.shape[1], a.shape[1], _p(out), a.shape[1])
    return out


def bf16_bits_to_f64(a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint16)
    out = np.empty(a.shape, dtype=np.float64)
    lib().bcd_bf16_to_f64(_p(a), a.shape[0], a.shape[1], a.shape[1], _p(out), a.shape[1])
    return out


def widen(a: np.ndarray) -> np.ndarray:
    """Exact FP64 values of a stored block (float64, float32 or BF16 bits)."""
    if a.dtype == np.uint16:
        return bf16_bits_to_f64(a)
    return np.asarray(a, dtype=np.float64)


def planted_support(seed: int, n: int, k: int) -> np.ndarray:
    """k distinct indices, uniform without replacement, ascending."""
    keys = uniform_vector(seed, S_SUPPORT, n)
    return np.sort(np.argsort(keys, kind="stable")[:k]).astype(np.int64)


def sparse_predict(A: np.ndarray, idx: np.ndarray, val: np.ndarray) -> np.ndarray:
    A = np.ascontiguousarray(A)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    val = np.ascontiguousarray(val, dtype=np.float64)
    out = np.empty(A.shape[0], dtype=np.float64)
    if A.dtype == np.float32:
        lib().bcd_sparse_predict_f32(_p(A), A.shape[0], A.shape[1], _p(idx), _p(val), len(idx), _p(out))
    elif A.dtype == np.float64:
        lib().bcd_sparse_predict_f64(_p(A), A.shape[0], A.shape[1], _p(idx), _p(val), len(idx), _p(out))
    else:
        return widen(A)[:, idx] @ val
    return out


# ---------------------------------------------------------------- workloads
@dataclass
class Workload:
    """A sample-partitioned sparse-fit problem and its solver parameters."""
    name: str
    loss: int
    A: List[np.ndarray]           # one m_i x n block per partition (float64/float32/uint16 bf16)
    b: List[np.ndarray]           # float64 targets, +-1 labels, or int32 class ids
    n: int
    kappa: int
    n_blocks: int
    n_classes: int = 1
    gamma: float = 10.0
    rho_c: float = 1.0
    rho_b: float = 0.5
    rho_l: float = 1.0
    max_iters: int = 100
    inner_iters: int = 5
    dtype: str = "f64"            # storage precision of A: f64, f32, bf16
    x_true: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return len(self.A)

    @property
    def rows(self) -> List[int]:
        return [a.shape[0] for a in self.A]

    def params(self) -> dict:
        return dict(loss=self.loss, n=self.n, n_classes=self.n_classes, N=self.N,
                    M=self.n_blocks, kappa=self.kappa, gamma=self.gamma, rho_c=self.rho_c,
                    rho_b=self.rho_b, rho_l=self.rho_l, max_iters=self.max_iters,
                    inner_iters=self.inner_iters)


def split_rows(m: int, N: int) -> List[int]:
    """m rows over N partitions; the first m mod N partitions get one extra row."""
    q, r = divmod(m, N)
    return [q + (1 if i < r else 0) for i in range(N)]


def linear_model(seed: int, n: int, k_true: int):
    """Planted model of the sparse linear recipe: k_true indices uniform without
    replacement, values +-U(1,2)."""
    supp = planted_support(seed, n, k_true)
    mag = 1.0 + uniform_vector(seed, S_VALUES, k_true)
    sgn = np.where(uniform_vector(seed, S_SIGNS, k_true) < 0.5, -1.0, 1.0)
    return supp, sgn * mag


def linear_partition(seed: int, i: int, m: int, n: int, supp, val, noise: float,
                     dtype: str = "f64", normalize: bool = False):
    """Partition i of the sparse linear recipe: A_i iid N(0,1) (optionally unit-norm
    columns, normalised in FP64), stored in `dtype` ("f64", "f32", "bf16" bits, or
    "f32+bf16" for both roundings of the same data); b_i = A_i x* + N(0, noise^2)
    with A_i the canonical (FP64, else FP32) matrix.  Returns (A, b), A a tuple
    (A32, Abf16) for "f32+bf16"."""
    if dtype == "f64":
        G = normal_matrix(seed, S_A + i, m, n)
        if normalize:
            lib().bcd_normalize_columns(_p(G), m, n, n)
        Ai = Aval = G
    else:
        # drawn straight to FP32 (and BF16), normalised with FP64 column sums
        A32 = np.empty((m, n), dtype=np.float32)
        Abf = np.empty((m, n), dtype=np.uint16) if dtype != "f32" else None
        lib().bcd_gaussian_block(seed, S_A + i, m, n, 0, int(normalize), _p(A32),
                                 _p(Abf) if Abf is not None else None, n)
        Aval = A32                      # targets use the canonical FP32 matrix
        Ai = {"f32": A32, "bf16": Abf}.get(dtype, (A32, Abf))
    pred = sparse_predict(Aval, supp, val)
    b = pred + noise * normal_vector(seed, S_NOISE + i, m)
    return Ai, b


def linear_targets(seed: int, i: int, A: np.ndarray, supp, val, noise: float) -> np.ndarray:
    """b_i = A_i x* + N(0, noise^2) for partition i of the sparse linear recipe, from
    an already drawn (canonical) A_i: the same targets linear_partition returns,
    for another planted model on the same matrix."""
    return sparse_predict(A, supp, val) + noise * normal_vector(seed, S_NOISE + i, A.shape[0])


def linear_workload(seed: int, N: int, m_per, n: int, kappa: int, k_true: int, noise: float,
                    n_blocks: int, dtype: str = "f64", normalize: bool = False,
                    max_iters: int = 200, inner_iters: int = 5, rho: float = 1.0,
                    gamma: float = 10.0, name: str = "linear") -> Workload:
    """Sparse linear regression: A_i iid N(0,1) (optionally unit-norm columns per
    partition), planted x* with values +-U(1,2), b_i = A_i x* + N(0, noise^2)."""
    rows = m_per if isinstance(m_per, (list, tuple)) else [m_per] * N
    supp, val = linear_model(seed, n, k_true)
    x_true = np.zeros(n)
    x_true[supp] = val
    A_out, b_out = [], []
    for i, m in enumerate(rows):
        Ai, b = linear_partition(seed, i, m, n, supp, val, noise, dtype, normalize)
        A_out.append(Ai)
        b_out.append(b)
    return Workload(name=name, loss=LOSS_SQUARED, A=A_out, b=b_out, n=n, kappa=kappa,
                    n_blocks=n_blocks, dtype=dtype, x_true=x_true, max_iters=max_iters,
                    inner_iters=inner_iters, rho_c=rho, rho_b=0.5 * rho, rho_l=rho, gamma=gamma,
                    meta=dict(seed=seed, noise=noise, normalize=normalize))


def logistic_workload(seed: int, N: int, m_per, n: int, kappa: int, k_true: int,
                      n_blocks: int, dtype: str = "f32", ar: float = 0.3,
                      max_iters: int = 100, inner_iters: int = 5, rho: float = 1.0,
                      gamma: float = 10.0, name: str = "logistic") -> Workload:
    """Sparse logistic regression: rows N(0, Sigma) with Sigma_ij = ar^|i-j| (AR(1)
    along the row), planted x* with N(0,1) values, labels +1 with probability
    sigmoid(a_k^T x*) else -1."""
    rows = m_per if isinstance(m_per, (list, tuple)) else [m_per] * N
    supp = planted_support(seed, n, k_true)
    val = normal_vector(seed, S_VALUES, k_true)
    x_true = np.zeros(n)
    x_true[supp] = val
    A_out, b_out = [], []
    for i, m in enumerate(rows):
        G = normal_matrix(seed, S_A + i, m, n)
        lib().bcd_ar1_rows(_p(G), m, n, n, ar)
        if dtype == "f64":
            Ai, Aval = G, G
        else:
            A32 = to_f32(G)
            del G
            Ai = A32 if dtype == "f32" else f32_to_bf16_bits(A32)
            Aval = A32
        logit = sparse_predict(Aval, supp, val)
        u = uniform_vector(seed, S_LABEL + i, m)
        prob = 1.0 / (1.0 + np.exp(-logit))
        b = np.where(u < prob, 1.0, -1.0)
        A_out.append(Ai)
        b_out.append(b)
    return Workload(name=name, loss=LOSS_LOGISTIC, A=A_out, b=b_out, n=n, kappa=kappa,
                    n_blocks=n_blocks, dtype=dtype, x_true=x_true, max_iters=max_iters,
                    inner_iters=inner_iters, rho_c=rho, rho_b=0.5 * rho, rho_l=rho, gamma=gamma,
                    meta=dict(seed=seed, ar=ar))


def svm_workload(seed: int, N: int, m_per, n: int, kappa: int, k_true: int, n_blocks: int,
                 dtype: str = "f32", noise: float = 0.5, max_iters: int = 100,
                 inner_iters: int = 5, rho: float = 1.0, gamma: float = 10.0,
                 name: str = "svm") -> Workload:
    """Sparse SVM (hinge loss): A_i iid N(0,1), planted x* with values +-U(1,2),
    labels b_k = +1 if a_k^T x* + N(0, noise^2) >= 0 else -1."""
    rows = m_per if isinstance(m_per, (list, tuple)) else [m_per] * N
    supp, val = linear_model(seed, n, k_true)
    x_true = np.zeros(n)
    x_true[supp] = val
    A_out, b_out = [], []
    for i, m in enumerate(rows):
        G = normal_matrix(seed, S_A + i, m, n)
        if dtype == "f64":
            Ai, Aval = G, G
        else:
            A32 = to_f32(G)
            del G
            Ai = A32 if dtype == "f32" else f32_to_bf16_bits(A32)
            Aval = A32
        score = sparse_predict(Aval, supp, val) + noise * normal_vector(seed, S_LABEL + i, m)
        A_out.append(Ai)
        b_out.append(np.where(score >= 0, 1.0, -1.0))
    return Workload(name=name, loss=LOSS_HINGE, A=A_out, b=b_out, n=n, kappa=kappa,
                    n_blocks=n_blocks, dtype=dtype, x_true=x_true, max_iters=max_iters,
                    inner_iters=inner_iters, rho_c=rho, rho_b=0.5 * rho, rho_l=rho, gamma=gamma,
                    meta=dict(seed=seed, noise=noise))


def softmax_workload(seed: int, N: int, m_per, n: int, C: int, kappa: int, k_true: int,
                     n_blocks: int, dtype: str = "f32", max_iters: int = 100,
                     inner_iters: int = 5, rho: float = 1.0, gamma: float = 10.0,
                     name: str = "softmax") -> Workload:
    """Sparse softmax regression: rows N(0, I), planted W* (n x C) with k_true
    nonzero rows of N(0,1) entries, class y_k = argmax_c (a_k^T W*)_c + Gumbel."""
    rows = m_per if isinstance(m_per, (list, tuple)) else [m_per] * N
    supp = planted_support(seed, n, k_true)
    W = np.zeros((n, C))
    W[supp, :] = normal_matrix(seed, S_VALUES, k_true, C)
    A_out, b_out = [], []
    for i, m in enumerate(rows):
        G = normal_matrix(seed, S_A + i, m, n)
        if dtype == "f64":
            Ai, Aval = G, G
        else:
            A32 = to_f32(G)
            del G
            Ai = A32 if dtype == "f32" else f32_to_bf16_bits(A32)
            Aval = A32
        scores = widen(Aval)[:, supp] @ W[supp, :]
        Uu = np.empty((m, C))
        for c in range(C):
            Uu[:, c] = uniform_vector(seed, S_LABEL + i, m, row=c + 1)
        gumbel = -np.log(-np.log(Uu))
        y = np.argmax(scores + gumbel, axis=1).astype(np.int32)
        A_out.append(Ai)
        b_out.append(y)
    return Workload(name=name, loss=LOSS_SOFTMAX, A=A_out, b=b_out, n=n, kappa=kappa,
                    n_blocks=n_blocks, n_classes=C, dtype=dtype, x_true=W, max_iters=max_iters,
                    inner_iters=inner_iters, rho_c=rho, rho_b=0.5 * rho, rho_l=rho, gamma=gamma,
                    meta=dict(seed=seed))


# ------------------------------------------------------------ named workloads
def config0(seed: int = 0) -> Workload:
    """Plain sparse linear regression, FP64: 4 partitions of 500 x 200, kappa = 10,
    2 feature blocks, rho = 1, 200 iterations."""
    return linear_workload(seed, N=4, m_per=500, n=200, kappa=10, k_true=10, noise=0.01,
                           n_blocks=2, dtype="f64", max_iters=200, inner_iters=5,
                           name="slinr_4x500x200_f64")


def config1(seed: int = 1, N: int = 8, m_per: int = 50000, n: int = 5000, kappa: int = 50,
            n_blocks: int = 4, max_iters: int = 100) -> Workload:
    """Plain sparse logistic regression, FP32: 8 partitions of 50,000 x 5,000 with
    Toeplitz row covariance 0.3^|i-j|, planted 50-sparse N(0,1) model, kappa = 50,
    4 feature blocks, 100 iterations.  Smaller shapes of the same recipe are used
    as parity cases."""
    return logistic_workload(seed, N=N, m_per=m_per, n=n, kappa=kappa, k_true=kappa,
                             n_blocks=n_blocks, dtype="f32", max_iters=max_iters,
                             inner_iters=5, name="slogr_%dx%dx%d_f32" % (N, m_per, n))


def config2(seed: int = 2, N: int = 16, m_per: int = 100000, n: int = 10000, kappa: int = 100,
            dtype: str = "bf16", max_iters: int = 100) -> Workload:
    """Precision form: sparse linear regression with unit-norm columns per
    partition, planted 100-sparse +-U(1,2) model, noise 0.05, kappa = 100,
    4 feature blocks; A stored as BF16 (or the canonical FP32 it was rounded from)."""
    return linear_workload(seed, N=N, m_per=m_per, n=n, kappa=kappa, k_true=kappa, noise=0.05,
                           n_blocks=4, dtype=dtype, normalize=True, max_iters=max_iters,
                           inner_iters=5, name="slinr_%dx%dx%d_%s" % (N, m_per, n, dtype))


def instance_sizes(seed: int, count: int, m_lo=500, m_hi=20000, n_lo=50, n_hi=2000):
    """Log-uniform (m, n) per instance."""
    um = uniform_vector(seed, S_SIZES, count, row=0)
    un = uniform_vector(seed, S_SIZES, count, row=1)
    m = np.rint(np.exp(np.log(m_lo) + um * (np.log(m_hi) - np.log(m_lo)))).astype(np.int64)
    n = np.rint(np.exp(np.log(n_lo) + un * (np.log(n_hi) - np.log(n_lo)))).astype(np.int64)
    return m, n


def batched_instance(r: int, m: int, n: int, base_seed: int = 3000, max_iters: int = 100,
                     dtype: str = "f32") -> Workload:
    """Instance r of the batched workload: even r squared loss (linear recipe),
    odd r logistic (AR(1) recipe); 4 partitions, 2 feature blocks,
    kappa = max(5, n // 20)."""
    kappa = max(5, n // 20)
    rows = split_rows(m, 4)
    if r % 2 == 0:
        return linear_workload(base_seed + r, N=4, m_per=rows, n=n, kappa=kappa, k_true=kappa,
                               noise=0.01, n_blocks=2, dtype=dtype, max_iters=max_iters,
                               name="inst%d_slinr_%dx%d" % (r, m, n))
    return logistic_workload(base_seed + r, N=4, m_per=rows, n=n, kappa=kappa, k_true=kappa,
                             n_blocks=2, dtype=dtype, max_iters=max_iters,
                             name="inst%d_slogr_%dx%d" % (r, m, n))


def config3_sizes(seed: int = 3, count: int = 512):
    return instance_sizes(seed, count)


def softmax_request(seed: int, m: int = 20000, n: int = 1000, C: int = 10, kappa: int = 30,
                    max_iters: int = 100, dtype: str = "f32") -> Workload:
    """Serving softmax request: 4 partitions of m/4 rows, n features, C classes,
    planted 30-row-sparse W*, kappa = 30 rows, 2 feature blocks."""
    return softmax_workload(seed, N=4, m_per=split_rows(m, 4), n=n, C=C, kappa=kappa,
                            k_true=kappa, n_blocks=2, dtype=dtype, max_iters=max_iters,
                            name="ssr_%dx%dx%d" % (m, n, C))
