"""FP64 CPU oracle for the pre-packed TSMM -- test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The product library never does, and this package imports
nothing from the product package: the two share no code.

The arithmetic lives in ``tsmm_oracle.c`` (plain C99 loops in binary64, one
rounding per operation, built with ``-ffp-contract=off``).  This module only
builds and loads that library and marshals numpy arrays into it:

* :func:`gemm_n` -- C = alpha*A*B + beta*C0, A m x k, B k x n (AutoTSMM
  Sec. I, Eq. (1); Algorithm 1 output);
* :func:`gemm_t` -- C = alpha*A^T*B + beta*C0, A K x m, B K x n (the same
  definition with A transposed, the reduction shape over a long shared
  dimension);
* :func:`split_bf16` -- binary32 -> bfloat16 residual split, bit-level
  round-to-nearest-even;
* :func:`column_scale_exp` -- power-of-two exponent per column;
* :func:`pack_a` -- Algorithm 1's PACKA scaling of A by alpha, followed (in
  the split-bf16 modes) by the residual split.

Floating inputs of narrower types are widened to binary64 exactly before
the call (bfloat16 values arrive as their uint16 bit patterns).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsmm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-std=c99", "-O3", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra"]

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, dbl, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        for name in ("oracle_gemm_n_f64", "oracle_gemm_t_f64"):
            f = getattr(lib, name)
            f.argtypes = [i64, i64, i64, dbl, vp, vp, dbl, vp, vp, ci]
            f.restype = ci
        lib.oracle_split_bf16.argtypes = [vp, i64, ci, vp]
        lib.oracle_split_bf16.restype = ci
        lib.oracle_column_scale_exp.argtypes = [vp, i64, i64, vp]
        lib.oracle_column_scale_exp.restype = ci
        _lib = lib
    return _lib


def bf16_bits_to_f64(bits: np.ndarray) -> np.ndarray:
    """Exact widening of bfloat16 bit patterns (uint16) to binary64."""
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def _as_f64(x):
    if x is None:
        return None
    x = np.asarray(x)
    if x.dtype == np.uint16:  # bfloat16 bit patterns
        return bf16_bits_to_f64(x)
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(threads):
    if threads is None:
        return len(os.sched_getaffinity(0))
    return int(threads)


def gemm_n(A, B, C0=None, alpha=1.0, beta=0.0, threads=None) -> np.ndarray:
    """C = alpha*A*B + beta*C0 in binary64; A is m x k, B is k x n."""
    A, B, C0 = _as_f64(A), _as_f64(B), _as_f64(C0)
    m, k = A.shape
    k2, n = B.shape
    if k2 != k:
        raise ValueError("inner dimensions differ: %d vs %d" % (k, k2))
    if beta != 0.0 and (C0 is None or C0.shape != (m, n)):
        raise ValueError("beta != 0 needs C0 of shape (m, n)")
    C = np.empty((m, n), dtype=np.float64)
    rc = _load().oracle_gemm_n_f64(m, n, k, float(alpha), _ptr(A), _ptr(B), float(beta),
                                   _ptr(C0 if beta != 0.0 else None), _ptr(C), _threads(threads))
    if rc != 0:
        raise ValueError("oracle_gemm_n_f64 rejected its arguments")
    return C


def gemm_t(A, B, C0=None, alpha=1.0, beta=0.0, threads=None) -> np.ndarray:
    """C = alpha*A^T*B + beta*C0 in binary64; A is K x m, B is K x n."""
    A, B, C0 = _as_f64(A), _as_f64(B), _as_f64(C0)
    K, m = A.shape
    K2, n = B.shape
    if K2 != K:
        raise ValueError("shared dimensions differ: %d vs %d" % (K, K2))
    if beta != 0.0 and (C0 is None or C0.shape != (m, n)):
        raise ValueError("beta != 0 needs C0 of shape (m, n)")
    C = np.empty((m, n), dtype=np.float64)
    rc = _load().oracle_gemm_t_f64(m, n, K, float(alpha), _ptr(A), _ptr(B), float(beta),
                                   _ptr(C0 if beta != 0.0 else None), _ptr(C), _threads(threads))
    if rc != 0:
        raise ValueError("oracle_gemm_t_f64 rejected its arguments")
    return C


def split_bf16(x, terms: int) -> np.ndarray:
    """Residual split of binary32 values into `terms` bfloat16 planes.

    Returns uint16 bit patterns of shape (terms,) + x.shape.
    """
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty((terms,) + x.shape, dtype=np.uint16)
    rc = _load().oracle_split_bf16(_ptr(x), x.size, int(terms), _ptr(out))
    if rc != 0:
        raise ValueError("oracle_split_bf16 rejected its arguments")
    return out


def pack_a(A, alpha: float, terms: int = 0) -> np.ndarray:
    """Algorithm 1, PACKA: A scaled by alpha as it is packed.

    Each product alpha*a is taken in binary64 and rounded once to A's type
    (binary64 or binary32).  terms = 0 returns the scaled matrix; terms = 2
    or 3 (binary32 A, the split-bf16 modes) returns its bfloat16 residual
    split: uint16 planes of shape (terms,) + A.shape.
    """
    A = np.asarray(A)
    if A.dtype == np.float64:
        scaled = np.float64(alpha) * A
    elif A.dtype == np.float32:
        scaled = (np.float64(alpha) * A.astype(np.float64)).astype(np.float32)
    else:
        raise TypeError("pack_a takes binary64 or binary32 A")
    if terms == 0:
        return scaled
    if A.dtype != np.float32:
        raise TypeError("the split takes binary32 A")
    return split_bf16(scaled, terms)


def column_scale_exp(B) -> np.ndarray:
    """Per-column exponent e_j with 1 <= max_i |B[i, j]| * 2**-e_j < 2."""
    B = np.ascontiguousarray(B, dtype=np.float32)
    k, n = B.shape
    e = np.empty(n, dtype=np.int32)
    rc = _load().oracle_column_scale_exp(_ptr(B), k, n, _ptr(e))
    if rc != 0:
        raise ValueError("oracle_column_scale_exp rejected its arguments")
    return e


def normwise_rel_err(C_hat, C_ref) -> float:
    """Frobenius-norm relative error ||C_hat - C_ref|| / ||C_ref|| in binary64.

    A reference of norm zero requires C_hat to be exactly zero (returns 0.0
    or inf).
    """
    Ch = _as_f64(C_hat)
    Cr = _as_f64(C_ref)
    d = np.linalg.norm((Ch - Cr).ravel())
    r = np.linalg.norm(Cr.ravel())
    if r == 0.0:
        return 0.0 if d == 0.0 else float("inf")
    return float(d / r)
