"""ctypes wrapper of the C oracle ``fht_oracle.c`` (test infrastructure only).

``build()`` compiles it with gcc and OpenMP into ``oracle/liboracle.so``.  The
functions mirror ``fht_oracle.py`` and return NumPy arrays; the outputs of the
four quadrants come back as a list in q order (V+, V-, H+, H-).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fht_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle; returns the path of the shared library."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fopenmp", "-shared", "-fPIC",
                        "-Wall", "-Wextra", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        p, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        lib.orc_patterns.argtypes = [i32, i32, p]
        lib.orc_nonleaf_width_sum.argtypes = [i32, i32]
        lib.orc_nonleaf_width_sum.restype = i64
        lib.orc_hough_u8.argtypes = [p, i32, i32, i32, p]
        lib.orc_hough_f64.argtypes = [p, i32, i32, i32, p, p]
        lib.orc_hough_sample_u8.argtypes = [p, i32, i32, i32, i64, p, p, p, p]
        lib.orc_hough_sample_f64.argtypes = [p, i32, i32, i32, i64, p, p, p, p, p]
        lib.orc_error_numerators.argtypes = [i32, i32, p]
        lib.orc_num_threads.argtypes = []
        lib.orc_alg1_u8_batch.argtypes = [p, i32, i32, i32, i32, p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dims(R: int, C: int):
    return [(R, C), (R, C), (C, R), (C, R)]


def patterns(n: int, split: int) -> np.ndarray:
    out = np.empty((n, n), dtype=np.int32)
    if _load().orc_patterns(n, split, _ptr(out)) != 0:
        raise ValueError("orc_patterns failed")
    return out


def nonleaf_width_sum(w: int, split: int) -> int:
    return int(_load().orc_nonleaf_width_sum(w, split))


def hough4_u8(img: np.ndarray, split: int):
    img = np.ascontiguousarray(img, dtype=np.uint8)
    R, C = img.shape
    out = np.empty(4 * R * C, dtype=np.int64)
    if _load().orc_hough_u8(_ptr(img), R, C, split, _ptr(out)) != 0:
        raise ValueError("orc_hough_u8 failed")
    res, off = [], 0
    for W, H in _dims(R, C):
        res.append(out[off:off + W * H].reshape(W, H))
        off += W * H
    return res


def hough4_f64(img: np.ndarray, split: int):
    """Returns (outputs, abs_sums), each a list of four float64 arrays."""
    img = np.ascontiguousarray(img, dtype=np.float64)
    R, C = img.shape
    out = np.empty(4 * R * C, dtype=np.float64)
    ab = np.empty_like(out)
    if _load().orc_hough_f64(_ptr(img), R, C, split, _ptr(out), _ptr(ab)) != 0:
        raise ValueError("orc_hough_f64 failed")
    res, absr, off = [], [], 0
    for W, H in _dims(R, C):
        res.append(out[off:off + W * H].reshape(W, H))
        absr.append(ab[off:off + W * H].reshape(W, H))
        off += W * H
    return res, absr


def sample_u8(img: np.ndarray, split: int, q, t, s) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    q, t, s = (np.ascontiguousarray(v, dtype=np.int32) for v in (q, t, s))
    out = np.empty(q.shape[0], dtype=np.int64)
    R, C = img.shape
    if _load().orc_hough_sample_u8(_ptr(img), R, C, split, q.shape[0], _ptr(q), _ptr(t),
                                   _ptr(s), _ptr(out)) != 0:
        raise ValueError("orc_hough_sample_u8 failed")
    return out


def sample_f64(img: np.ndarray, split: int, q, t, s):
    img = np.ascontiguousarray(img, dtype=np.float64)
    q, t, s = (np.ascontiguousarray(v, dtype=np.int32) for v in (q, t, s))
    out = np.empty(q.shape[0], dtype=np.float64)
    ab = np.empty_like(out)
    R, C = img.shape
    if _load().orc_hough_sample_f64(_ptr(img), R, C, split, q.shape[0], _ptr(q), _ptr(t),
                                    _ptr(s), _ptr(out), _ptr(ab)) != 0:
        raise ValueError("orc_hough_sample_f64 failed")
    return out, ab


def error_numerators(nmax: int, split: int) -> np.ndarray:
    """num[n] with E(n) = num[n] / (n - 1) for n in [2, nmax] (num[0] = num[1] = 0)."""
    num = np.zeros(nmax + 1, dtype=np.int64)
    if _load().orc_error_numerators(nmax, split, _ptr(num)) != 0:
        raise ValueError("orc_error_numerators failed")
    return num


def alg1_u8_batch(imgs: np.ndarray, split: int) -> np.ndarray:
    """Alg. 1's recursion (C, OpenMP over images and quadrants) for n uint8
    images of one shape: returns (n, 4 R C) int32, quadrants in q order."""
    imgs = np.ascontiguousarray(imgs, dtype=np.uint8)
    if imgs.ndim == 2:
        imgs = imgs[None]
    n, R, C = imgs.shape
    out = np.empty((n, 4 * R * C), dtype=np.int32)
    if _load().orc_alg1_u8_batch(_ptr(imgs), n, R, C, split, _ptr(out)) != 0:
        raise ValueError("orc_alg1_u8_batch failed")
    return out


def num_threads() -> int:
    """OpenMP threads the C oracle runs on."""
    return int(_load().orc_num_threads())
