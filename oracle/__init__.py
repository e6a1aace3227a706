"""CPU oracle for the GF(2) Toeplitz hash.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library and does not import it; both sides are fed inputs by
``synth`` (which holds no hash arithmetic).

Definition followed (paper section 2.1, Eq. 1 with the relabelling below, and
section 2.3, steps 1-2, in the column-vector orientation ``y = T x``): for a
seed ``s`` of ``n+m-1`` bits the m x n Toeplitz matrix is

    T[i][j] = s[i - j + n - 1]

and ``y_i = XOR_j T[i][j] AND x_j``.  Readings of the paper that fix this
(section 3, step 3 takes outputs "n .. n+k-1" of the product, read 1-based with
k = l = m; Eq. 1 names the first column t_0..t_{n-1} and the first row
t_0, t_n, ..., t_{2n-2}) are recorded with the tests that pin them.

Three implementations of the same definition:

* ``toeplitz_matrix`` / ``hash_matrix`` (O1): build T explicitly, numpy
  matrix-vector product mod 2.  Tiny sizes only.
* ``hash_bits`` (O2, C): double loop over (i, j), one bit at a time.
* ``hash_words`` (O3, C): the same sum 64 key bits per step, multi-threaded.
* ``hash_select``: selected output bits (spot checks at any size).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "toeplitz_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle into oracle/liboracle.so with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        lib.oracle_hash_bits.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p]
        lib.oracle_hash_bits.restype = None
        lib.oracle_hash_words.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p,
                                          ctypes.c_int]
        lib.oracle_hash_words.restype = ctypes.c_int
        lib.oracle_hash_select.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint64, u64p, u64p,
                                           ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint8)]
        lib.oracle_hash_select.restype = ctypes.c_int
        _lib = lib
    return _lib


def _words(a: np.ndarray, nbits: int) -> np.ndarray:
    need = (nbits + 63) // 64
    a = np.ascontiguousarray(a, dtype=np.uint64)
    if a.size < need:
        raise ValueError(f"bit array holds {a.size} words, needs {need}")
    return a


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _check(n: int, m: int):
    if n < 1 or m < 1:
        raise ValueError("n and m must be >= 1")


# ---------------------------------------------------------------- O1 (numpy)

def toeplitz_matrix(seed_bits: np.ndarray, n: int, m: int) -> np.ndarray:
    """Explicit m x n matrix with T[i][j] = s[i - j + n - 1] (0/1 uint8)."""
    s = np.asarray(seed_bits, dtype=np.uint8)
    if s.size < n + m - 1:
        raise ValueError("seed shorter than n+m-1 bits")
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    return s[i - j + n - 1]


def hash_matrix(seed_bits: np.ndarray, n: int, m: int, key_bits: np.ndarray) -> np.ndarray:
    """O1: y = T x mod 2 on unpacked 0/1 arrays.  Returns 0/1 uint8 of length m."""
    _check(n, m)
    T = toeplitz_matrix(seed_bits, n, m).astype(np.int64)
    x = np.asarray(key_bits, dtype=np.int64)[:n]
    return ((T @ x) % 2).astype(np.uint8)


# ----------------------------------------------------------------- O2 / O3 (C)

def hash_bits(seed: np.ndarray, n: int, m: int, key: np.ndarray) -> np.ndarray:
    """O2 on packed words.  Returns packed output words (tail bits zero)."""
    _check(n, m)
    lib = _load()
    s = _words(seed, n + m - 1)
    k = _words(key, n)
    out = np.zeros((m + 63) // 64, dtype=np.uint64)
    lib.oracle_hash_bits(_p(s), n, m, _p(k), _p(out))
    return out


def hash_words(seed: np.ndarray, n: int, m: int, key: np.ndarray, threads: int | None = None) -> np.ndarray:
    """O3 on packed words, multi-threaded.  Returns packed output words."""
    _check(n, m)
    lib = _load()
    s = _words(seed, n + m - 1)
    k = _words(key, n)
    out = np.zeros((m + 63) // 64, dtype=np.uint64)
    if threads is None:
        threads = default_threads()
    if lib.oracle_hash_words(_p(s), n, m, _p(k), _p(out), int(threads)) != 0:
        raise MemoryError("oracle_hash_words: allocation failed")
    return out


def hash_select(seed: np.ndarray, n: int, m: int, key: np.ndarray, idx) -> np.ndarray:
    """Selected output bits y_i for i in idx (0/1 uint8)."""
    _check(n, m)
    lib = _load()
    s = _words(seed, n + m - 1)
    k = _words(key, n)
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    out = np.zeros(idx.size, dtype=np.uint8)
    rc = lib.oracle_hash_select(_p(s), n, m, _p(k), _p(idx), idx.size,
                                out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)))
    if rc != 0:
        raise MemoryError("oracle_hash_select: allocation failed")
    return out


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return max(1, os.cpu_count() or 1)
