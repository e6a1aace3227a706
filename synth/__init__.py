"""Seeded synthetic inputs for the Toeplitz-hash path.

This module only draws bits.  It holds none of the hash arithmetic, so the
CPU oracle and the GPU path can both be fed from it without sharing any
computation.

Bit format (used everywhere in this repository): a bit string of length
``nbits`` is a little-endian array of ``uint64`` words, LSB-first, i.e. bit
``k`` is ``(w[k >> 6] >> (k & 63)) & 1``.  Bits at positions ``>= nbits`` in
the last word are zero.

Generator: NumPy's ``default_rng(seed)`` (PCG64).  Each random word is one
draw of ``Generator.integers(0, 2**64, dtype=uint64)``; i.i.d. uniform bits.
The paper's keys are reconciled CV-QKD keys that are not public, so i.i.d.
uniform bits stand in for them (the distribution does not change the cost of
the exact path; it does change floating-point error, which is exercised
separately with the structured patterns below).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "words_for", "mask_tail", "gen_bits", "bits_to_array", "array_to_bits",
    "get_bit", "Problem", "single_config", "batch_jobs", "serving_stream",
    "pattern_bits", "CONFIGS",
]


def words_for(nbits: int) -> int:
    return (int(nbits) + 63) // 64


def mask_tail(words: np.ndarray, nbits: int) -> np.ndarray:
    """Zero the bits at positions >= nbits (in place) and return the array."""
    nw = words_for(nbits)
    if nw and nbits % 64:
        words[nw - 1] &= np.uint64((1 << (nbits % 64)) - 1)
    return words


def gen_bits(rng: np.random.Generator, nbits: int) -> np.ndarray:
    """``nbits`` i.i.d. uniform bits packed LSB-first into uint64 words."""
    nw = words_for(nbits)
    w = rng.integers(0, 2**64, size=nw, dtype=np.uint64)
    return mask_tail(w, nbits)


def bits_to_array(words: np.ndarray, nbits: int) -> np.ndarray:
    """Unpack to a uint8 array of 0/1 values (length nbits)."""
    b = np.unpackbits(np.ascontiguousarray(words, dtype="<u8").view(np.uint8),
                      bitorder="little")
    return b[:nbits].copy()


def array_to_bits(bits: np.ndarray) -> np.ndarray:
    """Pack a 0/1 array into uint64 words (LSB-first)."""
    bits = np.asarray(bits, dtype=np.uint8) & 1
    nb = bits.size
    nw = words_for(nb)
    pad = np.zeros(nw * 64, dtype=np.uint8)
    pad[:nb] = bits
    return np.packbits(pad, bitorder="little").view("<u8").astype(np.uint64)


def get_bit(words: np.ndarray, k: int) -> int:
    return int((int(words[k >> 6]) >> (k & 63)) & 1)


@dataclass
class Problem:
    """One hash job: seed has n+m-1 bits, key n bits, output m bits."""
    n: int
    m: int
    seed: np.ndarray
    key: np.ndarray
    name: str = ""


# The five workloads the measurements are quoted on.
CONFIGS = {
    "c1": dict(rng_seed=0, n=131072, m=16384),
    "c2": dict(rng_seed=1, n=1_000_000, m=200_000),
    "c3": dict(rng_seed=2, n=12_345_679, m=1_234_567),
}


def single_config(name: str) -> Problem:
    """Seed bits are drawn first, then key bits, from default_rng(rng_seed)."""
    c = CONFIGS[name]
    rng = np.random.default_rng(c["rng_seed"])
    n, m = c["n"], c["m"]
    seed = gen_bits(rng, n + m - 1)
    key = gen_bits(rng, n)
    return Problem(n, m, seed, key, name)


def random_problem(rng: np.random.Generator, n: int, m: int, name: str = "") -> Problem:
    seed = gen_bits(rng, n + m - 1)
    key = gen_bits(rng, n)
    return Problem(n, m, seed, key, name)


def batch_shapes(count: int = 64, rng_seed: int = 3, nlo: float = 1e5, nhi: float = 1e7,
                 rlo: float = 0.05, rhi: float = 0.5):
    """Job sizes: n log-uniform in [nlo, nhi], m/n uniform in [rlo, rhi]."""
    rng = np.random.default_rng(rng_seed)
    u = rng.random(count)
    v = rng.random(count)
    a, b = math.log10(nlo), math.log10(nhi)
    ns = np.floor(10.0 ** (a + (b - a) * u)).astype(np.int64)
    ms = np.maximum(1, np.floor(ns * (rlo + (rhi - rlo) * v))).astype(np.int64)
    return rng, [(int(n), int(m)) for n, m in zip(ns, ms)]


def batch_jobs(count: int = 64, rng_seed: int = 3, **kw) -> list[Problem]:
    """Batch workload: ``count`` independent jobs with their own seeds/keys."""
    rng, shapes = batch_shapes(count, rng_seed, **kw)
    return [random_problem(rng, n, m, f"job{i}") for i, (n, m) in enumerate(shapes)]


def serving_stream(count: int = 2000, rng_seed: int = 4, n_seeds: int = 8,
                   seed_bits: int = 150_000_000, nlo: float = 1e5, nhi: float = 1e8,
                   rlo: float = 0.02, rhi: float = 0.5, rate_hz: float = 100.0,
                   make_seeds: bool = True):
    """Serving workload.

    Returns (seeds, requests) where seeds is a list of ``n_seeds`` resident seed
    bit strings of ``seed_bits`` bits, and each request is a dict with
    ``t`` (arrival time, s; exponential inter-arrivals at ``rate_hz``),
    ``n``, ``m`` (n log-uniform, m/n uniform, n+m-1 <= seed_bits),
    ``seed_id`` and ``key_seed`` (the RNG seed its key bits are drawn from with
    ``request_key``).
    """
    rng = np.random.default_rng(rng_seed)
    seeds = [gen_bits(rng, seed_bits) for _ in range(n_seeds)] if make_seeds else None
    a, b = math.log10(nlo), math.log10(nhi)
    reqs = []
    t = 0.0
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_hz))
        n = int(math.floor(10.0 ** (a + (b - a) * float(rng.random()))))
        m = int(math.floor(n * (rlo + (rhi - rlo) * float(rng.random()))))
        m = max(1, min(m, seed_bits - n + 1))
        reqs.append(dict(t=t, n=n, m=m, seed_id=int(rng.integers(0, n_seeds)),
                         key_seed=int(rng.integers(0, 2**31))))
    return seeds, reqs


def request_key(req) -> np.ndarray:
    return gen_bits(np.random.default_rng(req["key_seed"]), req["n"])


def pattern_bits(kind: str, nbits: int, rng: np.random.Generator | None = None) -> np.ndarray:
    """Structured bit strings used to stress floating-point error.

    ``ones``: all ones.  ``zeros``: all zeros.  ``period3``: 1,1,0 repeated.
    ``period2``: 1,0 repeated.  ``sparse``: one set bit every 4097 positions.
    ``block``: first half ones, second half zeros.
    """
    idx = np.arange(nbits, dtype=np.int64)
    if kind == "ones":
        b = np.ones(nbits, np.uint8)
    elif kind == "zeros":
        b = np.zeros(nbits, np.uint8)
    elif kind == "period3":
        b = (idx % 3 != 2).astype(np.uint8)
    elif kind == "period2":
        b = (idx % 2 == 0).astype(np.uint8)
    elif kind == "sparse":
        b = (idx % 4097 == 0).astype(np.uint8)
    elif kind == "block":
        b = (idx < nbits // 2).astype(np.uint8)
    else:
        raise ValueError(kind)
    return array_to_bits(b)
