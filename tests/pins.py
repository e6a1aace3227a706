"""Checks that pin a Toeplitz-hash implementation to facts fixed by the paper
and by mathematics, independently of any implementation under test.

Each check takes ``H(seed_bits, n, m, key_bits) -> y_bits`` on unpacked 0/1
uint8 arrays and raises AssertionError when the candidate disagrees.  They are
run against every oracle implementation, and against deliberately broken
copies of the oracle to show that a plausible mistake fails at least one.

What fixes each check:

* ``pin_eq1_structure``: paper Eq. 1 writes the square matrix with first column
  t_0 .. t_{n-1} and first row t_0, t_n, t_{n+1}, ..., t_{2n-2}, lower part
  T[i][j] = t_{i-j}, upper part T[i][j] = t_{j-i+n-1}.  The seed ordering used
  here stores t_d at s[n-1+d] (d >= 0) and t_{n-1+e} at s[n-1-e] (e >= 1); the
  check rebuilds Eq. 1 from the t labels and compares column by column through
  unit keys.
* ``pin_convolve``: section 3, step 3 computes the hash as a polynomial
  product (FFT, product, inverse FFT) and keeps outputs n .. n+l-1 (1-based),
  then reduces mod 2 (Eq. 7).  np.convolve is the library convolution; its
  window [n-1, n+m-1) mod 2 must equal the hash.
* ``pin_clmul``: the same window of the carry-less (GF(2)[z]) product of the
  two bit strings, computed with Python integer shifts and XORs.
* ``pin_closed_forms``: zero key -> 0; all-ones seed -> every output is the
  parity of the key's weight; all-ones key -> y_i is the parity of
  s[i .. i+n-1]; unit key e_j -> column j = s[n-1-j .. n-1-j+m).
* ``pin_linearity``: T(x xor z) = Tx xor Tz.
* ``pin_block_split``: paper Eq. 4-7 (split the key into blocks, hash each
  block with its slice of T, XOR the intermediate keys) and the output split
  (section 3 allows splitting the matrix columns as well).
* ``pin_universal``: every nonzero difference d is mapped to 0 by exactly
  2^(n-1) of the 2^(n+m-1) seeds (collision probability exactly 2^-m for the
  full Toeplitz family; section 2.1 quotes a looser n*2^(-m+1)).
"""
from __future__ import annotations

import itertools

import numpy as np


def _rand_bits(rng, k):
    return rng.integers(0, 2, size=k, dtype=np.uint8)


def _eq(a, b, what):
    a = np.asarray(a, dtype=np.uint8)
    b = np.asarray(b, dtype=np.uint8)
    if a.shape != b.shape or not np.array_equal(a, b):
        bad = np.flatnonzero(a != b)[:8] if a.shape == b.shape else "shape"
        raise AssertionError(f"{what}: mismatch at {bad}")


def pin_eq1_structure(H, sizes=(1, 2, 3, 5, 8)):
    rng = np.random.default_rng(101)
    for n in sizes:
        t = _rand_bits(rng, 2 * n - 1)          # t_0 .. t_{2n-2}
        T = np.zeros((n, n), np.uint8)
        for i in range(n):
            for j in range(n):
                T[i, j] = t[i - j] if i >= j else t[j - i + n - 1]
        # Eq. 1: first column and first row as printed
        assert list(T[:, 0]) == list(t[:n])
        assert list(T[0, 1:]) == list(t[n:2 * n - 1])
        s = np.zeros(2 * n - 1, np.uint8)
        for d in range(n):
            s[n - 1 + d] = t[d]
        for e in range(1, n):
            s[n - 1 - e] = t[n - 1 + e]
        for j in range(n):
            e_j = np.zeros(n, np.uint8)
            e_j[j] = 1
            _eq(H(s, n, n, e_j), T[:, j], f"Eq.1 column {j} (n={n})")


def pin_convolve(H, shapes=((1, 1), (1, 7), (7, 1), (5, 3), (64, 64), (65, 63), (100, 37),
                            (37, 100), (129, 257), (300, 1))):
    rng = np.random.default_rng(202)
    for n, m in shapes:
        s = _rand_bits(rng, n + m - 1)
        x = _rand_bits(rng, n)
        ref = (np.convolve(s.astype(np.int64), x.astype(np.int64))[n - 1:n + m - 1] % 2)
        _eq(H(s, n, m, x), ref.astype(np.uint8), f"np.convolve window n={n} m={m}")


def _clmul(a: int, b: int) -> int:
    r = 0
    while b:
        low = b & -b
        r ^= a << (low.bit_length() - 1)
        b ^= low
    return r


def pin_clmul(H, shapes=((3, 4), (64, 1), (70, 70), (200, 50), (33, 190))):
    rng = np.random.default_rng(303)
    for n, m in shapes:
        s = _rand_bits(rng, n + m - 1)
        x = _rand_bits(rng, n)
        S = sum(int(b) << k for k, b in enumerate(s))
        X = sum(int(b) << k for k, b in enumerate(x))
        P = _clmul(S, X)
        ref = np.array([(P >> (i + n - 1)) & 1 for i in range(m)], np.uint8)
        _eq(H(s, n, m, x), ref, f"carry-less product window n={n} m={m}")


def pin_closed_forms(H, shapes=((1, 1), (9, 4), (64, 20), (77, 130))):
    rng = np.random.default_rng(404)
    for n, m in shapes:
        s = _rand_bits(rng, n + m - 1)
        x = _rand_bits(rng, n)
        _eq(H(s, n, m, np.zeros(n, np.uint8)), np.zeros(m, np.uint8), "zero key")
        par = int(x.sum()) & 1
        _eq(H(np.ones(n + m - 1, np.uint8), n, m, x), np.full(m, par, np.uint8), "all-ones seed")
        ref = np.array([int(s[i:i + n].sum()) & 1 for i in range(m)], np.uint8)
        _eq(H(s, n, m, np.ones(n, np.uint8)), ref, "all-ones key")
        for j in sorted({0, n // 2, n - 1}):
            e = np.zeros(n, np.uint8)
            e[j] = 1
            _eq(H(s, n, m, e), s[n - 1 - j:n - 1 - j + m], f"unit key e_{j}")


def pin_linearity(H, shapes=((13, 7), (64, 64), (150, 90))):
    rng = np.random.default_rng(505)
    for n, m in shapes:
        s = _rand_bits(rng, n + m - 1)
        x = _rand_bits(rng, n)
        z = _rand_bits(rng, n)
        _eq(H(s, n, m, x ^ z), H(s, n, m, x) ^ H(s, n, m, z), f"linearity n={n} m={m}")


def pin_block_split(H, shapes=((10, 4), (100, 30), (129, 65))):
    rng = np.random.default_rng(606)
    for n, m in shapes:
        s = _rand_bits(rng, n + m - 1)
        x = _rand_bits(rng, n)
        full = H(s, n, m, x)
        for n1 in sorted({1, n // 3, n - 1}):
            n2 = n - n1
            a = H(s[n2:n2 + n1 + m - 1], n1, m, x[:n1])
            b = H(s[:n2 + m - 1], n2, m, x[n1:])
            _eq(full, a ^ b, f"Eq.4-7 key split n1={n1} (n={n}, m={m})")
        for lo, hi in [(0, 1), (1, m), (m // 2, m)]:
            if hi <= lo:
                continue
            part = H(s[lo:lo + n + (hi - lo) - 1], n, hi - lo, x)
            _eq(full[lo:hi], part, f"output split [{lo},{hi})")


def pin_universal(H, shapes=((3, 2), (4, 3), (2, 4))):
    for n, m in shapes:
        L = n + m - 1
        seeds = [np.array(bits, np.uint8) for bits in itertools.product((0, 1), repeat=L)]
        for dv in itertools.product((0, 1), repeat=n):
            d = np.array(dv, np.uint8)
            if not d.any():
                continue
            zeros = sum(1 for s in seeds if not H(s, n, m, d).any())
            assert zeros == 2 ** (L - m), f"universality n={n} m={m} d={dv}: {zeros}"


ALL_PINS = [pin_eq1_structure, pin_convolve, pin_clmul, pin_closed_forms, pin_linearity,
            pin_block_split, pin_universal]
