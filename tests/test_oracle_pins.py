"""The oracle pinned to the paper and to mathematics (CPU only)."""
import numpy as np
import pytest

import oracle
import synth
from pins import ALL_PINS


def _o1(s, n, m, x):
    return oracle.hash_matrix(s, n, m, x)


def _packed(fn):
    def H(s, n, m, x):
        out = fn(synth.array_to_bits(s), n, m, synth.array_to_bits(x))
        return synth.bits_to_array(out, m)
    return H


def _o3_1(seed, n, m, key):
    return oracle.hash_words(seed, n, m, key, threads=1)


def _o3_4(seed, n, m, key):
    return oracle.hash_words(seed, n, m, key, threads=4)


def _sel(seed, n, m, key):
    bits = oracle.hash_select(seed, n, m, key, np.arange(m))
    return synth.array_to_bits(bits)


IMPLS = {
    "O1-matrix": _o1,
    "O2-bits": _packed(oracle.hash_bits),
    "O3-words-1t": _packed(_o3_1),
    "O3-words-4t": _packed(_o3_4),
    "select": _packed(_sel),
}


@pytest.mark.parametrize("impl", list(IMPLS))
@pytest.mark.parametrize("pin", ALL_PINS, ids=[p.__name__ for p in ALL_PINS])
def test_pin(impl, pin):
    pin(IMPLS[impl])


SHAPES = [(1, 1), (1, 200), (200, 1), (63, 65), (64, 64), (65, 63), (127, 129), (640, 64),
          (1000, 333), (333, 1000), (4097, 511), (5000, 5000), (131, 9973)]


@pytest.mark.parametrize("n,m", SHAPES)
def test_oracle_levels_agree(n, m):
    rng = np.random.default_rng(n * 7919 + m)
    p = synth.random_problem(rng, n, m)
    o2 = oracle.hash_bits(p.seed, n, m, p.key)
    o3 = oracle.hash_words(p.seed, n, m, p.key, threads=3)
    assert np.array_equal(o2, o3)
    if n * m <= 2_000_000:
        o1 = oracle.hash_matrix(synth.bits_to_array(p.seed, n + m - 1), n, m,
                                synth.bits_to_array(p.key, n))
        assert np.array_equal(synth.array_to_bits(o1), o2)
    # tail bits beyond m are zero
    if m % 64:
        assert int(o3[-1]) >> (m % 64) == 0


def test_seed_tail_bits_ignored():
    """Bits beyond n+m-1 in the seed's last word and beyond n in the key's are
    not part of the input."""
    rng = np.random.default_rng(9)
    n, m = 70, 30
    p = synth.random_problem(rng, n, m)
    ref = oracle.hash_words(p.seed, n, m, p.key)
    s2 = p.seed.copy()
    s2[-1] |= np.uint64(~((1 << ((n + m - 1) % 64)) - 1) & (2**64 - 1))
    k2 = p.key.copy()
    k2[-1] |= np.uint64(~((1 << (n % 64)) - 1) & (2**64 - 1))
    assert np.array_equal(oracle.hash_words(s2, n, m, k2), ref)
    assert np.array_equal(oracle.hash_bits(s2, n, m, k2), ref)


def test_select_matches_full():
    p = synth.single_config("c1")
    full = oracle.hash_words(p.seed, p.n, p.m, p.key)
    idx = np.array([0, 1, 63, 64, 1000, p.m - 1, p.m + 5])
    sel = oracle.hash_select(p.seed, p.n, p.m, p.key, idx)
    bits = synth.bits_to_array(full, p.m)
    assert list(sel[:-1]) == [int(bits[i]) for i in idx[:-1]]
    assert sel[-1] == 0


def test_invalid_sizes():
    with pytest.raises(ValueError):
        oracle.hash_words(np.zeros(1, np.uint64), 0, 1, np.zeros(1, np.uint64))
    with pytest.raises(ValueError):
        oracle.hash_words(np.zeros(1, np.uint64), 100, 1, np.zeros(1, np.uint64))
