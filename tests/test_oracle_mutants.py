"""Plausible mistakes planted in copies of the oracle (CPU only) must each fail
at least one pin: the pins are strong enough to catch a wrong index, sign,
orientation or window."""
import numpy as np
import pytest

from pins import ALL_PINS


def _mk(index_fn, window=0, rev_key=False):
    def H(s, n, m, x):
        s = np.asarray(s, np.int64)
        x = np.asarray(x, np.int64)[:n]
        if rev_key:
            x = x[::-1]
        i = np.arange(m)[:, None] + window
        j = np.arange(n)[None, :]
        k = index_fn(i, j, n, m)
        ok = (k >= 0) & (k < s.size)
        T = np.where(ok, s[np.clip(k, 0, s.size - 1)], 0)
        return ((T @ x) % 2).astype(np.uint8)
    return H


MUTANTS = {
    "transposed_orientation": _mk(lambda i, j, n, m: j - i + m - 1),
    "off_by_one_up": _mk(lambda i, j, n, m: i - j + n),
    "off_by_one_down": _mk(lambda i, j, n, m: i - j + n - 2),
    "hankel_not_toeplitz": _mk(lambda i, j, n, m: i + j),
    "reversed_key": _mk(lambda i, j, n, m: i - j + n - 1, rev_key=True),
    "window_shift": _mk(lambda i, j, n, m: i - j + n - 1, window=1),
    "zero_based_window": _mk(lambda i, j, n, m: i - j + n - 1, window=-1),
}


def _mutant_and(a_fn):
    # AND instead of XOR accumulation: y = OR of products
    def H(s, n, m, x):
        s = np.asarray(s, np.int64)
        x = np.asarray(x, np.int64)[:n]
        i = np.arange(m)[:, None]
        j = np.arange(n)[None, :]
        T = s[i - j + n - 1]
        return ((T @ x) > 0).astype(np.uint8)
    return H


MUTANTS["or_instead_of_xor"] = _mutant_and(None)


@pytest.mark.parametrize("name", list(MUTANTS))
def test_mutant_is_caught(name):
    H = MUTANTS[name]
    failed = []
    for pin in ALL_PINS:
        try:
            pin(H)
        except (AssertionError, IndexError, ValueError):
            failed.append(pin.__name__)
    assert failed, f"mutant {name} passed every pin"


def test_correct_copy_passes():
    H = _mk(lambda i, j, n, m: i - j + n - 1)
    for pin in ALL_PINS:
        pin(H)
