"""GPU path vs the CPU oracle, bit-exact, through the C ABI (MI355X)."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "digests.json")))


@pytest.fixture(scope="module")
def pa():
    from paper_1805_02372_amd import pa as _pa
    return _pa


@pytest.fixture(scope="module")
def ctx(pa):
    import torch
    assert torch.cuda.is_available()
    c = pa.pa_create(0, 0, None)
    yield c
    pa.pa_destroy(c)


def _run(pa, ctx, p, flags):
    from gpu_util import gpu_hash
    print(f"case n={p.n} m={p.m} flags={flags:#x}", flush=True)
    return gpu_hash(pa, ctx, p.seed, p.n, p.m, p.key, flags)


SMALL = [(1, 1), (1, 100), (100, 1), (2, 3), (63, 65), (64, 64), (65, 63), (1000, 333), (333, 1000),
         (4097, 511), (5000, 5000), (100_000, 3000), (70_000, 70_001), (131_071, 1), (1, 131_071)]


def _flags(pa, prec):
    return {"fp64": pa.PA_PREC_FP64, "fp32": pa.PA_PREC_FP32_SEG, "auto": pa.PA_PREC_AUTO,
            "ntt": pa.PA_PREC_NTT}[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "auto", "ntt"])
@pytest.mark.parametrize("n,m", SMALL)
def test_small_shapes(pa, ctx, prec, n, m):
    from gpu_util import describe
    flags = _flags(pa, prec)
    rng = np.random.default_rng(n * 1000003 + m)
    p = synth.random_problem(rng, n, m)
    st, y = _run(pa, ctx, p, flags)
    assert st == pa.PA_OK, pa.pa_strerror(st)
    ref = oracle.hash_words(p.seed, n, m, p.key)
    assert np.array_equal(y, ref), describe(y, ref, m)
    s = pa.pa_last_stats(ctx)
    assert s["max_residual"] <= 0.125


@pytest.mark.parametrize("cap,n,m", [(12, 20_000, 900), (12, 9000, 20_000), (13, 50_000, 30_000),
                                     (12, 4096, 1), (12, 1, 5000), (14, 200_003, 100_001)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "ntt"])
def test_forced_tiling(pa, ctx, cap, n, m, prec, monkeypatch):
    """Key chunks (Eq. 4-7) and output windows at small sizes by capping the
    FFT length class."""
    from gpu_util import describe
    monkeypatch.setenv("PA_MAX_LOG2_LEN", str(cap))
    flags = _flags(pa, prec)
    plan = pa.pa_plan_query(n, m, flags)
    rng = np.random.default_rng(cap * 7 + n + 3 * m)
    p = synth.random_problem(rng, n, m)
    st, y = _run(pa, ctx, p, flags)
    assert st == pa.PA_OK, pa.pa_strerror(st)
    ref = oracle.hash_words(p.seed, n, m, p.key)
    assert np.array_equal(y, ref), describe(y, ref, m) + f" plan {plan}"
    s = pa.pa_last_stats(ctx)
    assert s["tiles"] == plan["chunks"] * plan["windows"]
    if prec == "fp32":
        assert s["max_residual"] <= s["bound"], s   # the error model holds on random inputs
    assert plan["log2_len"] <= cap


# Long classes (2^20..2^24, rows of 8192, wave-level transforms): key chunks,
# output windows and the two-wave column split of n2 = 2048, pinned by the
# class bounds.
LONG = [(20, 20, 2_000_003, 600_001), (20, 20, 300_000, 1_500_000), (21, 21, 1_500_000, 1_000_000),
        (22, 22, 3_000_000, 700_000), (23, 23, 5_000_000, 2_000_000), (24, 24, 9_000_000, 3_000_000)]


@pytest.mark.parametrize("lo,hi,n,m", LONG)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "ntt"])
def test_long_classes(pa, ctx, lo, hi, n, m, prec, monkeypatch):
    from gpu_util import describe
    monkeypatch.setenv("PA_MIN_LOG2_LEN", str(lo))
    monkeypatch.setenv("PA_MAX_LOG2_LEN", str(hi))
    flags = _flags(pa, prec)
    plan = pa.pa_plan_query(n, m, flags)
    assert plan["log2_len"] == hi
    rng = np.random.default_rng(lo * 1000 + n % 997 + m % 991)
    p = synth.random_problem(rng, n, m)
    st, y = _run(pa, ctx, p, flags)
    assert st == pa.PA_OK, pa.pa_strerror(st)
    if n * m <= 3e12:  # full oracle (about n*m/64 word steps)
        ref = oracle.hash_words(p.seed, n, m, p.key)
        assert np.array_equal(y, ref), describe(y, ref, m) + f" plan {plan}"
    else:  # sampled outputs, each by the word-parallel definition
        idx = np.unique(np.concatenate([np.arange(64), np.arange(m - 64, m),
                                        np.random.default_rng(5).integers(0, m, 4000)]))
        ref = oracle.hash_select(p.seed, n, m, p.key, idx)
        got = synth.bits_to_array(y, m)[idx]
        assert np.array_equal(got, ref), f"{int((got != ref).sum())} sampled bits differ, plan {plan}"
        assert int(y[-1]) >> (m % 64) == 0 if m % 64 else True
    s = pa.pa_last_stats(ctx)
    assert s["tiles"] == plan["chunks"] * plan["windows"]
    if prec == "fp32":
        assert s["max_residual"] <= s["bound"], s   # the error model holds on random inputs
    print(prec, lo, n, m, "residual", s["max_residual"], flush=True)


def _digest(words):
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<u8").tobytes()).hexdigest()


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
@pytest.mark.parametrize("prec", ["fp64", "auto", "ntt"])
def test_configs_golden(pa, ctx, name, prec):
    flags = _flags(pa, prec)
    p = synth.single_config(name)
    st, y = _run(pa, ctx, p, flags)
    assert st == pa.PA_OK, pa.pa_strerror(st)
    g = GOLDEN[name]
    assert _digest(y) == g["sha256"], f"{name} {prec}: weight {int(np.unpackbits(y.view(np.uint8)).sum())} vs {g['weight']}"
    s = pa.pa_last_stats(ctx)
    print(name, prec, s, flush=True)


def test_c1_vs_oracle(pa, ctx):
    from gpu_util import describe
    p = synth.single_config("c1")
    st, y = _run(pa, ctx, p, pa.PA_PREC_FP64)
    assert st == pa.PA_OK
    ref = oracle.hash_words(p.seed, p.n, p.m, p.key)
    assert np.array_equal(y, ref), describe(y, ref, p.m)


def test_host_pointers(pa, ctx):
    rng = np.random.default_rng(77)
    p = synth.random_problem(rng, 30_000, 7000)
    out = np.zeros(synth.words_for(p.m), np.uint64)
    st = pa.pa_hash(ctx, p.seed, p.n, p.m, p.key, out, pa.PA_PREC_AUTO)
    assert st == pa.PA_OK
    assert np.array_equal(out, oracle.hash_words(p.seed, p.n, p.m, p.key))


def test_invalid_arguments(pa, ctx):
    from gpu_util import to_dev, empty_dev
    s = to_dev(np.zeros(4, np.uint64))
    k = to_dev(np.zeros(4, np.uint64))
    o = empty_dev(4)
    assert pa.pa_hash(ctx, s, 0, 5, k, o, 0) == pa.PA_EINVAL
    assert pa.pa_hash(ctx, s, 5, 0, k, o, 0) == pa.PA_EINVAL
    assert pa.pa_hash(ctx, 0, 5, 5, k, o, pa.PA_DEVICE_PTRS) == pa.PA_EINVAL
    assert pa.pa_hash(ctx, s, 5, 5, k, o, 0x00F0) == pa.PA_EINVAL


def _random_shapes(count=24, seed=2027):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(10 ** rng.uniform(0, 6.5))
        m = int(10 ** rng.uniform(0, 6.5))
        if n * m <= 2e11:   # the oracle stays well under a second
            out.append((max(1, n), max(1, m)))
    return out


@pytest.mark.parametrize("n,m", _random_shapes())
def test_random_shapes_every_path(pa, ctx, n, m):
    """Log-uniform random shapes (1 .. 3e6 bits each side), every precision
    path against the oracle: FP32 tiles, plain FP64, NTT, the direct product
    and AUTO's choice."""
    from gpu_util import describe
    rng = np.random.default_rng(n * 31 + m)
    p = synth.random_problem(rng, n, m)
    ref = oracle.hash_words(p.seed, n, m, p.key)
    for prec in ("fp32", "fp64", "ntt", "direct", "auto"):
        flags = pa.PA_PREC_DIRECT if prec == "direct" else _flags(pa, prec)
        st, y = _run(pa, ctx, p, flags)
        assert st == pa.PA_OK, (prec, pa.pa_strerror(st))
        assert np.array_equal(y, ref), f"{prec}: " + describe(y, ref, m)
        s = pa.pa_last_stats(ctx)
        if prec in ("ntt", "direct") or s["prec"] in (pa.PA_PREC_NTT, pa.PA_PREC_DIRECT):
            assert s["certified"] == pa.PA_CERT_EXACT, (prec, s)
        else:
            a_priori = s["rigorous_bound"] < 0.5
            assert s["certified"] == (pa.PA_CERT_A_PRIORI if a_priori else pa.PA_CERT_A_POSTERIORI), (prec, s)
            assert s["max_residual"] <= s["rigorous_bound"], (prec, s)


GUARD = 8
SENTINEL = np.uint64(0xA5A5A5A5A5A5A5A5)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "ntt", "direct", "auto"])
@pytest.mark.parametrize("n,m", [(70_000, 9_001), (3_000_001, 300_007), (5, 64), (200_003, 1)])
def test_guard_words_untouched(pa, ctx, prec, n, m):
    """The output's ceil(m/64) words are written (bits past m as 0) and the
    guard words after them are never touched, on every path, including key
    chunks XOR-accumulated under a capped class (2^20)."""
    import torch
    from gpu_util import to_dev, from_dev
    flags = pa.PA_PREC_DIRECT if prec == "direct" else _flags(pa, prec)
    rng = np.random.default_rng(n + 7 * m)
    p = synth.random_problem(rng, n, m)
    w = synth.words_for(m)
    out = to_dev(np.full(w + GUARD, SENTINEL, np.uint64))
    old = os.environ.get("PA_MAX_LOG2_LEN")
    os.environ["PA_MAX_LOG2_LEN"] = "20"
    try:
        st = pa.pa_hash(ctx, to_dev(p.seed), n, m, to_dev(p.key), out, flags)
        torch.cuda.synchronize()
    finally:
        if old is None:
            del os.environ["PA_MAX_LOG2_LEN"]
        else:
            os.environ["PA_MAX_LOG2_LEN"] = old
    assert st == pa.PA_OK, pa.pa_strerror(st)
    y = from_dev(out)
    assert np.array_equal(y[:w], oracle.hash_words(p.seed, n, m, p.key))
    assert np.all(y[w:] == SENTINEL), "guard words written"
