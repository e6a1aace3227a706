"""Mixed-radix length classes (L = 3, 5, 7 times 2^k) against the oracle.

Every mixed-radix class of FP32 and FP64 is pinned with PA_ONLY_LEN and run
on two random jobs: one that fills a single tile (n + m - 1 close to L) and
one with several key chunks (XOR-accumulated, Eq. 4-7) and several output
windows.  Outputs are compared with the oracle in full where it finishes in
seconds, else at both ends, around every window boundary and at random
positions (selected-output evaluation of the definition).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

CLASS_LENS = sorted(p << k for p in (3, 5, 7) for k in range(11, 23) if (1 << 14) < (p << k) < (1 << 24))
FULL_ORACLE_NM = 2e12


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


def _check(p, y, window_bits, rng, what):
    from gpu_util import describe
    from test_gpu_scale import oracle_select, sample_indices
    n, m = p.n, p.m
    if m % 64:
        assert int(y[-1]) >> (m % 64) == 0, f"{what}: bits past m are set"
    if n * m <= FULL_ORACLE_NM:
        ref = oracle.hash_words(p.seed, n, m, p.key)
        assert np.array_equal(y, ref), f"{what}: " + describe(y, ref, m)
        return m
    idx = sample_indices(m, window_bits, rng, random_count=1500)
    ref = oracle_select(p.seed, n, m, p.key, idx)
    got = synth.bits_to_array(y, m)[idx.astype(np.int64)]
    bad = np.flatnonzero(got != ref)
    assert bad.size == 0, f"{what}: {bad.size} of {idx.size} sampled bits differ, first at {idx[bad[:8]].tolist()}"
    return int(idx.size)


@pytest.mark.parametrize("L", CLASS_LENS)
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_mixed_radix_class(pa, ctx, prec, L, monkeypatch):
    from gpu_util import gpu_hash
    monkeypatch.setenv("PA_ONLY_LEN", str(L))
    flags = pa.PA_PREC_FP32_SEG if prec == "fp32" else pa.PA_PREC_FP64
    rng = np.random.default_rng(L + (7 if prec == "fp32" else 0))
    n1 = int(L * rng.uniform(0.3, 0.7))
    shapes = [(n1, L - n1 + 1 - int(rng.integers(0, 64))),              # one tile, n + m - 1 close to L
              (int(L * rng.uniform(1.3, 2.2)), int(L * rng.uniform(0.55, 0.9)))]   # chunks x windows
    for n, m in shapes:
        plan = pa.pa_plan_query(n, m, flags)
        assert plan["fft_len"] == L, plan
        p = synth.random_problem(rng, n, m)
        print(f"{prec} L={L} n={n} m={m} plan {plan['chunks']}x{plan['windows']}", flush=True)
        st, y = gpu_hash(pa, ctx, p.seed, n, m, p.key, flags)
        assert st == pa.PA_OK, pa.pa_strerror(st)
        s = pa.pa_last_stats(ctx)
        assert s["fft_len"] == L and s["n1"] * s["n2"] == L, s
        if prec == "fp64":
            assert s["certified"] == pa.PA_CERT_A_PRIORI and s["max_residual"] < 1e-6, s
        checked = _check(p, y, plan["window_bits"], rng, f"{prec} L={L} n={n} m={m}")
        print(f"  ok: {checked} outputs checked, residual {s['max_residual']:.3g}, "
              f"fallback {s['fallback_tiles']}", flush=True)


def test_configs_take_mixed_radix_tiles(pa, ctx, monkeypatch):
    """c1-c3 on one FP64 tile of the shortest class that holds them (5 * 2^15,
    5 * 2^18 and 7 * 2^21 points); each output is the oracle's (golden
    digests)."""
    import hashlib
    import json
    import os
    from gpu_util import gpu_hash
    here = os.path.dirname(os.path.abspath(__file__))
    golden = json.load(open(os.path.join(here, "golden", "digests.json")))
    for name, want in (("c1", 163_840), ("c2", 1_310_720), ("c3", 14_680_064)):
        monkeypatch.setenv("PA_ONLY_LEN", str(want))
        p = synth.single_config(name)
        st, y = gpu_hash(pa, ctx, p.seed, p.n, p.m, p.key, pa.PA_PREC_FP64)
        assert st == pa.PA_OK
        s = pa.pa_last_stats(ctx)
        assert s["fft_len"] == want and s["tiles"] == 1, s
        digest = hashlib.sha256(np.ascontiguousarray(y, dtype="<u8").tobytes()).hexdigest()
        assert digest == golden[name]["sha256"], name


@pytest.mark.parametrize("L", [3 << 22, 5 << 21, 7 << 21])
def test_mixed_radix_fallback_accumulated(pa, ctx, L, monkeypatch):
    """All-ones key and seed in the mixed-radix classes whose FP64 column
    passes exchange real and imaginary parts in turn (n2 = 1536, 1280, 1792).
    Every key chunk weighs more than 2^20, so every FP32 tile fails its
    certificate and is re-run in FP64 with the key chunks XOR-accumulated
    (Eq. 4-7).  Closed form: every output is the parity of n."""
    from gpu_util import gpu_hash
    monkeypatch.setenv("PA_ONLY_LEN", str(L))
    n, m = L * 3 // 2 + 1, 1_000_003
    seed = synth.pattern_bits("ones", n + m - 1)
    key = synth.pattern_bits("ones", n)
    plan = pa.pa_plan_query(n, m, pa.PA_PREC_FP32_SEG)
    assert plan["fft_len"] == L and plan["chunks"] > 1, plan
    print(f"L={L} n={n} m={m} plan {plan['chunks']}x{plan['windows']}", flush=True)
    st, y = gpu_hash(pa, ctx, seed, n, m, key, pa.PA_PREC_FP32_SEG)
    assert st == pa.PA_OK, pa.pa_strerror(st)
    s = pa.pa_last_stats(ctx)
    assert s["fallback_tiles"] >= plan["chunks"] * plan["windows"], s
    assert np.array_equal(synth.bits_to_array(y, m), np.full(m, n & 1, np.uint8)), s
