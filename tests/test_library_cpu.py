"""Host-side checks of libpa (no GPU needed): the library loads, exports every
entry point include/pa.h declares, and its planner obeys the tiling rules."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


@pytest.fixture(scope="module")
def pa():
    from paper_1805_02372_amd import pa as _pa
    return _pa


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(pa):
    names = declared_symbols()
    assert len(names) >= 13
    lib = ctypes.CDLL(pa.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(names) == set(pa.EXPORTED)


def test_strerror(pa):
    assert pa.pa_strerror(pa.PA_OK) == "PA_OK"
    for s in range(1, 7):
        assert pa.pa_strerror(s).startswith("PA_E")
    assert "unknown" in pa.pa_strerror(99)


def test_create_without_device(pa):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(pa.PAError) as e:
        pa.pa_create(0)
    assert e.value.status == pa.PA_EDEVICE


def tiles_of(n, m, plan):
    """Tile geometry as include/pa.h documents it for pa_plan_query."""
    Bi, Bo = plan["chunk_bits"], plan["window_bits"]
    out = []
    for b in range(plan["chunks"]):
        hi = n - b * Bi
        lo = max(0, hi - Bi)
        for o in range(plan["windows"]):
            i0 = o * Bo
            bo = min(Bo, m - i0)
            sigma = i0 + n - hi
            out.append((lo, hi - lo, i0, bo, sigma))
    return out


# FFT lengths of the classes: 2^12 .. 2^24, and 3, 5, 7 times 2^k between
# 2^14 and 2^24 (FP32 and FP64)
CLASS_LENS = {1 << k for k in range(12, 25)} | {p << k for p in (3, 5, 7) for k in range(11, 23)
                                                if (1 << 14) < (p << k) < (1 << 24)}

SHAPES = [(1, 1), (5, 3), (131072, 16384), (1_000_000, 200_000), (12_345_679, 1_234_567),
          (100_000_000, 50_000_000), (3, 40_000_000), (40_000_000, 3), (16_777_216, 1), (2**24, 2**24)]


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("prec", ["auto", "fp32", "fp64"])
def test_plan_covers_every_pair_once(pa, n, m, prec):
    flags = {"auto": pa.PA_PREC_AUTO, "fp32": pa.PA_PREC_FP32_SEG, "fp64": pa.PA_PREC_FP64}[prec]
    p = pa.pa_plan_query(n, m, flags)
    L = p["fft_len"]
    assert p["n1"] * p["n2"] == L and 1 << p["log2_len"] >= L > 1 << (p["log2_len"] - 1)
    assert L in CLASS_LENS
    Bi, Bo = p["chunk_bits"], p["window_bits"]
    assert p["chunks"] == -(-n // Bi) and p["windows"] == -(-m // Bo)
    assert Bi + Bo - 1 <= L                       # no wrap into the kept window
    if p["windows"] > 1:
        assert Bo % 64 == 0                        # windows start on word boundaries
    if prec == "fp64" and n + m - 1 <= 2**24:
        assert p["chunks"] == 1 and p["windows"] == 1   # the plain single-tile path
    if flags != pa.PA_PREC_FP64:
        assert p["bound"] < 0.25
    tiles = tiles_of(n, m, p)
    # key chunks tile [0, n) exactly, windows tile [0, m) exactly
    chunks = sorted({(lo, bi) for lo, bi, *_ in tiles})
    assert chunks[0][0] == 0 and all(a[0] + a[1] == b[0] for a, b in zip(chunks, chunks[1:]))
    assert chunks[-1][0] + chunks[-1][1] == n
    wins = sorted({(i0, bo) for _, _, i0, bo, _ in tiles})
    assert wins[0][0] == 0 and all(a[0] + a[1] == b[0] for a, b in zip(wins, wins[1:]))
    assert wins[-1][0] + wins[-1][1] == m
    for lo, bi, i0, bo, sigma in tiles:
        assert 0 <= sigma and sigma + bi + bo - 1 <= n + m - 1   # seed slice in range
        assert bi >= 1 and bo >= 1 and bi + bo - 1 <= L


def test_plan_invariants_random_shapes(pa):
    """Property check over random shapes (hypothesis, a fixed number of cases):
    every plan's chunks tile the key and its windows tile the output once, no
    tile wraps (Bi + Bo - 1 <= L), window starts are word aligned, and FP plans
    respect the error limit."""
    hyp = pytest.importorskip("hypothesis")
    st = hyp.strategies

    @hyp.settings(max_examples=300, deadline=None, derandomize=True)
    @hyp.given(n=st.integers(1, 1 << 34), m=st.integers(1, 1 << 30),
               f=st.sampled_from([pa.PA_PREC_AUTO, pa.PA_PREC_FP64, pa.PA_PREC_NTT]))
    def check(n, m, f):
        p = pa.pa_plan_query(n, m, f)
        L = p["fft_len"]
        assert p["n1"] * p["n2"] == L and L in CLASS_LENS
        if f == pa.PA_PREC_NTT:
            assert L & (L - 1) == 0               # the NTT has power-of-two classes only
        Bi, Bo, C, W = p["chunk_bits"], p["window_bits"], p["chunks"], p["windows"]
        assert Bi + Bo - 1 <= L
        assert C == -(-n // Bi) and W == -(-m // Bo) and (C - 1) * Bi < n and (W - 1) * Bo < m
        assert W == 1 or Bo % 64 == 0
        if f != pa.PA_PREC_NTT:
            assert p["bound"] <= 0.25

    check()


def test_tile_geometry_reproduces_the_hash():
    """The documented tile geometry (seed slice per tile, Eq. 4-7 XOR of key
    chunks, output windows) recomputes the definition exactly; checked with the
    explicit-matrix oracle on small shapes."""
    import oracle
    import synth
    rng = np.random.default_rng(42)
    for n, m, Bi, Bo in [(50, 20, 17, 20), (50, 20, 50, 8), (33, 70, 10, 64), (64, 64, 7, 11)]:
        s = rng.integers(0, 2, n + m - 1, dtype=np.uint8)
        x = rng.integers(0, 2, n, dtype=np.uint8)
        ref = oracle.hash_matrix(s, n, m, x)
        plan = dict(chunk_bits=Bi, window_bits=Bo, chunks=-(-n // Bi), windows=-(-m // Bo))
        y = np.zeros(m, np.uint8)
        for lo, bi, i0, bo, sigma in tiles_of(n, m, plan):
            w = s[sigma:sigma + bi + bo - 1].astype(np.int64)
            c = np.convolve(w, x[lo:lo + bi].astype(np.int64))[bi - 1:bi - 1 + bo]
            y[i0:i0 + bo] ^= (c % 2).astype(np.uint8)
        assert np.array_equal(y, ref), (n, m, Bi, Bo)
        _ = synth  # inputs drawn locally


def test_error_model_monotone(pa):
    f = pa.PA_PREC_FP32_SEG
    v = [pa.pa_error_model(f, 20, b) for b in (1 << 10, 1 << 16, 1 << 19)]   # Bi <= L/2
    assert v[0] < v[1] < v[2]
    assert pa.pa_error_model(f, 24, 1 << 20) > pa.pa_error_model(f, 16, 1 << 20)
    assert pa.pa_error_model(pa.PA_PREC_FP64, 24, 1 << 24) < 1e-8
    assert pa.pa_error_model(0x00F0, 20, 5) < 0


def _fp32_packed_conv_error(rng, logL, Bi, centre_key):
    """Max error over the kept window of the packed two-for-one FP32 FFT
    convolution of a 0/1 chunk (or the same chunk minus 1/2) with a +-1 seed,
    computed with scipy's single-precision FFT."""
    import scipy.fft as sf
    L = 1 << logL
    Bo = L - Bi + 1
    x = np.zeros(L)
    x[:Bi] = rng.integers(0, 2, Bi)
    if centre_key:
        x[:Bi] -= 0.5
    w = (1.0 - 2.0 * rng.integers(0, 2, L)).astype(np.float64)
    exact = np.fft.ifft(np.fft.fft(x) * np.fft.fft(w)).real
    Z = sf.fft((x + 1j * w).astype(np.complex64))
    Zr = np.conj(np.roll(Z[::-1], 1))
    P = ((Z + Zr) / 2 * ((Z - Zr) / np.complex64(2j))).astype(np.complex64)
    y = sf.ifft(P).real
    return float(np.abs(y - exact)[Bi - 1:Bi - 1 + Bo].max())


def test_error_model_covers_fp32_packed_convolution(pa):
    """The error model bounds the error of an FP32 packed convolution (here
    scipy's FFT, not the kernels), and its low-frequency term is real: the same
    convolution with the key's mean removed is several times more accurate."""
    rng = np.random.default_rng(7)
    f = pa.PA_PREC_FP32_SEG
    for logL, Bi in [(18, 1 << 17), (18, 3 << 15), (20, 1 << 19)]:
        err = _fp32_packed_conv_error(rng, logL, Bi, False)
        assert err <= pa.pa_error_model(f, logL, Bi), (logL, Bi, err)
    e01 = _fp32_packed_conv_error(np.random.default_rng(8), 20, 1 << 19, False)
    e_centred = _fp32_packed_conv_error(np.random.default_rng(8), 20, 1 << 19, True)
    assert e_centred * 1.5 < e01, (e01, e_centred)


def test_direct_path_choice(pa):
    """PA_PREC_DIRECT always takes the direct GF(2) path; AUTO takes it only
    where its modeled cost (linear in m and in n) is below the FFT plan's."""
    for n, m in SHAPES:
        assert pa.pa_plan_query(n, m, pa.PA_PREC_DIRECT)["direct"] == 1
        assert pa.pa_plan_query(n, m, pa.PA_PREC_FP32_SEG)["direct"] == 0
        q = pa.pa_plan_query(n, m, pa.PA_PREC_AUTO)
        assert q["direct"] == (1 if q["direct_cost"] < q["cost"] else 0)
    assert pa.pa_plan_query(1_000_000, 100, 0)["direct"] == 1
    assert pa.pa_plan_query(12_345_679, 1_234_567, 0)["direct"] == 0
    c = [pa.pa_plan_query(1 << 20, m, 0)["direct_cost"] for m in (256, 512, 1024)]
    assert c[0] < c[1] < c[2] and abs((c[2] - c[1]) - 2 * (c[1] - c[0])) < 1e-12
    assert pa.pa_error_model(pa.PA_PREC_DIRECT, 20, 1000) == 0.0


def test_size_limits(pa):
    """Plans exist up to n = 2^40 (key chunks) and m = 2^38 (2^14 windows of
    2^24 bits); longer outputs are rejected, not mis-planned."""
    for f in (pa.PA_PREC_AUTO, pa.PA_PREC_FP64, pa.PA_PREC_NTT):
        p = pa.pa_plan_query(1 << 40, 1, f)
        assert p["chunks"] * p["chunk_bits"] >= 1 << 40
        p = pa.pa_plan_query(5, 1 << 38, f)
        assert p["windows"] <= 1 << 14 and p["windows"] * p["window_bits"] >= 1 << 38
        with pytest.raises(pa.PAError):
            pa.pa_plan_query(5, (1 << 38) + (1 << 24), f)


def test_plan_query_rejects_bad_input(pa):
    with pytest.raises(pa.PAError):
        pa.pa_plan_query(0, 5, 0)
    with pytest.raises(pa.PAError):
        pa.pa_plan_query(5, 0, 0)
    with pytest.raises(pa.PAError):
        pa.pa_plan_query(5, 5, 0x00F0)


def test_class_caps(pa, monkeypatch):
    monkeypatch.setenv("PA_MAX_LOG2_LEN", "12")
    p = pa.pa_plan_query(100_000, 10_000, pa.PA_PREC_FP64)
    assert p["log2_len"] == 12 and p["chunks"] * p["windows"] > 1
    monkeypatch.setenv("PA_MIN_LOG2_LEN", "12")
    monkeypatch.setenv("PA_MAX_LOG2_LEN", "24")
    monkeypatch.setenv("PA_MIN_LOG2_LEN", "24")
    p = pa.pa_plan_query(1000, 1000, pa.PA_PREC_FP32_SEG)
    assert p["log2_len"] == 24


def test_rigorous_bound_fp64_margin_and_monotone(pa):
    """The worst-case rounding bound (Percival's form) certifies every FP64
    plan with a wide margin, grows with the tile's length and its key and
    output norms, and is zero for the exact NTT."""
    prev = 0.0
    for k in range(12, 25):
        n = (1 << k) // 2
        os.environ["PA_MAX_LOG2_LEN"] = str(k)   # 2^k is then the only class that holds n + n - 1 bits
        try:
            p = pa.pa_plan_query(n, n, pa.PA_PREC_FP64)
        finally:
            del os.environ["PA_MAX_LOG2_LEN"]
        assert p["log2_len"] == k and p["chunks"] == 1
        assert 0 < p["rigorous_bound"] < 1e-4, p      # 5000x below the rounding margin 0.5
        assert p["rigorous_bound"] > prev
        prev = p["rigorous_bound"]
    for n, m in SHAPES:
        assert pa.pa_plan_query(n, m, pa.PA_PREC_FP64)["rigorous_bound"] < 1e-4
        assert pa.pa_plan_query(n, m, pa.PA_PREC_NTT)["rigorous_bound"] == 0.0
    # at a fixed class, a longer key chunk or output window gives a larger bound
    os.environ["PA_MIN_LOG2_LEN"] = os.environ["PA_MAX_LOG2_LEN"] = "16"
    try:
        a = pa.pa_plan_query(10_000, 1000, pa.PA_PREC_FP64)["rigorous_bound"]
        b = pa.pa_plan_query(20_000, 1000, pa.PA_PREC_FP64)["rigorous_bound"]
        c = pa.pa_plan_query(20_000, 30_000, pa.PA_PREC_FP64)["rigorous_bound"]
    finally:
        del os.environ["PA_MIN_LOG2_LEN"], os.environ["PA_MAX_LOG2_LEN"]
    assert a < b < c


def test_rigorous_bound_fp32(pa):
    """FP32: short tiles are certified a priori, the long tiles the fast path
    uses are not (they rely on the run-time certificate); on full tiles the
    worst case lies far above the probabilistic model."""
    small = pa.pa_plan_query(1000, 333, pa.PA_PREC_FP32_SEG)
    assert small["rigorous_bound"] < 0.5, small
    c3 = pa.pa_plan_query(12_345_679, 1_234_567, pa.PA_PREC_FP32_SEG)
    assert c3["rigorous_bound"] > 0.5, c3
    assert c3["rigorous_bound"] > 100 * c3["bound"], c3


def test_mixed_radix_classes_shorten_the_plain_fp64_tile(pa, monkeypatch):
    """Section 3, step 1 pads the product to an arbitrary length.  The plain
    FP64 path runs one tile; the shortest class that holds n + m - 1 is
    within 1.25x of it with the classes 3, 5 and 7 times 2^k, and the path
    takes the cheapest single tile by the cost model (never longer than the
    next power of two)."""
    import math
    for n, m, want in [(131_072, 16_384, 163_840),          # c1: 5 * 2^15 (2^18 without)
                       (1_000_000, 200_000, 1_310_720),     # c2: 5 * 2^18 (2^21 without)
                       (12_345_679, 1_234_567, 14_680_064)]:  # c3: 7 * 2^21 (2^24 without)
        assert want == min(x for x in CLASS_LENS if x >= n + m - 1)
        monkeypatch.setenv("PA_ONLY_LEN", str(want))
        p = pa.pa_plan_query(n, m, pa.PA_PREC_FP64)
        assert p["fft_len"] == want and p["chunks"] == p["windows"] == 1, p
        assert p["log2_len"] == math.ceil(math.log2(want))
        monkeypatch.delenv("PA_ONLY_LEN")
    rng = np.random.default_rng(5)
    for _ in range(200):
        n, m = int(rng.integers(1, 1 << 23)), int(rng.integers(1, 1 << 23))
        if n + m - 1 > 1 << 24 or n + m - 1 <= 1 << 14:
            continue
        p = pa.pa_plan_query(n, m, pa.PA_PREC_FP64)
        L = p["fft_len"]
        assert p["chunks"] == p["windows"] == 1 and n + m - 1 <= L <= 1 << math.ceil(math.log2(n + m - 1)), (n, m, L)


def test_class_filters(pa, monkeypatch):
    """PA_POW2_ONLY keeps the power-of-two classes; PA_ONLY_LEN pins one class."""
    monkeypatch.setenv("PA_POW2_ONLY", "1")
    assert pa.pa_plan_query(12_345_679, 1_234_567, pa.PA_PREC_FP64)["fft_len"] == 1 << 24
    monkeypatch.delenv("PA_POW2_ONLY")
    monkeypatch.setenv("PA_ONLY_LEN", str(3 << 16))
    for f in (pa.PA_PREC_FP32_SEG, pa.PA_PREC_FP64):
        p = pa.pa_plan_query(1_000_000, 300_000, f)
        assert p["fft_len"] == 3 << 16 and p["chunks"] * p["windows"] > 1, p


def test_shipped_tuning_table(pa):
    """The cost table measured on MI355X (pa_tune, one- and four-tile launches
    per class) ships beside libpa.so and covers every class: per class the
    marginal cost of a tile and the rest of a one-tile launch."""
    import json
    path = os.path.join(os.path.dirname(pa.LIB_PATH), "tune_mi355x.json")
    t = json.load(open(path))
    assert 0 < t["launch"] < 1e-3 and 0 < t["direct"] < 1e-9
    for prec, lens in (("fp32", CLASS_LENS), ("fp64", CLASS_LENS), ("ntt", {1 << k for k in range(12, 25)})):
        assert {int(k) for k in t[prec]} == lens, prec
        for L, (tile, first) in t[prec].items():
            assert 0 < tile < 0.1 and 0 <= first < 0.01, (prec, L, tile, first)


def test_plans_from_the_shipped_table_stay_valid(pa):
    """With the shipped table or the built-in model (PA_TUNE_DEFAULT=0, in a
    process of its own), every plan satisfies the tiling invariants."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r); from paper_1805_02372_amd import pa; "
            "print([pa.pa_plan_query(n, m, f)['fft_len'] for n, m in [(131072, 16384), (1000000, 200000), "
            "(12345679, 1234567)] for f in (0, 0x20)])") % ROOT
    out = {}
    for v in ("1", "0"):
        env = dict(os.environ, PA_TUNE_DEFAULT=v)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0, r.stderr[-2000:]
        out[v] = eval(r.stdout.strip().splitlines()[-1])
        assert all(L in CLASS_LENS for L in out[v])
