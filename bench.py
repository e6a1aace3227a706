#!/usr/bin/env python3
"""Benchmark: input-key Gbps of the Toeplitz-hash path on one MI355X.

Workload (default): one hash with n = 12,345,679 key bits and m = 1,234,567
output bits, i.i.d. uniform bits from seed 2 (synth.single_config("c3")),
inputs resident in HBM before timing starts.  A step is one complete pa_hash
call (plan, every tile's three kernel passes with the XOR merge, certificate
read-back), timed over K steps between device synchronisations.

Reported: the headline FP32-segmented (auto) throughput, the plain FP64
single-tile path and the 64-job batched launch beside it, per-call latency
percentiles, the dominant kernel's achieved bandwidth against the 8 TB/s HBM
peak (kernel durations from HIP events on the library's own stream), and the
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "input-key Gbps (bit-exact) at n=1e7; batched FP32 vs plain FP64 path, p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "traffic_c3.json")
PROFILE_VALU = os.path.join(ROOT, "profiles", "valu_c3.json")
# vector instructions a CU issues per second: 4 SIMDs, one 64-lane instruction each per 4 cycles
VALU_WAVE_INSTR_PEAK = 256 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("conv_fp32.hip", "conv_fp64.hip", "conv_fp32_p3.hip", "conv_fp32_p5.hip", "conv_fp32_p7.hip",
                  "conv_fp64_p3.hip", "conv_fp64_p5.hip", "conv_fp64_p7.hip", "conv_kernels.hpp", "conv_v2.hpp",
                  "fft_core.hpp", "wave_fft.hpp", "ntt.hip", "pa_internal.hpp", "tile_fused.hpp")


def kernel_source_digest() -> str:
    """Digest of the device-code sources: HBM counters taken on other kernels
    are not reported."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1805_02372_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:16]


def launch_bytes(st: dict, n: int, m: int) -> list[float]:
    """Algorithmic HBM bytes of one launch of each pass over all tiles of a
    job (e = 8 for FP32, 16 for FP64; L the FFT length; T tiles = C chunks x
    W windows):
      pass 1: reads each tile's key chunk and seed slice, writes the complex
              array (and clears the output when C > 1):
              e L T + (2 W n + C m) / 8 [+ m / 8]
      pass 2: reads the array, writes half of it: 1.5 e L T
      pass 3: reads the half, writes (C = 1) or XORs in (C > 1) each tile's
              output window: 0.5 e L T + C m / 8
    The fourth entry (the former merge) is 0: chunks are XOR-accumulated."""
    e = 16 if st["prec"] == 0x20 else 8
    L = float(st["fft_len"])
    C = -(-n // st["chunk_bits"])
    W = -(-m // st["window_bits"])
    T = C * W
    clear = m / 8 if C > 1 else 0.0
    return [e * L * T + (2 * W * n + C * m) / 8 + clear, 1.5 * e * L * T, 0.5 * e * L * T + C * m / 8, 0.0]


def run_single(pa, ctx, torch, prob, flags, steps, warmup):
    s = torch.from_numpy(prob.seed.view(np.int64).copy()).to("cuda:0")
    k = torch.from_numpy(prob.key.view(np.int64).copy()).to("cuda:0")
    o = torch.zeros(((prob.m + 63) // 64,), dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()   # the library's stream is not ordered after torch's
    for _ in range(warmup):
        st = pa.pa_hash(ctx, s, prob.n, prob.m, k, o, flags)
        assert st == pa.PA_OK, pa.pa_strerror(st)
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        st = pa.pa_hash(ctx, s, prob.n, prob.m, k, o, flags)
        if flags & pa.PA_ASYNC:
            torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
        assert st == pa.PA_OK, pa.pa_strerror(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stats = pa.pa_last_stats(ctx)
    # per-kernel durations: HIP events around each launch on the library stream
    kms = np.zeros(4)
    reps = max(3, min(steps, 10))
    for _ in range(reps):
        st = pa.pa_hash(ctx, s, prob.n, prob.m, k, o, flags | pa.PA_TIMING)
        assert st == pa.PA_OK
        kms += np.array(pa.pa_last_stats(ctx)["ms_pass"])
    kms /= reps
    torch.cuda.synchronize()
    out = o.cpu().numpy().view(np.uint64).copy()
    return dict(elapsed=el, lat=np.array(lat), stats=stats, kernel_ms=kms.tolist(), out=out)


def run_latency_c1(pa, ctx, torch, calls: int = 200, warmup: int = 20):
    """c1 (n = 131,072, m = 16,384) on the plain FP64 path: a latency-bound
    single hash.  Per-call wall time (launches, kernels, certificate read-back)
    over `calls` synchronous calls, inputs resident in HBM."""
    import synth
    prob = synth.single_config("c1")
    r = run_single(pa, ctx, torch, prob, pa.PA_PREC_FP64, calls, warmup)
    st = r["stats"]
    return prob, {"n": prob.n, "m": prob.m, "path": "fp64_plain",
                  "p50_us": round(float(np.percentile(r["lat"], 50)) * 1e6, 1),
                  "p99_us": round(float(np.percentile(r["lat"], 99)) * 1e6, 1),
                  "mean_us": round(r["elapsed"] / calls * 1e6, 1),
                  "kernel_us": [round(x * 1e3, 2) for x in r["kernel_ms"][:3]],
                  "gbps": round(prob.n * calls / r["elapsed"] / 1e9, 3),
                  "fft_len": st["fft_len"], "tiles": st["tiles"],
                  "rigorous_bound": st["rigorous_bound"], "certified": CERT_NAMES[st["certified"]],
                  "out": r["out"]}


def run_c2(pa, ctx, torch, steps, warmup):
    """c2 (n = 10^6, m = 2 * 10^5): the FP64 full-length single tile against
    the FP32 segmented plan, with each plan's length, chunk, window, model
    bound and worst-case bound."""
    import synth
    prob = synth.single_config("c2")
    out = {"n": prob.n, "m": prob.m}
    outs = {}
    for name, flags in (("fp64_plain", pa.PA_PREC_FP64), ("fp32_segmented", pa.PA_PREC_FP32_SEG)):
        r = run_single(pa, ctx, torch, prob, flags, steps, warmup)
        st = r["stats"]
        out[name] = {"gbps": round(prob.n * steps / r["elapsed"] / 1e9, 3),
                     "ms_per_call": round(r["elapsed"] / steps * 1e3, 4),
                     "p99_ms": round(float(np.percentile(r["lat"], 99)) * 1e3, 4),
                     "kernel_ms": [round(x, 5) for x in r["kernel_ms"][:3]],
                     "fft_len": st["fft_len"], "chunk_bits": st["chunk_bits"], "window_bits": st["window_bits"],
                     "tiles": st["tiles"], "model_bound": st["bound"], "rigorous_bound": st["rigorous_bound"],
                     "max_residual": st["max_residual"], "fallback_tiles": st["fallback_tiles"],
                     "certified": CERT_NAMES[st["certified"]]}
        outs[name] = r["out"]
    return prob, out, outs


def run_batch(pa, ctx, torch, jobs, flags, steps, warmup):
    dev = []
    for p in jobs:
        s = torch.from_numpy(p.seed.view(np.int64).copy()).to("cuda:0")
        k = torch.from_numpy(p.key.view(np.int64).copy()).to("cuda:0")
        o = torch.zeros(((p.m + 63) // 64,), dtype=torch.int64, device="cuda:0")
        dev.append((s, k, o, p.n, p.m))
    torch.cuda.synchronize()
    jb = pa.JobBatch(dev)   # the 64 descriptors, packed once (the buffers do not change)
    for _ in range(warmup):
        st, per = pa.pa_hash_batch(ctx, jb, flags)
        assert st == pa.PA_OK, pa.pa_strerror(st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st, per = pa.pa_hash_batch(ctx, jb, flags)
        assert st == pa.PA_OK
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    outs = [d[2].cpu().numpy().view(np.uint64).copy() for d in dev]
    return dict(elapsed=el, stats=pa.pa_last_stats(ctx), outs=outs)


def run_serving(pa, chk_ctx, torch, count: int, load: float = 0.7, budget_gib: int = 8):
    """Serving workload: `count` requests, n log-uniform in [1e5, 1e8], m/n
    uniform in [0.02, 0.5], seeds = 8 resident 1.5e8-bit strings, Poisson
    arrivals.  Request keys are prefixes of 8 resident random 1e8-bit
    buffers (key k uses buffer k mod 8).  The arrival rate is `load` times the
    capacity measured on a back-to-back burst of the same requests, on a
    context of its own with an HBM budget of `budget_gib` GiB.  Beside the
    main leg: a sweep of the load (0.5 and 0.9, 500 requests each) and the
    same 500 requests at 0.7 under a 1 GiB budget, where admission binds.
    Exactness: 256 outputs of each of 16 requests recomputed by
    pa_hash_select (the direct GF(2) product, no transform) on chk_ctx."""
    import synth
    seeds, reqs = synth.serving_stream(count)
    rng = np.random.default_rng(5)
    keys = [synth.gen_bits(rng, 100_000_000) for _ in range(8)]
    dseeds = [torch.from_numpy(sd.view(np.int64).copy()).to("cuda:0") for sd in seeds]
    dkeys = [torch.from_numpy(k.view(np.int64).copy()).to("cuda:0") for k in keys]
    outs = [torch.empty(((r["m"] + 63) // 64,), dtype=torch.int64, device="cuda:0") for r in reqs]
    torch.cuda.synchronize()
    mean_n = float(np.mean([r["n"] for r in reqs]))
    spacing = reqs[-1]["t"] / len(reqs)          # synth arrivals are at 100/s; rescaled below

    def new_ctx(gib):
        c = pa.pa_create(0, gib << 30, None)
        return c, [pa.pa_seed_register(c, d, 150_000_000) for d in dseeds]

    def submit(c, sids, k):
        r = reqs[k]
        st, t = pa.pa_submit(c, sids[r["seed_id"]], r["n"], r["m"], dkeys[k % 8], outs[k])
        assert st == pa.PA_OK, pa.pa_strerror(st)
        return t

    def play(c, sids, idx, rate):
        t0 = time.perf_counter()
        tickets = []
        for k in idx:
            due = t0 + (reqs[k]["t"] - reqs[idx[0]]["t"]) / (spacing * rate)
            while True:
                dt = due - time.perf_counter()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.002))
            tickets.append(submit(c, sids, k))
        status = [pa.pa_wait(c, t) for t in tickets]
        wall = time.perf_counter() - t0
        assert all(s == pa.PA_OK for s in status), [pa.pa_strerror(s) for s in set(status)]
        lat = np.array([pa.pa_ticket_latency(c, t) for t in tickets])
        total_n = sum(reqs[k]["n"] for k in idx)
        return {"requests": len(idx), "offered_rate_per_s": round(rate, 1),
                "sustained_gbps": round(total_n / wall / 1e9, 3),
                "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "wall_s": round(wall, 3)}

    ctx, sids = new_ctx(budget_gib)
    try:
        # capacity on a burst of the first requests (256: enough for the
        # class batches of both lanes to fill the device)
        burst = list(range(min(256, count)))
        a = time.perf_counter()
        tk = [submit(ctx, sids, k) for k in burst]
        for t in tk:
            st = pa.pa_wait(ctx, t)
            assert st == pa.PA_OK, pa.pa_strerror(st)
        cap = sum(reqs[k]["n"] for k in burst) / (time.perf_counter() - a)
        torch.cuda.synchronize()
        log(f"[bench] serving: capacity {cap / 1e9:.2f} Gbps on a burst")
        main = play(ctx, sids, list(range(count)), load * cap / mean_n)
        ss = pa.pa_serve_stats(ctx)
        main.update({"load": load, "hbm_budget_gib": budget_gib, "burst_capacity_gbps": round(cap / 1e9, 3),
                     "tiles": ss["tiles"], "fallback_tiles": ss["fallback_tiles"],
                     "fallback_rate": round(ss["fallback_tiles"] / max(1, ss["tiles"]), 6),
                     "direct_jobs": ss["direct_jobs"]})
        sub = list(range(min(500, count)))
        sweep = []
        for lf in (0.5, 0.9):
            r = play(ctx, sids, sub, lf * cap / mean_n)
            r["load"] = lf
            sweep.append(r)
            log(f"[bench] serving sweep: {r}")
    finally:
        pa.pa_destroy(ctx)
    tctx, tsids = new_ctx(1)
    try:
        tight = play(tctx, tsids, sub, load * cap / mean_n)
        tight.update({"load": load, "hbm_budget_gib": 1})
        log(f"[bench] serving tight budget: {tight}")
    finally:
        pa.pa_destroy(tctx)
    # exactness spot check on the device by the direct path
    chk = np.random.default_rng(6).choice(len(reqs), size=min(16, len(reqs)), replace=False)
    exact = True
    for k in chk:
        r = reqs[int(k)]
        idx = np.random.default_rng(int(k)).integers(0, r["m"], 256)
        st, ref = pa.pa_hash_select(chk_ctx, dseeds[r["seed_id"]], r["n"], r["m"], dkeys[int(k) % 8], idx)
        assert st == pa.PA_OK, pa.pa_strerror(st)
        got = synth.bits_to_array(outs[int(k)].cpu().numpy().view(np.uint64), r["m"])[idx]
        exact = exact and bool(np.array_equal(ref, got))
    main["spot_check_exact"] = exact
    main["spot_check"] = "256 outputs of 16 requests recomputed by pa_hash_select (direct GF(2) product)"
    main["sweep"] = sweep
    main["tight_budget"] = tight
    return main


def run_host_pointers(pa, ctx, prob, steps: int = 40):
    """The c3 job from host memory (numpy arrays): each call copies seed and key
    to the device and the output back, over PCIe.  Reported beside the
    resident-input rate, never as the headline.  Calls are timed one by one:
    the host side shows occasional multi-millisecond stalls, so the median
    and the mean are both given."""
    out = np.zeros((prob.m + 63) // 64, np.uint64)
    for _ in range(3):
        assert pa.pa_hash(ctx, prob.seed, prob.n, prob.m, prob.key, out, pa.PA_PREC_AUTO) == pa.PA_OK
    ts = []
    for _ in range(steps):
        t0 = time.perf_counter()
        assert pa.pa_hash(ctx, prob.seed, prob.n, prob.m, prob.key, out, pa.PA_PREC_AUTO) == pa.PA_OK
        ts.append(time.perf_counter() - t0)
    med, mean = float(np.median(ts)), float(np.mean(ts))
    return {"gbps_including_copies": round(prob.n / med / 1e9, 3), "ms_per_call_median": round(med * 1e3, 4),
            "ms_per_call_mean": round(mean * 1e3, 4), "ms_per_call_max": round(max(ts) * 1e3, 3),
            "gbps_at_mean": round(prob.n / mean / 1e9, 3), "calls": steps,
            "bytes_copied": int(((prob.n + prob.m - 1 + 63) // 64 + (prob.n + 63) // 64 + (prob.m + 63) // 64) * 8),
            "out": out}


CERT_NAMES = {0: "none", 1: "exact", 2: "a-priori", 3: "a-posteriori"}
VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz


def run_direct_leg(pa, ctx, torch, steps, warmup, m: int = 1000):
    """The c3 key (n = 12,345,679) with a short output (m = 1000): the direct
    GF(2) path against the FP32 FFT path on the same job.  Both are product
    paths; their outputs must agree bit for bit.  The direct kernel does two
    VALU operations per output and 32-bit key word; its ALU roofline is the
    vector rate of the chip."""
    import synth
    rng = np.random.default_rng(2)
    prob = synth.random_problem(rng, 12_345_679, m)
    rd = run_single(pa, ctx, torch, prob, pa.PA_PREC_DIRECT, steps, warmup)
    rf = run_single(pa, ctx, torch, prob, pa.PA_PREC_FP32_SEG, steps, warmup)
    key_words = -(-(-(-prob.n // 32)) // 4) * 4          # ceil(n / 32) rounded up to 4
    steps_word = (-(-m // 256) * 256) * key_words       # outputs in blocks of 256
    kms = rd["kernel_ms"][1]   # the product kernel (ms_pass[0] is the key-reversal prep)
    ops = 2.0 * steps_word / (kms * 1e-3)
    return {"n": prob.n, "m": m,
            "direct_gbps": round(prob.n * steps / rd["elapsed"] / 1e9, 3),
            "direct_ms_per_call": round(rd["elapsed"] / steps * 1e3, 4),
            "fft_fp32_gbps": round(prob.n * steps / rf["elapsed"] / 1e9, 3),
            "fft_ms_per_call": round(rf["elapsed"] / steps * 1e3, 4),
            "outputs_agree": bool(np.array_equal(rd["out"], rf["out"])),
            "roofline": {"bound": "alu", "kernel": "k_direct", "achieved": round(ops / 1e12, 2),
                         "peak": round(VALU_LANE_OPS / 1e12, 2), "unit": "T lane-ops/s",
                         "frac": round(ops / VALU_LANE_OPS, 4), "kernel_ms": round(kms, 5)}}


# Table 1 of the paper (NVIDIA TITAN Xp, FP32 FFT, m = 0.1 n): Gbps per input length
PAPER_TABLE1 = {4: 1.25, 8: 1.33, 16: 1.37, 32: 1.38, 64: 1.38, 128: 1.35}


def run_table1(pa, ctx, torch, reps: int = 5):
    """The paper's Table 1 shapes on this GPU: n = 4..128 Mbit (10^6 bits),
    m = 0.1 n, random bits, PA_PREC_AUTO.  Each result is checked on 256
    random outputs by pa_hash_select (the direct product)."""
    import synth
    out = []
    rng = np.random.default_rng(7)
    for mb, paper in PAPER_TABLE1.items():
        n = mb * 1_000_000
        m = n // 10
        prob = synth.random_problem(rng, n, m)
        r = run_single(pa, ctx, torch, prob, pa.PA_PREC_AUTO, reps, 2)
        idx = rng.integers(0, m, 256)
        s = torch.from_numpy(prob.seed.view(np.int64).copy()).to("cuda:0")
        k = torch.from_numpy(prob.key.view(np.int64).copy()).to("cuda:0")
        st, ref = pa.pa_hash_select(ctx, s, n, m, k, idx)
        assert st == pa.PA_OK, pa.pa_strerror(st)
        ok = bool(np.array_equal(ref, synth.bits_to_array(r["out"], m)[idx]))
        row = {"mbit": mb, "n": n, "m": m, "gbps": round(n * reps / r["elapsed"] / 1e9, 2),
               "ms_per_call": round(r["elapsed"] / reps * 1e3, 3), "fft_len": r["stats"]["fft_len"],
               "tiles": r["stats"]["tiles"], "spot_check_exact": ok, "paper_titan_xp_gbps": paper}
        log(f"[bench] table-1 shape: {row}")
        out.append(row)
    return out


def run_stream_leg(pa, ctx, torch, n: int = 128_000_000, m: int = 1_000_000, block: int = 16_000_000):
    """Block-serial hashing from host memory (the paper's Fig. 1-3 flow): a
    128 Mbit key with m = 10^6, fed in 16 Mbit blocks through pa_stream_feed
    (each block's key bits and seed slice copied over PCIe, hashed, XOR-merged
    on the device).  The rate includes the copies.  Checked on 256 outputs by
    pa_hash_select with the whole seed and key in device memory."""
    import synth
    rng = np.random.default_rng(9)
    prob = synth.random_problem(rng, n, m)
    keyb = synth.bits_to_array(prob.key, n)
    seedb = synth.bits_to_array(prob.seed, n + m - 1)
    blocks = []
    for lo in range(0, n, block):
        ln = min(block, n - lo)
        blocks.append((lo, ln, synth.array_to_bits(keyb[lo:lo + ln]),
                       synth.array_to_bits(seedb[n - lo - ln:n - lo + m - 1])))
    out = np.zeros(synth.words_for(m), np.uint64)
    times = []
    for rep in range(3):
        t0 = time.perf_counter()
        st, h = pa.pa_stream_open(ctx, n, m, pa.PA_PREC_AUTO)
        assert st == pa.PA_OK, pa.pa_strerror(st)
        for lo, ln, kb, sb in blocks:
            st = pa.pa_stream_feed(h, kb, lo, ln, sb)
            assert st == pa.PA_OK, pa.pa_strerror(st)
        st = pa.pa_stream_close(h, out)
        assert st == pa.PA_OK, pa.pa_strerror(st)
        times.append(time.perf_counter() - t0)
    el = float(np.median(times))
    s = torch.from_numpy(prob.seed.view(np.int64).copy()).to("cuda:0")
    k = torch.from_numpy(prob.key.view(np.int64).copy()).to("cuda:0")
    idx = rng.integers(0, m, 256)
    st, ref = pa.pa_hash_select(ctx, s, n, m, k, idx)
    assert st == pa.PA_OK
    return {"n": n, "m": m, "block_bits": block, "blocks": len(blocks), "source": "host memory (PCIe)",
            "gbps_including_copies": round(n / el / 1e9, 3), "ms": round(el * 1e3, 3),
            "spot_check_exact": bool(np.array_equal(ref, synth.bits_to_array(out, m)[idx]))}


def cpu_baseline(prob, target_s: float = 12.0, whole_s: float = 30.0, extra=None):
    """Oracle on a prefix of the outputs (full key): by the constant diagonals
    y[0:m'] is the hash with seed bits [0, n+m'-1) and m' outputs; its cost is
    linear in m', so the full job's time is t * m / m'.  When the whole job is
    projected to take at most whole_s seconds, the whole job is timed."""
    import oracle
    threads = oracle.default_threads()
    m_try = 4096
    t = 0.0
    while True:
        a = time.perf_counter()
        oracle.hash_words(prob.seed, prob.n, m_try, prob.key, threads=threads)
        t = time.perf_counter() - a
        if m_try >= prob.m:
            break
        if t * prob.m / m_try <= whole_s:
            m_try = prob.m
            continue
        if t >= target_s:
            break
        m_try = min(prob.m, int(m_try * min(8.0, max(2.0, target_s / max(t, 1e-3)))))
    full = t * prob.m / m_try
    others = {}
    for name, q in (extra or {}).items():   # small whole jobs (c1, c2), timed in full
        a = time.perf_counter()
        oracle.hash_words(q.seed, q.n, q.m, q.key, threads=threads)
        dt = time.perf_counter() - a
        others[name] = {"seconds": round(dt, 4), "gbps": round(q.n / dt / 1e9, 6), "n": q.n, "m": q.m}
    return {"value": prob.n / full / 1e9, "unit": "Gbps", "cores": threads, "kind": "oracle",
            "other_configs": others,
            "sample": (f"word-parallel oracle on the whole job ({prob.m} outputs, full key), {t:.2f} s"
                       if m_try >= prob.m else
                       f"word-parallel oracle on outputs [0, {m_try}) of {prob.m} (full key), "
                       f"{t:.2f} s, scaled by m/m' to {full:.1f} s for the whole job")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-job batch measurement")
    ap.add_argument("--serve", type=int, default=2000, help="requests in the serving leg (0: skip)")
    ap.add_argument("--only", choices=["fp32", "fp64"], default=None, help="run one path only (profiling)")
    ap.add_argument("--no-direct", action="store_true", help="skip the direct-path (short output) leg")
    ap.add_argument("--no-table1", action="store_true", help="skip the 4-128 Mbit sweep")
    ap.add_argument("--no-stream", action="store_true", help="skip the block-serial host streaming leg")
    ap.add_argument("--no-host", action="store_true", help="skip the c3 leg from host memory (PCIe copies)")
    ap.add_argument("--no-small", action="store_true", help="skip the c1 latency and c2 precision legs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 512 MiB device copy (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus > 1 or world > 1:
        print(json.dumps({"error": "the hash runs on one GPU here (how it would shard is a design note); "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_1805_02372_amd import pa

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    ctx = pa.pa_create(0, 0, None)
    golden = json.load(open(os.path.join(ROOT, "tests", "golden", "digests.json")))

    prob = synth.single_config("c3")
    res = {}
    paths = [("fp32", pa.PA_PREC_AUTO), ("fp64", pa.PA_PREC_FP64 | pa.PA_ASYNC)]
    if args.only:
        paths = [p for p in paths if p[0] == args.only]
    for name, flags in paths:
        log(f"[bench] c3 {name}: warmup {args.warmup}, steps {args.steps}")
        r = run_single(pa, ctx, torch, prob, flags, args.steps, args.warmup)
        ok = hashlib.sha256(r["out"].astype("<u8").tobytes()).hexdigest() == golden["c3"]["sha256"]
        r["bit_exact"] = ok
        res[name] = r
        log(f"[bench] c3 {name}: {prob.n * args.steps / r['elapsed'] / 1e9:.2f} Gbps, bit-exact={ok}, "
            f"kernel ms {r['kernel_ms']}")

    host = None
    if not args.only and not args.no_host:
        host = run_host_pointers(pa, ctx, prob)
        host["bit_exact"] = hashlib.sha256(host.pop("out").astype("<u8").tobytes()).hexdigest() == golden["c3"]["sha256"]
        log(f"[bench] c3 from host memory: {host}")

    c1 = c2 = None
    c1_prob = c2_prob = None
    if not args.only and not args.no_small:
        c1_prob, c1 = run_latency_c1(pa, ctx, torch)
        c1["bit_exact"] = hashlib.sha256(c1.pop("out").astype("<u8").tobytes()).hexdigest() == golden["c1"]["sha256"]
        log(f"[bench] c1 latency: {c1}")
        c2_prob, c2, c2_outs = run_c2(pa, ctx, torch, args.steps, args.warmup)
        for name, o in c2_outs.items():
            c2[name]["bit_exact"] = hashlib.sha256(o.astype("<u8").tobytes()).hexdigest() == golden["c2"]["sha256"]
        log(f"[bench] c2: {c2}")

    batch = None
    if not args.no_batch and not args.only:
        jobs = synth.batch_jobs()
        log(f"[bench] c4 batch of {len(jobs)} jobs")
        bsteps = max(10, args.steps)
        # segment sizes from the tuner: a context of its own measures the class
        # costs first (the headline context keeps the built-in model)
        bctx = pa.pa_create(0, 0, None)
        a = time.perf_counter()
        assert pa.pa_tune(bctx, pa.PA_PREC_AUTO, 3) == pa.PA_OK
        tune_s = time.perf_counter() - a
        try:
            batch = run_batch(pa, bctx, torch, jobs, pa.PA_PREC_AUTO, bsteps, max(1, args.warmup // 2))
        finally:
            pa.pa_destroy(bctx)
        batch["tune_s"] = tune_s
        g = golden.get("c4", [])
        bexact = len(g) == len(jobs) and all(
            hashlib.sha256(o.astype("<u8").tobytes()).hexdigest() == gg["sha256"]
            for o, gg in zip(batch["outs"], g))
        batch["bit_exact"] = bexact
        batch["gbps"] = sum(p.n for p in jobs) * bsteps / batch["elapsed"] / 1e9
        log(f"[bench] c4: {batch['gbps']:.2f} Gbps bit-exact={bexact}")

    direct = None
    if not args.only and not args.no_direct:
        direct = run_direct_leg(pa, ctx, torch, args.steps, args.warmup)
        log(f"[bench] direct leg: {direct}")
    table1 = None
    if not args.only and not args.no_table1:
        table1 = run_table1(pa, ctx, torch)
    stream = None
    if not args.only and not args.no_stream:
        stream = run_stream_leg(pa, ctx, torch)
        log(f"[bench] block-serial stream from host: {stream}")

    serving = None
    if args.serve and not args.only:
        log(f"[bench] serving leg, {args.serve} requests")
        serving = run_serving(pa, ctx, torch, args.serve)
        log(f"[bench] serving: {serving}")

    if args.calib_copy:
        a = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()

    head = res.get("fp32") or res.get("fp64")
    head_name = "fp32" if "fp32" in res else "fp64"
    st = head["stats"]
    value = prob.n * args.steps / head["elapsed"] / 1e9
    # roofline of the dominant kernel
    pb = launch_bytes(st, prob.n, prob.m)
    kms = head["kernel_ms"][:3]
    dom = int(np.argmax(kms))
    tiles = st["tiles"]
    achieved = pb[dom] / (kms[dom] * 1e-3) / 1e9
    traffic = None
    if os.path.exists(PROFILE_TRAFFIC):
        tr = json.load(open(PROFILE_TRAFFIC))
        if tr.get("kernel_digest") == kernel_source_digest():
            traffic = tr.get("bytes_per_launch", {}).get(f"pass{dom + 1}")
    valu = None   # the same kernel against the vector-ALU issue rate (counters of the same sources)
    if head_name == "fp32" and os.path.exists(PROFILE_VALU):
        vc = json.load(open(PROFILE_VALU))
        instr = vc.get("valu_wave_instructions_per_launch", {}).get(f"pass{dom + 1}")
        if vc.get("kernel_digest") == kernel_source_digest() and instr:
            rate = instr / (kms[dom] * 1e-3)
            valu = {"bound": "alu", "kernel": f"pass{dom + 1}", "achieved": round(rate / 1e9, 1),
                    "peak": round(VALU_WAVE_INSTR_PEAK / 1e9, 1), "unit": "G wave-instructions/s",
                    "frac": round(rate / VALU_WAVE_INSTR_PEAK, 4), "instructions": instr}
    pipeline_ms = sum(kms)
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gbps",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head_name == "fp32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "c3: one Toeplitz hash, n=12,345,679 key bits, m=1,234,567 output bits, "
                        "i.i.d. uniform bits (seed 2), inputs resident in HBM",
            "n": prob.n, "m": prob.m, "path": head_name,
            "plan": {"fft_len": st["fft_len"], "n1": st["n1"], "n2": st["n2"], "tiles": tiles,
                     "chunk_bits": st["chunk_bits"], "window_bits": st["window_bits"]},
        },
        "roofline": {
            "bound": "hbm", "kernel": f"pass{dom + 1}",
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel_ms": round(kms[dom], 5), "bytes_per_launch": round(pb[dom]),
        },
        "roofline_valu": valu,
        "pipeline": {
            "kernel_ms": [round(x, 5) for x in head["kernel_ms"]],
            "model_bytes": st["model_bytes"],
            "model_GBs": round(st["model_bytes"] / (pipeline_ms * 1e-3) / 1e9, 1),
            "model_frac": round(st["model_bytes"] / (pipeline_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        },
        "latency_ms": {"p50": round(float(np.percentile(head["lat"], 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(head["lat"], 99)) * 1e3, 4)},
        "bit_exact": bool(head["bit_exact"]),
        "max_residual": st["max_residual"],
        "fallback_tiles": st["fallback_tiles"],
        "precision": {"certified": CERT_NAMES[st["certified"]], "model_bound": st["bound"],
                      "rigorous_bound": st["rigorous_bound"], "max_residual": st["max_residual"],
                      "fallback_tiles": st["fallback_tiles"], "tiles": st["tiles"]},
    }
    if c1 is not None:
        line["c1_latency"] = c1
    if c2 is not None:
        line["c2_precision"] = c2
    if "fp64" in res and head_name != "fp64":
        r = res["fp64"]
        line["fp64_plain"] = {
            "gbps": round(prob.n * args.steps / r["elapsed"] / 1e9, 3),
            "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 4),
            "kernel_ms": [round(x, 5) for x in r["kernel_ms"]],
            "fft_len": r["stats"]["fft_len"], "tiles": r["stats"]["tiles"],
            "bit_exact": bool(r["bit_exact"]),
            "p99_ms": round(float(np.percentile(r["lat"], 99)) * 1e3, 4),
        }
    if batch is not None:
        line["batch_c4"] = {"jobs": 64, "gbps": round(batch["gbps"], 3), "tiles": batch["stats"]["tiles"],
                            "largest_fft_len": batch["stats"]["fft_len"], "bit_exact": bool(batch["bit_exact"]),
                            "fallback_tiles": batch["stats"]["fallback_tiles"],
                            "launches_per_batch": batch["stats"]["launches"],
                            "tuned": True, "tune_s": round(batch["tune_s"], 3),
                            "certified": CERT_NAMES[batch["stats"]["certified"]]}
    if host is not None:
        line["c3_host_pointers"] = host
    if batch is not None:
        line["batch_c4"]["direct_jobs"] = batch["stats"]["direct_jobs"]
    if direct is not None:
        line["direct_short_output"] = direct
    if table1 is not None:
        line["table1_sweep"] = table1
    if stream is not None:
        line["block_serial_host"] = stream
    if serving is not None:
        line["serving_c5"] = serving
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        extra = {k: v for k, v in (("c1", c1_prob), ("c2", c2_prob)) if v is not None}
        line["cpu_baseline"] = cpu_baseline(prob, extra=extra)
    pa.pa_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
