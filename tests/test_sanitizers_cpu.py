"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the planner (plan, batch groups, error model, direct-path cost) and, in a
separate program, the oracle's C loops.  Each harness is compiled with g++/gcc
and must run clean."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_02372_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]

PLANNER_HARNESS = r"""
#include "planner.hpp"
#include "pa.h"
#include <cstdio>
#include <vector>
using namespace pa;
int main() {
    CostModel cm;
    uint64_t sizes[] = {1, 2, 63, 64, 65, 1000, 4097, 131072, 1000003, 12345679, 100000000, 1ull << 30};
    int policies[] = {PREC_FP32, PREC_FP64, PREC_NTT};
    unsigned long long plans = 0;
    for (uint64_t n : sizes)
        for (uint64_t m : sizes)
            for (int p : policies) {
                TilePlan tp;
                if (plan_job(n, m, p, cm, &tp)) {
                    ++plans;
                    if (tp.Bi + tp.Bo - 1 > tp.L || tp.L != class_len(tp.cls)) return 2;
                    (void)choose_direct(PA_PREC_AUTO, n, m, cm, tp);
                }
                (void)direct_cost(n, m, cm);
            }
    for (int id = kMinClassId; id <= kMaxClassId; ++id) {
        const uint64_t L = class_len(id);
        if (L == 0) continue;
        for (uint64_t bi : {(uint64_t)1, (uint64_t)1000, L / 2, L - 1}) {
            (void)error_bound(PREC_FP32, L, bi);
            (void)rigorous_bound(PREC_FP64, L, bi, L - bi + 1);
        }
    }
    std::vector<uint64_t> ns, ms;
    for (int i = 0; i < 64; ++i) {
        ns.push_back(100000 + 154321ull * i);
        ms.push_back(1 + 9973ull * i);
    }
    std::vector<BatchGroup> g;
    if (!plan_batch_groups(ns, ms, PREC_FP32, cm, &g)) return 3;
    std::printf("plans %llu groups %zu\n", plans, g.size());
    return 0;
}
"""

ORACLE_HARNESS = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
void oracle_hash_bits(const uint64_t*, uint64_t, uint64_t, const uint64_t*, uint64_t*);
int oracle_hash_words(const uint64_t*, uint64_t, uint64_t, const uint64_t*, uint64_t*, int);
int oracle_hash_select(const uint64_t*, uint64_t, uint64_t, const uint64_t*, const uint64_t*, uint64_t, uint8_t*);
static uint64_t rnd(uint64_t* s) { *s ^= *s << 13; *s ^= *s >> 7; *s ^= *s << 17; return *s; }
int main(void) {
    uint64_t st = 88172645463325252ull;
    const uint64_t shapes[][2] = {{1, 1}, {1, 130}, {130, 1}, {63, 65}, {64, 64}, {65, 63}, {777, 1333}, {4097, 95}};
    for (unsigned c = 0; c < sizeof shapes / sizeof shapes[0]; ++c) {
        const uint64_t n = shapes[c][0], m = shapes[c][1];
        const uint64_t sw = (n + m - 1 + 63) / 64, kw = (n + 63) / 64, ow = (m + 63) / 64;
        uint64_t *s = malloc(sw * 8), *k = malloc(kw * 8), *a = malloc(ow * 8), *b = malloc(ow * 8);
        uint64_t* idx = malloc(m * 8);
        uint8_t* bits = malloc(m);
        for (uint64_t i = 0; i < sw; ++i) s[i] = rnd(&st);
        for (uint64_t i = 0; i < kw; ++i) k[i] = rnd(&st);
        for (uint64_t i = 0; i < m; ++i) idx[i] = i;
        oracle_hash_bits(s, n, m, k, a);
        if (oracle_hash_words(s, n, m, k, b, 3) != 0) return 2;
        if (oracle_hash_select(s, n, m, k, idx, m, bits) != 0) return 3;
        for (uint64_t i = 0; i < ow; ++i) if (a[i] != b[i]) return 4;
        for (uint64_t i = 0; i < m; ++i) if (bits[i] != ((a[i >> 6] >> (i & 63)) & 1)) return 5;
        free(s); free(k); free(a); free(b); free(idx); free(bits);
    }
    printf("oracle clean\n");
    return 0;
}
"""


def _run(tmp_path, name, src, compiler, sources, extra):
    cc = shutil.which(compiler)
    if cc is None:
        pytest.skip(f"{compiler} not available")
    main_src = tmp_path / (f"{name}.cpp" if compiler == "g++" else f"{name}.c")
    main_src.write_text(src)
    exe = tmp_path / name
    cmd = [cc, *SAN, *extra, str(main_src), *sources, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    if "does not come first in initial library list" in out.stderr:
        pytest.skip("the environment preloads a library ahead of the sanitizer runtime")
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert "runtime error" not in out.stderr and "AddressSanitizer" not in out.stderr, out.stderr[-4000:]
    return out.stdout


def test_planner_under_sanitizers(tmp_path):
    out = _run(tmp_path, "planner_san", PLANNER_HARNESS, "g++",
               [os.path.join(CSRC, "planner.cpp")],
               ["-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include")])
    assert out.startswith("plans ")


def test_oracle_under_sanitizers(tmp_path):
    out = _run(tmp_path, "oracle_san", ORACLE_HARNESS, "gcc",
               [os.path.join(ROOT, "oracle", "toeplitz_oracle.c")], ["-std=c11", "-pthread"])
    assert "oracle clean" in out
