"""Helpers for GPU tests: device buffers (torch) and calls through the C ABI."""
from __future__ import annotations

import numpy as np

import synth


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU")
    return torch


def to_dev(words: np.ndarray):
    torch = torch_cuda()
    a = np.ascontiguousarray(words, dtype=np.uint64).view(np.int64)
    t = torch.from_numpy(a.copy()).to("cuda:0")
    torch.cuda.synchronize()   # the library's stream is not ordered after torch's
    return t


def from_dev(t) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint64).copy()


def empty_dev(words: int, fill: int = -1):
    torch = torch_cuda()
    # filled with ones so that untouched words are caught
    t = torch.full((max(1, words),), fill, dtype=torch.int64, device="cuda:0")
    torch.cuda.synchronize()   # the fill must land before the library's stream writes
    return t


def gpu_hash(pa, ctx, seed, n, m, key, flags=0):
    """Hash on the device; returns (status, output words)."""
    ds, dk = to_dev(seed), to_dev(key)
    out = empty_dev(synth.words_for(m))
    st = pa.pa_hash(ctx, ds, n, m, dk, out, flags)
    torch_cuda().cuda.synchronize()
    return st, from_dev(out)[: synth.words_for(m)]


def describe(words_a, words_b, m):
    a = synth.bits_to_array(words_a, m)
    b = synth.bits_to_array(words_b, m)
    bad = np.flatnonzero(a != b)
    return f"{bad.size} of {m} bits differ; first {bad[:10].tolist()}"
