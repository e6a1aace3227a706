"""ctypes binding of libpa (include/pa.h), same entry-point names.

Argument marshalling only: every step of the hash runs in the HIP library.
Bit strings are uint64 arrays (LSB-first).  Device buffers are torch tensors
on the context's device (pass them with PA_DEVICE_PTRS); host buffers are
numpy arrays.  If libpa.so is missing this module raises on import: there is
no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpa.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1805_02372_amd.build`")

# PyTorch bundles its own HIP runtime.  Load it first so that libpa binds to
# that same runtime (same soname) instead of pulling a second copy into the
# process; two runtimes in one process cannot share the device.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - the library also works without torch
    torch = None

_lib = ctypes.CDLL(LIB_PATH)

# ---- constants (mirror include/pa.h)
PA_OK, PA_EINVAL, PA_ENOMEM, PA_EDEVICE, PA_EPRECISION, PA_EBUSY, PA_ENOTREADY, PA_ESCRATCH = range(8)
PA_DEVICE_PTRS = 0x0001
PA_PREC_AUTO = 0x0000
PA_PREC_FP32_SEG = 0x0010
PA_PREC_FP64 = 0x0020
PA_PREC_NTT = 0x0030
PA_PREC_DIRECT = 0x0040
PA_PREC_MASK = 0x00F0
PA_NO_FALLBACK = 0x0100
PA_ASYNC = 0x0200
PA_TIMING = 0x0400
PA_CERT_NONE, PA_CERT_EXACT, PA_CERT_A_PRIORI, PA_CERT_A_POSTERIORI = range(4)

_u64p = ctypes.POINTER(ctypes.c_uint64)


class pa_job(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_void_p), ("key", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("m", ctypes.c_uint64)]


class pa_stats(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_uint32), ("log2_len", ctypes.c_uint32), ("n1", ctypes.c_uint32),
                ("n2", ctypes.c_uint32), ("chunk_bits", ctypes.c_uint64), ("window_bits", ctypes.c_uint64),
                ("tiles", ctypes.c_uint64), ("fallback_tiles", ctypes.c_uint64),
                ("max_residual", ctypes.c_double), ("max_abs", ctypes.c_double), ("bound", ctypes.c_double),
                ("ms_pass", ctypes.c_double * 4), ("model_bytes", ctypes.c_uint64), ("launches", ctypes.c_uint64),
                ("direct_jobs", ctypes.c_uint64), ("rigorous_bound", ctypes.c_double), ("certified", ctypes.c_uint32),
                ("fft_len", ctypes.c_uint32), ("live_requests", ctypes.c_uint64)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["ms_pass"] = list(self.ms_pass)
        return d


class pa_plan(ctypes.Structure):
    _fields_ = [("prec", ctypes.c_uint32), ("log2_len", ctypes.c_uint32), ("n1", ctypes.c_uint32),
                ("n2", ctypes.c_uint32), ("chunk_bits", ctypes.c_uint64), ("window_bits", ctypes.c_uint64),
                ("chunks", ctypes.c_uint64), ("windows", ctypes.c_uint64), ("bound", ctypes.c_double),
                ("cost", ctypes.c_double), ("direct_cost", ctypes.c_double), ("direct", ctypes.c_uint32),
                ("fft_len", ctypes.c_uint32), ("rigorous_bound", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_sig = {
    "pa_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.c_uint64, _P]),
    "pa_destroy": (None, [_P]),
    "pa_hash": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P, _P, ctypes.c_uint32]),
    "pa_hash_noalloc": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P, _P, ctypes.c_uint32]),
    "pa_hash_batch": (ctypes.c_int, [_P, ctypes.POINTER(pa_job), ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.POINTER(ctypes.c_int)]),
    "pa_hash_select": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P, _P, ctypes.c_uint64, _P,
                                      ctypes.c_uint32]),
    "pa_stream_open": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(_P)]),
    "pa_stream_feed": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint64, _P]),
    "pa_stream_state": (ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "pa_stream_resume": (ctypes.c_int, [_P, _P, ctypes.c_uint64]),
    "pa_stream_close": (ctypes.c_int, [_P, _P]),
    "pa_seed_register": (ctypes.c_int, [_P, _P, ctypes.c_uint64, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_uint32)]),
    "pa_submit": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, _P, _P,
                                 ctypes.POINTER(ctypes.c_uint64)]),
    "pa_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]),
    "pa_wait": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "pa_ticket_latency": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "pa_ticket_release": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "pa_last_stats": (ctypes.c_int, [_P, ctypes.POINTER(pa_stats)]),
    "pa_serve_stats": (ctypes.c_int, [_P, ctypes.POINTER(pa_stats)]),
    "pa_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "pa_plan_query": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.POINTER(pa_plan)]),
    "pa_error_model": (ctypes.c_double, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]),
    "pa_tune": (ctypes.c_int, [_P, ctypes.c_uint32, ctypes.c_int, ctypes.c_char_p]),
    "pa_tune_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = sorted(_sig)


class PAError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        self.status = status
        super().__init__(f"{where}: {pa_strerror(status)}")


def _check(st: int, where: str):
    if st != PA_OK:
        raise PAError(st, where)


def _ptr(buf) -> int:
    """Address of a torch tensor or numpy array."""
    if buf is None:
        return 0
    if isinstance(buf, int):
        return buf
    if hasattr(buf, "data_ptr"):
        return int(buf.data_ptr())
    if isinstance(buf, np.ndarray):
        if not buf.flags["C_CONTIGUOUS"]:
            raise ValueError("array must be contiguous")
        return int(buf.ctypes.data)
    raise TypeError(f"unsupported buffer type {type(buf)}")


def _is_device(buf) -> bool:
    return hasattr(buf, "is_cuda") and bool(buf.is_cuda)


# ------------------------------------------------------------------ API

def pa_strerror(status: int) -> str:
    return _lib.pa_strerror(int(status)).decode()


def pa_create(device: int = 0, hbm_budget_bytes: int = 0, stream=None):
    """Context on `device`.  stream: a torch.cuda.Stream / raw hipStream_t or None."""
    raw = 0
    if stream is not None:
        raw = int(getattr(stream, "cuda_stream", stream))
    ctx = _P()
    _check(_lib.pa_create(ctypes.byref(ctx), int(device), int(hbm_budget_bytes), raw or None), "pa_create")
    return ctx


def pa_destroy(ctx) -> None:
    if ctx:
        _lib.pa_destroy(ctx)


def pa_hash(ctx, seed, n: int, m: int, key, out, flags: int = 0) -> int:
    """out = T(seed) key.  Device tensors need PA_DEVICE_PTRS (added
    automatically when all three are device tensors).  Returns the status."""
    if _is_device(seed) and _is_device(key) and _is_device(out):
        flags |= PA_DEVICE_PTRS
    return _lib.pa_hash(ctx, _ptr(seed), int(n), int(m), _ptr(key), _ptr(out), int(flags))


def pa_hash_noalloc(ctx, seed, n: int, m: int, key, out, flags: int = 0) -> int:
    """pa_hash without device allocation (device tensors only; PA_DEVICE_PTRS
    is added).  Returns the status."""
    return _lib.pa_hash_noalloc(ctx, _ptr(seed), int(n), int(m), _ptr(key), _ptr(out), int(flags) | PA_DEVICE_PTRS)


class JobBatch:
    """The pa_job descriptors of a list of (seed, key, out, n, m), packed once.
    Repeated pa_hash_batch calls over the same buffers can pass this instead
    of the list, which skips re-reading 3 addresses per job (about 1 us per
    job in Python)."""

    def __init__(self, jobs):
        self.count = len(jobs)
        self.arr = (pa_job * max(1, self.count))()
        dev = self.count > 0
        for i, (seed, key, out, n, m) in enumerate(jobs):
            self.arr[i] = pa_job(_ptr(seed), _ptr(key), _ptr(out), int(n), int(m))
            dev = dev and _is_device(seed) and _is_device(key) and _is_device(out)
        self.device = dev
        self.jobs = list(jobs)   # keeps the buffers alive with the descriptors


def pa_hash_batch(ctx, jobs, flags: int = 0):
    """jobs: list of (seed, key, out, n, m), or a JobBatch of such a list.
    Returns (status, per-job statuses)."""
    if not isinstance(jobs, JobBatch):
        jobs = JobBatch(jobs)
    if jobs.device:
        flags |= PA_DEVICE_PTRS
    per = (ctypes.c_int * max(1, jobs.count))()
    st = _lib.pa_hash_batch(ctx, jobs.arr, jobs.count, int(flags), per)
    return st, list(per)[:jobs.count]


def pa_hash_select(ctx, seed, n: int, m: int, key, idx, flags: int = 0):
    """Output bits y[idx[k]] by the direct GF(2) product on the device.
    seed/key: device tensors (PA_DEVICE_PTRS added) or host arrays; idx: a
    sequence of indices < m.  Returns (status, uint8 array of bits)."""
    if _is_device(seed) and _is_device(key):
        flags |= PA_DEVICE_PTRS
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
    bits = np.zeros(len(ix), np.uint8)
    st = _lib.pa_hash_select(ctx, _ptr(seed), int(n), int(m), _ptr(key), _ptr(ix) if len(ix) else None,
                             len(ix), _ptr(bits) if len(ix) else None, int(flags))
    return st, bits


def pa_stream_open(ctx, n: int, m: int, flags: int = 0):
    """Block-serial hashing of an (n, m) job.  Returns (status, stream)."""
    h = _P()
    st = _lib.pa_stream_open(ctx, int(n), int(m), int(flags), ctypes.byref(h))
    return st, h


def pa_stream_feed(stream, key_block, lo: int, length: int, seed_block) -> int:
    """XOR the partial hash of key bits [lo, lo+length) into the accumulator
    (seed_block: seed bits [n-lo-length, n-lo+m-1))."""
    return _lib.pa_stream_feed(stream, _ptr(key_block), int(lo), int(length), _ptr(seed_block))


def pa_stream_state(stream, acc=None):
    """Copy the accumulator into acc (if given); returns (status, fed_bits)."""
    fed = ctypes.c_uint64(0)
    st = _lib.pa_stream_state(stream, _ptr(acc) if acc is not None else None, ctypes.byref(fed))
    return st, int(fed.value)


def pa_stream_resume(stream, acc, fed_bits: int) -> int:
    return _lib.pa_stream_resume(stream, _ptr(acc), int(fed_bits))


def pa_stream_close(stream, out=None) -> int:
    return _lib.pa_stream_close(stream, _ptr(out) if out is not None else None)


def pa_seed_register(ctx, seed, nbits: int, flags: int = 0) -> int:
    if _is_device(seed):
        flags |= PA_DEVICE_PTRS
    sid = ctypes.c_uint32()
    _check(_lib.pa_seed_register(ctx, _ptr(seed), int(nbits), int(flags), ctypes.byref(sid)), "pa_seed_register")
    return int(sid.value)


def pa_submit(ctx, seed_id: int, n: int, m: int, key, out) -> tuple[int, int]:
    """Returns (status, ticket)."""
    t = ctypes.c_uint64()
    st = _lib.pa_submit(ctx, int(seed_id), int(n), int(m), _ptr(key), _ptr(out), ctypes.byref(t))
    return st, int(t.value)


def pa_poll(ctx, ticket: int) -> bool:
    d = ctypes.c_int()
    _check(_lib.pa_poll(ctx, int(ticket), ctypes.byref(d)), "pa_poll")
    return bool(d.value)


def pa_wait(ctx, ticket: int) -> int:
    return _lib.pa_wait(ctx, int(ticket))


def pa_ticket_latency(ctx, ticket: int) -> float:
    s = ctypes.c_double()
    _check(_lib.pa_ticket_latency(ctx, int(ticket), ctypes.byref(s)), "pa_ticket_latency")
    return float(s.value)


def pa_ticket_release(ctx, ticket: int) -> int:
    """Free a finished ticket's record.  Returns the status."""
    return _lib.pa_ticket_release(ctx, int(ticket))


def pa_last_stats(ctx) -> dict:
    s = pa_stats()
    _check(_lib.pa_last_stats(ctx, ctypes.byref(s)), "pa_last_stats")
    return s.as_dict()


def pa_serve_stats(ctx) -> dict:
    s = pa_stats()
    _check(_lib.pa_serve_stats(ctx, ctypes.byref(s)), "pa_serve_stats")
    return s.as_dict()


def pa_plan_query(n: int, m: int, flags: int = 0) -> dict:
    p = pa_plan()
    _check(_lib.pa_plan_query(int(n), int(m), int(flags), ctypes.byref(p)), "pa_plan_query")
    return p.as_dict()


def pa_tune(ctx, flags: int = 0, reps: int = 3, path: str | None = None) -> int:
    """Measure per-tile class costs for this context's planner (and write them
    to `path` as JSON when given).  Returns the status."""
    return _lib.pa_tune(ctx, int(flags), int(reps), path.encode() if path else None)


def pa_tune_load(ctx, path: str) -> int:
    return _lib.pa_tune_load(ctx, path.encode())


def pa_error_model(prec: int, log2_len: int, chunk_bits: int) -> float:
    return float(_lib.pa_error_model(int(prec), int(log2_len), int(chunk_bits)))
