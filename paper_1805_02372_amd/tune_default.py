"""Measure the default tuning table that ships beside libpa.so.

Usage (on an MI355X): python -m paper_1805_02372_amd.tune_default [out.json]

Runs pa_tune for FP32, FP64 and the direct path (PA_PREC_AUTO) and for the
NTT, each class timed with one-tile and four-tile launches, and writes one
table in pa_tune's format.  Contexts load it as their starting cost model
(tune_mi355x.json next to libpa.so); pa_tune or PA_TUNE_CACHE replace it.
"""
from __future__ import annotations

import json
import os
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune_mi355x.json")


def main(out: str = DEFAULT_OUT, reps: int = 5) -> dict:
    from paper_1805_02372_amd import pa
    os.environ["PA_TUNE_DEFAULT"] = "0"   # measure from the built-in model, not the table being replaced
    merged: dict = {}
    with tempfile.TemporaryDirectory() as tmp:
        for name, flags in (("auto", pa.PA_PREC_AUTO), ("ntt", pa.PA_PREC_NTT)):
            ctx = pa.pa_create(0, 0, None)
            try:
                path = os.path.join(tmp, name + ".json")
                st = pa.pa_tune(ctx, flags, reps, path)
                if st != pa.PA_OK:
                    raise RuntimeError(f"pa_tune({name}): {pa.pa_strerror(st)}")
                part = json.load(open(path))
            finally:
                pa.pa_destroy(ctx)
            for k, v in part.items():
                if k in ("launch", "direct", "direct_launch") and k in merged and name == "ntt":
                    continue   # launch and direct-path costs from the FP32/FP64 run
                merged[k] = v
    with open(out, "w") as f:
        json.dump(merged, f, indent=1, sort_keys=True)
        f.write("\n")
    return merged


if __name__ == "__main__":
    t = main(sys.argv[1] if len(sys.argv) > 1 else DEFAULT_OUT)
    print("classes:", {k: len(v) for k, v in t.items() if isinstance(v, dict)}, "launch", t["launch"])
