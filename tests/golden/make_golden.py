"""Write tests/golden/digests.json from the CPU oracle (only ``oracle`` and
``synth`` are called).

The paper prints no worked example with bit values, so no stored value here
comes from the paper.  These digests let GPU tests at full size compare whole
outputs without re-running the oracle there.  Each entry: SHA-256 of the
output words as little-endian bytes (tail bits beyond m zero), the output
weight, and the first output word.

Usage:  python tests/golden/make_golden.py [c1 c2 c3 c4]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "digests.json")


def digest(words: np.ndarray) -> dict:
    w = np.ascontiguousarray(words, dtype="<u8")
    return {
        "sha256": hashlib.sha256(w.tobytes()).hexdigest(),
        "weight": int(np.unpackbits(w.view(np.uint8)).sum()),
        "word0": f"{int(w[0]):016x}",
    }


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        if name == "c4":
            jobs = synth.batch_jobs()
            data["c4"] = []
            for p in jobs:
                y = oracle.hash_words(p.seed, p.n, p.m, p.key)
                data["c4"].append(dict(n=p.n, m=p.m, **digest(y)))
        else:
            p = synth.single_config(name)
            y = oracle.hash_words(p.seed, p.n, p.m, p.key)
            data[name] = dict(n=p.n, m=p.m, **digest(y))
        print(f"{name}: {time.time() - t0:.1f} s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1", "c2", "c3"])
