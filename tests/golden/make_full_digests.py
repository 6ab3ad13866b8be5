"""Write tests/golden/full_digests.json: SHA-256 digests of the oracle's
whole-field results on the full-size workloads, so that GPU tests can compare
every point of a full run with the oracle without running the oracle there.

Calls only oracle/ (and the seeded input generators of workloads.py).  Each
run is the plain full-grid step-by-step definition; at 8 host threads the
three runs take about 20 minutes.

    python tests/golden/make_full_digests.py
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "full_digests.json")


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def cases():
    """(name, description, function returning the oracle's field)."""
    wh, wk = workloads.WORKLOADS["heat_large"], workloads.WORKLOADS["ks"]
    return [
        ("heat_large_f64", "heat N=2^24 f64 r=0.25 20000 steps, u0 = initial('heat_large')",
         lambda: oracle.heat(workloads.initial("heat_large"), wh["nsteps"], wh["r"])),
        ("heat_large_f32", "heat N=2^24 f32 r=0.25 20000 steps, u0 = initial('heat_large', f32)",
         lambda: oracle.heat(workloads.initial("heat_large", np.float32), wh["nsteps"], wh["r"])),
        ("ks", "KS N=2^20 dt=0.005 dx=0.5 50000 steps, u0 = initial('ks')",
         lambda: oracle.ks(workloads.initial("ks"), wk["nsteps"], wk["dt"], wk["dx"])),
    ]


def main():
    oracle.build(force=False)
    rec = {}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            rec = json.load(fh)
    want = sys.argv[1:]
    for name, desc, fn in cases():
        if want and name not in want:
            continue
        t0 = time.time()
        u = fn()
        rec[name] = {"workload": desc, "dtype": str(u.dtype), "n": int(u.size),
                     "sha256": digest(u), "max_abs": float(np.abs(u).max()),
                     "oracle_threads": oracle.max_threads()}
        print("%s: %s (%.0f s)" % (name, rec[name]["sha256"], time.time() - t0), flush=True)
        with open(OUT, "w") as fh:
            json.dump(rec, fh, indent=1, sort_keys=True)
            fh.write("\n")


if __name__ == "__main__":
    main()
