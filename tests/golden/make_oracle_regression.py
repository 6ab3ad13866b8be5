"""Write tests/golden/oracle_regression.json: the oracle's outputs on a few
tiny seeded cases, as hexadecimal binary64 (or binary32) values.

The file calls only oracle/ and workloads.py (the seeded input generators).
It is a regression record of the oracle's arithmetic, not a pin: the pins
in tests/test_oracle_pins.py tie the oracle to the paper and to closed forms;
this file makes any later change to the oracle's bits visible in review.

    python tests/golden/make_oracle_regression.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle      # noqa: E402
import workloads   # noqa: E402


def cases():
    """(name, inputs, callable producing the oracle output)."""
    u = workloads.white_noise(16, seed=1)
    yield "heat_f64_n16_s10_r0.25", lambda: oracle.heat(u, 10, 0.25)
    u32 = workloads.white_noise(16, seed=2, dtype=np.float32)
    yield "heat_f32_n16_s10_r0.3", lambda: oracle.heat(u32, 10, 0.3)
    v = workloads.smoothed_noise(16, seed=3)
    yield "ks_n16_s5", lambda: oracle.ks(v, 5, workloads.KS_DT, workloads.KS_DX)
    q = workloads.euler_smooth(8, seed=4)
    yield "euler_n8_s3", lambda: oracle.euler(q, 3, workloads.EULER_CFL / 8, 1.0 / 8,
                                              workloads.EULER_GAMMA)
    w = 3 * workloads.smoothed_noise(12, seed=5)
    yield "ks_adjoint_n12_s4_first2", lambda: oracle.ks_adjoint(
        w, 4, workloads.KS_DT, workloads.KS_DX, 2, 1.0 / 60)


def hexes(a):
    a = np.asarray(a)
    return [float(x).hex() for x in a.ravel()], str(a.dtype), list(a.shape)


def main():
    oracle.build(force=False)
    out = {}
    for name, fn in cases():
        vals, dtype, shape = hexes(fn())
        out[name] = {"dtype": dtype, "shape": shape, "values": vals}
    with open(os.path.join(HERE, "oracle_regression.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
