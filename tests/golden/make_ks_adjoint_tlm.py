"""Write tests/golden/ks_adjoint_tlm.json: for the KS adjoint workload (2^16
points, dt = 0.005, dx = 0.5, 20,000 steps, J = mean of u^2 over the final
2,000 steps), J itself and its derivative along each of the 16 seeded unit
directions of workloads.adjoint_directions, by the oracle's tangent-linear
model (forward-mode stepping, no truncation error).

Calls only oracle/ (and the seeded generators of workloads.py).

    python tests/golden/make_ks_adjoint_tlm.py
"""
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "ks_adjoint_tlm.json")


def main(nsteps=None):
    oracle.build(force=False)
    w = workloads.WORKLOADS["ks_adjoint"]
    n, dt, dx = w["n"], w["dt"], w["dx"]
    nsteps = w["nsteps"] if nsteps is None else nsteps
    window = workloads.KS_ADJOINT_WINDOW
    n0 = nsteps - window + 1
    wgt = 1.0 / (window * n)
    u0 = workloads.initial("ks_adjoint")
    dirs = workloads.adjoint_directions(n)
    t0 = time.time()
    dJ = oracle.ks_tlm(u0, nsteps, dt, dx, n0, wgt, dirs)
    t_tlm = time.time() - t0
    # J itself: the oracle's fields at steps n0 .. nsteps, each summed exactly
    u = oracle.ks(u0, n0 - 1, dt, dx)
    terms = []
    for _ in range(window):
        u = oracle.ks(u, 1, dt, dx)
        terms.append(math.fsum(u * u))
    J = wgt * math.fsum(terms)
    rec = {"workload": "KS N=2^16 dt=0.005 dx=0.5, %d steps, J = mean of u^2 over steps "
                       "%d..%d; u0 = initial('ks_adjoint'); directions = "
                       "adjoint_directions(2^16) (16 unit vectors, seed 1104)" % (nsteps, n0, nsteps),
           "n": n, "nsteps": nsteps, "window_first": n0, "window_weight": wgt,
           "J": J.hex(), "J_float": J,
           "dJ": [float(x).hex() for x in dJ], "dJ_float": [float(x) for x in dJ],
           "tlm_seconds": t_tlm, "oracle_threads": oracle.max_threads()}
    with open(OUT, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print("J = %.17g; dJ[0..3] = %s (%.0f s)" % (J, list(dJ[:4]), t_tlm))


if __name__ == "__main__":
    main()
