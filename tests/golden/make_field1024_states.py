"""Write field1024_states.json: states of the FP64 oracle's weighted-GS run
on the 1024 x 1024, 400-spot workload (field1024), for one-step parity
tests at iterations 1, 10 and 99.

The state entering iteration k is (phi_k, W_k) with phi_k = arg F_c^{-1}
y_{k-1}; it is stored as the farfield projection y_{k-1} (400 complex
numbers) and the weights W_k, so a test rebuilds phi_k with one oracle
adjoint instead of reading a megapixel phase.  Only the oracle and the
seeded input generators are used.

Usage: python tests/golden/make_field1024_states.py   (about 15-20 minutes
on 8 cores)
"""

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

KEEP = (1, 10, 99)


def main():
    d = workloads.field1024()
    geom = oracle.Geometry(d["nx"], d["ny"])
    basis = oracle.ZernikeBasis(d["modes"])
    amp = d["amp"].astype(np.float32).astype(np.float64)
    t = d["t"].astype(np.float32).astype(np.float64)
    phi = d["phi0"].astype(np.float32).astype(np.float64)
    W = np.ones(len(t))
    states, stats = {}, []
    t0 = time.time()
    for it in range(max(KEEP)):
        phi, W, E, st, y = oracle.wgs_step(phi, W, t, amp, d["w"], basis,
                                           geom, return_y=True)
        stats.append([float(v) for v in st])
        if it + 1 in KEEP:
            states[str(it + 1)] = {
                "y_re": [float(v) for v in y.real],
                "y_im": [float(v) for v in y.imag],
                "W": [float(v) for v in W]}
        print("iteration %d: efficiency %.5f uniformity %.5f (%.0f s)"
              % (it, st[0], st[1], time.time() - t0), flush=True)
    out = {"workload": "field1024", "seed": workloads.BASE_SEED + 2,
           "note": "state entering iteration k: W_k and the projection "
                   "y_{k-1}, phi_k = arg(oracle.adjoint(y_{k-1}))",
           "states": states,
           "stats_per_iteration": stats}
    with open(os.path.join(HERE, "field1024_states.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
