"""Write the oracle-derived golden files of tests/golden/ (calls only oracle/).

The paper prints no worked example, so these files are not values from the
paper: they record the FP64 oracle's own trajectory on the 100^3, 10^4-entry,
J=(5,5,5) planted workload (seed 0, lambda 0.01, 5 iterations, Alg. 2 without
the final QR) so that later changes to the oracle are caught.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    p = synth.make_c1()
    G = p.core.astype(np.float64)
    A0 = [a.astype(np.float64) for a in p.factors]
    val = p.val.astype(np.float64)
    sse0 = oracle.sse(G, A0, p.idx, val)
    A, L, S = oracle.fit(G, A0, p.idx, val, p.lam, p.iters)
    out = {
        "workload": "c1: 100x100x100, 10^4 distinct uniform cells, J=(5,5,5), "
                    "planted N(0,1) + N(0,0.01), lambda=0.01, seed 0",
        "source": "FP64 oracle (oracle/ptk_oracle.c), Alg. 2 iterations",
        "sse_init": sse0,
        "sse_per_iter": S.tolist(),
        "loss_after_mode": L.tolist(),
        "rows_mode0_first5": A[0][:5].tolist(),
        "rows_mode2_last5": A[2][-5:].tolist(),
    }
    with open(os.path.join(HERE, "c1_oracle_trajectory.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
