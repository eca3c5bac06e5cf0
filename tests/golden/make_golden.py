"""Write stored oracle results used by the GPU parity tests at full size.

Calls only the FP64 oracle (oracle/) on the seeded workloads; nothing here
comes from the HIP path.  Usage:
    python tests/golden/make_golden.py phantom64      # ~20 min on 8 cores
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import solve  # noqa: E402
from paper_2105_01028_amd import workloads as W  # noqa: E402


def phantom64():
    """Per-step detector records and budget of the 64^3 x 192 x 1000-step phantom."""
    p = W.config2()
    t0 = time.time()
    S = solve.build(p)
    state = None
    det = np.zeros((p.ndet, p.steps))
    budget = np.zeros((p.steps, 4))
    for m in range(p.steps):
        r = solve.forward(p, steps=1, S=S, state0=state, start_step=m)
        state = r.state
        det[:, m] = r.det[:, 0]
        budget[m] = (r.injected[0], r.absorbed[0], r.escaped[0].sum(), r.in_domain[0])
        if m % 50 == 0:
            print(f"step {m} {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, "phantom64_oracle.npz"), det=det, budget=budget,
                        dt=S.dt, steps=p.steps)


if __name__ == "__main__":
    {"phantom64": phantom64}[sys.argv[1]]()
