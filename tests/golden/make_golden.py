"""Write stored oracle results used by the GPU parity tests at full size.

Calls only the FP64 oracle (oracle/) on the seeded workloads; nothing here
comes from the HIP path.  Usage:
    python tests/golden/make_golden.py phantom64      # ~20 min on 8 cores
    python tests/golden/make_golden.py retarded64     # ~30 min on 8 cores
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import medium, retarded, solve  # noqa: E402
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


RETARDED_STEPS = 600


def retarded64():
    """The same phantom stepped at a fifth of the voxel crossing time with the
    retarded history: per-step detector records and budget of 600 steps."""
    p = W.config2()
    p = p.copy(advance="retarded",
               dt_ps=0.2 * p.dx_mm * float(p.n.flat[0]) / medium.C0_MM_PER_PS)
    t0 = time.time()
    r = retarded.forward(p, RETARDED_STEPS)
    print(f"{RETARDED_STEPS} steps {time.time() - t0:.0f} s", flush=True)
    budget = np.stack([r.injected, r.absorbed, r.escaped.sum(axis=1), r.in_domain], axis=1)
    np.savez_compressed(os.path.join(HERE, "retarded64_oracle.npz"), det=r.det, budget=budget,
                        dt=r.setup.dt, steps=RETARDED_STEPS, history=r.setup.H)


if __name__ == "__main__":
    {"phantom64": phantom64, "retarded64": retarded64}[sys.argv[1]]()
