"""Benchmark of the TRINITY time step on one MI355X.

A step is one pass of the whole hot path (inject, scattering contraction,
transport sweep, tallies) over the phantom-scale workload: a 64^3 voxel grid
with +-5% voxel noise, 192 HEALPix directions (the Sec. 3.1 phantom shape on
synthetic data).  The metric is voxel x direction x step updates per second,
with the state resident in HBM.  Kernel durations come from HIP events
recorded around every kernel on the medium's stream inside the timed region.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("voxel·direction·step updates/s (FP32 vs BF16-split); "
          "p50/p99 solve latency")
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16split": 2500.0}


def kernel_rooflines(prof, prob, precision):
    """Achieved rates of the collide (MFMA) and sweep (HBM) kernels from their
    average launch durations and the algorithmic work per launch."""
    N, V = prob.ndir, prob.nvox
    out = {}
    ms, n = prof["collide"]
    if n:
        t = ms / n * 1e-3
        flop = 2.0 * N * N * V * (3 if precision == "bf16split" else 1)
        out["collide"] = {"bound": "mfma", "achieved": flop / t / 1e12,
                          "peak": PEAK_TFLOPS[precision], "unit": "TFLOP/s",
                          "frac": flop / t / 1e12 / PEAK_TFLOPS[precision],
                          "avg_ms": ms / n, "work_per_launch": flop, "traffic": None}
    ms, n = prof["sweep"]
    if n:
        t = ms / n * 1e-3
        byt = 8.0 * N * V
        out["sweep"] = {"bound": "hbm", "achieved": byt / t / 1e9, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": byt / t / 1e9 / PEAK_HBM_GBS,
                        "avg_ms": ms / n, "work_per_launch": byt, "traffic": None}
    return out


def timed_run(prob, steps, warmup, stream):
    import torch

    from paper_2105_01028_amd import trinity as T
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(prob)
        m.solve(warmup)
        # instrumented timed region: HIP events around every kernel
        m.reset()
        m.profile_begin(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = m.profile_end()
        budget = m.read_budget()
        # the same steps replayed from captured graphs, no events
        m.reset()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        torch.cuda.synchronize()
        g1 = time.perf_counter()
        m.close()
    inj = budget[:, 0].sum()
    closure = abs(inj - budget[:, 1].sum() - budget[:, 3:].sum() - budget[-1, 2]) / max(inj, 1e-300)
    return t1 - t0, g1 - g0, prof, closure


def latency(prob, solves, stream):
    """Wall time of complete solves (create excluded): p50 / p99 in ms."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    times = []
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(prob)
        m.solve(prob.steps)
        for _ in range(solves):
            m.reset()
            t0 = time.perf_counter()
            m.solve(prob.steps)
            m.read_detectors()
            times.append((time.perf_counter() - t0) * 1e3)
        m.close()
    return float(np.percentile(times, 50)), float(np.percentile(times, 99))


def cpu_baseline(prob, budget_s=15.0):
    """The FP64 oracle on the host cores, on the first steps of the same workload."""
    from oracle import solve
    t_setup = time.perf_counter()
    S = solve.build(prob)
    t0 = time.perf_counter()
    res = None
    steps = 0
    while time.perf_counter() - t0 < budget_s or steps < 2:
        res = solve.forward(prob, steps=1, S=S, state0=None if res is None else res.state,
                            start_step=steps)
        steps += 1
    el = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count()
    return {"value": prob.nvox * prob.ndir * steps / el, "unit": "updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"first {steps} steps of the same 64^3 x 192 workload, FP64 NumPy "
                      f"(set-up {t0 - t_setup:.1f} s excluded)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16split"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design, not part of this build)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2105_01028_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    stream = torch.cuda.Stream()
    prob = W.config2().copy(precision=args.precision)
    K, Wm = args.steps, args.warmup
    el, el_graph, prof, closure = timed_run(prob, K, Wm, stream)
    updates = prob.nvox * prob.ndir * K
    roof = kernel_rooflines(prof, prob, args.precision)
    dom = max(("collide", "sweep"), key=lambda k: prof[k][0])
    rl = dict(roof[dom])
    rl["kernel"] = dom
    rl = {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                             "avg_ms", "work_per_launch")}
    out = {
        "metric": METRIC, "value": updates / el, "unit": "updates/s", "n_gpus": 1,
        "steps": K, "warmup": Wm, "ms_per_step": el / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3-f32acc",
        "data": "synthetic",
        "config": {"workload": "phantom 64^3, 1 mm voxels, +-5% noise, 192 directions "
                               "(nside 4), phase advance", "grid": [64, 64, 64], "ndir": 192,
                   "precision": args.precision},
        "roofline": rl,
        "kernels": {k: {"avg_ms": v[0] / v[1] if v[1] else 0.0, "launches": v[1]}
                    for k, v in prof.items()},
        "kernel_rooflines": roof,
        "graph_replay": {"value": updates / el_graph, "ms_per_step": el_graph / K * 1e3},
        "budget_closure": closure,
    }
    if not args.no_extras:
        other = "bf16split" if args.precision == "fp32" else "fp32"
        e2, g2, p2, c2 = timed_run(prob.copy(precision=other), K, Wm, stream)
        out[other] = {"value": updates / e2, "ms_per_step": e2 / K * 1e3,
                      "graph_value": updates / g2, "kernel_rooflines":
                      kernel_rooflines(p2, prob, other), "budget_closure": c2}
        p50, p99 = latency(W.config1(), 30, stream)
        out["latency_uniform16"] = {"p50_ms": p50, "p99_ms": p99, "solves": 30,
                                    "workload": "16^3, 48 directions, 200 steps"}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
