"""Benchmark of the TRINITY time step on one MI355X.

A step is one pass of the whole hot path (inject, scattering contraction,
transport with Fresnel interception and gather, tallies) over the
heterogeneous refraction workload: a 128^3 voxel grid at 1 mm with an air
cylinder (n = 1.0) inside n = 1.4 tissue and three absorbing spheres,
768 HEALPix directions (nside 8), split advance (the air-hole study of
Sec. 3.3 on synthetic data).  The headline is the FP32 solve; the BF16-split
contraction of the same workload is reported beside it.  The metric is
voxel x direction x step updates per second with the state resident in HBM.
Kernel durations come from HIP events recorded around every kernel on the
medium's stream inside the timed region.

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
PEAK_TFLOPS = {"fp32": 157.3, "bf16split": 2500.0}   # dense MFMA peaks


def bf16_products(ndir):
    """bf16 MFMA products per term of the BF16-split contraction: P_hi x_hi,
    P_hi x_lo, P_lo x_hi, and P_lo x_lo where P is resident in LDS (up to 192
    directions); the kernels that stream P leave the last one out (its column
    totals go to the diagonal)."""
    return 4 if ndir <= 192 else 3


def bf16_dtype(ndir):
    return f"bf16x{bf16_products(ndir)}-f32acc"


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_collide_sweep.txt")


def kernel_source_hash(kernel="collide"):
    """First 16 hex digits of the sha256 of the source file that holds `kernel`."""
    import hashlib
    src = "twolevel.hip" if kernel in ("coarse_sum", "apply") else "kernels.hip"
    with open(os.path.join(ROOT, "paper_2105_01028_amd", "csrc", src), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, precision, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a plain copy of known size), or None when there is none
    or the kernel source has changed since the counters were taken."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rows = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kv = dict(item.split("=", 1) for item in line.split())
        rows[(kv.get("workload"), kv.get("kernel"), kv.get("precision"))] = kv
    kv = rows.get((workload, kernel, precision))
    if kv is None or kv.get("source") != kernel_source_hash(kernel):
        return None
    return (float(kv["fetch_kib"]) * float(kv["fetch_scale"]) +
            float(kv["write_kib"]) * float(kv["write_scale"])) * 1024.0


def copy_probe(nbytes):
    """A plain device copy of known size (the calibration of the HBM counters)."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                      "copies": 5}), flush=True)


def copy_bandwidth(sizes=(1 << 30, 4 << 30, 12 << 30), reps=10):
    """What plain device copies, reductions and fills reach on this GPU (torch's
    own kernels, HIP events): the practical ceiling beside the 8 TB/s peak the
    rooflines are priced against, per buffer size."""
    import torch
    out = {}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for nbytes in sizes:
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        out[str(nbytes)] = {
            "copy_TBps_read_plus_write": 2 * nbytes / timed(lambda: b.copy_(a)) / 1e9,
            "sum_TBps_read": nbytes / timed(lambda: a.sum()) / 1e9,
            "fill_TBps_write": nbytes / timed(lambda: b.fill_(1.0)) / 1e9}
        del a, b
    return out


def mfma_ceiling():
    """What the two MFMA shapes of the collision kernels deliver here
    (tr_probe_mfma: back-to-back register-operand MFMAs, two wavefronts per
    SIMD), beside the datasheet peaks the rooflines quote."""
    from paper_2105_01028_amd import trinity as T
    f32, f32_ms = T.probe_mfma(T.TR_PROBE_MFMA_F32, iters=20000)
    b16, b16_ms = T.probe_mfma(T.TR_PROBE_MFMA_BF16, iters=40000)
    return {"fp32_32x32x2_tflops": f32, "fp32_frac_of_peak": f32 / PEAK_TFLOPS["fp32"],
            "bf16_32x32x16_tflops": b16, "bf16_frac_of_peak": b16 / PEAK_TFLOPS["bf16split"],
            "probe_ms": {"fp32": f32_ms, "bf16": b16_ms}}


def kernel_rooflines(prof, prob, precision, workload="phantom64"):
    """Achieved rates of the collide and sweep kernels from their average
    launch durations and the algorithmic work per launch.  With the phase
    moves in the collision kernel there is no sweep kernel: the collide kernel
    also moves every value to its downwind voxel, within the same 8 N V bytes.

    collide, FP32: 2 N^2 V FLOP on the FP32 MFMA peak.  collide, BF16-split:
    the hi/lo products execute 2 bf16_products(N) N^2 V bf16 FLOP; at few directions the
    kernel is bound by its 8 N V bytes (read X, write Y) instead, and the
    binding roofline (the larger fraction) is reported, with the effective
    FP32-equivalent rate 2 N^2 V / t beside it.  sweep: 8 N V bytes (read the
    collided field once, write the new one once) on the HBM peak."""
    N, V = prob.ndir, prob.nvox
    out = {}
    ms, n = prof["collide"]
    if n:
        t = ms / n * 1e-3
        if precision == "fp32":
            flop = 2.0 * N * N * V
            out["collide"] = {"bound": "mfma", "achieved": flop / t / 1e12, "peak": 157.3,
                              "unit": "TFLOP/s", "frac": flop / t / 1e12 / 157.3,
                              "avg_ms": ms / n, "work_per_launch": flop}
        else:
            flop = 2.0 * bf16_products(N) * N * N * V
            byt = 8.0 * N * V
            f_mfma = flop / t / 1e12 / PEAK_TFLOPS["bf16split"]
            f_hbm = byt / t / 1e9 / PEAK_HBM_GBS
            if f_mfma >= f_hbm:
                out["collide"] = {"bound": "mfma", "achieved": flop / t / 1e12,
                                  "peak": PEAK_TFLOPS["bf16split"], "unit": "TFLOP/s",
                                  "frac": f_mfma, "avg_ms": ms / n, "work_per_launch": flop}
            else:
                out["collide"] = {"bound": "hbm", "achieved": byt / t / 1e9, "peak": PEAK_HBM_GBS,
                                  "unit": "GB/s", "frac": f_hbm, "avg_ms": ms / n,
                                  "work_per_launch": byt}
            out["collide"]["effective_fp32_equiv_tflops"] = 2.0 * N * N * V / t / 1e12
        out["collide"]["traffic"] = measured_traffic("collide", precision, workload)
    ms, n = prof["sweep"]
    if n:
        t = ms / n * 1e-3
        byt = 8.0 * N * V
        out["sweep"] = {"bound": "hbm", "achieved": byt / t / 1e9, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": byt / t / 1e9 / PEAK_HBM_GBS,
                        "avg_ms": ms / n, "work_per_launch": byt,
                        "traffic": measured_traffic("sweep", precision, workload)}
    return out


def step_roofline(prob, precision, ms_per_step):
    """The whole step against its own bound: the larger of the contraction's
    2 N^2 V FLOP on the FP32 MFMA peak (FP32; BF16-split executes 8 N^2 V bf16
    FLOP on the bf16 peak) and the transport's 8 N V bytes on the HBM peak
    (read the field once, write it once), whatever kernels the step runs."""
    N, V = prob.ndir, prob.nvox
    if precision == "fp32":
        t_mfma = 2.0 * N * N * V / (PEAK_TFLOPS["fp32"] * 1e12)
    else:
        t_mfma = 2.0 * bf16_products(N) * N * N * V / (PEAK_TFLOPS["bf16split"] * 1e12)
    t_hbm = 8.0 * N * V / (PEAK_HBM_GBS * 1e9)
    t_min = max(t_mfma, t_hbm)
    return {"bound": "mfma" if t_mfma >= t_hbm else "hbm", "min_ms": t_min * 1e3,
            "ms_per_step": ms_per_step, "frac": t_min * 1e3 / ms_per_step}


def stored_oracle(name):
    """Records of a stored FP64 oracle run (tests/golden/make_golden.py), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", name + "_oracle.npz")
    return np.load(path) if os.path.exists(path) else None


def rel_l2_above(got, ref, floor=1e-6):
    """Relative L2 over the bins whose reference exceeds floor * (its peak)."""
    import numpy as np
    mask = ref > floor * ref.max()
    if not mask.any():
        return None
    return float(np.linalg.norm(got[mask] - ref[mask]) / np.linalg.norm(ref[mask]))


def oracle_error(name, det_steps):
    """Relative L2 error of per-step detector records against the first k steps
    of the stored FP64 oracle run of the same workload (k = the steps run; bins
    above 1e-6 of the compared records' peak).  None without stored records or
    signal."""
    z = stored_oracle(name)
    if z is None:
        return None
    ref = z["det"]
    k = min(ref.shape[1], det_steps.shape[1])
    return rel_l2_above(det_steps[:, :k].ravel(), ref[:, :k].ravel())


def timed_run(prob, steps, warmup, stream):
    import torch

    from paper_2105_01028_amd import trinity as T
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(prob)
        fused = m.info().moves_fused
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
        det_steps = m.read_detector_steps()
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
    return t1 - t0, g1 - g0, prof, closure, det_steps, fused


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


def serving(stream, count=200, count_low=50):
    """Batched server on the seeded serving stream (Poisson arrivals at 200/s,
    grids 32^3 .. 96^3, 192 directions, 500-1500 steps): p50/p99 latency with
    queueing over the first `count` arrivals at the offered rate (far above
    capacity: 200 arrivals are one second of traffic), and over the first
    `count_low` arrivals stretched to 0.8 x the capacity measured in the first
    run."""
    import numpy as np

    from paper_2105_01028_amd import serve
    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    import torch
    reqs = W.serving_stream(count, seed=4)
    work = [r.problem.nvox * 192 * r.problem.steps for r in reqs]
    count_low = min(count, count_low)
    out = {"requests": count, "updates": float(sum(work)), "requests_at_0.8_capacity": count_low}
    with torch.cuda.stream(stream):
        srv = T.Server(nside=4, g=0.85, budget_bytes=32 << 30, max_slots=16)
        sat = serve.run_stream(srv, reqs, chunk_steps=64)
        cap = sum(work) / sat["wall_s"]
        print(f"serving: {count} requests at the offered rate in {sat['wall_s']:.1f} s",
              file=sys.stderr, flush=True)
        low_reqs = reqs[:count_low]
        ts = 200.0 * (sum(work[:count_low]) / count_low) / (0.8 * cap)
        low = serve.run_stream(srv, low_reqs, chunk_steps=64, time_scale=ts)
        srv.close()
    for key, r in (("offered_200_per_s", sat), ("offered_0.8_capacity", low)):
        lat = r["latency_s"] * 1e3
        out[key] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                    "wall_s": r["wall_s"], "completed": r["completed"]}
    out["capacity_updates_per_s"] = cap
    out["arrival_stretch_0.8"] = ts
    return out


def adjoint_timing(stream):
    """Forward solve with checkpoints every 50 steps and the adjoint, on the
    64^3 / 192-direction / 500-step adjoint medium."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.config5()
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(p)
        m.solve_checkpointed(p.steps, 50)
        y = m.read_detectors()
        m.backward(np.ones_like(y))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.solve_checkpointed(p.steps, 50)
        y = m.read_detectors()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m.backward(np.ones_like(y))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        m.close()
    upd = p.nvox * p.ndir * p.steps
    return {"forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3,
            "backward_over_forward": (t2 - t1) / (t1 - t0),
            "forward_updates_per_s": upd / (t1 - t0), "checkpoint_every": 50,
            "workload": "64^3, 192 directions, 500 steps, three absorbing spheres"}


def refraction128(stream, steps=20, precisions=("fp32", "bf16split")):
    """The 128^3 / 768-direction heterogeneous medium with an air cylinder
    (split advance, Fresnel interfaces): ms per step in FP32 and BF16-split."""
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.config3()
    out = {"workload": "128^3, 768 directions (nside 8), air cylinder + 3 spheres, split advance",
           "steps": steps}
    for prec in precisions:
        q = p.copy(precision=prec)
        with torch.cuda.stream(stream):
            m = T.Medium.from_problem(q)
            m.solve(3)
            m.reset()
            m.profile_begin(steps)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.step(steps)
            m.synchronize()
            t1 = time.perf_counter()
            prof = m.profile_end()
            m.close()
        out[prec] = {"ms_per_step": (t1 - t0) / steps * 1e3,
                     "updates_per_s": q.nvox * q.ndir * steps / (t1 - t0),
                     "kernel_rooflines": kernel_rooflines(prof, q, prec, "refraction128"),
                     "kernels_ms": {k: v[0] / v[1] if v[1] else 0.0 for k, v in prof.items()}}
    return out


def implicit_source(stream, steps=200):
    """The phantom with the implicit source (S1 of Eq. 10 from the outgoing
    intensity, closed form per voxel): ms per step and kernel rooflines."""
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.config2().copy(source="implicit")
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(p)
        m.solve(10)
        m.reset()
        m.profile_begin(steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t1 = time.perf_counter()
        prof = m.profile_end()
        b = m.read_budget()
        m.close()
    inj = b[:, 0].sum()
    ms, n = prof["collide"]
    t = ms / n * 1e-3
    flop = 4.0 * p.ndir * p.ndir * p.nvox      # two products with V
    return {"ms_per_step": (t1 - t0) / steps * 1e3,
            "updates_per_s": p.nvox * p.ndir * steps / (t1 - t0),
            "collide": {"avg_ms": ms / n, "achieved_tflops": flop / t / 1e12, "peak": 157.3,
                        "frac": flop / t / 1e12 / 157.3},
            "budget_closure": abs(inj - b[:, 1].sum() - b[:, 3:].sum() - b[-1, 2]) / inj,
            "workload": "phantom 64^3, 192 directions, implicit source, 200 steps"}


def two_level_rooflines(prof, prob, nc):
    """Rates of the kernels of a two-level step (N fine, nc coarse directions):
    coarse_sum reads the fine field and writes the coarse one (4 V (N + nc)
    bytes); the coarse contraction is 2 nc^2 V FLOP on the FP32 MFMA peak;
    apply reads the fine and coarse fields and writes the fine one
    (4 V (2 N + nc) bytes); sweep is 8 N V bytes as in the one-level step."""
    N, V = prob.ndir, prob.nvox
    work = {"coarse_sum": ("hbm", 4.0 * V * (N + nc)),
            "collide": ("mfma", 2.0 * nc * nc * V),
            "apply": ("hbm", 4.0 * V * (2 * N + nc)),
            "sweep": ("hbm", 8.0 * N * V)}
    out = {}
    for k, (bound, w) in work.items():
        ms, n = prof[k]
        if not n:
            continue
        t = ms / n * 1e-3
        if bound == "hbm":
            out[k] = {"bound": "hbm", "achieved": w / t / 1e9, "peak": PEAK_HBM_GBS,
                      "unit": "GB/s", "frac": w / t / 1e9 / PEAK_HBM_GBS}
        else:
            out[k] = {"bound": "mfma", "achieved": w / t / 1e12, "peak": 157.3,
                      "unit": "TFLOP/s", "frac": w / t / 1e12 / 157.3}
        out[k].update({"avg_ms": ms / n, "work_per_launch": w,
                       "traffic": measured_traffic(k, "fp32", "twolevel64")})
    return out


def two_level(stream, steps=20):
    """The paper's fiducial angular set-up on the phantom: transport on 3072
    directions (nside 16), scattering on 192 (nside 4)."""
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.config2().copy(nside=16, nside_scatter=4)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        m = T.Medium.from_problem(p)
        t1 = time.perf_counter()
        m.solve(3)
        m.reset()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t3 = time.perf_counter()
        m.reset()
        m.profile_begin(steps)
        m.step(steps)
        prof = m.profile_end()
        b = m.read_budget()
        m.close()
    inj = b[:, 0].sum()
    return {"workload": "phantom 64^3, transport 3072 directions (nside 16), scattering 192 "
                        "(nside 4)", "setup_s": t1 - t0, "steps": steps,
            "ms_per_step": (t3 - t2) / steps * 1e3,
            "updates_per_s": p.nvox * p.ndir * steps / (t3 - t2),
            "kernels_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
            "kernel_rooflines": two_level_rooflines(prof, p, 12 * 4 * 4),
            "budget_closure": abs(inj - b[:, 1].sum() - b[:, 3:].sum() - b[-1, 2]) / max(inj, 1e-300)}


def retarded_rooflines(prof, prob, phi_nonzero):
    """Rates of the kernels of a retarded step: the hop collide does the
    2 N^2 V FLOP of the contraction (FP32 MFMA peak); the retarded sweep reads
    two history slots (one where the hop is a whole number of steps) and
    writes the new field: (8 + 4 [phi_d > 0]) V bytes per direction."""
    N, V = prob.ndir, prob.nvox
    out = {}
    ms, n = prof["collide"]
    if n:
        t = ms / n * 1e-3
        flop = 2.0 * N * N * V
        out["collide"] = {"bound": "mfma", "achieved": flop / t / 1e12, "peak": 157.3,
                          "unit": "TFLOP/s", "frac": flop / t / 1e12 / 157.3, "avg_ms": ms / n,
                          "work_per_launch": flop,
                          "traffic": measured_traffic("collide", "fp32", "retarded64")}
    ms, n = prof["sweep"]
    if n:
        t = ms / n * 1e-3
        byt = float(V) * (8.0 * N + 4.0 * phi_nonzero)
        out["sweep"] = {"bound": "hbm", "achieved": byt / t / 1e9, "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": byt / t / 1e9 / PEAK_HBM_GBS, "avg_ms": ms / n,
                        "work_per_launch": byt,
                        "traffic": measured_traffic("sweep", "fp32", "retarded64")}
    return out


def retarded(stream, steps=200, emptied=True):
    """The phantom stepped at a fifth of the voxel crossing time (the paper's
    phantom time step), with the retarded history: ms per step, updates/s,
    simulated ps per wall-clock second and kernel rooflines."""
    import math

    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.config2()
    n = float(p.n.flat[0])
    p = p.copy(advance="retarded", dt_ps=0.2 * p.dx_mm * n / 0.299792458)
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(p)
        info = m.info()
        dirs = T.host_directions(p.nside)
        m.solve(3 * info.history)
        m.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t1 = time.perf_counter()
        m.reset()
        nprof = min(steps, 100)
        m.profile_begin(nprof)
        m.step(nprof)
        prof = m.profile_end()
        m.close()
    # hop duration D_d = dx n / (|Omega_a| c0 dt) = 5 / |Omega_a|
    D = [5.0 / max(abs(x) for x in d) for d in dirs]
    phi_nonzero = sum(1 for x in D if x - math.floor(x + 1e-12) > 1e-12)
    return {"workload": "phantom 64^3, 192 directions, time step a fifth of the crossing "
                        "time (retarded history)", "history": info.history,
            "dt_ps": info.dt_ps, "steps": steps, "ms_per_step": (t1 - t0) / steps * 1e3,
            "updates_per_s": p.nvox * p.ndir * steps / (t1 - t0),
            "simulated_ps_per_s": info.dt_ps * steps / (t1 - t0),
            "kernels_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
            "kernel_rooflines": retarded_rooflines(prof, p, phi_nonzero),
            "device_gb": info.device_bytes / 1e9,
            "budget_until_emptied": {src: retarded_budget_emptied(stream, p, src)
                                     for src in ("target", "flux")} if emptied else None}


def retarded_budget_emptied(stream, p, source, steps=12000):
    """The retarded phantom run until its light has left (12000 steps of 1 ps:
    the slowest diffusion mode and absorption decay by e^-16), with the given
    source weighting: the photon budget imbalance (injected - absorbed -
    escaped - left in the box) / injected.  Light in transit between planes
    is in no tally until it lands, so only an emptied box shows what a form
    loses: the target-direction source O(dtau) per scattering where hops
    differ in length, the flux-weighted one nothing beyond FP32 rounding."""
    import torch

    from paper_2105_01028_amd import trinity as T
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(p.copy(retarded_source=source))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t1 = time.perf_counter()
        b = m.read_budget()
        m.close()
    inj = b[:, 0].sum()
    return {"steps": steps, "ms_per_step": (t1 - t0) / steps * 1e3,
            "left_in_box": b[-1, 2] / inj,
            "budget_imbalance": (inj - b[:, 1].sum() - b[:, 3:].sum() - b[-1, 2]) / inj}


def retarded_varying_index(stream, steps=50):
    """Stepping below Courant one with a varying refractive index (per-voxel
    hop durations, Fresnel interception at the air cylinder's wall), both
    source weightings: ms per step on the 64^3 refraction medium (air
    cylinder and spheres, 192 directions, a fifth of the crossing time in
    air), and the photon budget imbalance after a small medium has emptied
    (9 x 10 x 9, tissue around an air cylinder, 700 steps): the flux-weighted
    source conserves light, the target-direction form of Eq. 10 does not."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    C0 = 0.299792458
    out = {"workload": "64^3 refraction medium (air cylinder r = 3 mm, 3 spheres), "
                       "192 directions, dt = a fifth of the crossing time in air",
           "steps": steps}
    big = W.config3(nx=64).copy(nside=4, advance="retarded", dt_ps=0.2 / C0)
    z, y = np.meshgrid(np.arange(9) + 0.5, np.arange(10) + 0.5, indexing="ij")
    small = W.small_problem(nside=2, nx=9, ny=10, nz=9, mua=0.03, mus=2.0, g=0.8, n=1.4,
                            steps=700, seed=7, det_cone_deg=0.0, t0_ps=3.0, fwhm_ps=2.0)
    cyl = np.broadcast_to(((y - 5.0) ** 2 + (z - 4.95) ** 2 <= 2.7 ** 2)[:, :, None],
                          small.n.shape)
    n, mua, mus = small.n.copy(), small.mua.copy(), small.mus.copy()
    n[cyl], mua[cyl], mus[cyl] = 1.0, 0.0, 0.0
    small = small.copy(n=n, mua=mua, mus=mus, advance="retarded", dt_ps=0.2 / C0)
    for src in ("target", "flux"):
        q = big.copy(retarded_source=src)
        with torch.cuda.stream(stream):
            m = T.Medium.from_problem(q)
            info = m.info()
            m.solve(5)
            m.reset()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            m.step(steps)
            m.synchronize()
            t1 = time.perf_counter()
            m.reset()
            m.profile_begin(10)
            m.step(10)
            prof = m.profile_end()
            m.close()
            s = T.Medium.from_problem(small.copy(retarded_source=src))
            s.solve(small.steps)
            b = s.read_budget()
            s.close()
        inj = b[:, 0].sum()
        out[src] = {"ms_per_step": (t1 - t0) / steps * 1e3,
                    "updates_per_s": q.nvox * q.ndir * steps / (t1 - t0),
                    "history": info.history, "interceptions": info.ninterceptions,
                    "kernels_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
                    "budget_imbalance_small_medium_emptied":
                        float((inj - b[:, 1].sum() - b[:, 3:].sum() - b[-1, 2]) / inj),
                    "left_in_box": float(b[-1, 2] / inj)}
    return out


def paper_fiducial(stream, steps=20):
    """The paper's fiducial phantom configuration end to end on one GPU:
    101^3 voxels, 3072 transport / 192 source directions, 0.4 ps steps with the
    retarded history.  The paper states about 20 h per run of 8680 steps on
    64 Oakforest-PACS nodes (4352 Xeon Phi 7250 cores, Sec. 4), with the
    source iterated within each step; here the source is explicit.  Context,
    not a like-for-like target."""
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.fiducial101()
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        m = T.Medium.from_problem(p)
        info = m.info()
        t1 = time.perf_counter()
        m.solve(2 * info.history)
        m.reset()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t3 = time.perf_counter()
        m.reset()
        m.profile_begin(10)
        m.step(10)
        prof = m.profile_end()
        m.close()
    # the flux-weighted source (conserves light; the same kernels and traffic)
    with torch.cuda.stream(stream):
        m = T.Medium.from_problem(p.copy(retarded_source="flux"))
        m.solve(2 * info.history)
        m.reset()
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        m.step(steps)
        m.synchronize()
        t5 = time.perf_counter()
        m.close()
    ms = (t3 - t2) / steps * 1e3
    run_s = ms * p.steps / 1e3
    return {"workload": p.name, "history": info.history, "device_gb": info.device_bytes / 1e9,
            "flux_source_ms_per_step": (t5 - t4) / steps * 1e3,
            "setup_s": t1 - t0, "steps": steps, "ms_per_step": ms,
            "updates_per_s": p.nvox * p.ndir * steps / (t3 - t2),
            "kernels_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
            "projected_run_s_8680_steps": run_s,
            "paper_run": "about 20 h on 64 Oakforest-PACS nodes (4352 Xeon Phi 7250 cores), "
                         "source iterated per step",
            "paper_run_s_over_this": 20 * 3600.0 / run_s}


def paper_fiducial_run(stream, source="flux", chunk=500):
    """The paper's whole fiducial run on one GPU: 8680 steps of 0.4 ps on the
    101^3 phantom with 3072 / 192 directions and the retarded history, timed
    end to end (set-up apart), with a progress line on stderr every `chunk`
    steps.  Reports the photon budget at the end (the flux-weighted source
    conserves light; the target-direction form of Eq. 10 does not) and each
    detector's peak."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    p = W.fiducial101().copy(retarded_source=source)
    with torch.cuda.stream(stream):
        t0 = time.perf_counter()
        m = T.Medium.from_problem(p)
        info = m.info()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        done = 0
        while done < p.steps:
            n = min(chunk, p.steps - done)
            m.step(n)
            m.synchronize()
            done += n
            print(f"fiducial run ({source}): {done}/{p.steps} steps, "
                  f"{time.perf_counter() - t1:.1f} s", file=sys.stderr, flush=True)
        t2 = time.perf_counter()
        b = m.read_budget()
        det = m.read_detectors()
        m.close()
    inj = float(b[:, 0].sum())
    left = float(b[-1, 2])
    bins_ps = p.bin_ps
    return {"workload": p.name, "source": source, "steps": p.steps, "dt_ps": p.dt_ps,
            "simulated_ps": p.steps * p.dt_ps, "device_gb": info.device_bytes / 1e9,
            "setup_s": t1 - t0, "run_s": t2 - t1, "ms_per_step": (t2 - t1) / p.steps * 1e3,
            "updates_per_s": p.nvox * p.ndir * p.steps / (t2 - t1),
            "budget_imbalance": (inj - float(b[:, 1].sum()) - float(b[:, 3:].sum()) - left) / inj,
            "left_in_box": left / inj,
            "detector_peak_ps": [float((np.argmax(r) + 0.5) * bins_ps) for r in det],
            "detector_peak": [float(r.max()) for r in det],
            "paper_run": "about 20 h on 64 Oakforest-PACS nodes (4352 Xeon Phi 7250 cores), "
                         "source iterated per step"}


def c3_subbox(prob, x0=62, x1=66, y0=0, y1=128, z0=0, z1=128):
    """A sub-box of the 128^3 refraction medium: by default a slab four voxels
    thick across the cylinder's axis (x), so it holds the whole y-z cross
    section (the air cylinder's wall, tissue, the spheres the slab cuts) with
    about the full medium's density of interceptions (1.00 against 1.16 per
    voxel).  Source and detectors on the sub-box's own top face."""
    import numpy as np
    sl = (slice(z0, z1), slice(y0, y1), slice(x0, x1))
    nx, ny, nz = x1 - x0, y1 - y0, z1 - z0
    return prob.copy(nx=nx, ny=ny, nz=nz, mua=np.ascontiguousarray(prob.mua[sl]),
                     mus=np.ascontiguousarray(prob.mus[sl]), n=np.ascontiguousarray(prob.n[sl]),
                     src_ix=nx // 2 - 1, src_iy=ny // 2 - 1, det_face=[4, 4],
                     det_i=[nx // 2 + 4, nx // 2 + 8], det_j=[ny // 2, ny // 2])


def slab_share(stream, steps=50, warmup=3, z0=56, nzs=16):
    """The kernels at one GPU's share of a z-slab decomposition of the
    128^3 x 768 refraction medium over eight GPUs: the 128 x 128 x 16 slab
    z0 .. z0+15 (through the air cylinder), FP32 and BF16-split.  One GPU
    only; the halo a slab would exchange per face and step is reported as
    bytes, not timed."""
    from paper_2105_01028_amd import workloads as W
    sub = c3_subbox(W.config3(), 0, 128, 0, 128, z0, z0 + nzs)
    out = {"workload": f"128 x 128 x {nzs} slab (z {z0}..{z0 + nzs - 1}) of the 128^3 "
                       "refraction medium, 768 directions, split advance",
           "halo_bytes_per_face_per_step": sub.ndir * sub.nx * sub.ny * 4}
    for prec in ("fp32", "bf16split"):
        e, g, prof, clos, det, _ = timed_run(sub.copy(precision=prec), steps, warmup, stream)
        out[prec] = {"ms_per_step": g / steps * 1e3,
                     "updates_per_s": sub.nvox * sub.ndir * steps / g,
                     "kernels_ms": {k: v[0] / v[1] for k, v in prof.items() if v[1]},
                     "budget_closure": clos}
    return out


def cpu_baseline(prob, budget_s=15.0, single_budget_s=12.0):
    """The FP64 oracle on the host cores, on a bounded sample of the workload:
    the first steps of a sub-box of the same medium (c3_subbox), set-up
    excluded, scaled to updates/s (so the full-size figure is extrapolated
    from the sample).  Timed once with the BLAS pool at its default size and
    once single-threaded."""
    from oracle import solve
    from threadpoolctl import threadpool_info, threadpool_limits
    q = c3_subbox(prob)
    t_setup = time.perf_counter()
    S = solve.build(q, steps=64)
    setup_s = time.perf_counter() - t_setup

    def run(budget):
        t0 = time.perf_counter()
        res, steps = None, 0
        while time.perf_counter() - t0 < budget or steps < 2:
            res = solve.forward(q, steps=1, S=S, state0=None if res is None else res.state,
                                start_step=steps)
            steps += 1
        return steps, time.perf_counter() - t0

    pools = threadpool_info()
    threads = max([i.get("num_threads", 1) for i in pools] + [1])
    steps, el = run(budget_s)
    with threadpool_limits(limits=1):
        steps1, el1 = run(single_budget_s)
    try:
        affinity = len(os.sched_getaffinity(0))
    except Exception:
        affinity = os.cpu_count()
    upd = q.nvox * q.ndir
    return {"value": upd * steps / el, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"first {steps} steps of a {q.nx}x{q.ny}x{q.nz} slab of the 128^3 "
                      f"refraction medium across the air cylinder ({len(S.icpt)} interceptions), "
                      f"768 directions, FP64 NumPy with {threads} BLAS threads; set-up "
                      f"{setup_s:.1f} s excluded; the full-size rate is extrapolated from it",
            "nproc": os.cpu_count(), "cpus_available": affinity,
            "single_thread": {"value": upd * steps1 / el1, "unit": "updates/s", "cores": 1,
                              "steps": steps1}}


def c3_accuracy(stream, steps=300):
    """Detector records of the 128^3 x 768 refraction solve in BF16-split
    against the plain FP32 solve over the first `steps` steps (relative L2 on
    bins above 1e-6 of the FP32 peak), and both budget closures."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    out = {"steps": steps}
    recs = {}
    for prec in ("fp32", "bf16split"):
        with torch.cuda.stream(stream):
            m = T.Medium.from_problem(W.config3().copy(precision=prec))
            m.solve(steps)
            recs[prec] = m.read_detector_steps()
            b = m.read_budget()
            m.close()
        inj = b[:, 0].sum()
        out[prec + "_budget_closure"] = float(
            abs(inj - b[:, 1].sum() - b[:, 3:].sum() - b[-1, 2]) / inj)
    out["bf16split_vs_fp32_rel_l2"] = rel_l2_above(recs["bf16split"].ravel(),
                                                   recs["fp32"].ravel())
    out["fp32_detector_peak"] = float(recs["fp32"].max())
    return out


def refraction32_vs_oracle(stream):
    """The same path (768 directions, split advance, air cylinder with Fresnel
    interfaces, spheres) on the medium scaled to 32^3, where the FP64 oracle's
    stored 200-step run exists: detector rel L2 and the largest relative error
    of any voxel's energy density, FP32 and BF16-split."""
    import numpy as np
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    z = stored_oracle("refraction32")
    if z is None:
        return None
    steps = int(z["steps"])
    out = {"workload": "32^3 scaled refraction medium, 768 directions, split advance",
           "steps": steps}
    for prec in ("fp32", "bf16split"):
        with torch.cuda.stream(stream):
            m = T.Medium.from_problem(W.config3(nx=32).copy(precision=prec))
            m.solve(steps)
            det = m.read_detector_steps()
            E = m.read_energy().astype(np.float64)
            m.close()
        Eref = z["energy"]
        big = Eref > 1e-6 * Eref.max()
        out[prec] = {"rel_l2_vs_fp64_oracle": rel_l2_above(det.ravel(), z["det"].ravel()),
                     "energy_max_rel_error": float(np.max(np.abs(E[big] - Eref[big]) / Eref[big]))}
    return out


def phantom64_accuracy(stream):
    """The 64^3 x 192 phantom for its full 1000 steps in FP32 and BF16-split
    (moves in the collision kernel) against the stored FP64 oracle records."""
    import torch

    from paper_2105_01028_amd import trinity as T
    from paper_2105_01028_amd import workloads as W
    out = {}
    for prec in ("fp32", "bf16split"):
        p = W.config2().copy(precision=prec)
        with torch.cuda.stream(stream):
            m = T.Medium.from_problem(p)
            m.solve(p.steps)
            det = m.read_detector_steps()
            m.close()
        out[prec] = oracle_error("phantom64", det)
    return out


def phantom64(stream, K, Wm):
    """The 64^3 x 192 phantom (uniform n, phase advance: the moves in the
    collision kernel), FP32 and BF16-split, and both with the separate sweep
    kernel."""
    from paper_2105_01028_amd import workloads as W
    prob = W.config2()
    updates = prob.nvox * prob.ndir * K
    out = {"workload": "phantom 64^3, 1 mm voxels, +-5% noise, 192 directions (nside 4), "
                       "phase advance"}
    for prec in ("fp32", "bf16split"):
        e, g, p, c, d, fused = timed_run(prob.copy(precision=prec), K, Wm, stream)
        out[prec] = {"value": updates / g, "ms_per_step": g / K * 1e3,
                     "step_roofline": step_roofline(prob, prec, g / K * 1e3),
                     "kernels_ms": {k: v[0] / v[1] for k, v in p.items() if v[1]},
                     "instrumented_value": updates / e,
                     "kernel_rooflines": kernel_rooflines(
                         p, prob, prec, "phantom64" if fused else "phantom64-sweep"),
                     "budget_closure": c,
                     "rel_l2_vs_fp64_oracle_first_steps": oracle_error("phantom64", d)}
        e3, g3, p3, _, _, _ = timed_run(prob.copy(precision=prec, transport="sweep"), K, Wm,
                                        stream)
        out["separate_sweep_" + prec] = {
            "value": updates / g3, "ms_per_step": g3 / K * 1e3,
            "step_roofline": step_roofline(prob, prec, g3 / K * 1e3),
            "kernels_ms": {k: v[0] / v[1] for k, v in p3.items() if v[1]}}
    return out


C3_WORKLOAD = ("heterogeneous 128^3 at 1 mm: n = 1.4 tissue (mu_a 0.01, mu_s 10 /mm, g 0.9) "
               "with a 6 mm air cylinder (n = 1.0, Fresnel interfaces) and 3 absorbing spheres, "
               "768 directions (nside 8), split advance, dt = 3.336 ps")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16split"])
    ap.add_argument("--transport", default="auto", choices=["auto", "sweep"],
                    help="phantom64 workload only -- auto: phase moves in the collision kernel; "
                         "sweep: separate sweep kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--workload", default="refraction128",
                    choices=["refraction128", "refraction128-steps", "slab16", "phantom64",
                             "twolevel64",
                             "retarded64", "fiducial101", "fiducial101-run", "serving",
                             "adjoint64", "implicit64"],
                    help="refraction128: the headline line; fiducial101-run: the paper's "
                         "whole run, 8680 steps, both source forms; the others only time "
                         "that medium (profiling runs)")
    ap.add_argument("--serving-requests", type=int, default=200,
                    help="arrivals of the serving stream (workload 'serving' or the extra)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES (counter calibration)")
    ap.add_argument("--copy-bandwidth", action="store_true",
                    help="only time plain device copies, sums and fills of 1, 4 and 12 GiB")
    ap.add_argument("--mfma-probe", action="store_true",
                    help="only run the matrix-core rate probe (tr_probe_mfma)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design, not part of this build)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.copy_bandwidth:
        print(json.dumps(copy_bandwidth()), flush=True)
        return
    if args.mfma_probe:
        print(json.dumps(mfma_ceiling()), flush=True)
        return
    import torch
    if args.workload == "serving":
        print(json.dumps(serving(torch.cuda.Stream(), args.serving_requests)), flush=True)
        return
    if args.workload == "refraction128-steps":
        print(json.dumps(refraction128(torch.cuda.Stream(), args.steps, (args.precision,))),
              flush=True)
        return
    if args.workload == "adjoint64":
        print(json.dumps(adjoint_timing(torch.cuda.Stream())), flush=True)
        return
    if args.workload == "implicit64":
        print(json.dumps(implicit_source(torch.cuda.Stream(), args.steps)), flush=True)
        return
    if args.workload == "fiducial101":
        print(json.dumps(paper_fiducial(torch.cuda.Stream(), args.steps)), flush=True)
        return
    if args.workload == "slab16":
        print(json.dumps(slab_share(torch.cuda.Stream(), args.steps)), flush=True)
        return
    if args.workload == "fiducial101-run":
        # the whole run, both source forms (about three minutes each)
        for src in ("flux", "target"):
            print(json.dumps(paper_fiducial_run(torch.cuda.Stream(), src)), flush=True)
        return
    if args.workload == "retarded64":
        # the kernels alone (profiling runs); the budget until emptied is 24000
        # more steps, an accuracy figure of the full run
        print(json.dumps(retarded(torch.cuda.Stream(), args.steps, emptied=False)), flush=True)
        return
    if args.workload == "twolevel64":
        print(json.dumps(two_level(torch.cuda.Stream(), args.steps)), flush=True)
        return
    if args.workload == "phantom64":
        from paper_2105_01028_amd import workloads as W
        prob = W.config2().copy(precision=args.precision, transport=args.transport)
        e, g, p, c, d, fused = timed_run(prob, args.steps, args.warmup, torch.cuda.Stream())
        print(json.dumps({"workload": "phantom64", "precision": args.precision,
                          "ms_per_step": g / args.steps * 1e3,
                          "kernels_ms": {k: v[0] / v[1] for k, v in p.items() if v[1]},
                          "kernel_rooflines": kernel_rooflines(
                              p, prob, args.precision,
                              "phantom64" if fused else "phantom64-sweep")}), flush=True)
        return

    from paper_2105_01028_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    stream = torch.cuda.Stream()
    K, Wm = args.steps, args.warmup
    base = W.config3()
    prob = base.copy(precision=args.precision)
    el, el_graph, prof, closure, det_steps, _ = timed_run(prob, K, Wm, stream)
    updates = prob.nvox * prob.ndir * K
    roof = kernel_rooflines(prof, prob, args.precision, "refraction128")
    dom = max(("collide", "sweep"), key=lambda k: prof[k][0])
    rl = dict(roof[dom])
    rl["kernel"] = dom
    rl = {k: rl[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                             "avg_ms", "work_per_launch") if k in rl}
    out = {
        "metric": METRIC, "value": updates / el_graph, "unit": "updates/s", "n_gpus": 1,
        "steps": K, "warmup": Wm, "ms_per_step": el_graph / K * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else bf16_dtype(prob.ndir),
        "data": "synthetic",
        "config": {"workload": C3_WORKLOAD, "grid": [128, 128, 128], "ndir": 768,
                   "precision": args.precision, "steps_per_solve": base.steps},
        "roofline": rl,
        "kernels": {k: {"avg_ms": v[0] / v[1] if v[1] else 0.0, "launches": v[1]}
                    for k, v in prof.items()},
        "kernel_rooflines": roof,
        "step_roofline": step_roofline(prob, args.precision, el_graph / K * 1e3),
        "timing": "value: the K steps as the library runs them (tr_step replays captured "
                  "graphs); kernel durations: the same K steps queued kernel by kernel with "
                  "HIP events on the medium's stream (instrumented below)",
        "instrumented": {"value": updates / el, "ms_per_step": el / K * 1e3},
        "budget_closure": closure,
    }
    other = "bf16split" if args.precision == "fp32" else "fp32"
    e2, g2, p2, c2, d2, _ = timed_run(base.copy(precision=other), K, Wm, stream)
    out[other] = {"value": updates / g2, "ms_per_step": g2 / K * 1e3,
                  "dtype": "f32" if other == "fp32" else bf16_dtype(prob.ndir),
                  "step_roofline": step_roofline(prob, other, g2 / K * 1e3),
                  "kernels_ms": {k: v[0] / v[1] for k, v in p2.items() if v[1]},
                  "instrumented_value": updates / e2,
                  "kernel_rooflines": kernel_rooflines(p2, prob, other, "refraction128"),
                  "budget_closure": c2}
    ceil = mfma_ceiling()
    ceil["collide_fp32_frac_of_probe"] = (
        (out if args.precision == "fp32" else out[other])["kernel_rooflines"]["collide"]["achieved"]
        / ceil["fp32_32x32x2_tflops"])
    ceil["collide_bf16split_frac_of_probe"] = (
        (out if args.precision == "bf16split" else out[other])["kernel_rooflines"]["collide"]
        ["achieved"] / ceil["bf16_32x32x16_tflops"])
    out["mfma_ceiling"] = ceil
    print("headline and its other precision done", file=sys.stderr, flush=True)
    acc = {"full_size_bf16split_vs_fp32": c3_accuracy(stream),
           "scaled_32cube_vs_fp64_oracle": refraction32_vs_oracle(stream)}
    out["accuracy"] = acc
    print("accuracy done", file=sys.stderr, flush=True)
    if not args.no_extras:
        out["phantom64"] = phantom64(stream, K, Wm)
        out["phantom64"]["full_1000_steps_rel_l2_vs_fp64_oracle"] = phantom64_accuracy(stream)
        p50, p99 = latency(W.config1(), 30, stream)
        out["latency_uniform16"] = {"p50_ms": p50, "p99_ms": p99, "solves": 30,
                                    "workload": "16^3, 48 directions, 200 steps"}
        print("phantom and latency done", file=sys.stderr, flush=True)
        out["serving"] = serving(stream, args.serving_requests)
        out["adjoint"] = adjoint_timing(stream)
        out["implicit_source"] = implicit_source(stream)
        out["two_level_3072_192"] = two_level(stream)
        out["retarded_courant02"] = retarded(stream)
        out["retarded_varying_index"] = retarded_varying_index(stream)
        out["paper_fiducial_101"] = paper_fiducial(stream)
        out["slab_share_128x128x16"] = slab_share(stream)
        print("extras done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(base)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
