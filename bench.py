#!/usr/bin/env python3
"""Benchmark of the CME solver on one MI355X.

Workload (default): the batched detuning sweep -- 256 resonators of N = 2048
modes, D2 = 0.002, D3 = 2e-6, sigma_i evenly spaced in [-2, 10], pump 5x
threshold, noise 1e-6, classic RK4 with h = 5e-4 for 5e4 steps, FP64.  One
bench step is one full run of that horizon for the whole batch (one
persistent kernel launch, captured once in a hipGraph and replayed).  The metric is mode-steps/s = sum_i N_i x RK4
steps / wall time, valid only where the GPU matches the FP64 oracle to
<= 1e-10 relative L2 error.  That error is measured on the launch the
bench times: after the full 5e4 steps against the oracle states stored in
tests/golden/ (five instances: both detuning ends, two inside the
modulation-instability window, the middle; with the oracle's own spread
under a 1e-12 change of A(0)), and after 640 steps against the oracle run
live on 16 instances, whose timing (about 10 s) is the CPU baseline.  Errors are given
for the whole spectrum and for the sidebands mu != 0 alone.

Also reported on the same JSON line:
  roofline      counted FFT flops (8 transforms x 5 N log2 N per RK4 step)
                per launch / the launch's mean duration (HIP events on the
                launch stream) against the FP64 vector peak (78.6 TFLOP/s);
  cpu_baseline  the CPU oracle (O(N^2) direct sum) timed on a bounded
                sample of the same workload on this host's cores (one
                instance per thread), and a scaling sweep N = 64 ... 8192 of
                oracle and GPU cost per mode-step (the O(N) vs O(log N)
                per-mode cost of the direct sum and the transforms);
  adjoint       forward-with-checkpoints and adjoint times for the N = 2048,
                5000-step gradient workload and their ratio;
  single        single instances on one workgroup (plain N = 128, soliton
                ramp N = 1024), also as a fraction of one CU's FP64 peak;
  fp32          the same sweep in FP32 (FP64 time bookkeeping);
  uneven        the uneven-octave batch (512 instances, N in {1024, ..., 8192},
                h = 2e-4, 2e4 steps) in FP64 and FP32, classic RK4 on the
                instances it is stable for (the excluded count is reported),
                and all 512 with the interaction-picture RK4 (FP64); FP32
                against the GPU's FP64 run for every instance, and both
                against the stored oracle states of 32 sampled instances;
  staged        the four-step transforms through global memory: 128 x N=8192
                (beside the LDS-resident kernels: the one-transform wave
                kernel and rk4_stream), 64 x N=16384, 16 x N=65536,
                with algorithmic HBM GB/s, for RK4 and for the split-step map;
  padded        256 instances of N = 1024 with the alias-free truncated sum
                (2N-point transforms) beside the cyclic sum, 2000 steps;
  fig1          the paper's Fig. 1 ensemble (four N = 256 runs to normalised
                time 128 pi) with the split-step map in one launch, beside
                the paper's own 54 s (desktop CPU, split-step; its step size
                is not stated, h = 1e-3 here).
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "mode-steps/s (FP64, 1 GPU) at ≤1e-10 rel. error vs oracle; adjoint/forward ratio"
FP64_PEAK_TFLOPS = 78.6
COUNTERS = os.path.join(ROOT, "profiles", "rk4_duo_sweep_n2048_counters.txt")
# sources of the default N = 2048 kernel (rk4_duo)
KERNEL_SOURCES = ("cme_fft.hpp", "cme_internal.hpp", "cme_lean.hpp", "cme_duo.hip")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1307_3428_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic():
    """HBM bytes of one launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by what the counter reads for a
    1 GiB copy), or None if there is none or the kernel sources changed since.
    The state stays on chip for the whole run, so the bytes of a launch do not
    depend on how many RK4 steps it takes."""
    if not os.path.exists(COUNTERS):
        return None
    vals = {}
    with open(COUNTERS) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        fetch = float(vals["fetch_kib_per_dispatch_scaled"]) * 1024.0
        write = float(vals["write_kib_per_dispatch_scaled"]) * 1024.0
    except (KeyError, ValueError):
        return None
    return fetch + write


def counted_flops_per_step(n: int) -> float:
    return 8 * 5.0 * n * math.log2(n)


def spectrum_errors(y, ref):
    """Relative L2 errors of one instance's spectrum (centred order, pump mode
    mu = 0 at N/2): the whole vector, the sidebands mu != 0 alone, the power
    spectrum |A|^2 and its sidebands; and the share of ||ref|| the sidebands
    hold.  The pump mode dominates ||A|| on the CW + noise workloads, so the
    sideband figures are the ones that constrain the comb."""
    import numpy as np
    y = np.asarray(y, np.complex128)
    ref = np.asarray(ref, np.complex128)
    m = np.ones(ref.shape[0], bool)
    m[ref.shape[0] // 2] = False

    def rel(d, r):
        nr = float(np.linalg.norm(r))
        return float(np.linalg.norm(d)) / nr if nr > 0 else 0.0

    py, pr = np.abs(y) ** 2, np.abs(ref) ** 2
    return {"whole": rel(y - ref, ref), "side": rel((y - ref)[m], ref[m]),
            "power": rel(py - pr, pr), "power_side": rel((py - pr)[m], pr[m]),
            "side_frac": rel(ref[m], ref)}


def golden(name: str):
    """Stored oracle states (written by tests/golden/make_oracle_goldens.py,
    which runs only the CPU oracle), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{name}.npz")
    if not os.path.exists(path):
        return None
    d = np.load(path, allow_pickle=False)
    out = {k: d[k] for k in d.files if k != "meta"}
    out["meta"] = json.loads(str(d["meta"]))
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3, help="timed full runs")
    ap.add_argument("--warmup", type=int, default=1, help="untimed full runs")
    ap.add_argument("--rk-steps", type=int, default=None,
                    help="RK4 steps per run (default: the workload's 5e4)")
    ap.add_argument("--parity-steps", type=int, default=640,
                    help="RK4 steps of the live oracle sample (also the CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip adjoint / single-instance legs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--kernel", type=int, default=-1, help="force a kernel variant id")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only run the adjoint leg (profiling) and exit")
    ap.add_argument("--staged-case", type=int, default=0, metavar="N",
                    help="only run the staged kernel on the staged leg's batch of size N "
                         "(8192, 16384 or 65536) for --rk-steps steps (profiling) and exit")
    ap.add_argument("--profile-case", default="", metavar="N,B,KIND,PREC[,uniform]",
                    help="only run B seeded random instances of N modes on the first kernel "
                         "variant of that kind and precision (0 FP64, 1 FP32) for --rk-steps "
                         "steps (profiling) and exit; 'uniform': kappa the same for every mode "
                         "(as in the paper's normalised workloads) instead of per-mode kappa")
    ap.add_argument("--uneven-only", action="store_true",
                    help="only run the uneven-octave leg (profiling) and exit")
    ap.add_argument("--single-only", action="store_true",
                    help="only run the single-instance leg (profiling) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this solver benchmark runs on exactly one GPU; independent instances "
              "would be sharded across GPUs with no communication, which this benchmark does not "
              "launch. Run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1307_3428_amd import cme as C
    from paper_1307_3428_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)

    if args.copy_calibration:
        n = 1 << 27  # 2^27 complex64 = 1 GiB
        src = torch.ones(n, dtype=torch.complex64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 8}))
        return 0

    if args.adjoint_only:
        print(json.dumps(adjoint_leg(C, W, torch)))
        return 0

    if args.staged_case:
        print(json.dumps(staged_leg(C, W, torch, only=args.staged_case,
                                    steps=args.rk_steps or 20)))
        return 0

    if args.profile_case:
        fields = args.profile_case.split(",")
        n, b, kind, prec = (int(x) for x in fields[:4])
        uniform = len(fields) > 4 and fields[4] == "uniform"
        kid = next(k for k in C.cme_list_kernels(prec, n) if C.cme_kernel_info(k)["kind"] == kind)
        p = W.pack(W.random_batch(43, [n] * b, noise=1e-3, random_kappa=not uniform))
        steps = args.rk_steps or 200
        integ = C.CME_RK4IP if kind in (7, 8, 12, 14) else C.CME_RK4
        with C.Plan(p, 2e-4, precision=prec, integrator=integ) as plan:
            plan.select(n, kid)
            A = plan.state(p.a0)
            s = timed_run(plan, A, steps, torch)
            print(json.dumps({"case": args.profile_case, "kernel": plan.kernel(n)["name"],
                              "us_per_step": 1e6 * s / steps,
                              "mode_steps_per_s": p.total * steps / s}))
        return 0

    if args.uneven_only:
        print(json.dumps(uneven_leg(C, W, torch)))
        return 0

    if args.single_only:
        print(json.dumps(single_leg(C, W, torch)))
        return 0

    rk_steps = args.rk_steps or 50000
    wl = W.sweep_n2048(n_steps=rk_steps)
    p = W.pack(wl.instances)
    n_modes = 2048
    flags = 0 if args.no_autotune else C.CME_INIT_AUTOTUNE
    stream = torch.cuda.current_stream()
    plan = C.Plan(p, wl.h, flags=flags)
    if args.kernel >= 0:
        plan.select(n_modes, args.kernel)
    kinfo = plan.kernel(n_modes)
    A0 = plan.state(p.a0)

    # ---- parity at the full horizon against the stored oracle states, on the
    # launch the bench times (all 256 instances, one run from A(0)) ----
    horizon = None
    g2 = golden("c2_sweep")
    A = A0.clone()
    plan.run(A, rk_steps)
    torch.cuda.synchronize()
    if g2 is not None and int(g2["meta"]["n_steps"]) == rk_steps:
        y = A.cpu().numpy()
        rows = []
        for j, i in enumerate(g2["meta"]["indices"]):
            e = spectrum_errors(y[p.slice(i)], g2["states"][-1][j])
            e.update({"instance": int(i), "sigma": float(p.sigma0[i]),
                      "twin_separation": float(g2["sep_whole"][-1][j]),
                      "twin_separation_side": float(g2["sep_side"][-1][j])})
            rows.append(e)
        horizon = {"rk4_steps": rk_steps, "instances": rows,
                   "max_rel_l2_err": max(r["whole"] for r in rows),
                   "max_sideband_err": max(r["side"] for r in rows),
                   "tolerance": 1e-10,
                   "ok": max(r["whole"] for r in rows) <= 1e-10,
                   "reference": "oracle states stored by tests/golden/make_oracle_goldens.py "
                                "(CPU oracle only); twin_separation: the oracle's own spread "
                                "after perturbing A(0) by 1e-12"}

    # ---- live oracle sample on the same launch configuration (short horizon);
    # its timing is the CPU baseline: at least as many instances as threads,
    # so every thread runs one instance ----
    parity, cpu_s, threads, sub, pick = None, None, None, None, []
    if args.parity_steps > 0:
        import oracle
        threads = oracle.max_threads()
        n_pick = min(p.batch, max(16, threads))
        pick = sorted({round(k * (p.batch - 1) / (n_pick - 1)) for k in range(n_pick)})
        A = A0.clone()
        plan.run(A, args.parity_steps)
        torch.cuda.synchronize()
        y = A.cpu().numpy()
        sub = W.pack([wl.instances[i] for i in pick])
        t0 = time.perf_counter()
        ref, _ = oracle.run(sub, wl.h, args.parity_steps)
        cpu_s = time.perf_counter() - t0
        errs = [spectrum_errors(y[p.slice(i)], ref[sub.slice(j)]) for j, i in enumerate(pick)]
        # the same oracle on one core: one instance
        one = W.pack([wl.instances[pick[0]]])
        one_steps = max(10, args.parity_steps // 4)
        oracle.set_threads(1)
        t1 = time.perf_counter()
        oracle.run(one, wl.h, one_steps)
        cpu1_s = time.perf_counter() - t1
        oracle.set_threads(threads)
        parity = {"max_rel_l2_err": max(e["whole"] for e in errs),
                  "max_sideband_err": max(e["side"] for e in errs),
                  "max_power_err": max(e["power"] for e in errs),
                  "instances": pick, "rk4_steps": args.parity_steps,
                  "tolerance": 1e-10, "ok": max(e["whole"] for e in errs) <= 1e-10}
    flags_out = plan.status()

    # ---- timed runs: the persistent launch is captured once in a hipGraph
    # (on a side stream) and replayed on the current stream, one replay per
    # bench step ----
    A = A0.clone()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    plan.set_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        plan.run(A, rk_steps)
    plan.set_stream(None)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        graph.replay()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    launch_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
    mean_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    mode_steps = p.total * rk_steps * args.steps
    value = mode_steps / wall
    flops_per_launch = counted_flops_per_step(n_modes) * p.batch * rk_steps
    achieved = flops_per_launch / mean_launch_s / 1e12
    finite = not plan.status().any() and not flags_out.any()

    traffic = read_traffic()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "mode-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "sweep_n2048: 256 instances x N=2048 modes, RK4 h=5e-4, "
                        f"{rk_steps} steps per bench step, sigma in [-2,10], pump 5x threshold",
            "batch": p.batch, "n_modes": n_modes, "rk4_steps": rk_steps, "h": wl.h,
            "kernel": {**kinfo, "autotuned": not args.no_autotune and args.kernel < 0},
            "launch": "one persistent launch per bench step, captured once in a hipGraph "
                      "and replayed",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK_TFLOPS,
            "traffic": traffic,
            "counted_flops_per_launch": flops_per_launch,
            "mean_launch_ms": mean_launch_s * 1e3,
            "note": "counted flops = 8 FFTs x 5 N log2 N per RK4 step per instance; "
                    "FP64 vector peak",
        },
        "parity": parity,
        "parity_full_horizon": horizon,
        "all_finite": bool(finite),
    }
    if not args.no_cpu_baseline and cpu_s is not None:
        used = min(threads, len(pick))
        out["cpu_baseline"] = {
            "value": sub.total * args.parity_steps / cpu_s,
            "unit": "mode-steps/s",
            "cores": used,
            "kind": "oracle",
            "sample": f"{len(pick)} of the 256 N=2048 instances x {args.parity_steps} RK4 steps, "
                      f"one instance per thread (O(N^2) direct-sum FWM, FP64, OpenMP), "
                      f"{cpu_s:.1f} s",
            "cpu_model": cpu_model(),
            "one_core": {"value": 2048 * one_steps / cpu1_s, "cores": 1,
                         "sample": f"1 instance x {one_steps} RK4 steps, {cpu1_s:.1f} s"},
        }
        if not args.no_extras:
            out["cpu_baseline"]["scaling"] = scaling_sweep(C, W, torch, threads)
    plan.close()

    if not args.no_extras:
        out["adjoint"] = adjoint_leg(C, W, torch)
        out["single"] = single_leg(C, W, torch)
        out["fp32"] = fp32_leg(C, W, torch, rk_steps)
        out["uneven"] = uneven_leg(C, W, torch)
        out["fig1"] = fig1_leg(C, W, torch)
        out["padded"] = padded_leg(C, W, torch)
        out["staged"] = staged_leg(C, W, torch)
    print(json.dumps(out))
    return 0


def scaling_sweep(C, W, torch, threads):
    """Cost per mode-step against N (Sec. 2: the transform evaluation of the
    four-wave-mixing sum is O(N log N) per right-hand side, the direct sum
    O(N^2)): the CPU oracle (direct sum; one instance per thread) and the GPU
    (256 instances of N modes, default kernels), N = 64 ... 8192, seeded
    random parameters, classic RK4."""
    import numpy as np
    import oracle
    rows = []
    for n in (64, 128, 256, 512, 1024, 2048, 4096, 8192):
        insts = W.random_batch(97, [n] * 256, noise=1e-3)
        p = W.pack(insts)
        gpu_steps = max(20, (1 << 24) // (256 * n))
        with C.Plan(p, 1e-3) as plan:
            A = plan.state(p.a0)
            plan.run(A, 5)
            torch.cuda.synchronize()
            g = timed_run(plan, A, gpu_steps, torch)
            kname = plan.kernel(n)["name"]
        sub = W.pack(insts[:threads])
        cpu_steps = max(1, int(3e8 / (64.0 * n * n)))
        t0 = time.perf_counter()
        oracle.run(sub, 1e-3, cpu_steps)
        c = time.perf_counter() - t0
        rows.append({"n": n, "gpu_mode_steps_per_s": p.total * gpu_steps / g,
                     "oracle_mode_steps_per_s": sub.total * cpu_steps / c,
                     "gpu_kernel": kname, "oracle_steps": cpu_steps})
    for r in rows:
        r["gpu_over_oracle"] = r["gpu_mode_steps_per_s"] / r["oracle_mode_steps_per_s"]
    ns = np.log2([r["n"] for r in rows])
    fit = lambda key: float(np.polyfit(ns, np.log2([1.0 / r[key] for r in rows]), 1)[0])
    return {"workload": "256 random instances per N (GPU), one per thread (oracle), RK4 h=1e-3",
            "rows": rows,
            "slope_log2_time_per_mode_step_vs_log2_n": {"oracle": fit("oracle_mode_steps_per_s"),
                                                         "gpu": fit("gpu_mode_steps_per_s")}}


def adjoint_leg(C, W, torch):
    """N=2048, 5000 RK4 steps, checkpoints every 100: forward (with
    checkpoint writes) vs cme_adjoint (segment recompute + reverse sweep)."""
    wl = W.adjoint_n2048()
    p = W.pack(wl.instances)
    K = 100
    with C.Plan(p, wl.h) as plan:
        A0 = plan.state(p.a0)
        ck = torch.empty((wl.n_steps // K, p.total), dtype=torch.complex128, device="cuda")
        gT = torch.ones_like(A0)
        # warm-up
        A = A0.clone()
        plan.run(A, 200, ckpt_every=K, ckpt=ck[:2])
        plan.adjoint(A0, gT, 200, ckpt_every=K, ckpt=ck[:2])
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        A = A0.clone()
        e[0].record()
        plan.run(A, wl.n_steps, ckpt_every=K, ckpt=ck)
        e[1].record()
        plan.adjoint(A0, gT, wl.n_steps, ckpt_every=K, ckpt=ck)
        e[2].record()
        torch.cuda.synchronize()
        fwd, bwd = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
    return {"workload": "adjoint_n2048: N=2048, 5000 RK4 steps, checkpoints every 100",
            "forward_ms": fwd, "adjoint_ms": bwd, "adjoint_over_forward": bwd / fwd,
            "forward_plus_adjoint_over_forward": (fwd + bwd) / fwd}


def timed_run(plan, A, steps, torch):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    plan.run(A, steps)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def fp32_leg(C, W, torch, rk_steps):
    """The 256 x N=2048 sweep in FP32 (same horizon), autotuned."""
    wl = W.sweep_n2048(n_steps=rk_steps)
    p = W.pack(wl.instances)
    with C.Plan(p, wl.h, precision=C.CME_F32, flags=C.CME_INIT_AUTOTUNE) as plan:
        A = plan.state(p.a0)
        plan.run(A, 1000)
        torch.cuda.synchronize()
        s = timed_run(plan, A, rk_steps, torch)
        k = plan.kernel(2048)
    rate = p.total * rk_steps / s
    return {"workload": f"sweep_n2048 in FP32, {rk_steps} RK4 steps",
            "mode_steps_per_s": rate, "kernel": k["name"],
            "counted_TFLOPs": rate * counted_flops_per_step(2048) / 2048 / 1e12,
            "frac_fp32_vector_peak": rate * counted_flops_per_step(2048) / 2048 / 157.3e12}


def rk4_stable(inst, h):
    import numpy as np
    ok = True
    for sg in (inst.sigma0, inst.sigma1):
        z = h * (-0.5 * inst.kappa + 1j * (inst.omega - sg))
        ok &= bool(np.all(np.abs(1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24) <= 1 + 1e-12))
    return ok


def uneven_leg(C, W, torch, steps=20000):
    """The uneven-octave batch, FP64 and FP32, one plan per precision (size
    classes launched concurrently), on the classically RK4-stable instances.
    Also: every instance's FP32 result against the GPU's FP64 result after
    the full horizon (labelled as such), and the sampled instances against
    the stored oracle states after 2e3 steps (all four classes) and 2e4 steps
    (N <= 2048)."""
    import numpy as np
    wl = W.uneven_octave(n_steps=steps)
    keep_idx = [i for i, x in enumerate(wl.instances) if rk4_stable(x, wl.h)]
    keep = [wl.instances[i] for i in keep_idx]
    p = W.pack(keep)
    out = {"workload": f"uneven_octave: {len(keep)} of {len(wl.instances)} instances "
                       f"(classic RK4 stable), N in {{1024,2048,4096,8192}}, {steps} steps",
           "excluded_unstable": len(wl.instances) - len(keep),
           "by_n": {str(n): int(sum(1 for x in keep if x.n_modes == n))
                    for n in (1024, 2048, 4096, 8192)}}
    g3 = golden("c3_uneven")
    short = int(g3["meta"]["short"]) if g3 is not None else 2000
    finals, shorts = {}, {}
    for prec, name in ((C.CME_F64, "fp64"), (C.CME_F32, "fp32")):
        with C.Plan(p, wl.h, precision=prec, flags=C.CME_INIT_AUTOTUNE) as plan:
            A = plan.state(p.a0)
            plan.run(A, short)
            torch.cuda.synchronize()
            shorts[name] = A.cpu().numpy().astype(np.complex128)
            plan.run(A, steps - short, step0=short)
            torch.cuda.synchronize()
            finals[name] = A.cpu().numpy().astype(np.complex128)
            A = plan.state(p.a0)
            s = timed_run(plan, A, steps, torch)
            out[name] = {"mode_steps_per_s": p.total * steps / s, "seconds": s,
                         "all_finite": not bool(plan.status().any()),
                         "kernels": {str(n): plan.kernel(n)["name"] for n in (1024, 2048, 4096, 8192)}}
    # FP32 against the GPU's FP64 run, every instance, full horizon
    e32 = [spectrum_errors(finals["fp32"][p.slice(b)], finals["fp64"][p.slice(b)])
           for b in range(p.batch)]
    out["fp32_vs_gpu_fp64"] = {
        "note": "FP32 GPU result against the FP64 GPU result (not the oracle) after "
                f"{steps} steps, per instance in batch order (instance ids in 'ids')",
        "ids": keep_idx,
        "whole": [float("%.3g" % e["whole"]) for e in e32],
        "side": [float("%.3g" % e["side"]) for e in e32],
        "power": [float("%.3g" % e["power"]) for e in e32],
        "max_whole": max(e["whole"] for e in e32),
        "median_whole": float(np.median([e["whole"] for e in e32])),
        "max_side": max(e["side"] for e in e32),
        "median_side": float(np.median([e["side"] for e in e32])),
    }
    # both precisions against the stored oracle states
    if g3 is not None and int(g3["meta"]["n_steps"]) == steps:
        pos = {i: b for b, i in enumerate(keep_idx)}
        ref_short, ref_full = g3["states_short"], g3["states_full"]
        res = {}
        for name in ("fp64", "fp32"):
            rows, o = [], 0
            for i in g3["meta"]["indices_short"]:
                n = wl.instances[i].n_modes
                e = spectrum_errors(shorts[name][p.slice(pos[i])], ref_short[o:o + n])
                rows.append({"instance": i, "n": n, "steps": short, **e})
                o += n
            o = 0
            for i in g3["meta"]["indices_full"]:
                n = wl.instances[i].n_modes
                e = spectrum_errors(finals[name][p.slice(pos[i])], ref_full[o:o + n])
                rows.append({"instance": i, "n": n, "steps": steps, **e})
                o += n
            res[name] = {"max_whole": max(r["whole"] for r in rows),
                         "max_side": max(r["side"] for r in rows),
                         "rows": [{k: (float("%.3g" % v) if isinstance(v, float) else v)
                                   for k, v in r.items()} for r in rows]}
        out["vs_oracle"] = res
    # all 512 instances, the ones classic RK4 refuses included, with the
    # interaction-picture RK4 (the linear part integrated exactly)
    pa = W.pack(wl.instances)
    with C.Plan(pa, wl.h, integrator=C.CME_RK4IP, flags=C.CME_INIT_AUTOTUNE) as plan:
        A = plan.state(pa.a0)
        plan.run(A, 200)
        torch.cuda.synchronize()
        A = plan.state(pa.a0)
        s = timed_run(plan, A, steps, torch)
        out["fp64_rk4ip_all"] = {
            "instances": pa.batch, "mode_steps_per_s": pa.total * steps / s, "seconds": s,
            "all_finite": not bool(plan.status().any()),
            "kernels": {str(n): plan.kernel(n)["name"] for n in (1024, 2048, 4096, 8192)}}
    return out


# HBM bytes per mode and RK4 step of the staged kernels (per-mode kappa, as in
# the seeded batches of this leg): per stage the column kernel reads S, kappa,
# omega' and stage 1: y; stage 2: y, k_1; stage 3: y, k_1, k_2; stage 4: P, u_4,
# and writes S and stage 1: k_1; stage 2: k_2; stage 3: P, u_4; stage 4: y;
# the row kernel reads and writes S.  16 B per complex value, 8 per real.
STAGED_BYTES_PER_MODE_STEP = (16 * 4 + 16) + (16 * 5 + 16) + (16 * 7 + 16) + (16 * 5 + 16) + 4 * 32
# split-step on the staged transforms: the row kernel reads and writes S, the
# column kernel reads and writes S and reads kappa and omega'
SPLIT_STAGED_BYTES_PER_MODE_STEP = 32 + 32 + 16


def staged_leg(C, W, torch, only=0, steps=None):
    """The staged path (four-step transforms through global memory): FP64,
    N = 8192 against the LDS-resident kernel, and N = 16384 / 65536, where it
    is the only kernel; about 10^6 modes per plan (seeded random instances,
    RK4 h = 2e-4).  only = N: just the first staged kernel of that size."""
    out = {"bytes_per_mode_step": STAGED_BYTES_PER_MODE_STEP, "peak_GBps": 8000.0, "cases": []}
    for n, b, default_steps in ((8192, 128, 200), (16384, 64, 200), (65536, 16, 100)):
        if only and n != only:
            continue
        nsteps = steps or default_steps
        p = W.pack(W.random_batch(43, [n] * b, noise=1e-3))
        ids = [k for k in C.cme_list_kernels(C.CME_F64, n)
               if C.cme_kernel_info(k)["kind"] in ((6,) if only else (1, 6, 13))][:1 if only else None]
        for kid in ids:
            with C.Plan(p, 2e-4) as plan:
                plan.select(n, kid)
                A = plan.state(p.a0)
                plan.run(A, 10)
                torch.cuda.synchronize()
                s = timed_run(plan, A, nsteps, torch)
                name = plan.kernel(n)["name"]
            rate = p.total * nsteps / s
            case = {"workload": f"{b} x N={n}, {nsteps} RK4 steps", "kernel": name,
                    "mode_steps_per_s": rate, "us_per_step": 1e6 * s / nsteps}
            if name.startswith("rk4_staged"):
                gbps = rate * STAGED_BYTES_PER_MODE_STEP / 1e9
                case.update({"algorithmic_GBps": gbps, "frac_hbm_peak": gbps / 8000.0})
            out["cases"].append(case)
        if only:
            continue
        if n == 8192:
            # rk4_stream skips the kappa loads where kappa is the same for every
            # mode (the paper's normalised workloads): the same batch so
            q = W.pack(W.random_batch(43, [n] * b, noise=1e-3, random_kappa=False))
            kid = next(k for k in C.cme_list_kernels(C.CME_F64, n)
                       if C.cme_kernel_info(k)["kind"] == 13)
            with C.Plan(q, 2e-4) as plan:
                plan.select(n, kid)
                A = plan.state(q.a0)
                plan.run(A, 10)
                torch.cuda.synchronize()
                s = timed_run(plan, A, nsteps, torch)
                out["cases"].append({"workload": f"{b} x N={n}, {nsteps} RK4 steps, kappa the same "
                                                 "for every mode", "kernel": plan.kernel(n)["name"],
                                     "mode_steps_per_s": q.total * nsteps / s,
                                     "us_per_step": 1e6 * s / nsteps})
        # the split-step map on the same transforms: two launches per step
        with C.Plan(p, 2e-4, integrator=C.CME_SPLIT_STEP) as plan:
            A = plan.state(p.a0)
            plan.run(A, 10)
            torch.cuda.synchronize()
            s = timed_run(plan, A, 4 * nsteps, torch)
            rate = p.total * 4 * nsteps / s
            gbps = rate * SPLIT_STAGED_BYTES_PER_MODE_STEP / 1e9
            out["cases"].append({"workload": f"{b} x N={n}, {4 * nsteps} split steps",
                                 "kernel": plan.kernel(n)["name"], "mode_steps_per_s": rate,
                                 "us_per_step": 1e6 * s / (4 * nsteps), "algorithmic_GBps": gbps,
                                 "frac_hbm_peak": gbps / 8000.0})
    return out


def padded_leg(C, W, torch, steps=2000):
    """256 x N=1024 (seeded random parameters): padded vs cyclic FWM sum."""
    insts = W.random_batch(41, [1024] * 256, noise=1e-3)
    p = W.pack(insts)
    out = {"workload": f"256 x N=1024 random instances, {steps} RK4 steps of h=1e-3"}
    for fwm, name in ((C.CME_FWM_PADDED, "padded"), (C.CME_FWM_CYCLIC, "cyclic")):
        with C.Plan(p, 1e-3, fwm=fwm) as plan:
            A = plan.state(p.a0)
            plan.run(A, 100)
            torch.cuda.synchronize()
            s = timed_run(plan, A, steps, torch)
            out[name] = {"mode_steps_per_s": p.total * steps / s, "kernel": plan.kernel(1024)["name"]}
    return out


def fig1_leg(C, W, torch):
    """Fig. 1 ensemble, full horizon, split-step (CME_SPLIT_STEP), FP64."""
    wl = W.fig1_ensemble()
    p = W.pack(wl.instances)
    with C.Plan(p, wl.h, integrator=C.CME_SPLIT_STEP) as plan:
        A = plan.state(p.a0)
        plan.run(A, 100)
        torch.cuda.synchronize()
        A = plan.state(p.a0)
        s = timed_run(plan, A, wl.n_steps, torch)
        finite = not plan.status().any()
        k = plan.kernel(256)["name"]
    return {"workload": f"fig1_ensemble: 4 x N=256, {wl.n_steps} split-step steps of h={wl.h} "
                        "(tau = 256 pi, normalised time 128 pi)",
            "seconds": s, "mode_steps_per_s": p.total * wl.n_steps / s, "kernel": k,
            "all_finite": bool(finite),
            "paper": "54 s for the four runs on a desktop CPU (Fig. 1 caption); step not stated"}


def single_leg(C, W, torch):
    """Single instances, each on one workgroup (one CU): the plain N=128
    workload and the N=1024 soliton ramp, 20000 RK4 steps each.  Reported
    against one CU's FP64 vector peak (128 flop/clk at 2.4 GHz) as well as
    the device's: one instance cannot use more than one CU."""
    steps = 20000
    cu_peak = 128 * 2.4e9
    out = {}
    for name, wl in (("plain_n128", W.plain_n128(n_steps=steps)),
                     ("soliton_ramp_n1024", W.soliton_ramp_n1024(n_steps=steps))):
        p = W.pack(wl.instances)
        n = int(p.n_modes[0])
        with C.Plan(p, wl.h, flags=C.CME_INIT_AUTOTUNE) as plan:
            A = plan.state(p.a0)
            plan.run(A, 1000)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.run(A, steps, step0=1000)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1)
            k = plan.kernel(n)
        flops = counted_flops_per_step(n) * steps / (ms / 1e3)
        out[name] = {"workload": f"{name} (one instance), {steps} RK4 steps",
                     "mode_steps_per_s": n * steps / (ms / 1e3), "us_per_rk4_step": ms * 1e3 / steps,
                     "counted_GFLOPs": flops / 1e9, "frac_one_cu_fp64_peak": flops / cu_peak,
                     "frac_device_fp64_peak": flops / 78.6e12, "kernel": k["name"]}
    return out


if __name__ == "__main__":
    sys.exit(main())
