#!/usr/bin/env python3
"""Benchmark: one RK4 step of 3D forced isotropic turbulence at 512^3 in FP32.

Workload (synthetic, seeded): random-phase solenoidal velocity with
E(k) ~ k^4 exp(-2 (k/4)^2), unit energy (seed 1); nu = 2e-4, dt = 1e-3;
constant-power forcing P = 5e-3 on 2 <= |k| <= 3; 2/3-rule dealiasing.

Prints ONE JSON line on stdout.  `value` is nanoseconds per grid point per
RK4 step (lower is better).  Inputs are resident in device memory before the
timed region.  Every kernel of the timed steps is bracketed by HIP events on
the stream it runs on; the per-kernel averages give the roofline figures of
the dominant kernel.  The FP64 CPU oracle is timed on a bounded sample on the
host's cores for reference.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RK4 step ns/gridpoint at 512³ FP32, % HBM roofline; closure-LES vs DNS speedup"
HBM_PEAK_GBS = 8000.0
NU, DT, POWER, KMIN, KMAX, SEED = 2e-4, 1e-3, 5e-3, 2.0, 3.0, 1
TRAFFIC_FILES = {"plain": os.path.join(ROOT, "profiles", "traffic_3d_512.txt"),
                 "boussinesq": os.path.join(ROOT, "profiles", "traffic_3d_512_boussinesq.txt")}
KERNEL_SOURCES = ["fft_core.h", "ns_common.h", "ns3d_kernels.h", "ops3d_impl.h"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1807_01769_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(variant="plain"):
    """Measured HBM bytes per launch of a workload (plain flow, or stratified
    Boussinesq flow without rotation) from its counter summary: the line that
    starts with "DATA " holds {"n", "source_hash", "bytes_per_launch"}."""
    path = TRAFFIC_FILES.get(variant)
    if path is None or not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("DATA "):
                return json.loads(line[5:])
    return None


def algorithmic_bytes(n: int, steps: int, elem: int = 8, nc: int = 3) -> dict:
    """Bytes each kernel class must move in `steps` steps if only kept modes
    travel (the dealias-pruned model): per field, Us = M*M*H (state), Uzm =
    N*M*H (after the z pass), Uzn = N*N*H (after the y pass) complex values,
    with K = (N-1)//3, M = 2K+1, H = K+1.  The x pass reads six fields (u,
    w) and writes three (u x w); the z pass writes five of the six (the
    vertical vorticity, which needs no kz, is formed by the inverse y pass
    from ux, uy).  nc = 4: Boussinesq flow (u, b), one more inverse field and
    three more forward ones (u b)."""
    K = (n - 1) // 3
    M, H = 2 * K + 1, K + 1
    Us, Uzm, Uzn = M * M * H * elem, n * M * H * elem, n * n * H * elem
    fi, ff = (6, 3) if nc == 3 else (7, 6)
    fz = fi - 1
    launches = {"y_inverse": 4 * steps, "x_c2r_product_r2c": 4 * steps,
                "y_forward": 4 * steps, "z_stage": 4 * steps, "p1": 1}
    total = {
        "y_inverse": 4 * steps * (fz * Uzm + fi * Uzn),
        "x_c2r_product_r2c": 4 * steps * (fi * Uzn + ff * Uzn),
        "y_forward": 4 * steps * (ff * Uzn + ff * Uzm),
        # read the products, write the next stage's inverse fields (not after
        # the last stage), RK4 state/accumulator traffic 10 Us per component
        # and step
        "z_stage": 4 * steps * ff * Uzm + (4 * steps - 1) * fz * Uzm + steps * 10 * nc * Us,
        "p1": nc * Us + fz * Uzm,
    }
    return {k: (total[k], launches[k]) for k in total}


def unfused_model_bytes(n: int) -> float:
    """Bytes per step of the unfused pruned schedule (separate passes per
    stage: z inverse reads 3 and writes 6 kept-column fields, y inverse 6/6,
    x 6/3, y forward 3/3, z forward reads 3; the RK4 epilogue 42 field
    traffics per step), with f = M/N the kept fraction per full axis and C
    the bytes of one real single-precision field, 4 N^3:
    (4 (3 f^3 + 18 f^2 + 18 f) + 42 f^3) C, about 385 B per grid point."""
    K = (n - 1) // 3
    f = (2 * K + 1) / n
    return (4 * (3 * f ** 3 + 18 * f ** 2 + 18 * f) + 42 * f ** 3) * 4.0 * n ** 3


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n: int = 512) -> dict:
    """The oracle as it stands (plain FP64 C, OpenMP over transform lines, all
    host threads), wall time: one RK4 step of the forced recipe at n^3 (the
    headline size: no warm-up step, which would double the time), then the
    two small reference workloads: 10 steps of the 3D Taylor-Green vortex at
    128^3 and 100 FP64 steps of the 2D Taylor-Green + noise case at 128^2, and
    one 128^3 step on a single thread."""
    import numpy as np
    import oracle
    from paper_1807_01769_amd import inputs as I

    cores = oracle.get_threads()
    u = I.random_solenoidal_3d(n, seed=SEED).astype(np.complex64).astype(np.complex128)
    t0 = time.perf_counter()
    oracle.step3d(u, NU, DT, 1, power=POWER, kf_min=KMIN, kf_max=KMAX)
    t_head = time.perf_counter() - t0
    del u
    log(f"oracle: one {n}^3 step {t_head:.1f} s on {cores} threads")
    tg = I.taylor_green_3d(128)
    oracle.step3d(tg, 1.0 / 1600, 2e-3, 1)
    t0 = time.perf_counter()
    oracle.step3d(tg, 1.0 / 1600, 2e-3, 10)
    t_m1 = time.perf_counter() - t0
    w = I.tg_plus_noise_2d(128, seed=0)
    t0 = time.perf_counter()
    oracle.step2d(w, 1e-3, 1e-3, 100)
    t_m0 = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.step3d(tg, 1.0 / 1600, 2e-3, 1)
    t_1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    return {"value": t_head / n ** 3 * 1e9, "unit": "ns/gridpoint/step", "cores": cores,
            "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count(),
            "sample": f"1 FP64 RK4 step of the same forced-turbulence recipe at {n}^3 on {cores} "
                      f"threads ({t_head:.1f} s, no warm-up)",
            "taylor_green_3d_128_10_steps": {"seconds": t_m1,
                                             "ns_per_gridpoint_step": t_m1 / 10 / 128 ** 3 * 1e9},
            "tg_noise_2d_128_fp64_100_steps": {"seconds": t_m0,
                                               "ns_per_gridpoint_step": t_m0 / 100 / 128 ** 2 * 1e9},
            "single_thread_128_ns_per_gridpoint_step": t_1 / 128 ** 3 * 1e9}


LES_DT_FACTOR = 8  # LES step = 8 DNS steps (grid ratio 512 / 64)


def closure_les_speed(fs, torch, plan, state, nc, steps, dns_ms_per_step):
    """Wall time of the closure LES step (network of the closure's
    architecture, random initial weights: the cost does not depend on their
    values) on the nc^3 cutoff of the DNS state, against the DNS step, per
    unit of simulated time."""
    coarse = fs.Plan(nc, nu=NU, dt=DT * LES_DT_FACTOR, ndim=3, precision="f32",
                     forcing_power=POWER, forcing_kmin=KMIN, forcing_kmax=KMAX)
    closure = fs.Closure(plan, coarse)
    uc, A, tau = closure.samples(state)
    m = closure.moments(A, tau).cpu().numpy()
    net = fs.Mlp(seed=7)
    les = fs.Les(coarse, net, float(m[:9].mean() ** 0.5), [float(v ** 0.5) for v in m[9:]], 6.0)
    les.step(uc, 5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    les.step(uc, steps)
    torch.cuda.synchronize()
    les_ms = (time.perf_counter() - t0) * 1e3 / steps
    _, e, _ = coarse.energy_spectrum(uc)
    finite = math.isfinite(float(e.cpu()))
    log(f"closure LES {nc}^3: {les_ms:.3f} ms/step (dt x{LES_DT_FACTOR})")
    out = {"les_n": nc, "les_dt": DT * LES_DT_FACTOR, "les_ms_per_step": les_ms,
           "les_steps": steps, "dns_ms_per_step": dns_ms_per_step,
           "speedup_per_simulated_time": (dns_ms_per_step / DT) / (les_ms / (DT * LES_DT_FACTOR)),
           "network": "9-64-64-6 GELU, BF16 MFMA, random initial weights", "finite": finite}
    for o in (les, net, closure, coarse):
        o.close()
    return out


ENS_NU, ENS_DT = 1e-4, 5e-4


RESIDENT_SIZES = (64, 128)  # classes advanced block-resident by default


def ensemble_alg_bytes(sizes, resident=RESIDENT_SIZES) -> float:
    """Bytes one 2D RK4 step of the ensemble must move if only kept modes
    travel: per stage the x pass reads 3 fields and writes 2 (N x H each), the
    y pass reads those 2, the state and accumulator (M x H) and writes 3
    fields and the accumulator; the state is written once per step.  A
    block-resident run keeps the N x H fields in LDS and moves only the state
    and accumulator: 3 state and 3 accumulator reads, 3 accumulator writes
    and one state write per step."""
    tot = 0.0
    for n in sizes:
        K = (n - 1) // 3
        M, H = 2 * K + 1, K + 1
        un, us = n * H * 8.0, M * H * 8.0
        if n in resident:
            tot += 10 * us
        else:
            tot += 4 * (3 * un + 2 * un + 2 * un + 3 * un + 3 * us) + us
    return tot


def time_ensemble(fs, torch, I, np, steps):
    """256 independent 2D runs (128 at 128^2, 96 at 256^2, 32 at 512^2), FP32,
    nu = 1e-4, dt = 5e-4, `steps` RK4 steps: one graph launch per size class,
    the classes on streams of their own (the 128^2 class block-resident);
    then the same with direct launches, and with the 128^2 class
    class-batched."""
    sizes = I.ensemble_sizes()
    fields = [I.ensemble_vorticity(r, n).astype(np.complex64) for r, n in enumerate(sizes)]
    log("ensemble inputs ready")
    t0 = time.perf_counter()
    ens = fs.Ensemble(sizes, nu=ENS_NU, dt=ENS_DT)
    log(f"ensemble created and tuned in {time.perf_counter() - t0:.2f} s: {ens.schedule()}")
    st = ens.pack(fields)
    ens.step(st, steps)  # warm-up: captures and runs the graph once
    torch.cuda.synchronize()
    st = ens.pack(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(st, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pts = sum(n * n for n in sizes)
    alg = ensemble_alg_bytes(sizes) * steps
    res = {"gridpoint_steps_per_s": pts * steps / (t1 - t0), "ms_total": (t1 - t0) * 1e3,
           "steps": steps, "gridpoints": pts,
           "alg_bytes_per_step": alg / steps, "alg_GBps": alg / (t1 - t0) / 1e9,
           "finite": bool(torch.isfinite(torch.view_as_real(st)).all()),
           "schedule": ens.schedule()}
    ens.close()
    # the same steps launched directly, each class's chain on its own stream
    ens = fs.Ensemble(sizes, nu=ENS_NU, dt=ENS_DT, graphs=False)
    st2 = ens.pack(fields)
    ens.step(st2, 2)
    st2 = ens.pack(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(st2, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res["direct_streams"] = {"gridpoint_steps_per_s": pts * steps / (t1 - t0),
                             "ms_total": (t1 - t0) * 1e3,
                             "same_result": bool(torch.equal(st, st2))}
    ens.close()
    # the 128^2 class class-batched too (two passes per stage through HBM)
    # instead of block-resident, one graph per class
    ens = fs.Ensemble(sizes, nu=ENS_NU, dt=ENS_DT, resident=False)
    st3 = ens.pack(fields)
    ens.step(st3, steps)
    st3 = ens.pack(fields)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(st3, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res["class_batched_small"] = {"gridpoint_steps_per_s": pts * steps / (t1 - t0),
                                  "ms_total": (t1 - t0) * 1e3,
                                  "same_result": bool(torch.equal(st, st3)),
                                  "schedule": ens.schedule()}
    ens.close()
    res["counters"] = read_ensemble_counters()
    return res, sizes, fields


ENSEMBLE_COUNTERS = os.path.join(ROOT, "profiles", "ensemble_2d_counters.md")


def read_ensemble_counters():
    """L2 and memory-side traffic of the ensemble step from its counter
    summary (the line that starts with "DATA "), or None."""
    if not os.path.exists(ENSEMBLE_COUNTERS):
        return None
    with open(ENSEMBLE_COUNTERS) as fh:
        for line in fh:
            if line.startswith("DATA "):
                return json.loads(line[5:])
    return None


def bench_ensemble(args) -> int:
    import numpy as np
    import torch
    from paper_1807_01769_amd import fs, inputs as I

    nu, dt, steps = ENS_NU, ENS_DT, args.ens_steps
    if args.ens_counter_pass:
        # only the step's kernels: default schedules (no tuning launches),
        # direct launches, for counter collection
        sizes = I.ensemble_sizes()
        fields = [I.ensemble_vorticity(r, n).astype(np.complex64) for r, n in enumerate(sizes)]
        ens = fs.Ensemble(sizes, nu=nu, dt=dt, autotune=False, graphs=False)
        st = ens.pack(fields)
        ens.step(st, steps)
        torch.cuda.synchronize()
        ens.close()
        log(f"ensemble counter pass: {steps} steps")
        return 0
    res, sizes, fields = time_ensemble(fs, torch, I, np, steps)
    rate, pts, finite = res["gridpoint_steps_per_s"], res["gridpoints"], res["finite"]
    cpu = None
    if not args.no_cpu:
        import oracle
        w = fields[0].astype(np.complex128)
        t = time.perf_counter()
        k = 0
        while time.perf_counter() - t < 8.0:
            w = oracle.step2d(w, nu, dt, 1)
            k += 1
        el = time.perf_counter() - t
        cpu = {"value": 128 * 128 * k / el, "unit": "gridpoint-steps/s", "cores": oracle.get_threads(),
               "kind": "oracle", "sample": f"{k} FP64 RK4 steps of ensemble run 0 (128^2) in {el:.1f} s"}
    out = {"metric": "2D ensemble throughput (256 uneven runs, one graph launch per size class)",
           "value": rate,
           "unit": "gridpoint-steps/s", "n_gpus": 1, "steps": steps, "ms_total": res["ms_total"],
           "higher_is_better": True, "dtype": "f32", "data": "synthetic", "finite": finite,
           "config": {"workload": "2D NS ensemble: 128 runs at 128^2, 96 at 256^2, 32 at 512^2, "
                                  "FP32, nu=1e-4, dt=5e-4, E(k)~k exp(-(k/6)^2), seeds 1000+r",
                      "gridpoints": pts},
           "alg_GBps": res["alg_GBps"], "schedule": res["schedule"],
           "direct_streams": res["direct_streams"],
           "class_batched_small": res["class_batched_small"], "counters": res["counters"],
           "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)
    return 0


MLP_FLOP_PER_POINT = 2 * (9 * 64 + 64 * 64 + 64 * 6)  # forward multiply-adds x 2


def time_mlp(fs, torch, points=64 ** 3, batch=8192, reps=20):
    """Forward TFLOP/s of the closure network over one 64^3 field of features
    and the rate of full Adam training steps (forward, backward, reduction,
    update) on minibatches; random inputs, BF16 matrix cores."""
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    x = torch.randn((points, 16), generator=g, device="cuda").to(torch.bfloat16)
    x[:, 9:] = 0
    t = torch.randn((points, 6), generator=g, device="cuda")
    net = fs.Mlp(seed=7)
    net.forward(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / reps
    xb, tb = x[:batch].contiguous(), t[:batch].contiguous()
    net.train_step(xb, tb, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps * 5):
        net.train_step(xb, tb, 1e-4)
    torch.cuda.synchronize()
    trn = (time.perf_counter() - t0) / (reps * 5)
    net.close()
    return {"forward_points": points, "forward_us": fwd * 1e6,
            "forward_TFLOPs": MLP_FLOP_PER_POINT * points / fwd / 1e12,
            "train_batch": batch, "train_step_us": trn * 1e6,
            "train_TFLOPs": 3 * MLP_FLOP_PER_POINT * batch / trn / 1e12,
            "peak_TFLOPs_bf16": 2500.0,
            "note": "flop = 2 x multiply-adds of the three layers (GELU and biases not counted); "
                    "training counted as 3 x forward"}


def copy_ceiling(torch, gib=2.0, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second)."""
    nb = int(gib * 2 ** 30) // 4
    a = torch.ones(nb, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    del a, b
    return {"GBps": 2 * nb * 4 / el / 1e9, "bytes_per_copy": nb * 4, "kind": "torch copy_"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50,
                    help="timed graph-launched steps, split into --reps repetitions")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5,
                    help="repetitions of the timed steps; ms_per_step is their median")
    ap.add_argument("--breakdown-steps", type=int, default=10,
                    help="steps of the per-kernel event pass after the timed region (0 = skip)")
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--cpu-n", type=int, default=512,
                    help="grid of the oracle's timed step (the CPU baseline)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", choices=["3d", "ensemble"], default="3d")
    ap.add_argument("--ens-steps", type=int, default=200)
    ap.add_argument("--ens-counter-pass", action="store_true",
                    help="ensemble workload: run --ens-steps steps of the default schedules "
                         "with direct launches and print nothing (for counter collection)")
    ap.add_argument("--les-n", type=int, default=64,
                    help="LES grid of the closure speedup measurement (0 = skip)")
    ap.add_argument("--les-steps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the copy ceiling, network and ensemble measurements")
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--boussinesq", action="store_true",
                    help="3D Boussinesq flow (a buoyancy field b beside u), squared "
                         "buoyancy frequency --n2; no LES or CPU leg")
    ap.add_argument("--n2", type=float, default=4.0)
    ap.add_argument("--rotation", type=float, default=0.0,
                    help="Coriolis parameter f of a frame rotating about z; no LES or CPU leg")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE {world})", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_1807_01769_amd import fs, inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        return 1
    if args.workload == "ensemble":
        return bench_ensemble(args)
    n = args.n
    dev = torch.device("cuda:0")
    if args.calib_copy_gib > 0:
        nb = int(args.calib_copy_gib * 2 ** 30) // 4
        a = torch.ones(nb, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"calibration copy: {nb * 4} bytes read, {nb * 4} bytes written")
        del a, b
    log(f"generating the {n}^3 initial field")
    t0 = time.perf_counter()
    u0 = I.random_solenoidal_3d(n, seed=SEED, dtype=np.complex64)
    if args.boussinesq:
        # b: one solenoidal component of a second draw (same spectrum)
        b0 = I.random_solenoidal_3d(n, seed=SEED + 1, dtype=np.complex64)[2]
        u0 = np.concatenate([u0, b0[None]])
        del b0
    state = torch.from_numpy(u0).to(dev)
    del u0
    log(f"initial field ready ({time.perf_counter() - t0:.1f} s)")
    plain = not args.boussinesq and args.rotation == 0.0
    variant_opts = dict(boussinesq=args.boussinesq, n2=args.n2 if args.boussinesq else 0.0,
                        rotation=args.rotation)
    plan = fs.Plan(n, nu=NU, dt=DT, ndim=3, precision="f32", forcing_power=POWER,
                   forcing_kmin=KMIN, forcing_kmax=KMAX, **variant_opts)
    plan.step(state, args.warmup)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # Timed region: exactly K graph-launched steps, in R repetitions of about
    # K / R steps, each bracketed by HIP events on the plan's stream (torch's
    # current stream, on which the plan was created); ms_per_step is the
    # median over the repetitions of their time per step.
    reps = max(1, min(args.reps, args.steps))
    chunks = [args.steps // reps + (1 if r < args.steps % reps else 0) for r in range(reps)]
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in chunks]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (e0, e1), c in zip(evs, chunks):
        e0.record()
        plan.step(state, c)
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rep_ms = [e0.elapsed_time(e1) / c for (e0, e1), c in zip(evs, chunks)]
    ms_per_step = float(np.median(rep_ms))
    host_ms_per_step = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps in {reps} repetitions: median {ms_per_step:.3f} ms/step "
        f"(repetitions {', '.join(f'{v:.3f}' for v in rep_ms)}; host clock {host_ms_per_step:.3f})")

    _, e, z = plan.energy_spectrum(state)
    energy, enstrophy = float(e.cpu()), float(z.cpu())
    if not (math.isfinite(energy) and math.isfinite(enstrophy)):
        print("non-finite state after the timed steps", file=sys.stderr)
        return 1

    # Per-kernel breakdown: the same step on a plan that launches its kernels
    # directly and brackets each with HIP events on the plan's stream, for
    # `--breakdown-steps` steps right after the timed region; the roofline of
    # the dominant kernel uses these per-launch averages.
    kernels, roofline = {}, None
    tvariant = "plain" if plain else (
        "boussinesq" if args.boussinesq and args.rotation == 0.0 else None)
    tr = read_traffic(tvariant)
    tr_ok = bool(tr and tr.get("source_hash") == kernel_source_hash() and tr.get("n") == n)
    bsteps = args.breakdown_steps
    if bsteps > 0:
        plan.close()
        plan = fs.Plan(n, nu=NU, dt=DT, ndim=3, precision="f32", forcing_power=POWER,
                       forcing_kmin=KMIN, forcing_kmax=KMAX, profile=True, **variant_opts)
        plan.step(state, 1)
        torch.cuda.synchronize()
        plan.profile_read()
        tb0 = time.perf_counter()
        plan.step(state, bsteps)
        torch.cuda.synchronize()
        prof_ms_per_step = (time.perf_counter() - tb0) * 1e3 / bsteps
        prof = plan.profile_read()
        alg = algorithmic_bytes(n, bsteps, nc=4 if args.boussinesq else 3)
        for name, (ms, cnt) in prof.items():
            rec = {"ms_total": ms, "launches": cnt, "ms_avg": ms / cnt}
            if name in alg and alg[name][1] == cnt:
                tot, _ = alg[name]
                rec["alg_bytes_per_launch"] = tot / cnt
                rec["alg_GBps"] = tot / cnt / (ms / cnt * 1e-3) / 1e9
            kernels[name] = rec
        dom = max((k for k in kernels if "alg_GBps" in kernels[k]), key=lambda k: kernels[k]["ms_total"])
        traffic = tr.get("bytes_per_launch", {}).get(dom) if tr_ok else None
        ach = kernels[dom]["alg_GBps"]
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "alg_bytes_per_launch": kernels[dom]["alg_bytes_per_launch"],
                    "ms_avg": kernels[dom]["ms_avg"],
                    "kernel_timing": f"HIP events around every launch on the plan's stream, "
                                     f"{bsteps} directly launched steps after the timed region "
                                     f"({prof_ms_per_step:.3f} ms/step on the host clock)"}
        step_alg = sum(v[0] for k, v in alg.items() if k != "p1") / bsteps
        roofline["step_alg_GBps"] = round(step_alg / (ms_per_step * 1e-3) / 1e9, 1)
        roofline["step_alg_frac"] = round(roofline["step_alg_GBps"] / HBM_PEAK_GBS, 4)
        if not args.boussinesq:
            roofline["step_unfused_model_frac"] = round(
                unfused_model_bytes(n) / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)

        if tr_ok:
            bpl = tr.get("bytes_per_launch", {})
            names = [k for k in ("z_stage", "x_c2r_product_r2c", "y_inverse", "y_forward")
                     if k in bpl and k in kernels]
            step_bytes = sum(bpl[k] * kernels[k]["launches"] for k in names) / bsteps
            roofline["step_measured_GBps"] = round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1)
            roofline["step_measured_frac"] = round(roofline["step_measured_GBps"] / HBM_PEAK_GBS, 4)

    les = None
    if plain and args.les_n > 0 and args.les_n < n:
        les = closure_les_speed(fs, torch, plan, state, args.les_n, args.les_steps, ms_per_step)
    extras = {}
    if not args.no_extras:
        plan.close()
        del state
        torch.cuda.empty_cache()
        extras["copy_ceiling"] = copy_ceiling(torch)
        log(f"copy ceiling {extras['copy_ceiling']['GBps']:.0f} GB/s")
        extras["mlp"] = time_mlp(fs, torch)
        log(f"closure network: forward {extras['mlp']['forward_TFLOPs']:.1f} TFLOP/s")
        ens, _, _ = time_ensemble(fs, torch, I, np, args.ens_steps)
        extras["ensemble"] = ens
        log(f"ensemble: {ens['gridpoint_steps_per_s']:.3e} gridpoint-steps/s")

    cpu = None
    if plain and not args.no_cpu:
        log("timing the FP64 CPU oracle on a bounded sample")
        cpu = cpu_baseline(args.cpu_n)

    # the stratified and rotating variants are other workloads: their own metric
    # name and a structured variant, so that no collector mixes them with the
    # headline forced-turbulence step
    variant = None if plain else {"boussinesq": bool(args.boussinesq),
                                  "n2": args.n2 if args.boussinesq else 0.0,
                                  "rotation_f": args.rotation}
    metric = METRIC if plain else (
        "RK4 step ns/gridpoint, 3D " + ("rotating " if args.rotation else "")
        + ("Boussinesq (stratified) " if args.boussinesq else "") + f"flow {n}^3 FP32")
    out = {
        "metric": metric,
        "value": ms_per_step * 1e6 / n ** 3,
        "unit": "ns/gridpoint/step",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_repetitions": rep_ms,
        "host_ms_per_step": host_ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3D forced isotropic turbulence {n}^3, velocity form, FP32, "
                               "nu=2e-4, dt=1e-3, random solenoidal E(k)~k^4 exp(-2(k/4)^2) unit "
                               "energy seed 1, constant-power forcing 5e-3 on 2<=|k|<=3, "
                               "2/3 dealiasing, Lawson IF-RK4"
                               + (f", Boussinesq N^2={args.n2} (b: second draw, seed 2)"
                                  if args.boussinesq else "")
                               + (f", rotating frame f={args.rotation}" if args.rotation else ""),
                   "n": n,
                   "timing": f"graph-launched steps, median of {reps} repetitions of "
                             f"{'/'.join(str(c) for c in chunks)} steps (HIP events)",
                   "variant": variant},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "closure_les": les,
        **extras,
        "kernels": kernels,
        "energy_after": energy,
        "enstrophy_after": enstrophy,
    }
    print(json.dumps(out), flush=True)
    if args.no_extras:
        plan.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
