#!/usr/bin/env python3
"""Benchmark of the batched Jacobi SVD / randomized SVD hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

One step = one call of the library over the whole synthetic batch, inputs resident in HBM.
Prints one JSON line (rank 0) with throughput, the roofline figure of the dominant kernel (timed with
HIP events on the stream the library launches on) and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "batched SVDs/s + GFLOP/s (% roofline), mixed+learned vs plain FP64 at 1e-6 err"
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def jacobi_model_flops(M, N, sweeps):
    """Flop model of one-sided Jacobi: each sweep tests N(N-1)/2 pairs (three length-M dot products,
    6M flops) and, in every sweep but the last, rotates them (6M flops on the working columns and 6N
    on the V columns). Rotations skipped before the last sweep are not subtracted."""
    P = N * (N - 1) // 2
    sweeps = np.asarray(sweeps, dtype=np.float64)
    return float(np.sum(sweeps * P * 6 * M + np.maximum(sweeps - 1, 0) * P * (6 * M + 6 * N)))


def wl_c1():
    return dict(name="jacobi_wave_f64_1000x32x32", batch=1000, m=32, n=32, seed=1)


def run_c1(args, torch, P, synth):
    w = wl_c1()
    A_np = synth.batch_gaussian(w["batch"], w["m"], w["n"], seed=w["seed"])
    A = torch.from_numpy(A_np).cuda()
    b, m, n = A.shape
    k = min(m, n)
    Acm = P.colmajor(A)
    S = torch.empty((b, k), dtype=A.dtype, device="cuda")
    U = torch.empty((b, k, m), dtype=A.dtype, device="cuda")
    V = torch.empty((b, k, n), dtype=A.dtype, device="cuda")
    sw = torch.empty(b, dtype=torch.int32, device="cuda")
    info = torch.empty(b, dtype=torch.int32, device="cuda")
    ptr = lambda t: t.data_ptr() + t.stride(0) * t.element_size() * np.arange(b, dtype=np.uint64)
    args_c = (np.full(b, m), np.full(b, n), ptr(Acm), np.full(b, m), ptr(S), ptr(U), np.full(b, m), ptr(V),
              np.full(b, n))

    def step():
        P.batched_svd(*args_c, sweeps=sw, info=info)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        step()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
    assert int(info.max().item()) == 0, "non-zero info in benchmark batch"
    sweeps = sw.cpu().numpy()
    flops = jacobi_model_flops(m, n, sweeps)
    # parity spot check on sampled instances
    import oracle
    idx = np.random.default_rng(0).choice(b, 16, replace=False)
    So = oracle.batched_jacobi_svd(A_np[idx], want_vectors=False)[0]
    err = float(np.max(np.abs(S.cpu().numpy()[idx] - So) / So[:, :1]))
    assert err <= 1e-12, err

    ms_per_step = wall * 1e3 / args.steps
    achieved = flops / (kern_ms * 1e-3) / 1e12
    res = dict(value=b / (ms_per_step * 1e-3), unit="SVDs/s", ms_per_step=ms_per_step, dtype="f64",
               config=dict(workload=w["name"], batch=b, m=m, n=n, tol=1e-15, seed=w["seed"],
                           mean_sweeps=float(sweeps.mean()), gflops_model=flops / 1e9,
                           gflop_per_s=flops / (ms_per_step * 1e-3) / 1e9, max_sigma_err_sampled=err),
               roofline=dict(bound="alu", achieved=achieved, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                             frac=achieved / FP64_PEAK_TFLOPS, traffic=None, kernel="jacobi_wave_kernel<double,32,32>",
                             kernel_ms=kern_ms))
    if args.cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_jacobi(A_np, oracle)
    return res


def cpu_baseline_jacobi(A_np, oracle):
    """The oracle (OpenMP across instances, as written) on the same batch: SVDs/s."""
    b = A_np.shape[0]
    best = None
    t_total = 0.0
    reps = 0
    while t_total < 10.0 and reps < 20:
        t0 = time.perf_counter()
        oracle.batched_jacobi_svd(A_np)
        dt = time.perf_counter() - t0
        t_total += dt
        reps += 1
        best = dt if best is None else min(best, dt)
    return dict(value=b / best, unit="SVDs/s", cores=oracle.num_threads(), kind="oracle",
                sample="full batch of %d instances, best of %d runs (%.1f s CPU wall total)" % (b, reps, t_total))


def run_c2(args, torch, P, synth):
    """10,000 graded 64 x 64 plus 20,000 graded 128 x 32 (sigma_i = 10^(-8(i-1)/(n-1))): Householder
    QR, one-sided Jacobi of R (rows), U = Q U_R; one call per shape group, both in a step."""
    import oracle
    from paper_1707_05141_amd import _lib
    groups = []
    for (b, m, n) in [(10000, 64, 64), (20000, 128, 32)]:
        A_np = synth.batch_prescribed(b, m, n, synth.graded_sigma_log(n, 8.0), seed=2)
        A = torch.from_numpy(A_np).cuda()
        k = min(m, n)
        Acm = P.colmajor(A)
        S = torch.empty((b, k), dtype=A.dtype, device="cuda")
        U = torch.empty((b, k, m), dtype=A.dtype, device="cuda")
        V = torch.empty((b, k, n), dtype=A.dtype, device="cuda")
        sw = torch.empty(b, dtype=torch.int32, device="cuda")
        info = torch.empty(b, dtype=torch.int32, device="cuda")
        ptr = lambda t, b=b: t.data_ptr() + t.stride(0) * t.element_size() * np.arange(b, dtype=np.uint64)
        groups.append(dict(A_np=A_np, A=A, Acm=Acm, S=S, U=U, V=V, sw=sw, info=info, m=m, n=n, b=b,
                           args=(np.full(b, m), np.full(b, n), ptr(Acm), np.full(b, m), ptr(S), ptr(U), np.full(b, m),
                                 ptr(V), np.full(b, n))))

    def step():
        for g in groups:
            P.batched_svd(*g["args"], sweeps=g["sw"], info=g["info"], flags=_lib.SVD_QR_FIRST)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record()
        step()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = float(np.mean([s.elapsed_time(e) for s, e in ev]))
    flops = 0.0
    errs = []
    for g in groups:
        assert int(g["info"].max().item()) == 0
        sw = g["sw"].cpu().numpy()
        m, n = g["m"], g["n"]
        qr_fl = 2 * (2 * m * n * n - 2 * n ** 3 / 3)  # factorisation + thin Q
        flops += g["b"] * qr_fl + jacobi_model_flops(n, n, sw) + g["b"] * 2 * m * n * n
        sig = synth.graded_sigma_log(n, 8.0)
        errs.append(float(np.max(np.abs(g["S"].cpu().numpy() - sig[None, :]))))
    assert max(errs) <= 1e-12, errs
    total = sum(g["b"] for g in groups)
    ms_per_step = wall * 1e3 / args.steps
    achieved = flops / (step_ms * 1e-3) / 1e12
    res = dict(value=total / (ms_per_step * 1e-3), unit="SVDs/s", ms_per_step=ms_per_step, dtype="f64",
               config=dict(workload="qr_jacobi_f64_10000x64x64_20000x128x32", batch=total, kappa=1e8,
                           mean_sweeps={"%dx%d" % (g["m"], g["n"]): float(g["sw"].float().mean().item()) for g in groups},
                           gflops_model=flops / 1e9, gflop_per_s=flops / (ms_per_step * 1e-3) / 1e9,
                           max_sigma_err=max(errs)),
               roofline=dict(bound="alu", achieved=achieved, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                             frac=achieved / FP64_PEAK_TFLOPS, traffic=None, kernel="whole step (QR + Jacobi + GEMM)",
                             kernel_ms=step_ms))
    return res


WORKLOADS = {"c1": run_c1, "c2": run_c2}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c1", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on exactly one GPU; --gpus %d is not supported "
              "(independent instances would shard across GPUs with no exchange)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1707_05141_amd as P
    from paper_1707_05141_amd import synth
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    res = WORKLOADS[args.workload](args, torch, P, synth)
    out = dict(metric=METRIC, value=res["value"], unit=res["unit"], n_gpus=1, steps=args.steps, warmup=args.warmup,
               ms_per_step=res["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None,
               dtype=res["dtype"], data="synthetic", config=res["config"], roofline=res["roofline"])
    if "cpu_baseline" in res:
        out["cpu_baseline"] = res["cpu_baseline"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
