#!/usr/bin/env python3
"""Throughput of the MGARD+ hot path on one MI355X.

Workload: a 513^3 float32 Gaussian random field with a turbulence-like
spectrum P(k) ~ k^-11/3 (NYX-shaped), decomposed fully (L = 8, down to
3^3), quantized level-wise at tau = 1e-3 * range, dequantized and
recomposed.  One step = decompose + quantize + dequantize + recompose,
with the input already resident in HBM.  value = 2 * N * 4 bytes / step
time (the paper's size/time metric for the decompose and the recompose of
one field; quantization is inside the timed step, so the figure is
conservative for decompose+recompose alone, which is reported beside it).

Prints one JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decompose+recompose GB/s on 513^3 fp32 + % HBM roofline; batched vs plain"
HBM_PEAK_GBPS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2010_05872_amd", "csrc", "kernels.hip")


def level_sizes(shape, L, l):
    out = 1
    for n in shape:
        out *= (n - 1) // 2 ** (L - l) + 1
    return out


def algorithmic_bytes(name, level, shape, L, s):
    """Bytes one launch must move at minimum (each operand read or written once)."""
    if level < 0:
        N = 1
        for n in shape:
            N *= n
        return N * (s + 4)  # quantize / dequantize: coefficients + int32 labels
    Nl = level_sizes(shape, L, level)
    Nc = level_sizes(shape, L, level - 1)
    table = {
        "load_vector_dec": 2 * Nl,        # read Q_l u; write coefficients (N_l - N_c) and load vector (N_c)
        "load_vector_rec": Nl,            # read coefficients (N_l - N_c); write load vector (N_c)
        "interp_add": 2 * Nl,             # read nodal (N_c) + coefficients (N_l - N_c); write Q_l u
        "solve_contig": 2 * Nc,           # load vector in, solved rows out
        "solve_strided": 2 * Nc,
        "solve_strided_store": 2 * Nc,    # read load vector, write Q_{l-1} u
        "solve_strided_apply": 3 * Nc,    # read load vector + nodal, write nodal
        "finish_1d": 3 * Nc,
    }
    return table[name] * s


def kernel_source_sha():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, level, shape):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    if data.get("kernel_sha") != kernel_source_sha():
        return None
    key = f"{kernel}@{level}:{'x'.join(map(str, shape))}"
    ent = data.get("kernels", {}).get(key)
    return None if ent is None else ent.get("bytes_per_launch")


def cpu_baseline(u_gpu, rel_tol):
    """The FP64 oracle, as it stands, on a bounded sample of the same field:
    the 257^3 corner sub-box, one full step."""
    import numpy as np

    import oracle
    sub = u_gpu[:257, :257, :257].double().cpu().numpy()
    tol = rel_tol * float(sub.max() - sub.min())
    t0 = time.perf_counter()
    v = oracle.decompose(sub)
    labels, code = oracle.quantize(v, tol)
    vq = oracle.dequantize(labels, tol)
    r = oracle.recompose(vq)
    dt = time.perf_counter() - t0
    err = float(np.abs(r - sub).max())
    nbytes = 2 * sub.size * 4
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": "257^3 corner sub-box of the benchmark field, one step (decompose, quantize, "
                      "dequantize, recompose), FP64 single-threaded C oracle; bytes counted as 2*N*4",
            "seconds": dt, "max_err_over_tau": err / tol, "quantize_status": int(code)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--rel-tol", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of the field (counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; multi-GPU runs are not "
                                   "part of this build (fields shard across GPUs without exchange)"}))
        sys.exit(2)

    import torch

    import paper_2010_05872_amd as mgx
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    shape = (n, n, n)
    u = workloads.turbulence_field(n, device=dev, dtype=torch.float32)
    torch.cuda.synchronize()
    rng = float((u.max() - u.min()).item())
    tol = args.rel_tol * rng
    L = mgx.num_levels(shape)
    umc = torch.empty_like(u)
    uq = torch.empty_like(u)
    ut = torch.empty_like(u)
    labels = torch.empty(shape, dtype=torch.int32, device=dev)
    ws = torch.empty(mgx.workspace_size(mgx.MGX_F32, shape, 0), dtype=torch.uint8, device=dev)

    def step():
        mgx.decompose(u, out=umc, workspace=ws)
        mgx.quantize(umc, tol, out=labels)
        mgx.dequantize(labels, tol, torch.float32, out=uq)
        mgx.recompose(uq, out=ut, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---- timed region ----
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) / args.steps * 1e3
    N = u.numel()
    value = 2 * N * 4 / (ms_per_step * 1e-3) / 1e9

    # ---- per-operation times (events on the stream the library launches on) ----
    ops = {
        "decompose": lambda: mgx.decompose(u, out=umc, workspace=ws),
        "quantize": lambda: mgx.quantize(umc, tol, out=labels),
        "dequantize": lambda: mgx.dequantize(labels, tol, torch.float32, out=uq),
        "recompose": lambda: mgx.recompose(uq, out=ut, workspace=ws),
    }
    op_ms = {}
    for name, fn in ops.items():
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        op_ms[name] = e0.elapsed_time(e1) / args.steps

    # ---- kernel durations: HIP events around every launch, same stream ----
    mgx.trace_enable(True)
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ktimes = mgx.trace_read()
    mgx.trace_enable(False)
    traced_ms_per_step = (t3 - t2) / args.steps * 1e3
    dom = max(ktimes, key=lambda k: k["total_ms"])
    avg_ms = dom["total_ms"] / dom["count"]
    alg = algorithmic_bytes(dom["name"], dom["level"], shape, L, 4)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom["name"], dom["level"], shape)
    total_alg = sum(algorithmic_bytes(k["name"], k["level"], shape, L, 4) * k["count"] for k in ktimes)
    kernel_sum_ms = sum(k["total_ms"] for k in ktimes) / args.steps

    if args.copy_calibration:
        # a plain copy kernel of known size (N * 4 bytes read, N * 4 written)
        ut.copy_(u)
        torch.cuda.synchronize()

    # ---- correctness of the measured run ----
    err = float((ut.double() - u.double()).abs().max().item())

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{n}^3 fp32 Gaussian random field P(k)~k^-11/3 (NYX-shaped), full decomposition "
                        f"L={L} to 3^3, level-wise quantization at tau={args.rel_tol:g}*range",
            "step": "decompose+quantize+dequantize+recompose",
            "bytes_counted_per_step": 2 * N * 4,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom['name']}@level{dom['level']}",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg,
            "avg_launch_ms": round(avg_ms, 5),
        },
        "op_ms": {k: round(v, 4) for k, v in op_ms.items()},
        "dec_rec_GBps": round(2 * N * 4 / ((op_ms["decompose"] + op_ms["recompose"]) * 1e-3) / 1e9, 2),
        "step_algorithmic_GB": round(total_alg / args.steps / 1e9, 4),
        "step_kernel_sum_ms": round(kernel_sum_ms, 4),
        "step_roofline_frac": round(total_alg / args.steps / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "traced_ms_per_step": round(traced_ms_per_step, 4),
        "kernels": sorted(({"name": k["name"], "level": k["level"], "avg_ms": round(k["total_ms"] / k["count"], 5)}
                           for k in ktimes), key=lambda k: -k["avg_ms"])[:12],
        "max_err_over_tau": round(err / tol, 5),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(u, args.rel_tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
