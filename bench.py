#!/usr/bin/env python3
"""Throughput of the MGARD+ hot path on one MI355X.

Workload: a 513^3 float32 Gaussian random field with a turbulence-like
spectrum P(k) ~ k^-11/3 (NYX-shaped), decomposed fully (L = 8, down to
3^3), quantized level-wise at tau = 1e-3 * range, dequantized and
recomposed.  One step = decompose + quantize + dequantize + recompose,
with the input already resident in HBM: the fused entry points, whose level
kernels write (decomposition) and read (recomposition) the labels
themselves, so the coefficients never make a separate trip through HBM.
value = 2 * N * 4 bytes / step time (the paper's size/time metric for the
decompose and the recompose of one field, with quantization inside the
timed step).  The four separate calls are timed beside it.

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
# the device code of the profiled 1-D to 3-D kernels: their source and the headers it includes
KERNEL_SRC = tuple(os.path.join(ROOT, "paper_2010_05872_amd", "csrc", f)
                   for f in ("kernels.hip", "kernels.hpp", "levelpos.hpp"))


def level_sizes(shape, L, l):
    out = 1
    for n in shape:
        out *= (n - 1) // 2 ** (L - l) + 1
    return out


def algorithmic_bytes(name, level, shape, L, s):
    """Bytes one launch must move at minimum (each operand read or written once).
    A "+q" kernel reads or writes int32 labels in place of the coefficients
    (4 bytes each, the same as a float32 coefficient)."""
    if name.endswith("+q"):
        if s != 4:
            raise ValueError("label-kernel byte counts are stated for float32 fields")
        name = name[:-2]
    if level < 0:
        N = 1
        for n in shape:
            N *= n
        Nfine = N - level_sizes(shape, L, L - 1)  # coefficients of the finest level
        if name.endswith("_finest"):
            return Nfine * (s + 4)
        if name.endswith("_coarse"):
            return (N - Nfine) * (s + 4)
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
        "tail_dec": 2 * Nl,               # levels lt..stop+1 in one workgroup: read Q_lt u, write its coefficients
        "tail_rec": 2 * Nl,               # read the coefficients of levels <= lt, write Q_lt u
        "copy_box": 2 * Nl,
    }
    return table[name] * s


def kernel_source_sha(paths=KERNEL_SRC):
    """sha256 of the kernels' code (source and headers, in order): comments
    dropped, whitespace collapsed (a comment edit leaves the measured kernels,
    and so their counters, valid)."""
    import re
    src = "\n".join(open(p).read() for p in paths)
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


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
    """The FP64 oracle, as it stands (single-threaded C), on the benchmark
    field itself: one full step, timed on one host core."""
    import numpy as np

    import oracle
    sub = u_gpu.double().cpu().numpy()
    tol = rel_tol * float(sub.max() - sub.min())
    t0 = time.perf_counter()
    v = oracle.decompose(sub)
    labels, code = oracle.quantize(v, tol)
    vq = oracle.dequantize(labels, tol)
    r = oracle.recompose(vq)
    dt = time.perf_counter() - t0
    err = float(np.abs(r - sub).max())
    nbytes = 2 * sub.size * 4
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": nbytes / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"the full {'x'.join(map(str, sub.shape))} benchmark field (promoted to FP64), one step "
                      "(decompose, quantize, dequantize, recompose); bytes counted as 2*N*4 like the GPU value",
            "seconds": dt, "host_cpu": cpu, "host_cores_available": len(os.sched_getaffinity(0)),
            "max_err_over_tau": err / tol, "quantize_status": int(code)}


def timed(torch, fn, reps):
    """Mean ms of fn() over reps calls, bracketed by device synchronizations."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps * 1e3


def batched_section(torch, mgx, workloads, dev, reps):
    """64 fp32 fields of uneven shapes (axes from {33,65,129,257}), k^-2..k^-4
    spectra, per-field tolerances log-uniform in [1e-4,1e-2]*range: decompose +
    quantize, then dequantize + recompose (labels written and read by the level
    kernels), per field (plain) or as one batch."""
    specs = workloads.batch_specs()
    us = [workloads.batch_field(s, device=dev) for s in specs]
    tols = [s["rel_tol"] * float((u.max() - u.min()).item()) for s, u in zip(specs, us)]
    mk = lambda: [torch.empty_like(u) for u in us]  # noqa: E731
    outs_p, rec_p = mk(), mk()
    outs_b, rec_b = mk(), mk()
    lab_p = [torch.empty(u.shape, dtype=torch.int32, device=dev) for u in us]
    lab_b = [torch.empty(u.shape, dtype=torch.int32, device=dev) for u in us]
    ws = torch.empty(max(mgx.workspace_size(mgx.MGX_F32, u.shape, 0) for u in us), dtype=torch.uint8, device=dev)

    def plain():  # one fused call per field and direction
        for u, o, lab, t in zip(us, outs_p, lab_p, tols):
            mgx.decompose_quantize(u, t, out=o, labels=lab, workspace=ws)
        for lab, r, t in zip(lab_p, rec_p, tols):
            mgx.dequantize_recompose(lab, t, torch.float32, out=r, workspace=ws)

    bd = mgx.Batch([{"in": u, "out": o, "tol": t, "labels": lab} for u, o, t, lab in zip(us, outs_b, tols, lab_b)])
    br = mgx.Batch([{"out": r, "tol": t, "labels": lab} for r, t, lab in zip(rec_b, tols, lab_b)])

    def batched():
        bd.decompose()
        br.recompose()

    for _ in range(2):  # warmup; the first batched call captures and tunes the graphs
        plain()
        batched()
    bd.decompose()
    info_d = mgx.batch_last_info()
    br.recompose()
    info_r = mgx.batch_last_info()
    plain_ms = timed(torch, plain, reps)
    batched_ms = timed(torch, batched, reps)
    same = all(torch.equal(a, b) for a, b in zip(rec_p, rec_b)) and all(torch.equal(a, b) for a, b in zip(lab_p, lab_b))
    N = sum(u.numel() for u in us)
    nbytes = 2 * N * 4
    return {"fields": len(us), "values": N, "bytes_counted": nbytes,
            "step": "decompose+quantize, dequantize+recompose of every field",
            "plain_ms": round(plain_ms, 4), "batched_ms": round(batched_ms, 4),
            "plain_GBps": round(nbytes / (plain_ms * 1e-3) / 1e9, 2),
            "batched_GBps": round(nbytes / (batched_ms * 1e-3) / 1e9, 2),
            "speedup": round(plain_ms / batched_ms, 3), "batched_equals_plain": bool(same),
            "graph_launches": {"decompose": info_d["launches"], "recompose": info_r["launches"]},
            "tuned_shape": {"decompose": [info_d["target_blocks"], info_d["min_zchunk"]],
                            "recompose": [info_r["target_blocks"], info_r["min_zchunk"]]},
            }


def adjoint_section(torch, mgx, workloads, dev, reps):
    """8 fp32 257^3 fields (k^-3): forward y = R(D x + delta) against the
    backward pass D^T R^T g of the autograd Function."""
    X = workloads.adjoint_fields(device=dev)
    delta = 1e-3 * torch.randn(X.shape, device=dev, generator=torch.Generator(device=dev).manual_seed(5))
    g = torch.randn(X.shape, device=dev, generator=torch.Generator(device=dev).manual_seed(6))
    ws = torch.empty(mgx.adjoint_workspace_size(mgx.MGX_F32, X.shape[1:], 0), dtype=torch.uint8, device=dev)
    c, y, gc, gx = (torch.empty_like(X) for _ in range(4))

    def forward():
        for i in range(X.shape[0]):
            mgx.decompose(X[i], out=c[i], workspace=ws)
            c[i].add_(delta[i])
            mgx.recompose(c[i], out=y[i], workspace=ws)

    def backward():
        for i in range(X.shape[0]):
            mgx.recompose_adjoint(g[i], out=gc[i], workspace=ws)
            mgx.decompose_adjoint(gc[i], out=gx[i], workspace=ws)

    forward()
    backward()
    f_ms = timed(torch, forward, reps)
    b_ms = timed(torch, backward, reps)
    N = X.numel()
    # D^T R^T = (R D)^T = I: the backward pass of the linear part returns g
    ident_err = float((gx - g).abs().max().item() / g.abs().max().item())
    nbytes = 2 * N * 4
    return {"fields": X.shape[0], "shape": list(X.shape[1:]), "values": N,
            "forward_ms": round(f_ms, 4), "backward_ms": round(b_ms, 4),
            "forward_GBps": round(nbytes / (f_ms * 1e-3) / 1e9, 2),
            "backward_GBps": round(nbytes / (b_ms * 1e-3) / 1e9, 2),
            "backward_over_forward": round(b_ms / f_ms, 3),
            "rel_err_DtRt_identity": ident_err}


def progressive_section(torch, mgx, u, umc, ws, reps):
    """Progressive recomposition of the benchmark field: Q_t u on the level-t
    grid for every target t, against the full recomposition.  Bytes counted:
    the coefficients of levels <= t read once (the level-t box of u_mc) and
    the level-t box written once."""
    L = mgx.num_levels(u.shape)
    out = {}
    for t in range(max(L - 4, 0), L + 1):
        box = mgx.level_shape(u.shape, t)
        n = 1
        for m in box:
            n *= m
        dst = torch.empty(box, dtype=u.dtype, device=u.device)
        fn = lambda: mgx.recompose_to(umc, t, out=dst, workspace=ws)  # noqa: E731
        fn()
        ms = timed(torch, fn, reps)
        out[str(t)] = {"box": list(box), "ms": round(ms, 4), "GBps": round(2 * n * 4 / (ms * 1e-3) / 1e9, 2)}
    full = mgx.recompose(umc, workspace=ws)
    torch.cuda.synchronize()
    same = bool(torch.equal(mgx.recompose_to(umc, L, workspace=ws), full))
    return {"targets": out, "target_L_equals_recompose": same}


def adaptive_section(torch, mgx, u, umc, ws, reps):
    """Adaptive decomposition of the benchmark field at three tolerances:
    the stop level chosen and the time, against the full decomposition; and
    of a field of the same shape that is a sum of three products of two
    one-axis waves (period 2 pi n / 8 nodes), which Lorenzo's predictor
    reproduces up to rounding, so that the estimate stops the decomposition
    early (the time of the levels gated off included)."""
    rng = float((u.max() - u.min()).item())
    out = {}
    for rel in (1e-2, 1e-3, 1e-4):
        res = {}
        fn = lambda: res.update(stop=mgx.decompose_adaptive(u, rel * rng, out=umc, workspace=ws)[1])  # noqa: E731
        fn()
        ms = timed(torch, fn, reps)
        out[f"{rel:g}"] = {"stop_level": res["stop"], "ms": round(ms, 4)}
    full_ms = timed(torch, lambda: mgx.decompose(u, out=umc, workspace=ws), reps)
    s = u.shape[0] / 8
    z, y, x = (torch.arange(k, device=u.device, dtype=torch.float64) / s for k in u.shape)
    z, y, x = z[:, None, None], y[None, :, None], x[None, None, :]
    wave = (torch.sin(x) * torch.cos(y) + torch.sin(y + 1) * torch.cos(z) + torch.cos(x) * torch.sin(z)).to(u.dtype)
    del x, y, z
    wrng = float((wave.max() - wave.min()).item())
    res = {}
    fn = lambda: res.update(stop=mgx.decompose_adaptive(wave, 1e-3 * wrng, out=umc, workspace=ws)[1])  # noqa: E731
    fn()
    wave_ms = timed(torch, fn, reps)
    del wave
    return {"tau_over_range": out, "full_decompose_ms": round(full_ms, 4),
            "two_axis_waves_1e-3": {"stop_level": res["stop"], "ms": round(wave_ms, 4)}}


def entropy_section(torch, mgx, u, labels, tol, reps):
    """Per-level entropy of the step's labels (L-infinity schedule) and the
    estimated size of the labels in bits per value (Sec. 4.1's cost
    estimate), with the time of the entropy pass, alone and given the
    fused quantizer's per-level maxima (one read of the labels); the same
    for the L2
    schedule with the library's default C_L2, at an L2 tolerance whose
    root-mean-square error over the domain equals the L-infinity tolerance
    (tau_L2 = tol * sqrt(|Omega|), |Omega| = 512^3 on unit spacing)."""
    L = mgx.num_levels(u.shape)
    counts, prev = [], 0
    for l in range(L + 1):
        box = 1
        for m in mgx.level_shape(u.shape, l):
            box *= m
        counts.append(box - prev)
        prev = box
    ws = torch.empty(mgx.lib().mgx_label_entropy_workspace_size(3, mgx._dims(u.shape), 0), dtype=torch.uint8,
                     device=u.device)
    H = mgx.label_entropy(labels, 0, workspace=ws)
    ms = timed(torch, lambda: mgx.label_entropy(labels, 0, workspace=ws), reps)
    wsd = torch.empty(mgx.workspace_size(mgx.MGX_F32, u.shape, 0), dtype=torch.uint8, device=u.device)
    _, lab_s, st, _ = mgx.decompose_quantize(u, tol, labels=torch.empty_like(labels), workspace=wsd,
                                             keep_coef=False, stats=True)
    del wsd
    same = bool(torch.equal(lab_s, labels))
    Hb = mgx.label_entropy(lab_s, 0, workspace=ws, stats=st)
    ms_b = timed(torch, lambda: mgx.label_entropy(lab_s, 0, workspace=ws, stats=st), reps)
    del lab_s
    bits = float(sum(c * h for c, h in zip(counts, H)) / u.numel())
    umc = mgx.decompose(u)
    vol = 1.0
    for n in u.shape:
        vol *= n - 1
    tol_l2 = tol * vol ** 0.5
    tau2 = mgx.level_tolerances_l2(u.shape, tol_l2)
    H2 = mgx.label_entropy(mgx.quantize_levels(umc, tau2), 0, workspace=ws)
    bits2 = float(sum(c * h for c, h in zip(counts, H2)) / u.numel())
    return {"linf_bits_per_level": [round(float(h), 4) for h in H], "linf_bits_per_value": round(bits, 4),
            "l2_c": mgx.l2_constant(u.shape), "l2_tol_over_sqrt_volume": tol,
            "l2_bits_per_value": round(bits2, 4), "entropy_ms": round(ms, 3),
            "entropy_given_maxima_ms": round(ms_b, 3),
            "given_maxima_equal": bool(same and list(Hb) == list(H))}


def four_d_section(torch, mgx, workloads, dev, reps):
    """The 4-D workload: a field shaped like Table 2's QMCPACK data
    (288 x 115 x 69 x 69 fp32), padded with dummy nodes to 513 x 129 x 129 x 129,
    one step = pad, decompose+quantize and dequantize+recompose (the fused
    calls, labels only), crop.  Bytes counted: 2 x the real field (and 2 x
    the padded field)."""
    shape = (288, 115, 69, 69)
    u = workloads.orbital_field(shape, device=dev)
    p = mgx.pad(u)
    pshape = tuple(p.shape)
    L = mgx.num_levels(pshape)
    tol = 1e-3 * float((u.max() - u.min()).item())
    rec = torch.empty_like(p)
    labels = torch.empty(pshape, dtype=torch.int32, device=dev)
    back = torch.empty_like(u)
    ws = torch.empty(mgx.workspace_size(mgx.MGX_F32, pshape, 0), dtype=torch.uint8, device=dev)

    def step():
        mgx.pad(u, out=p)
        mgx.decompose_quantize(p, tol, labels=labels, workspace=ws, keep_coef=False)
        mgx.dequantize_recompose(labels, tol, torch.float32, out=rec, workspace=ws)
        mgx.crop(rec, shape, out=back)

    step()
    ms = timed(torch, step, reps)
    mgx.trace_enable(True)
    for _ in range(reps):
        step()
    torch.cuda.synchronize()
    kt = mgx.trace_read()
    mgx.trace_enable(False)
    err = float((back.double() - u.double()).abs().max().item())
    N, P = u.numel(), p.numel()
    kernels = sorted(({"name": k["name"], "level": k["level"], "avg_ms": round(k["total_ms"] / k["count"], 5)}
                      for k in kt), key=lambda k: -k["avg_ms"])[:8]
    # algorithmic bytes of the finest level's largest passes (fp32): the
    # decomposition's coefficient pass reads the level box and writes its
    # coefficient nodes' labels (15/16 of it) and the first load-vector sweep
    # (half of it); the recomposition's first sweep reads the labels and
    # writes half the box, its last pass reads the labels and writes the box
    fin = {k["name"]: k["total_ms"] / k["count"] for k in kt if k["level"] == L}
    per_unit = {"coef4_dec+q": 1 + 15 / 16 + 0.5, "sweep4_gather+q": 15 / 16 + 0.5,
                "coef4_rec+q": 15 / 16 + 1}
    rates = {k: round(P * f * 4 / (fin[k] * 1e-3) / 1e9, 1) for k, f in per_unit.items() if k in fin}
    out = {
        "shape": list(shape), "padded": list(pshape), "levels": L,
        "step": "pad, decompose+quantize, dequantize+recompose (fused calls, labels only), crop "
                "(tau = 1e-3 * range)",
        "ms": round(ms, 3),
        "GBps_real": round(2 * N * 4 / (ms * 1e-3) / 1e9, 2),
        "GBps_padded": round(2 * P * 4 / (ms * 1e-3) / 1e9, 2),
        "max_err_over_tau": round(err / tol, 5),
        "kernels": kernels,
        "finest_level_GBps": rates,
    }
    del u, p, rec, labels, back, ws
    torch.cuda.empty_cache()
    return out


def _event_ms(torch, fn, reps):
    """Mean ms per call of fn() from HIP events on the current stream (where
    the library launches)."""
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _dominant(mgx, torch, fn, reps, shape, L, s):
    """The longest kernel of fn() by HIP events (per launch), its algorithmic
    bytes and HBM rate."""
    mgx.trace_enable(True)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    kt = mgx.trace_read()
    mgx.trace_enable(False)
    dom = max(kt, key=lambda k: k["total_ms"])
    avg = dom["total_ms"] / dom["count"]
    alg = algorithmic_bytes(dom["name"], dom["level"], shape, L, s)
    return {"kernel": f"{dom['name']}@level{dom['level']}", "avg_launch_ms": round(avg, 5),
            "algorithmic_bytes_per_launch": alg, "achieved": round(alg / (avg * 1e-3) / 1e9, 1),
            "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": round(alg / (avg * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}


def config1_section(torch, mgx, workloads, dev, reps):
    """65^3 fp64 sum of three sinusoids plus noise, full decomposition (L = 5,
    to 3^3), tau = 1e-3 * range: the four separate operations (launch-bound,
    2.2 MB: the field stays in the caches)."""
    u = torch.as_tensor(workloads.sinusoid_field(65), dtype=torch.float64, device=dev)
    tol = 1e-3 * float((u.max() - u.min()).item())
    ws = torch.empty(mgx.workspace_size(mgx.MGX_F64, u.shape, 0), dtype=torch.uint8, device=dev)
    umc, uq, ut = torch.empty_like(u), torch.empty_like(u), torch.empty_like(u)
    lab = torch.empty(u.shape, dtype=torch.int32, device=dev)
    ops = {"decompose": lambda: mgx.decompose(u, out=umc, workspace=ws),
           "quantize": lambda: mgx.quantize(umc, tol, out=lab),
           "dequantize": lambda: mgx.dequantize(lab, tol, torch.float64, out=uq),
           "recompose": lambda: mgx.recompose(uq, out=ut, workspace=ws)}
    ms = {k: _event_ms(torch, f, reps) for k, f in ops.items()}
    err = float((ut - u).abs().max().item())
    nb = u.numel() * 8
    return {"shape": [65, 65, 65], "dtype": "f64", "tau_over_range": 1e-3,
            "op_ms": {k: round(v, 4) for k, v in ms.items()},
            "op_GBps": {k: round(nb / (v * 1e-3) / 1e9, 2) for k, v in ms.items()},
            "dec_rec_GBps": round(2 * nb / ((ms["decompose"] + ms["recompose"]) * 1e-3) / 1e9, 2),
            "max_err_over_tau": round(err / tol, 5)}


def config2_variants_section(torch, mgx, u, labels, ut, ws, reps):
    """The benchmark field at the other tolerances of its configuration
    (1e-2 and 1e-4 * range, full decomposition) and with the decomposition
    stopped at level 4 (a 33^3 box kept, at 1e-3 * range): the fused step's
    time, rate and error."""
    rng = float((u.max() - u.min()).item())
    out = {}
    N = u.numel()
    for rel, stop in ((1e-2, 0), (1e-4, 0), (1e-3, 4)):
        tol = rel * rng
        w = ws if stop == 0 else torch.empty(mgx.workspace_size(mgx.MGX_F32, u.shape, stop), dtype=torch.uint8,
                                             device=u.device)

        def step():
            mgx.decompose_quantize(u, tol, None, stop, labels=labels, workspace=w, keep_coef=False)
            mgx.dequantize_recompose(labels, tol, torch.float32, None, stop, out=ut, workspace=w)

        ms = _event_ms(torch, step, reps)
        err = float((ut.double() - u.double()).abs().max().item())
        out[f"tau{rel:g}_stop{stop}"] = {"ms_per_step": round(ms, 4), "GBps": round(2 * N * 4 / (ms * 1e-3) / 1e9, 2),
                                         "max_err_over_tau": round(err / tol, 5)}
    return out


def config3_section(torch, mgx, workloads, dev, reps):
    """257 x 1025 x 1025 fp32, tanh-stretched vertical axis (spacing ratio 20),
    layered log-normal field: decompose and recompose (L = 7, to 3 x 9 x 9),
    and the fused step at tau = 1e-3 * range, with the roofline figure of the
    dominant kernel of decompose + recompose."""
    u, coords = workloads.layered_lognormal_field(device=dev)
    shape = tuple(u.shape)
    L = mgx.num_levels(shape)
    tol = 1e-3 * float((u.max() - u.min()).item())
    ws = torch.empty(mgx.workspace_size(mgx.MGX_F32, shape, 0), dtype=torch.uint8, device=dev)
    umc, ut = torch.empty_like(u), torch.empty_like(u)
    lab = torch.empty(shape, dtype=torch.int32, device=dev)
    dec = lambda: mgx.decompose(u, coords, out=umc, workspace=ws)  # noqa: E731
    rec = lambda: mgx.recompose(umc, coords, out=ut, workspace=ws)  # noqa: E731
    t_dec = _event_ms(torch, dec, reps)
    t_rec = _event_ms(torch, rec, reps)

    def step():
        mgx.decompose_quantize(u, tol, coords, labels=lab, workspace=ws, keep_coef=False)
        mgx.dequantize_recompose(lab, tol, torch.float32, coords, out=ut, workspace=ws)

    t_step = _event_ms(torch, step, reps)
    err = float((ut.double() - u.double()).abs().max().item())
    roof = _dominant(mgx, torch, lambda: (dec(), rec()), max(2, reps // 2), shape, L, 4)
    N = u.numel()
    out = {"shape": list(shape), "levels": L, "decompose_ms": round(t_dec, 4), "recompose_ms": round(t_rec, 4),
           "dec_rec_GBps": round(2 * N * 4 / ((t_dec + t_rec) * 1e-3) / 1e9, 2),
           "fused_step_ms": round(t_step, 4), "fused_step_GBps": round(2 * N * 4 / (t_step * 1e-3) / 1e9, 2),
           "max_err_over_tau": round(err / tol, 5), "roofline": roof}
    del u, umc, ut, lab, ws
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=513)
    ap.add_argument("--rel-tol", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extensions", action="store_true", help="skip the batched and adjoint comparisons")
    ap.add_argument("--four-d-only", action="store_true",
                    help="run only the 4-D workload section (its own JSON line), e.g. under a profiler")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain device copy of the field (counter calibration)")
    ap.add_argument("--only", choices=["entropy", "adaptive", "batched", "adjoint", "config1", "config3"],
                    help="run only this section (its own JSON line), e.g. under a profiler")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; runs on several GPUs are not "
                                   "supported (fields shard across GPUs without exchange)"}))
        sys.exit(2)

    import torch

    import paper_2010_05872_amd as mgx
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.four_d_only:
        print(json.dumps({"four_d": four_d_section(torch, mgx, workloads, dev, args.steps)}), flush=True)
        return
    reps_x = max(3, args.steps // 4)
    if args.only in ("batched", "adjoint", "config1", "config3"):
        fn = {"batched": batched_section, "adjoint": adjoint_section, "config1": config1_section,
              "config3": config3_section}[args.only]
        print(json.dumps({args.only: fn(torch, mgx, workloads, dev, reps_x)}), flush=True)
        return
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
        mgx.decompose_quantize(u, tol, labels=labels, workspace=ws, keep_coef=False)
        mgx.dequantize_recompose(labels, tol, torch.float32, out=ut, workspace=ws)

    if args.only == "entropy":
        mgx.decompose_quantize(u, tol, labels=labels, workspace=ws, keep_coef=False)
        print(json.dumps({"entropy": entropy_section(torch, mgx, u, labels, tol, reps_x)}), flush=True)
        return
    if args.only == "adaptive":
        print(json.dumps({"adaptive": adaptive_section(torch, mgx, u, umc, ws, reps_x)}), flush=True)
        return

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
        "decompose_quantize": lambda: mgx.decompose_quantize(u, tol, labels=labels, workspace=ws, keep_coef=False),
        "dequantize_recompose": lambda: mgx.dequantize_recompose(labels, tol, torch.float32, out=ut, workspace=ws),
        "decompose_quantize_keep_coef": lambda: mgx.decompose_quantize(u, tol, out=umc, labels=labels,
                                                                       workspace=ws),
        # with statistics: out-of-range counts, per-level max |label| and the status (waits for the stream)
        "decompose_quantize_stats": lambda: mgx.decompose_quantize(u, tol, labels=labels, workspace=ws,
                                                                   keep_coef=False, stats=True),
        "dequantize_recompose_keep_coef": lambda: mgx.dequantize_recompose(labels, tol, torch.float32, coef=uq,
                                                                           out=ut, workspace=ws),
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
            "step": "decompose+quantize+dequantize+recompose (fused entry points, labels only)",
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
        "unfused_step_ms": round(sum(op_ms[k] for k in ("decompose", "quantize", "dequantize", "recompose")), 4),
        "step_algorithmic_GB": round(total_alg / args.steps / 1e9, 4),
        "step_kernel_sum_ms": round(kernel_sum_ms, 4),
        "step_roofline_frac": round(total_alg / args.steps / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "traced_ms_per_step": round(traced_ms_per_step, 4),
        "kernels": sorted(({"name": k["name"], "level": k["level"], "avg_ms": round(k["total_ms"] / k["count"], 5)}
                           for k in ktimes), key=lambda k: -k["avg_ms"])[:12],
        "max_err_over_tau": round(err / tol, 5),
    }
    if not args.no_extensions:
        reps = max(3, args.steps // 4)
        out["config1"] = config1_section(torch, mgx, workloads, dev, max(5, args.steps))
        out["config2_variants"] = config2_variants_section(torch, mgx, u, labels, ut, ws, reps)
        out["config3"] = config3_section(torch, mgx, workloads, dev, reps)
        mgx.decompose(u, out=umc, workspace=ws)
        out["progressive"] = progressive_section(torch, mgx, u, umc, ws, max(3, args.steps // 4))
        out["adaptive"] = adaptive_section(torch, mgx, u, umc, ws, max(3, args.steps // 4))
        mgx.decompose_quantize(u, tol, labels=labels, workspace=ws, keep_coef=False)
        out["entropy"] = entropy_section(torch, mgx, u, labels, tol, 3)
        out["batched"] = batched_section(torch, mgx, workloads, dev, max(3, args.steps // 4))
        out["adjoint"] = adjoint_section(torch, mgx, workloads, dev, max(3, args.steps // 4))
        out["four_d"] = four_d_section(torch, mgx, workloads, dev, max(3, args.steps // 4))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(u, args.rel_tol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
