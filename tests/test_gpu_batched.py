"""Batched fields: many uneven fields in one captured graph of multi-field
launches (mgx_decompose_batched / mgx_recompose_batched).

The batched results must equal the single-field calls bit for bit (the same
kernel bodies; tiling does not change any summation order), and every field
meets the oracle to the parity bars in every direction: decomposition,
labels, recomposition from coefficients and from labels.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


SPECS = [
    ((33, 65, 33), torch.float32, None, 0),
    ((65, 33, 129), torch.float32, "random", 0),
    ((129, 129, 65), torch.float32, None, 1),
    ((33, 33, 33), torch.float64, "tanh", 0),
    ((17, 257), torch.float32, None, 0),
    ((1025,), torch.float64, "random", 2),
    ((65, 65, 65), torch.float64, None, 5),   # stop = L: copy only
    ((257, 33, 65), torch.float32, "tanh", 0),
    ((65, 65, 65), torch.float32, "random", 4),  # stop box outside the single-workgroup tail
    ((1025, 17), torch.float32, None, 0),     # 513-long strided lines: the segmented solve
    ((33, 65, 129), torch.float32, "random", 0),  # contiguous-axis lines of 65 coarse nodes
]


def _coords(shape, kind, seed):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


def _fields():
    out = []
    for i, (shape, dt, kind, stop) in enumerate(SPECS):
        u = workloads.gaussian_random_field(shape, slope=2.0 + (i % 3), seed=900 + i)
        out.append(dict(u=torch.as_tensor(u, dtype=dt, device="cuda"), coords=_coords(shape, kind, 10 * i),
                        stop=stop, tol=10 ** (-2 - (i % 3)) * float(u.max() - u.min())))
    return out


@pytest.mark.parametrize("autotune", [True, False])
def test_batched_equals_single(autotune):
    _say(f"[batched] autotune={autotune}")
    mgx.batch_set_autotune(autotune)
    try:
        F = _fields()
        outs = [torch.empty_like(f["u"]) for f in F]
        labels = [torch.empty(f["u"].shape, dtype=torch.int32, device="cuda") for f in F]
        b = mgx.Batch([dict(**{"in": f["u"]}, out=o, coords=f["coords"], stop_level=f["stop"], tol=f["tol"],
                            labels=lab) for f, o, lab in zip(F, outs, labels)])
        b.decompose()
        torch.cuda.synchronize()
        info = mgx.batch_last_info()
        _say("info", info)
        assert info["launches"] > 0
        for f, o, lab in zip(F, outs, labels):
            ref = mgx.decompose(f["u"], f["coords"], f["stop"])
            assert torch.equal(o, ref)
            rl = mgx.quantize(ref, f["tol"], f["coords"], f["stop"])
            assert torch.equal(lab, rl)
        # replay with new input values in the same buffers
        for f in F:
            f["u"].mul_(-0.5).add_(0.25)
        b.decompose()
        torch.cuda.synchronize()
        for f, o, lab in zip(F, outs, labels):
            ref = mgx.decompose(f["u"], f["coords"], f["stop"])
            assert torch.equal(o, ref)
            assert torch.equal(lab, mgx.quantize(ref, f["tol"], f["coords"], f["stop"]))
        # recomposition from the coefficients
        recs = [torch.empty_like(f["u"]) for f in F]
        r = mgx.Batch([dict(**{"in": o}, out=rr, coords=f["coords"], stop_level=f["stop"])
                       for f, o, rr in zip(F, outs, recs)])
        r.recompose()
        torch.cuda.synchronize()
        for f, o, rr in zip(F, outs, recs):
            assert torch.equal(rr, mgx.recompose(o, f["coords"], f["stop"]))
        # recomposition from labels (dequantize into coef, then recompose)
        coefs = [torch.empty_like(f["u"]) for f in F]
        recs2 = [torch.empty_like(f["u"]) for f in F]
        # labels still hold the first input's quantization
        r2 = mgx.Batch([dict(out=rr, coords=f["coords"], stop_level=f["stop"], tol=f["tol"], labels=lab, coef=c)
                        for f, lab, c, rr in zip(F, labels, coefs, recs2)])
        r2.recompose()
        torch.cuda.synchronize()
        for f, lab, c, rr in zip(F, labels, coefs, recs2):
            dq = mgx.dequantize(lab, f["tol"], f["u"].dtype, f["coords"], f["stop"])
            assert torch.equal(c, dq)
            assert torch.equal(rr, mgx.recompose(dq, f["coords"], f["stop"]))
        # recomposition straight from the labels (no coef): the level kernels dequantize
        recs3 = [torch.full_like(f["u"], float("nan")) for f in F]
        r3 = mgx.Batch([dict(out=rr, coords=f["coords"], stop_level=f["stop"], tol=f["tol"], labels=lab)
                        for f, lab, rr in zip(F, labels, recs3)])
        r3.recompose()
        torch.cuda.synchronize()
        for f, lab, rr, want in zip(F, labels, recs3, recs2):
            assert torch.equal(rr, want)
            assert torch.equal(rr, mgx.dequantize_recompose(lab, f["tol"], f["u"].dtype, f["coords"], f["stop"]))
    finally:
        mgx.batch_set_autotune(True)


def _bar(dtype):
    return 1e-12 if dtype == torch.float64 else 1e-5


def test_batched_parity_with_oracle():
    """Every field of the batch, in every direction, against the oracle:
    decomposition (coefficients), labels from the same coefficients
    (bit-exact), recomposition from the coefficients, and recomposition from
    the labels, with the dequantized coefficients written to coef and
    straight from the labels in the level kernels (both against the oracle's
    recomposition of its own dequantization of the same labels)."""
    _say("[batched] oracle, all fields and directions")
    F = _fields()
    # the oracle's constant on both sides: labels and dequantized values then compare bit for bit
    for f in F:
        f["C"] = oracle.linf_constant(tuple(f["u"].shape), f["coords"], f["stop"])
    outs = [torch.empty_like(f["u"]) for f in F]
    labels = [torch.empty(f["u"].shape, dtype=torch.int32, device="cuda") for f in F]
    b = mgx.Batch([dict(**{"in": f["u"]}, out=o, coords=f["coords"], stop_level=f["stop"], tol=f["tol"],
                        c_linf=f["C"], labels=lab) for f, o, lab in zip(F, outs, labels)])
    b.decompose()
    recs = [torch.empty_like(f["u"]) for f in F]
    mgx.Batch([dict(**{"in": o}, out=rr, coords=f["coords"], stop_level=f["stop"])
               for f, o, rr in zip(F, outs, recs)]).recompose()
    coefs = [torch.empty_like(f["u"]) for f in F]
    recs_c = [torch.empty_like(f["u"]) for f in F]
    mgx.Batch([dict(out=rr, coords=f["coords"], stop_level=f["stop"], tol=f["tol"], c_linf=f["C"],
                         labels=lab, coef=c) for f, lab, c, rr in zip(F, labels, coefs, recs_c)]).recompose()
    recs_l = [torch.full_like(f["u"], float("nan")) for f in F]
    mgx.Batch([dict(out=rr, coords=f["coords"], stop_level=f["stop"], tol=f["tol"], c_linf=f["C"],
                         labels=lab) for f, lab, rr in zip(F, labels, recs_l)]).recompose()
    torch.cuda.synchronize()
    for i, f in enumerate(F):
        shape, stop, coords, tol = tuple(f["u"].shape), f["stop"], f["coords"], f["tol"]
        _say(f"  field {i}: {shape} {f['u'].dtype} stop={stop}")
        u64 = f["u"].double().cpu().numpy()
        scale = np.abs(u64).max()
        bar = _bar(f["u"].dtype) * scale
        ref = oracle.to_level_centric(oracle.decompose(u64, coords, stop), stop)
        g64 = outs[i].double().cpu().numpy()
        assert np.abs(g64 - ref).max() <= bar, ("decompose", i)
        g_int = oracle.from_level_centric(g64, stop)
        rref = oracle.recompose(g_int, coords, stop)
        assert np.abs(recs[i].double().cpu().numpy() - rref).max() <= bar, ("recompose", i)
        lref, code = oracle.quantize(g_int, tol, coords, stop, c_linf=f["C"])
        assert code == 0
        assert np.array_equal(labels[i].cpu().numpy(), oracle.to_level_centric(lref, stop)), ("labels", i)
        dq = oracle.dequantize(lref, tol, coords, stop, c_linf=f["C"])
        np_dt = np.float32 if f["u"].dtype == torch.float32 else np.float64
        assert np.array_equal(coefs[i].cpu().numpy(), oracle.to_level_centric(dq, stop).astype(np_dt)), ("coef", i)
        qref = oracle.recompose(dq, coords, stop)
        for name, got in (("labels->coef->recompose", recs_c[i]), ("labels->recompose", recs_l[i])):
            assert np.abs(got.double().cpu().numpy() - qref).max() <= bar, (name, i)
        # and the quantized round trip honours the L-infinity bound
        assert np.abs(recs_l[i].double().cpu().numpy() - u64).max() <= tol, ("bound", i)


def test_batched_errors():
    u = torch.zeros((33, 33, 33), dtype=torch.float32, device="cuda")
    o = torch.empty_like(u)
    b = mgx.Batch([dict(**{"in": u}, out=o)], workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    with pytest.raises(mgx.MgxError) as e:
        b.decompose()
    assert e.value.code == 7
    with pytest.raises(mgx.MgxError) as e:
        mgx.Batch([dict(**{"in": u}, out=u)]).decompose()
    assert e.value.code == 1


def test_tune_cache_persists(tmp_path, monkeypatch):
    """MGX_TUNE_CACHE: a batch timed once appends its shape to the file; the
    same field shapes at other addresses, after the in-process caches are
    dropped, are built from the file without timing and give the same
    results; malformed lines are skipped."""
    _say("[batched] tune cache")
    path = tmp_path / "tune.txt"
    path.write_text("not a line\n0123 1 2\n")
    monkeypatch.setenv("MGX_TUNE_CACHE", str(path))
    specs = [((33, 17, 65), torch.float32), ((65, 33), torch.float64), ((17, 129, 17), torch.float32)]

    def run():
        us = [torch.as_tensor(workloads.gaussian_random_field(s, slope=3.0, seed=70 + i), dtype=dt, device="cuda")
              for i, (s, dt) in enumerate(specs)]
        outs = [torch.empty_like(u) for u in us]
        mgx.Batch([dict(**{"in": u}, out=o) for u, o in zip(us, outs)]).decompose()
        torch.cuda.synchronize()
        for u, o in zip(us, outs):
            assert torch.equal(o, mgx.decompose(u))
        return mgx.batch_last_info()

    mgx.batch_set_autotune(True)
    try:
        mgx.release_cached()
        first = run()
        assert first["tune_source"] == 1
        lines = [ln.split() for ln in path.read_text().splitlines() if len(ln.split()) == 5]
        assert len(lines) == 1
        assert int(lines[0][1]) == first["target_blocks"] and int(lines[0][2]) == first["min_zchunk"]
        mgx.release_cached()
        second = run()
        assert second["tune_source"] == 2
        assert second["target_blocks"] == first["target_blocks"]
        assert second["min_zchunk"] == first["min_zchunk"]
        assert second["tuned_ms"] == pytest.approx(float(lines[0][4]), rel=1e-6)
        assert len([ln for ln in path.read_text().splitlines() if len(ln.split()) == 5]) == 1
    finally:
        monkeypatch.delenv("MGX_TUNE_CACHE")
        mgx.release_cached()
