"""Fused decompose+quantize and dequantize+recompose (labels written and read
by the level kernels themselves): results equal the separate calls bit for
bit, with and without u_mc, on shapes with and without the single-workgroup
tail, 1-D to 3-D, both dtypes, and every kind of stop level."""
import sys

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402

CASES = [
    ((65, 65, 65), torch.float32, None),
    ((33, 129, 65), torch.float64, "random"),
    ((17, 17, 17), torch.float32, None),      # all levels in the tail
    ((257, 129), torch.float32, "random"),
    ((4097,), torch.float64, None),
    ((129, 9, 33), torch.float32, "tanh"),
    ((9, 257, 5), torch.float64, None),      # level boxes never all within the tail
]


def _coords(shape, kind, seed):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}-{c[2]}")
def test_fused_equals_separate(case):
    shape, dt, kind = case
    print(f"[fused] {shape} {dt} {kind}", flush=True)
    sys.stdout.flush()
    coords = _coords(shape, kind, 4)
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=77), dtype=dt, device="cuda")
    tol = 1e-3 * float((u.max() - u.min()).item())
    L = mgx.num_levels(shape)
    for stop in sorted({0, L // 2, max(L - 1, 0), L}):
        umc, lab = mgx.decompose_quantize(u, tol, coords, stop)
        ref = mgx.decompose(u, coords, stop)
        rlab = mgx.quantize(ref, tol, coords, stop)
        torch.cuda.synchronize()
        assert torch.equal(umc, ref), stop
        assert torch.equal(lab, rlab), stop
        coef = torch.empty_like(u)
        out = mgx.dequantize_recompose(lab, tol, dt, coords, stop, coef=coef)
        dq = mgx.dequantize(rlab, tol, dt, coords, stop)
        rr = mgx.recompose(dq, coords, stop)
        torch.cuda.synchronize()
        assert torch.equal(coef, dq), stop
        assert torch.equal(out, rr), stop
        assert (out.double() - u.double()).abs().max().item() <= tol
        # labels only (no u_mc), and recomposition straight from the labels
        none, lab2 = mgx.decompose_quantize(u, tol, coords, stop, keep_coef=False)
        out2 = torch.full_like(u, float("nan"))
        mgx.dequantize_recompose(lab2, tol, dt, coords, stop, out=out2)
        torch.cuda.synchronize()
        assert none is None
        assert torch.equal(lab2, rlab), stop
        assert torch.equal(out2, rr), stop


def test_fused_back_to_back_reuse():
    """Repeated fused calls on one stream (the side stream and its events are
    reused) stay ordered with the caller's own work."""
    shape = (129, 129, 129)
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=2.5, seed=3), dtype=torch.float32,
                        device="cuda")
    tol = 1e-3 * float((u.max() - u.min()).item())
    umc = torch.empty_like(u)
    lab = torch.empty(shape, dtype=torch.int32, device="cuda")
    coef = torch.empty_like(u)
    out = torch.empty_like(u)
    ref = None
    for i in range(4):
        u.mul_(1.0 + 0.01 * i)  # the caller's work on the stream between calls
        mgx.decompose_quantize(u, tol, out=umc, labels=lab)
        mgx.dequantize_recompose(lab, tol, torch.float32, coef=coef, out=out)
        ref = mgx.recompose(mgx.dequantize(mgx.quantize(mgx.decompose(u), tol), tol, torch.float32))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), i


def test_fused_labels_back_to_back_smaller():
    """Coefficient-free calls that share one workspace, the second on a
    smaller field: the stop box held in the workspace is rewritten each call."""
    ws = torch.full((mgx.workspace_size(mgx.MGX_F32, (129, 129, 65), 0) // 4 + 64,), float("nan"),
                    dtype=torch.float32, device="cuda").view(torch.uint8)
    for shape, stop in (((129, 129, 65), 5), ((65, 33, 33), 4)):
        print(f"[fused-labels] {shape} stop {stop}", flush=True)
        u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=11), dtype=torch.float32,
                            device="cuda")
        tol = 1e-4 * float((u.max() - u.min()).item())
        _, lab = mgx.decompose_quantize(u, tol, None, stop, keep_coef=False, workspace=ws)
        out = mgx.dequantize_recompose(lab, tol, torch.float32, None, stop, workspace=ws)
        rlab = mgx.quantize(mgx.decompose(u, None, stop), tol, None, stop)
        rr = mgx.recompose(mgx.dequantize(rlab, tol, torch.float32, None, stop), None, stop)
        torch.cuda.synchronize()
        assert torch.equal(lab, rlab)
        assert torch.equal(out, rr)


def test_fused_labels_near_ties():
    """Finest-level coefficients placed on and around the quantizer's
    half-integer ties (and beyond the FP32 fast path's range): with the
    coarse nodes zero, each finest coefficient is the field value itself, so
    the labels the decomposition kernel writes must equal the FP64 division's
    decision of the separate pass at every such node."""
    shape = (65, 65, 65)
    L = mgx.num_levels(shape)
    stop = L - 1
    rng = np.random.default_rng(2024)
    tol = 1.0
    q = 2.0 * float(mgx.level_tolerances(shape, tol, None, stop)[-1])
    idx = np.indices(shape)
    coef_node = ((idx[0] | idx[1] | idx[2]) & 1).astype(bool)
    n = int(coef_node.sum())
    k = rng.integers(-3000, 3000, n).astype(np.float64)
    big = rng.random(n) < 0.1
    k[big] = rng.integers(60000, 70000, int(big.sum())) * rng.choice([-1.0, 1.0], int(big.sum()))
    huge = rng.random(n) < 0.02
    k[huge] = rng.integers(2 ** 20, 2 ** 28, int(huge.sum())).astype(np.float64)
    v = ((k + 0.5) * q).astype(np.float32)
    steps = rng.integers(-3, 4, n)
    for s in range(3):  # nudge by up to 3 ulps either way
        up, dn = steps > s, steps < -s
        v[up] = np.nextafter(v[up], np.float32(np.inf))
        v[dn] = np.nextafter(v[dn], np.float32(-np.inf))
    off = rng.random(n) < 0.2  # some far from ties
    v[off] = (rng.normal(size=int(off.sum())) * 1000 * q).astype(np.float32)
    host = np.zeros(shape, dtype=np.float32)
    host[coef_node] = v
    u = torch.as_tensor(host, device="cuda")
    _, lab = mgx.decompose_quantize(u, tol, None, stop, keep_coef=False)
    ref = mgx.decompose(u, None, stop)
    rlab = mgx.quantize(ref, tol, None, stop)
    torch.cuda.synchronize()
    assert torch.equal(lab, rlab)
    # the finest coefficients are the values themselves, at level-centric positions
    lc = [np.where(np.arange(m) % 2 == 1, (m + 1) // 2 + np.arange(m) // 2, np.arange(m) // 2) for m in shape]
    pos = lab.cpu().numpy()[np.ix_(*lc)]
    want = np.rint(host.astype(np.float64) / q).astype(np.int32)
    assert np.array_equal(pos[coef_node], want[coef_node])


RANGE_CASES = [
    ((17, 17, 17), torch.float32, 0),    # every level in the single-workgroup tail
    ((65, 65, 65), torch.float32, 0),    # tiled levels, then the tail
    ((65, 65, 65), torch.float32, 4),    # the stop box by the corner-box pass
    ((33, 65), torch.float64, 0),
    ((33, 33, 33), torch.float32, 4),    # stop = L: one flat pass
    ((9, 9, 9, 9), torch.float32, 0),    # four axes
    ((9, 17, 9, 9), torch.float64, 2),
]


def _range_field(shape, dt, bad):
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=12), dtype=dt, device="cuda")
    if bad:
        mid = tuple(n // 2 for n in shape)
        u[mid] = float("nan")
        u[(1,) * len(shape)] = 1e30 if dt == torch.float32 else 1e300
    return u


@pytest.mark.parametrize("case", RANGE_CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}-stop{c[2]}")
@pytest.mark.parametrize("bad", [True, False])
def test_fused_range_reporting(case, bad):
    """The fused call with statistics reports what the separate quantization
    reports: the same labels, the same per-level max |label|, the same
    overflow and non-finite counts, and MGX_ERR_RANGE exactly when they are
    nonzero (a NaN and a huge value in the input spread to many
    coefficients)."""
    shape, dt, stop = case
    print(f"[fused range] {shape} {dt} stop={stop} bad={bad}", flush=True)
    u = _range_field(shape, dt, bad)
    tol = 1e-3
    for keep in (True, False):
        _, lab, st, code = mgx.decompose_quantize(u, tol, None, stop, keep_coef=keep, stats=True)
        umc = mgx.decompose(u, None, stop)
        rlab, rst, rcode = mgx.quantize(umc, tol, None, stop, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(lab, rlab)
        assert st == rst, (st, rst)
        assert code == rcode == (6 if bad else 0)
        if bad:
            assert st["n_nonfinite"] > 0 and st["n_overflow"] > 0
        # without statistics the same labels come back and no status is raised
        _, lab2 = mgx.decompose_quantize(u, tol, None, stop, keep_coef=keep)
        torch.cuda.synchronize()
        assert torch.equal(lab2, rlab)


def test_batched_range_reporting():
    """Batched decomposition with labels: the fields that ask for statistics
    get the single-field call's, and the call returns MGX_ERR_RANGE when one
    of them overflowed; replaying the batch on clean inputs clears it."""
    print("[fused range] batched", flush=True)
    specs = [((17, 17, 17), torch.float32, 0, True), ((65, 33, 65), torch.float32, 0, False),
             ((33, 65), torch.float64, 1, True), ((65, 65, 65), torch.float32, 4, False)]
    us = [_range_field(s, dt, bad) for s, dt, _, bad in specs]
    outs = [torch.empty_like(u) for u in us]
    labs = [torch.empty(u.shape, dtype=torch.int32, device="cuda") for u in us]
    b = mgx.Batch([dict(**{"in": u}, out=o, stop_level=stop, tol=1e-3, labels=lab, stats=(i != 1))
                   for i, (u, o, lab, (_, _, stop, _)) in enumerate(zip(us, outs, labs, specs))])
    b.decompose()
    torch.cuda.synchronize()
    assert b.code == 6
    got = b.stats()
    assert sorted(got) == [0, 2, 3]
    for i in got:
        _, lab, st, code = mgx.decompose_quantize(us[i], 1e-3, None, specs[i][2], stats=True)
        torch.cuda.synchronize()
        assert torch.equal(labs[i], lab)
        assert got[i] == st, (i, got[i], st)
        assert code == (6 if specs[i][3] else 0)
    # the same batch on clean inputs: statistics cleared, status OK
    for u, (s, dt, _, bad) in zip(us, specs):
        if bad:
            u.copy_(_range_field(s, dt, False))
    b.decompose()
    torch.cuda.synchronize()
    assert b.code == 0
    for i, st in b.stats().items():
        assert st["n_overflow"] == 0 and st["n_nonfinite"] == 0
        _, _, ref, _ = mgx.decompose_quantize(us[i], 1e-3, None, specs[i][2], stats=True)
        assert st == ref
