"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars: max |gpu - oracle| <= 1e-12 max|u| (float64) and 1e-5 max|u| (float32,
oracle run on the promoted float32 input); labels bit-exact from identical
coefficients; dequantized values bit-exact; L-infinity bound end to end.
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


def tol_for(dtype):
    return 1e-12 if dtype == torch.float64 else 1e-5


def make_coords(shape, kind, seed=0):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    if kind == "mixed":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 2) + \
               [workloads.random_coordinates(shape[-1], seed)]
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


def make_field(shape, seed):
    rng = np.random.default_rng(seed)
    base = rng.standard_normal(shape)
    # smooth part + noise so that coefficients span several magnitudes
    grids = np.meshgrid(*[np.linspace(0, 1, n) for n in shape], indexing="ij")
    smooth = sum(np.sin(3.1 * (k + 1) * g + 0.3 * k) for k, g in enumerate(grids))
    return 2.0 * smooth + 0.1 * base


CASES = [
    ((65, 65, 65), torch.float64, None),
    ((33, 257, 65), torch.float32, None),
    ((33, 257, 65), torch.float64, None),
    ((17, 129, 65), torch.float64, "mixed"),
    ((17, 129, 65), torch.float32, "mixed"),
    ((65, 9, 33), torch.float32, "random"),
    ((9, 5, 17), torch.float64, "random"),
    ((5, 5, 5), torch.float64, None),
    ((3, 3, 3), torch.float64, None),
    ((129, 257), torch.float64, None),
    ((257, 129), torch.float32, "random"),
    ((1025,), torch.float64, None),
    ((8193,), torch.float64, "random"),
    ((33, 4097), torch.float32, None),
    ((513, 9, 17), torch.float32, None),       # 257-long strided lines (two-ended solve)
    ((17, 513, 33), torch.float32, "random"),
    ((513, 9, 9), torch.float64, None),        # fp64 257-long strided lines (chunked sweeps)
    ((9, 1025, 17), torch.float64, "tanh"),    # 513-long strided lines (chunked sweeps)
    # shaped like the thin-vertical weather grid (257 x 1025 x 1025, tanh-stretched axis 0) with the
    # contiguous axis cut to 33: fp32 1025-long strided lines on axis 1, the tanh axis 257 long
    ((257, 1025, 33), torch.float32, "tanh"),
    # strided lines of 513 (fp32) and 257 (fp64) nodes, the segmented solve's longest, as the last
    # solve; 1025 (fp32) and 513 (fp64) nodes take the chunked sweeps
    # 3-D fp32 boxes with wide coarse planes (contiguous-axis lines of 65 and 129 coarse nodes)
    ((33, 129, 257), torch.float32, "mixed"),
    ((17, 513, 129), torch.float32, "random"),
    ((1025, 65), torch.float32, "random"),
    ((513, 33), torch.float64, None),
    ((2049, 17), torch.float32, "random"),
    ((1025, 33), torch.float64, None),
]


def _id(c):
    shape, dt, kind = c
    return f"{'x'.join(map(str, shape))}-{str(dt).split('.')[-1]}-{kind}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_decompose_recompose_parity(case):
    shape, dtype, kind = case
    _say(f"[parity] {_id(case)}")
    coords = make_coords(shape, kind, seed=3)
    u = make_field(shape, seed=sum(shape))
    ud = torch.as_tensor(u, dtype=dtype, device="cuda")
    u64 = ud.double().cpu().numpy()
    scale = np.abs(u64).max()
    L = oracle.num_levels(shape)
    # every stop level for the weather-grid-shaped case, four for the others
    stops = list(range(L + 1)) if shape == (257, 1025, 33) else sorted({0, L // 2, max(L - 1, 0), L})
    for stop in stops:
        g = mgx.decompose(ud, coords, stop)
        torch.cuda.synchronize()
        ref = oracle.to_level_centric(oracle.decompose(u64, coords, stop), stop)
        err = np.abs(g.double().cpu().numpy() - ref).max()
        assert err <= tol_for(dtype) * scale, (stop, err / scale)
        # recomposition parity from the same coefficients
        r = mgx.recompose(g, coords, stop)
        torch.cuda.synchronize()
        g64 = oracle.from_level_centric(g.double().cpu().numpy(), stop)
        rref = oracle.recompose(g64, coords, stop)
        rerr = np.abs(r.double().cpu().numpy() - rref).max()
        assert rerr <= tol_for(dtype) * scale, (stop, rerr / scale)
        # round trip
        assert np.abs(r.double().cpu().numpy() - u64).max() <= tol_for(dtype) * scale


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_quantize_bit_exact(dtype):
    shape = (33, 65, 129)
    _say(f"[quant] {shape} {dtype}")
    coords = make_coords(shape, "mixed", 5)
    u = make_field(shape, seed=7) * 10
    ud = torch.as_tensor(u, dtype=dtype, device="cuda")
    for stop in (0, 2):
        umc = mgx.decompose(ud, coords, stop)
        C = oracle.linf_constant(shape, coords, stop)
        tol = 1e-3 * float(u.max() - u.min())
        labels, stats, code = mgx.quantize(umc, tol, coords, stop, c_linf=C, stats=True)
        assert code == 0
        umc64 = oracle.from_level_centric(umc.double().cpu().numpy(), stop)
        ref, rcode = oracle.quantize(umc64, tol, coords, stop, c_linf=C)
        assert rcode == 0
        ref_lc = oracle.to_level_centric(ref, stop)
        got = labels.cpu().numpy()
        assert np.array_equal(got, ref_lc)
        # statistics: per-level max |label|
        lev = oracle.to_level_centric(oracle.level_map(shape, stop), stop)
        want = [int(np.abs(ref_lc[lev == l]).max()) for l in range(stop, oracle.num_levels(shape) + 1)]
        assert stats["max_abs_label"] == want
        assert stats["n_overflow"] == 0 and stats["n_nonfinite"] == 0
        # dequantization bit-exact
        dq = mgx.dequantize(labels, tol, dtype, coords, stop, c_linf=C)
        dref = oracle.dequantize(ref, tol, coords, stop, c_linf=C)
        dref_lc = oracle.to_level_centric(dref, stop).astype(np.float32 if dtype == torch.float32 else np.float64)
        assert np.array_equal(dq.cpu().numpy(), dref_lc)
        # the default constant of the library equals the oracle's to rounding
        assert mgx.linf_constant(shape, coords, stop) == pytest.approx(C, rel=1e-13)


@pytest.mark.parametrize("dtype,rel", [(torch.float64, 1e-2), (torch.float64, 1e-3), (torch.float64, 1e-4),
                                       (torch.float32, 1e-3)])
def test_linf_bound_end_to_end(dtype, rel):
    shape = (65, 65, 65)
    _say(f"[linf] {dtype} {rel}")
    u = workloads.sinusoid_field(65)
    ud = torch.as_tensor(u, dtype=dtype, device="cuda")
    tol = rel * float(u.max() - u.min())
    for stop in (0, 3):
        umc = mgx.decompose(ud, None, stop)
        labels = mgx.quantize(umc, tol, None, stop)
        ut = mgx.recompose(mgx.dequantize(labels, tol, dtype, None, stop), None, stop)
        err = (ut.double() - ud.double()).abs().max().item()
        assert err <= tol, (stop, err / tol)


def test_quantize_range_errors():
    shape = (17, 17, 17)
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    x[3, 4, 5] = float("nan")
    x[1, 1, 1] = 1e30
    labels, stats, code = mgx.quantize(x, 1e-3, stats=True)
    assert code == 6
    assert stats["n_nonfinite"] == 1 and stats["n_overflow"] == 1
    lab = labels.cpu().numpy()
    assert lab[3, 4, 5] == np.iinfo(np.int32).min and lab[1, 1, 1] == np.iinfo(np.int32).min
    assert (lab[lab != np.iinfo(np.int32).min] == 0).all()


def test_determinism():
    shape = (65, 129, 129)
    u = torch.as_tensor(make_field(shape, 1), dtype=torch.float32, device="cuda")
    a = mgx.decompose(u)
    b = mgx.decompose(u)
    assert torch.equal(a, b)
    ra, rb = mgx.recompose(a), mgx.recompose(a)
    assert torch.equal(ra, rb)
    # the same after the library's caches (plans, device tables) are dropped
    torch.cuda.synchronize()
    mgx.release_cached()
    assert torch.equal(mgx.decompose(u), a)
    assert torch.equal(mgx.recompose(a), ra)


def test_error_status_on_device_calls():
    u = torch.zeros((33, 33, 33), dtype=torch.float32, device="cuda")
    with pytest.raises(mgx.MgxError) as e:
        mgx.decompose(u, stop_level=9)
    assert e.value.code == 4
    with pytest.raises(mgx.MgxError) as e:
        mgx.decompose(u, workspace=torch.empty(16, dtype=torch.uint8, device="cuda"))
    assert e.value.code == 7
    with pytest.raises(mgx.MgxError) as e:
        mgx.decompose(u, out=u)
    assert e.value.code == 1
    with pytest.raises(mgx.MgxError) as e:
        mgx.quantize(u, -1.0)
    assert e.value.code == 5
