"""4-D fields on the GPU (the four-axis QMCPACK field of Sec. 6, Table 2):
decomposition and recomposition against the FP64 oracle, quantization labels
bit-exact from the same coefficients, the L-infinity bound end to end, the
fused calls equal to the separate ones, and the padded non-dyadic path.

Bars: max |gpu - oracle| <= 1e-12 max|u| (float64) and 1e-5 max|u| (float32,
oracle run on the promoted float32 input), as for 1-D to 3-D fields."""
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
    if kind == "mixed":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 2) + \
               [workloads.random_coordinates(shape[-1], seed)]
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


def make_field(shape, seed):
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.linspace(0, 1, n) for n in shape], indexing="ij")
    smooth = sum(np.sin(2.3 * (k + 1) * g + 0.4 * k) for k, g in enumerate(grids))
    return 2.0 * smooth + 0.1 * rng.standard_normal(shape)


CASES = [
    ((9, 17, 9, 33), torch.float64, "random"),
    ((17, 9, 33, 9), torch.float32, None),
    ((33, 17, 9, 17), torch.float32, "mixed"),
    ((5, 5, 5, 5), torch.float64, None),
    ((3, 3, 3, 3), torch.float64, None),        # L = 0
    ((9, 9, 5, 257), torch.float32, "random"),  # 129-long contiguous solves
    ((513, 5, 5, 5), torch.float32, None),      # 257-long axis-0 lines (two-ended solve)
    ((513, 5, 5, 5), torch.float64, "random"),  # the same in fp64 (chunked sweeps)
    ((8193, 5, 5, 5), torch.float32, None),     # longest axis 0: 256 march chunks, 4097-long chunked solves
    ((5, 5, 5, 8193), torch.float64, "random"),  # longest contiguous axis: 4097-long wave-scan solves
]


def _id(c):
    shape, dt, kind = c
    return f"{'x'.join(map(str, shape))}-{str(dt).split('.')[-1]}-{kind}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_decompose_recompose_parity_4d(case):
    shape, dtype, kind = case
    _say(f"[4d parity] {_id(case)}")
    coords = make_coords(shape, kind, seed=5)
    u = make_field(shape, seed=sum(shape))
    ud = torch.as_tensor(u, dtype=dtype, device="cuda")
    u64 = ud.double().cpu().numpy()
    scale = np.abs(u64).max()
    L = oracle.num_levels(shape)
    assert mgx.num_levels(shape) == L
    for stop in sorted({0, L // 2, max(L - 1, 0), L}):
        g = mgx.decompose(ud, coords, stop)
        torch.cuda.synchronize()
        ref = oracle.to_level_centric(oracle.decompose(u64, coords, stop), stop)
        err = np.abs(g.double().cpu().numpy() - ref).max()
        assert err <= tol_for(dtype) * scale, (stop, err / scale)
        r = mgx.recompose(g, coords, stop)
        torch.cuda.synchronize()
        g64 = oracle.from_level_centric(g.double().cpu().numpy(), stop)
        rerr = np.abs(r.double().cpu().numpy() - oracle.recompose(g64, coords, stop)).max()
        assert rerr <= tol_for(dtype) * scale, (stop, rerr / scale)
        assert np.abs(r.double().cpu().numpy() - u64).max() <= tol_for(dtype) * scale


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_quantize_bit_exact_4d(dtype):
    shape = (17, 9, 33, 17)
    _say(f"[4d quant] {shape} {dtype}")
    coords = make_coords(shape, "random", 9)
    u = make_field(shape, seed=3) * 10
    ud = torch.as_tensor(u, dtype=dtype, device="cuda")
    L = oracle.num_levels(shape)
    for stop in (0, 1):
        umc = mgx.decompose(ud, coords, stop)
        C = oracle.linf_constant(shape, coords, stop)
        assert mgx.linf_constant(shape, coords, stop) == pytest.approx(C, rel=1e-13)
        tol = 1e-3 * float(u.max() - u.min())
        labels, stats, code = mgx.quantize(umc, tol, coords, stop, c_linf=C, stats=True)
        assert code == 0
        umc64 = oracle.from_level_centric(umc.double().cpu().numpy(), stop)
        ref, rcode = oracle.quantize(umc64, tol, coords, stop, c_linf=C)
        assert rcode == 0
        ref_lc = oracle.to_level_centric(ref, stop)
        assert np.array_equal(labels.cpu().numpy(), ref_lc)
        lev = oracle.to_level_centric(oracle.level_map(shape, stop), stop)
        want = [int(np.abs(ref_lc[lev == l]).max()) for l in range(stop, L + 1)]
        assert stats["max_abs_label"] == want
        assert stats["n_overflow"] == 0 and stats["n_nonfinite"] == 0
        dq = mgx.dequantize(labels, tol, dtype, coords, stop, c_linf=C)
        dref = oracle.to_level_centric(oracle.dequantize(ref, tol, coords, stop, c_linf=C), stop)
        assert np.array_equal(dq.cpu().numpy(), dref.astype(np.float32 if dtype == torch.float32 else np.float64))


def test_quantize_range_errors_4d():
    shape = (5, 5, 5, 5)
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    x[4, 4, 4, 4] = float("nan")
    x[3, 4, 4, 4] = 1e30
    labels, stats, code = mgx.quantize(x, 1e-3, stats=True)
    assert code == 6
    assert stats["n_nonfinite"] == 1 and stats["n_overflow"] == 1


@pytest.mark.parametrize("dtype,rel", [(torch.float64, 1e-2), (torch.float32, 1e-3), (torch.float32, 1e-5)])
def test_linf_bound_and_fused_4d(dtype, rel):
    shape = (33, 17, 17, 33)
    _say(f"[4d linf] {dtype} {rel}")
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.5, seed=12), dtype=dtype, device="cuda")
    tol = rel * float((u.max() - u.min()).item())
    L = mgx.num_levels(shape)
    for stop in (0, L - 1):
        umc = mgx.decompose(u, None, stop)
        labels = mgx.quantize(umc, tol, None, stop)
        coef = mgx.dequantize(labels, tol, dtype, None, stop)
        ut = mgx.recompose(coef, None, stop)
        err = (ut.double() - u.double()).abs().max().item()
        assert err <= tol, (stop, err / tol)
        # the fused calls give the separate calls' results, with and without u_mc
        umc2, lab2 = mgx.decompose_quantize(u, tol, None, stop)
        none, lab3 = mgx.decompose_quantize(u, tol, None, stop, keep_coef=False)
        out2 = mgx.dequantize_recompose(lab2, tol, dtype, None, stop)
        coef3 = torch.empty_like(u)
        out3 = mgx.dequantize_recompose(lab3, tol, dtype, None, stop, coef=coef3)
        torch.cuda.synchronize()
        assert none is None
        assert torch.equal(umc2, umc) and torch.equal(lab2, labels) and torch.equal(lab3, labels)
        assert torch.equal(out2, ut) and torch.equal(out3, ut) and torch.equal(coef3, coef)


def test_padded_4d_path():
    """A non-dyadic 4-D field shaped like a slice of Table 2's QMCPACK field:
    padding equal to the oracle's, and the whole path within the bound on the
    real nodes."""
    shape = (36, 15, 9, 9)
    _say(f"[4d padding] {shape}")
    u = workloads.orbital_field(shape, device="cuda")
    p = mgx.pad(u)
    torch.cuda.synchronize()
    assert tuple(p.shape) == oracle.dyadic_shape(shape) == (65, 17, 9, 9)
    assert np.array_equal(p.double().cpu().numpy(), oracle.pad_to_dyadic(u.double().cpu().numpy()))
    assert torch.equal(mgx.crop(p, shape), u)
    tol = 1e-3 * float((u.max() - u.min()).item())
    _, labels = mgx.decompose_quantize(p, tol, keep_coef=False)
    back = mgx.crop(mgx.dequantize_recompose(labels, tol, torch.float32), shape)
    torch.cuda.synchronize()
    assert (back.double() - u.double()).abs().max().item() <= tol


@pytest.mark.parametrize("shape,dt", [((6, 5, 2, 3), torch.float32), ((7, 3, 5, 2), torch.float64),
                                      ((10, 3, 4, 13), torch.float32), ((3, 2, 2, 2), torch.float64)],
                         ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v)[6:])
def test_pad4_bit_exact(shape, dt):
    """4-D padding equal to the oracle's for boxes whose padded rows are shorter
    than the four nodes a pad thread writes (quads crossing several row ends),
    and element counts that are not a multiple of four."""
    _say(f"[4d pad] {shape} {dt}")
    u = torch.as_tensor(make_field(shape, seed=len(shape) + shape[0]), dtype=dt, device="cuda")
    p = mgx.pad(u)
    torch.cuda.synchronize()
    assert tuple(p.shape) == oracle.dyadic_shape(shape)
    assert np.array_equal(p.double().cpu().numpy(), oracle.pad_to_dyadic(u.double().cpu().numpy()))
    assert torch.equal(mgx.crop(p, shape), u)


def test_back_to_back_smaller_4d():
    """Two calls sharing one workspace, the second on a smaller field."""
    ws = torch.full((mgx.workspace_size(mgx.MGX_F32, (17, 17, 33, 17), 0) // 4 + 64,), float("nan"),
                    dtype=torch.float32, device="cuda").view(torch.uint8)
    for shape in ((17, 17, 33, 17), (9, 5, 17, 9)):
        _say(f"[4d back-to-back] {shape}")
        u = torch.as_tensor(make_field(shape, seed=8), dtype=torch.float32, device="cuda")
        g = mgx.decompose(u, None, 0, workspace=ws)
        r = mgx.recompose(g, None, 0, workspace=ws)
        torch.cuda.synchronize()
        ref = oracle.to_level_centric(oracle.decompose(u.double().cpu().numpy(), None, 0), 0)
        scale = float(u.abs().max())
        assert np.abs(g.double().cpu().numpy() - ref).max() <= 1e-5 * scale
        assert (r.double() - u.double()).abs().max().item() <= 1e-5 * scale


@pytest.mark.parametrize("stop", [0, 1])
def test_progressive_and_entropy_4d(stop):
    """Progressive recomposition of a 4-D field to every level t (Q_t u on the
    level-t grid) and the per-level label entropy, against the oracle."""
    shape = (17, 9, 33, 17)
    _say(f"[4d progressive+entropy] {shape} stop {stop}")
    coords = make_coords(shape, "random", 3)
    u = make_field(shape, seed=4)
    ud = torch.as_tensor(u, dtype=torch.float64, device="cuda")
    scale = np.abs(u).max()
    L = mgx.num_levels(shape)
    g = mgx.decompose(ud, coords, stop)
    g64 = oracle.from_level_centric(g.cpu().numpy(), stop)
    for t in range(stop, L + 1):
        got = mgx.recompose_to(g, t, coords, stop)
        torch.cuda.synchronize()
        want = oracle.recompose_to(g64, t, coords, stop)
        assert got.shape == want.shape
        assert np.abs(got.cpu().numpy() - want).max() <= 1e-12 * scale, t
    tol = 1e-3 * float(u.max() - u.min())
    lab = mgx.quantize(g, tol, coords, stop)
    H = mgx.label_entropy(lab, stop)
    Href = oracle.label_entropy(oracle.from_level_centric(lab.cpu().numpy(), stop), stop)
    assert np.allclose(H, Href, rtol=1e-12, atol=1e-12), (H, Href)
    # labels too wide for the histogram: the sort path
    rng = np.random.default_rng(stop)
    wide = (rng.integers(-2 ** 30, 2 ** 30, size=shape) * rng.random(shape) ** 3).astype(np.int32)
    H = mgx.label_entropy(torch.as_tensor(wide, device="cuda"), stop)
    Href = oracle.label_entropy(oracle.from_level_centric(wide, stop), stop)
    assert np.allclose(H, Href, rtol=1e-12, atol=1e-12), (H, Href)
