"""GPU adjoints (transposes) of decompose and recompose, through the C ABI.

Parity against the oracle's adjoints (which are pinned on the CPU by the
dot-product identity and dense transposes), the dot-product identity of the
GPU pair itself, and finite differences through the autograd Function
(quantization straight-through).  Bars as for the forward maps: 1e-12 (fp64)
and 1e-5 (fp32) relative to the largest input magnitude.
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


def _coords(shape, kind, seed=0):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


CASES = [
    ((33, 33, 33), torch.float64, None),
    ((17, 65, 33), torch.float64, "random"),
    ((17, 65, 33), torch.float32, "random"),
    ((9, 129, 65), torch.float32, "tanh"),
    ((65, 9, 17), torch.float64, "tanh"),
    ((129, 257), torch.float64, None),
    ((257, 65), torch.float32, "random"),
    ((1025,), torch.float64, "random"),
    ((5, 5, 5), torch.float64, None),
    ((3, 3, 3), torch.float64, None),
    ((513, 9, 17), torch.float32, None),
]


def _id(c):
    shape, dt, kind = c
    return f"{'x'.join(map(str, shape))}-{str(dt).split('.')[-1]}-{kind}"


@pytest.mark.parametrize("case", CASES, ids=_id)
def test_adjoint_parity(case):
    shape, dtype, kind = case
    _say(f"[adjoint] {_id(case)}")
    coords = _coords(shape, kind, 2)
    rng = np.random.default_rng(sum(shape) + 11)
    g = torch.as_tensor(rng.standard_normal(shape), dtype=dtype, device="cuda")
    g64 = g.double().cpu().numpy()
    scale = np.abs(g64).max()
    bar = 1e-12 if dtype == torch.float64 else 1e-5
    L = oracle.num_levels(shape)
    for stop in sorted({0, L // 2, L}):
        # D^T: level-centric input -> natural output
        gu = mgx.decompose_adjoint(g, coords, stop)
        torch.cuda.synchronize()
        ref = oracle.decompose_adjoint(oracle.from_level_centric(g64, stop), coords, stop)
        rs = max(scale, np.abs(ref).max())
        err = np.abs(gu.double().cpu().numpy() - ref).max()
        assert err <= bar * rs, ("D^T", stop, err / rs)
        # R^T: natural input -> level-centric output
        gm = mgx.recompose_adjoint(g, coords, stop)
        torch.cuda.synchronize()
        ref = oracle.to_level_centric(oracle.recompose_adjoint(g64, coords, stop), stop)
        rs = max(scale, np.abs(ref).max())
        err = np.abs(gm.double().cpu().numpy() - ref).max()
        assert err <= bar * rs, ("R^T", stop, err / rs)


@pytest.mark.parametrize("shape", [(65, 65, 65), (33, 129, 17)])
def test_dot_product_identity_on_gpu(shape):
    _say(f"[dot] {shape}")
    gen = torch.Generator(device="cuda").manual_seed(7)
    x = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
    y = torch.randn(shape, dtype=torch.float64, device="cuda", generator=gen)
    for stop in (0, 2):
        lhs = torch.dot(mgx.decompose(x, None, stop).ravel(), y.ravel()).item()
        rhs = torch.dot(x.ravel(), mgx.decompose_adjoint(y, None, stop).ravel()).item()
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + x.norm().item() * y.norm().item() * 1e-3)
        lhs = torch.dot(mgx.recompose(x, None, stop).ravel(), y.ravel()).item()
        rhs = torch.dot(x.ravel(), mgx.recompose_adjoint(y, None, stop).ravel()).item()
        assert abs(lhs - rhs) <= 1e-11 * (abs(lhs) + x.norm().item() * y.norm().item() * 1e-3)
        # R^T is the inverse of D^T
        back = mgx.decompose_adjoint(mgx.recompose_adjoint(y, None, stop), None, stop)
        assert (back - y).abs().max().item() <= 1e-12 * y.abs().max().item()


def test_autograd_finite_differences():
    """loss = MSE(R(D x + delta), target) in fp64 on a 33^3 field with
    k^-3 spectrum; central differences with h = 1e-6 along 16 seeded random
    directions, for x and for delta."""
    _say("[fd] 33^3 fp64")
    n = 33
    x = torch.as_tensor(workloads.gaussian_random_field((n, n, n), slope=3.0, seed=501), dtype=torch.float64,
                        device="cuda")
    tgt = torch.as_tensor(workloads.gaussian_random_field((n, n, n), slope=3.0, seed=502), dtype=torch.float64,
                          device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(503)
    delta = 1e-3 * torch.randn((n, n, n), dtype=torch.float64, device="cuda", generator=gen)
    coords = [workloads.tanh_coordinates(n), None, None]

    def loss_of(xx, dd):
        y = mgx.MGXRoundTrip.apply(xx, dd, coords, 1, None)
        return ((y - tgt) ** 2).mean()

    xr = x.clone().requires_grad_(True)
    dr = delta.clone().requires_grad_(True)
    loss = loss_of(xr, dr)
    loss.backward()
    h = 1e-6
    for i in range(16):
        v = torch.randn((n, n, n), dtype=torch.float64, device="cuda", generator=gen)
        with torch.no_grad():
            fd_x = (loss_of(x + h * v, delta) - loss_of(x - h * v, delta)).item() / (2 * h)
            fd_d = (loss_of(x, delta + h * v) - loss_of(x, delta - h * v)).item() / (2 * h)
        an_x = torch.dot(xr.grad.ravel(), v.ravel()).item()
        an_d = torch.dot(dr.grad.ravel(), v.ravel()).item()
        assert abs(fd_x - an_x) <= 1e-6 * max(abs(an_x), 1e-3 * xr.grad.norm().item()), (i, fd_x, an_x)
        assert abs(fd_d - an_d) <= 1e-6 * max(abs(an_d), 1e-3 * dr.grad.norm().item()), (i, fd_d, an_d)


def test_straight_through_quantization_and_fp32_backward():
    """fp32 round trip with the quantizer: the gradient w.r.t. x is D^T R^T g
    (straight-through), compared with the oracle's adjoints."""
    _say("[ste] 65^3 fp32")
    n = 65
    x = torch.as_tensor(workloads.gaussian_random_field((n, n, n), slope=3.0, seed=601), dtype=torch.float32,
                        device="cuda").requires_grad_(True)
    delta = torch.zeros((n, n, n), dtype=torch.float32, device="cuda", requires_grad=True)
    tol = 1e-3 * (x.max() - x.min()).item()
    y = mgx.MGXRoundTrip.apply(x, delta, None, 0, tol)
    assert (y.detach() - x.detach()).abs().max().item() <= tol
    w = torch.linspace(-1, 1, n ** 3, device="cuda", dtype=torch.float32).reshape(n, n, n)
    (y * w).sum().backward()
    g64 = w.double().cpu().numpy()
    gc = oracle.recompose_adjoint(g64)
    gx = oracle.decompose_adjoint(gc)
    assert np.abs(delta.grad.double().cpu().numpy() - oracle.to_level_centric(gc)).max() <= 1e-5 * np.abs(gc).max()
    # D^T is applied to gc in fp32: the bar is relative to its input magnitude
    assert np.abs(x.grad.double().cpu().numpy() - gx).max() <= 1e-5 * np.abs(gc).max()


def test_adjoint_workspace_and_errors():
    u = torch.zeros((17, 17, 17), dtype=torch.float32, device="cuda")
    small = torch.empty(mgx.workspace_size(mgx.MGX_F32, u.shape, 0), dtype=torch.uint8, device="cuda")
    assert mgx.adjoint_workspace_size(mgx.MGX_F32, u.shape, 0) > small.numel()
    with pytest.raises(mgx.MgxError) as e:
        mgx.decompose_adjoint(u, workspace=small)
    assert e.value.code == 7
    with pytest.raises(mgx.MgxError) as e:
        mgx.recompose_adjoint(u, out=u)
    assert e.value.code == 1
