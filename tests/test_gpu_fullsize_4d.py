"""4-D parity at the benchmark's full size: the QMCPACK-shaped field of
Table 2 (288 x 115 x 69 x 69, fp32), padded with dummy nodes to
513 x 129 x 129 x 129 (1.1 G nodes, too large for the oracle in a test).

- the finest level's coefficients at sampled nodes against their definition
  (value minus the multilinear interpolant of its up to 16 nodal corners,
  computed here in FP64);
- a separable field f0 x f1 x f2 x f3 of the padded size: the coarsest box
  Q_0 u equals the outer product of the four 1-D oracle projections (the L2
  projection onto a tensor-product space factorizes), which checks every
  sweep and solve of all six levels;
- the round trip, the L-infinity bound on the real nodes after cropping, and
  the fused calls equal to the separate ones.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402

SHAPE = (288, 115, 69, 69)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def padded():
    u = workloads.orbital_field(SHAPE, device="cuda")
    p = mgx.pad(u)
    torch.cuda.synchronize()
    return u, p


def test_qmcpack_padded_finest_coefficients_sampled(padded):
    _say("[full 4d] sampled finest coefficients")
    u, p = padded
    shape = tuple(p.shape)
    assert shape == (513, 129, 129, 129)
    ws = torch.empty(mgx.workspace_size(mgx.MGX_F32, shape, 0), dtype=torch.uint8, device="cuda")
    g = mgx.decompose(p, None, 0, workspace=ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    n = 20000
    idx = np.stack([rng.integers(0, s, 4 * n) for s in shape], axis=1)
    idx = idx[(idx & 1).any(axis=1)][:n]  # coefficient nodes of the finest level
    strides = np.array([shape[1] * shape[2] * shape[3], shape[2] * shape[3], shape[3], 1])
    # every node's corners (weights 1/2 per odd axis on the unit grid)
    flat_p = p.view(-1)
    want = p.view(-1)[torch.as_tensor(idx @ strides, device="cuda")].double().cpu().numpy()
    for corner in range(16):
        bits = np.array([(corner >> k) & 1 for k in range(4)])
        odd = idx & 1
        use = ~((bits == 1) & (odd == 0)).any(axis=1)
        q = idx + np.where(odd == 1, 2 * bits - 1, 0)
        w = np.prod(np.where(odd == 1, 0.5, 1.0), axis=1)
        vals = flat_p[torch.as_tensor(np.where(use[:, None], q, 0) @ strides, device="cuda")].double().cpu().numpy()
        want -= np.where(use, w * vals, 0.0)
    c = np.array([(s + 1) // 2 for s in shape])
    pos = np.where(idx & 1, c + (idx - 1) // 2, idx // 2)
    got = g.view(-1)[torch.as_tensor(pos @ strides, device="cuda")].double().cpu().numpy()
    scale = float(p.abs().max())
    assert np.abs(got - want).max() <= 1e-5 * scale


def test_separable_full_size_coarsest_box():
    shape = (513, 129, 129, 129)
    _say(f"[full 4d] separable {shape}")
    L = mgx.num_levels(shape)
    rng = np.random.default_rng(23)
    fs = [np.sin(np.linspace(0, rng.uniform(2, 6), n) + rng.uniform(0, 3)) + 0.2 * rng.standard_normal(n) + 1.5
          for n in shape]
    t = [torch.as_tensor(f, dtype=torch.float32, device="cuda") for f in fs]
    u = (t[0][:, None, None, None] * t[1][None, :, None, None]) * (t[2][None, None, :, None] * t[3][None, None, None, :])
    u = u.contiguous()
    g = mgx.decompose(u, None, 0)
    torch.cuda.synchronize()
    parts = []
    for k, f in enumerate(fs):
        f32 = np.asarray(f, dtype=np.float32).astype(np.float64)
        off = oracle.num_levels((shape[k],)) - L
        parts.append(oracle.recompose_to(oracle.decompose(f32, None, off), off, None, off))
    want = np.einsum("a,b,c,d->abcd", *parts)
    got = g[:want.shape[0], :want.shape[1], :want.shape[2], :want.shape[3]].double().cpu().numpy()
    assert want.shape == (9, 3, 3, 3)
    assert np.abs(got - want).max() <= 1e-5 * float(u.abs().max())
    del u, g
    torch.cuda.empty_cache()


def test_qmcpack_round_trip_bound_and_fused(padded):
    _say("[full 4d] round trip, bound, fused")
    u, p = padded
    g = mgx.decompose(p)
    r = mgx.recompose(g)
    scale = float(p.abs().max())
    assert (r.double() - p.double()).abs().max().item() <= 1e-5 * scale
    del r
    for rel in (1e-2, 1e-4):
        tol = rel * float((u.max() - u.min()).item())
        labels = mgx.quantize(g, tol)
        umc2, lab2 = mgx.decompose_quantize(p, tol)
        torch.cuda.synchronize()
        assert torch.equal(lab2, labels) and torch.equal(umc2, g)
        del umc2
        back = mgx.crop(mgx.dequantize_recompose(labels, tol, torch.float32), SHAPE)
        err = (back.double() - u.double()).abs().max().item()
        assert err <= tol, (rel, err / tol)
        del back, labels, lab2
    del g
    torch.cuda.empty_cache()
