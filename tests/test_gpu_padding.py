"""Non-dyadic fields on the GPU: mgx_pad / mgx_crop bit-exact against the
oracle's padding, and the whole path on a padded field (decompose_quantize,
dequantize_recompose, crop) within the L-infinity bound on the real nodes,
1-D to 3-D, both dtypes, with continued non-uniform coordinates."""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402

CASES = [((50, 70, 90), torch.float32, None), ((100,), torch.float64, "random"), ((33, 100), torch.float32, "random"),
         ((20, 9, 300), torch.float64, None)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}-{c[2]}")
def test_padded_path(case):
    shape, dt, kind = case
    print(f"[padding] {shape} {dt} {kind}", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(3)
    u64 = np.cumsum(rng.standard_normal(shape), axis=-1) + 0.1 * rng.standard_normal(shape)
    u = torch.as_tensor(u64, dtype=dt, device="cuda")
    p = mgx.pad(u)
    torch.cuda.synchronize()
    assert np.array_equal(p.double().cpu().numpy(), oracle.pad_to_dyadic(u.double().cpu().numpy()))
    c = mgx.crop(p, shape)
    torch.cuda.synchronize()
    assert torch.equal(c, u)
    coords = None
    if kind == "random":
        coords = mgx.pad_coords([np.cumsum(rng.uniform(0.5, 1.5, n)) for n in shape], shape)
    tol = 1e-3 * float((u.max() - u.min()).item())
    _, labels = mgx.decompose_quantize(p, tol, coords, keep_coef=False)
    r = mgx.dequantize_recompose(labels, tol, dt, coords)
    back = mgx.crop(r, shape)
    torch.cuda.synchronize()
    err = (back.double() - u.double()).abs().max().item()
    assert err <= tol, (err, tol)


def test_pad_errors():
    u = torch.zeros((1, 5), device="cuda")
    with pytest.raises(mgx.MgxError):
        mgx.pad(u)
