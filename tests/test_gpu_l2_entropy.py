"""The L2 quantizer schedule and the label entropy on the GPU against the
oracle: labels from caller-given tolerances bit-exact (quantize and
dequantize), and the per-level entropies of the labels equal to the oracle's
(the counts are exact, so 1e-12 relative), on shapes with several levels,
both dtypes and two stop levels."""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402


@pytest.mark.parametrize("case", [((33, 65, 129), torch.float32), ((65, 65, 65), torch.float64), ((257, 129), torch.float32),
                                  ((4097,), torch.float64)],
                         ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}")
def test_l2_labels_and_entropy(case):
    shape, dt = case
    print(f"[l2-entropy] {shape} {dt}", flush=True)
    sys.stdout.flush()
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=31), dtype=dt, device="cuda")
    for stop in (0, 2):
        umc = mgx.decompose(u, None, stop)
        tau = mgx.level_tolerances_l2(shape, 1e-3 * float((u.max() - u.min()).item()), 4.0, None, stop)
        lab = mgx.quantize_levels(umc, tau, None, stop)
        back = mgx.dequantize_levels(lab, tau, dt, None, stop)
        torch.cuda.synchronize()
        umc64 = oracle.from_level_centric(umc.double().cpu().numpy(), stop)
        want = oracle.to_level_centric(oracle.quantize_levels(umc64, tau, stop), stop)
        assert np.array_equal(lab.cpu().numpy(), want)
        wback = oracle.to_level_centric(oracle.dequantize_levels(oracle.from_level_centric(want, stop), tau, stop),
                                        stop)
        assert np.array_equal(back.double().cpu().numpy(), wback.astype(np.float32 if dt == torch.float32 else
                                                                         np.float64).astype(np.float64))
        H = mgx.label_entropy(lab, stop)
        Href = oracle.label_entropy(oracle.from_level_centric(lab.cpu().numpy(), stop), stop)
        assert np.allclose(H, Href, rtol=1e-12, atol=1e-12), (stop, H, Href)


def test_entropy_workspace_errors():
    lab = torch.zeros((33, 33, 33), dtype=torch.int32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(mgx.MgxError):
        mgx.label_entropy(lab, 0, workspace=small)
    H = mgx.label_entropy(lab, 0)
    assert np.allclose(H, 0.0)


@pytest.mark.parametrize("spread", [100, 2 ** 20, 2 ** 30])
def test_entropy_histogram_and_sort_paths(spread):
    """Labels whose per-level ranges fit the histogram (the two smaller
    spreads) and ranges too wide for it (the radix-sort path, with the extreme
    labels INT32_MIN and INT32_MAX), against the oracle."""
    shape = (33, 65, 65)
    rng = np.random.default_rng(spread)
    lab = rng.integers(-spread, spread + 1, size=shape).astype(np.int64)
    lab = (lab * rng.random(shape) ** 3).astype(np.int32)  # many small values, a few large ones
    if spread > 2 ** 26:  # the extreme labels too (sort path)
        lab.flat[5] = np.iinfo(np.int32).min
        lab.flat[7] = np.iinfo(np.int32).max
    for stop in (0, 3):
        H = mgx.label_entropy(torch.as_tensor(lab, device="cuda"), stop)
        Href = oracle.label_entropy(oracle.from_level_centric(lab, stop), stop)
        assert np.allclose(H, Href, rtol=1e-12, atol=1e-12), (spread, stop, H, Href)


@pytest.mark.parametrize("case", [((65, 129, 33), torch.float32, 0), ((129, 65), torch.float64, 2),
                                  ((17, 9, 17, 9), torch.float32, 0)],
                         ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}-stop{c[2]}")
def test_entropy_with_quantizer_maxima(case):
    """label_entropy given the fused quantizer's statistics (one pass over the
    labels) equals the plain call and the oracle; maxima that are too small
    (labels beyond them) or statistics of another stop level or with
    out-of-range labels still give the exact entropies."""
    shape, dt, stop = case
    print(f"[entropy-bounded] {shape} {dt} stop {stop}", flush=True)
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=41), dtype=dt, device="cuda")
    tol = 1e-3 * float((u.max() - u.min()).item())
    _, lab, st, code = mgx.decompose_quantize(u, tol, stop_level=stop, stats=True)
    assert code == 0
    Href = oracle.label_entropy(oracle.from_level_centric(lab.cpu().numpy(), stop), stop)
    H0 = mgx.label_entropy(lab, stop)
    H1 = mgx.label_entropy(lab, stop, stats=st)
    assert np.array_equal(H0, H1)
    assert np.allclose(H1, Href, rtol=1e-12, atol=1e-12)
    # maxima one short on every level: the labels at the maxima are detected
    short = dict(st, max_abs_label=[max(m - 1, 0) for m in st["max_abs_label"]])
    assert np.array_equal(mgx.label_entropy(lab, stop, stats=short), H0)
    # larger maxima than needed: the same counts over wider key ranges
    wide = dict(st, max_abs_label=[2 * m + 5 for m in st["max_abs_label"]])
    assert np.allclose(mgx.label_entropy(lab, stop, stats=wide), H0, rtol=1e-12, atol=1e-12)
    # statistics that cannot be used are ignored
    assert np.array_equal(mgx.label_entropy(lab, stop, stats=dict(st, n_overflow=1)), H0)
    other = dict(st, first_level=stop + 1, max_abs_label=st["max_abs_label"][1:])
    assert np.array_equal(mgx.label_entropy(lab, stop, stats=other), H0)
