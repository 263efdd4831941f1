"""Adaptive decomposition on the GPU (Sec. 4.2, Alg. 1 lines 1-16) against
the FP64 oracle.

The estimate's sums on a level box are compared with the oracle's on the same
values (FP64 arithmetic on both sides, so 1e-10 relative to the sums;
sampled node counts exact).  The chosen stop level must equal the oracle's
where the two estimates are clearly apart, and the coefficients must meet the
decomposition's parity bars at that stop level."""
import sys

import numpy as np
import pytest

import oracle
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2010_05872_amd as mgx  # noqa: E402


def _coords(shape, kind, seed):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


@pytest.mark.parametrize("case", [((33, 33, 33), torch.float64, None), ((65, 33, 129), torch.float32, "random"),
                                  ((129, 65, 65), torch.float64, "tanh")],
                         ids=lambda c: f"{'x'.join(map(str, c[0]))}-{str(c[1])[6:]}-{c[2]}")
def test_estimate_matches_oracle(case):
    shape, dt, kind = case
    print(f"[adaptive-estimate] {shape} {dt} {kind}", flush=True)
    sys.stdout.flush()
    coords = _coords(shape, kind, 2)
    u = torch.as_tensor(workloads.gaussian_random_field(shape, slope=3.0, seed=12), dtype=dt, device="cuda")
    L = mgx.num_levels(shape)
    for l in range(1, L + 1):
        umc = mgx.decompose(u, coords, l)
        box = tuple(slice(0, n) for n in mgx.level_shape(shape, l))
        v = umc[box].contiguous()
        (sl, si), cnt = mgx.adaptive_estimate(v, shape, l, coords)
        s = 2 ** (L - l)
        w = np.zeros(shape)
        w[::s, ::s, ::s] = v.double().cpu().numpy()
        rl, ri, rcnt = oracle.adaptive_estimate(w, l, coords)
        assert list(cnt) == list(rcnt), l
        assert abs(sl - rl) <= 1e-10 * max(rl, 1e-300), (l, sl, rl)
        assert abs(si - ri) <= 1e-10 * max(ri, 1e-300), (l, si, ri)


def _fields(shape):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    smooth = np.sin(0.3 * x) * np.cos(0.2 * y) + (y * z) ** 2 / 100 + np.exp(0.05 * x) * z / 10
    rough = np.random.default_rng(4).standard_normal(shape)
    grf = workloads.gaussian_random_field(shape, slope=3.0, seed=21)
    return {"smooth": smooth, "rough": rough, "grf": grf}


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_decisions_and_coefficients_match_oracle(dt):
    shape = (65, 65, 65)
    L = mgx.num_levels(shape)
    fields = _fields(shape)
    cases = [("smooth", 1e-6), ("rough", 10.0), ("grf", 1e-2), ("grf", 1e-4), ("grf", 1e-6), ("smooth", 1e-2)]
    for name, rel in cases:
        print(f"[adaptive] {name} {rel} {dt}", flush=True)
        ud = torch.as_tensor(fields[name], dtype=dt, device="cuda")
        u64 = ud.double().cpu().numpy()
        tol = rel * float(np.ptp(u64))
        umc, stop = mgx.decompose_adaptive(ud, tol)
        torch.cuda.synchronize()
        ref, rstop = oracle.decompose_adaptive(u64, tol)
        if stop != rstop:
            # allowed only at a near tie: the oracle's margin at the level where the runs part
            l = max(stop, rstop)
            v = oracle.decompose(u64, None, l)
            sl, si, cnt = oracle.adaptive_estimate(v, l)
            tau0 = oracle.level_tolerances(shape, tol, None, l)[0]
            el, ei = oracle.adaptive_errors(sl, si, cnt, tau0)
            assert abs(el - ei) <= 1e-6 * max(el, ei), (name, rel, stop, rstop)
        scale = np.abs(u64).max()
        bar = (1e-12 if dt == torch.float64 else 1e-5) * scale
        want = oracle.to_level_centric(oracle.decompose(u64, None, stop), stop)
        assert np.abs(umc.double().cpu().numpy() - want).max() <= bar, (name, rel, stop)
        # the same coefficients as the fixed-level decomposition
        fixed = mgx.decompose(ud, None, stop)
        assert (umc - fixed).abs().max().item() <= bar
    assert 0 <= stop <= L


def test_adaptive_errors():
    u2 = torch.zeros((33, 33), dtype=torch.float32, device="cuda")
    with pytest.raises(mgx.MgxError):
        mgx.decompose_adaptive(u2, 1.0)
    u3 = torch.zeros((17, 17, 17), dtype=torch.float32, device="cuda")
    with pytest.raises(mgx.MgxError):
        mgx.decompose_adaptive(u3, -1.0)
