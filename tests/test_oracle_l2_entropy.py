"""Pins of the oracle's L2 quantizer schedule and label entropy (Sec. 4.1).

The schedule is pinned by the two facts the paper derives from it: the
tolerance grows by kappa = sqrt(2^d) per level on uniform grids, and the bin
widths meet the L2 budget with equality, sum_l #N*_l h_l^d tau_l^2 =
tol^2 / C_L2 (here on uniform and random coordinates).  The quantizer with
caller-given tolerances reproduces the pinned L-infinity quantizer when given
its schedule.  The entropy is pinned by closed forms (constant labels: 0 bits;
K equally likely labels: log2 K; probabilities 1/4, 3/4: 0.8113 bits).
"""
import math

import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("shape", [(65,), (33, 33), (17, 17, 17)])
def test_kappa_ratio_uniform(shape):
    tau = oracle.level_tolerances_l2(shape, 1.0, 3.0)
    kappa = math.sqrt(2 ** len(shape))
    assert np.allclose(tau[1:] / tau[:-1], kappa, rtol=1e-13, atol=0)


@pytest.mark.parametrize("shape,kind", [((33, 17, 65), "uniform"), ((17, 33, 9), "random"), ((129,), "random")])
@pytest.mark.parametrize("stop", [0, 2])
def test_l2_budget_met_with_equality(shape, kind, stop):
    rng = np.random.default_rng(2)
    coords = None if kind == "uniform" else [np.cumsum(rng.uniform(0.3, 2.0, n)) for n in shape]
    tol, C = 0.7, 5.5
    tau = oracle.level_tolerances_l2(shape, tol, C, coords, stop)
    L = oracle.num_levels(shape)
    Xs = [np.arange(n, dtype=float) if coords is None else coords[k] for k, n in enumerate(shape)]
    total, prev = 0.0, 0
    for i, l in enumerate(range(stop, L + 1)):
        m = [(n - 1) // 2 ** (L - l) + 1 for n in shape]
        box = int(np.prod(m))
        hd = np.prod([(X[-1] - X[0]) / (mm - 1) for X, mm in zip(Xs, m)])
        total += (box - prev) * hd * tau[i] ** 2
        prev = box
    assert total == pytest.approx(tol ** 2 / C, rel=1e-12)


def test_levels_quantizer_reproduces_linf_quantizer():
    rng = np.random.default_rng(9)
    shape = (17, 33, 17)
    u = rng.standard_normal(shape)
    for stop in (0, 2):
        c = oracle.decompose(u, None, stop)
        tol = 1e-2
        tau = oracle.level_tolerances(shape, tol, None, stop)
        want, code = oracle.quantize(c, tol, None, stop)
        assert code == 0
        got = oracle.quantize_levels(c, tau, stop)
        assert np.array_equal(got, want)
        back = oracle.dequantize_levels(got, tau, stop)
        lev = oracle.level_map(shape, stop)
        assert np.all(np.abs(back - c) <= tau[lev - stop] * (1 + 1e-12))


def test_entropy_closed_forms():
    shape = (9, 9, 9)
    lev = oracle.level_map(shape, 0)
    L = oracle.num_levels(shape)
    lab = np.zeros(shape, dtype=np.int32)
    assert np.allclose(oracle.label_entropy(lab, 0), 0.0)
    # level L: labels cycle through K values equally often
    K = 7
    fine = np.flatnonzero(lev.ravel() == L)
    n = len(fine) // K * K
    lab.ravel()[fine[:n]] = np.arange(n) % K
    lab.ravel()[fine[n:]] = -99  # a few extra nodes: checked separately below
    H = oracle.label_entropy(lab, 0)[L]
    cnt = np.array([n // K] * K + [len(fine) - n])
    cnt = cnt[cnt > 0]
    p = cnt / cnt.sum()
    assert H == pytest.approx(float(-(p * np.log2(p)).sum()), rel=1e-14)
    if len(fine) == n:
        assert H == pytest.approx(math.log2(K))
    lab2 = np.zeros(shape, dtype=np.int32)
    sel = np.flatnonzero(lev.ravel() == L)
    lab2.ravel()[sel[: len(sel) // 4]] = 5
    q = (len(sel) // 4) / len(sel)
    assert oracle.label_entropy(lab2, 0)[L] == pytest.approx(-(q * math.log2(q) + (1 - q) * math.log2(1 - q)))
    if len(sel) % 4 == 0:
        assert oracle.label_entropy(lab2, 0)[L] == pytest.approx(0.8112781244591328)


def test_library_l2_schedule_matches_oracle():
    """The library's host-side schedule (no GPU needed) against the oracle's."""
    import paper_2010_05872_amd as mgx
    rng = np.random.default_rng(4)
    for shape, kind in (((33, 17, 65), None), ((17, 33, 9), "random"), ((257,), None)):
        coords = None if kind is None else [np.cumsum(rng.uniform(0.3, 2.0, n)) for n in shape]
        for stop in (0, 1):
            a = mgx.level_tolerances_l2(shape, 0.7, 5.5, coords, stop)
            b = oracle.level_tolerances_l2(shape, 0.7, 5.5, coords, stop)
            assert np.allclose(a, b, rtol=1e-14, atol=0)
    with pytest.raises(mgx.MgxError):
        mgx.level_tolerances_l2((33, 33), 1.0, 0.0)
