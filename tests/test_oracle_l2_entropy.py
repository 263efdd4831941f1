"""Pins of the oracle's L2 quantizer schedule and label entropy (Sec. 4.1).

The schedule is pinned by the two facts the paper derives from it: the
tolerance grows by kappa = sqrt(2^d) per level on uniform grids, and the bin
widths meet the L2 budget with equality, sum_l #N*_l h_l^d tau_l^2 =
tol^2 / C_L2 (here on uniform and random coordinates).  The quantizer with
caller-given tolerances reproduces the pinned L-infinity quantizer when given
its schedule.  The entropy is pinned by closed forms (constant labels: 0 bits;
K equally likely labels: log2 K; probabilities 1/4, 3/4: 0.8113 bits).
The cell volume h_l^d on nonuniform axes and the default C_L2 are pinned by
hand-computed values, and C_L2 by brute force: the exact smallest constant of
the L2 estimator (dense recomposition, quadrature mass matrix) never exceeds
it, and a perturbation that spends the whole budget stays within tol.
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
            # the default constant, and the schedule taking it
            assert mgx.l2_constant(shape, coords, stop) == pytest.approx(oracle.l2_constant(shape, coords, stop),
                                                                         rel=1e-14)
            a0 = mgx.level_tolerances_l2(shape, 0.7, 0.0, coords, stop)
            assert np.allclose(a0, oracle.level_tolerances_l2(shape, 0.7, 0.0, coords, stop), rtol=1e-14, atol=0)
    assert mgx.l2_constant((5,), [[0.0, 1.0, 3.0, 4.0, 10.0]]) == pytest.approx(1.4, rel=1e-15)
    with pytest.raises(mgx.MgxError):
        mgx.level_tolerances_l2((33, 33), 1.0, float("nan"))
    with pytest.raises(mgx.MgxError):
        mgx.level_tolerances_l2((33, 33), -1.0, 1.0)


# ---- nonuniform cell volume and the default C_L2, against hand-computed values ----

def test_l2_schedule_nonuniform_hand_computed():
    """tau_l = tol / sqrt(C h_l^d #N_L) with h_l the level's mean spacing,
    worked out by hand.  1-D, X = (0, 1, 3, 4, 10), L = 1: level 1 has four
    intervals over an extent of 10 (h = 5/2), level 0 nodes (0, 3, 10) two
    (h = 5); with tol = 1, C = 2, #N_L = 5: tau_1 = 1/sqrt(25) = 1/5,
    tau_0 = 1/sqrt(50).  2-D, second axis (0, 1/2, 2, 5/2, 3): h = 3/4 and
    3/2, so tau_1 = 1/sqrt(2 * 15/8 * 25) and tau_0 = 1/sqrt(2 * 15/2 * 25)."""
    X0 = [0.0, 1.0, 3.0, 4.0, 10.0]
    X1 = [0.0, 0.5, 2.0, 2.5, 3.0]
    tau = oracle.level_tolerances_l2((5,), 1.0, 2.0, [X0])
    assert tau[1] == pytest.approx(0.2, rel=1e-15)
    assert tau[0] == pytest.approx(1.0 / math.sqrt(50.0), rel=1e-15)
    tau2 = oracle.level_tolerances_l2((5, 5), 1.0, 2.0, [X0, X1])
    assert tau2[1] == pytest.approx(1.0 / math.sqrt(93.75), rel=1e-15)
    assert tau2[0] == pytest.approx(1.0 / math.sqrt(375.0), rel=1e-15)


def test_l2_constant_hand_computed():
    """Row sums (h_{j-1} + h_j)/2 of the 1-D mass matrix over the mean
    spacing.  X = (0, 1, 3, 4, 10): level 1 spacings (1, 2, 1, 6), row sums
    (1/2, 3/2, 3/2, 7/2, 3), mean 5/2: 7/5; level 0 spacings (3, 7), row sums
    (3/2, 5, 7/2), mean 5: 1.  C = 7/5 from stop 0, and 7/5 from stop 1."""
    X0 = [0.0, 1.0, 3.0, 4.0, 10.0]
    assert oracle.l2_constant((5,), [X0], 0) == pytest.approx(1.4, rel=1e-15)
    assert oracle.l2_constant((5,), [X0], 1) == pytest.approx(1.4, rel=1e-15)
    for shape in ((65,), (17, 33), (9, 9, 17)):
        assert oracle.l2_constant(shape) == 1.0
    # the default enters the schedule when no constant is given
    tau = oracle.level_tolerances_l2((5,), 1.0, 0.0, [X0])
    assert tau[1] == pytest.approx(1.0 / math.sqrt(1.4 * 2.5 * 5), rel=1e-15)


def _dense_recomposition(shape, coords, stop):
    """Column x of R = the oracle's recomposition of the unit coefficient at
    interleaved node x."""
    n = int(np.prod(shape))
    R = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        R[:, i] = oracle.recompose(e.reshape(shape), coords, stop).ravel()
    return R


@pytest.mark.parametrize("shape,kind", [((17,), "random"), ((9, 5), "uniform"), ((5, 9), "random"),
                                        ((5, 5, 9), "uniform"), ((5, 9, 5), "random")])
@pytest.mark.parametrize("stop", [0, 1])
def test_l2_constant_bounds_exact_amplification(shape, kind, stop):
    """Brute force: the exact smallest constant of the L2 estimator,
    lambda_max(W^-1/2 R^T M R W^-1/2) with R the dense recomposition, M the
    fine grid's mass matrix by quadrature (tests/dense_ref) and W the weights
    h_l^d of each coefficient's level, is at most the default C_L2; and a
    perturbation that spends the whole budget reconstructs within tol in the
    exact L2 norm."""
    import dense_ref
    rng = np.random.default_rng(17)
    coords = None if kind == "uniform" else [np.cumsum(rng.uniform(0.2, 3.0, n)) for n in shape]
    Xs = [np.arange(n, dtype=float) if coords is None else coords[k] for k, n in enumerate(shape)]
    L = oracle.num_levels(shape)
    R = _dense_recomposition(shape, coords, stop)
    M = np.array([[1.0]])
    for X in Xs:
        M = np.kron(M, dense_ref.mixed_mass(np.asarray(X), np.asarray(X)))
    lev = oracle.level_map(shape, stop).ravel()
    hd = np.ones(L + 1)
    for l in range(L + 1):
        for X in Xs:
            Y = np.asarray(X)[:: 2 ** (L - l)]
            hd[l] *= (Y[-1] - Y[0]) / (len(Y) - 1)
    w = hd[lev]
    G = (R.T @ M @ R) / np.sqrt(np.outer(w, w))
    c_exact = float(np.linalg.eigvalsh(G).max())
    C = oracle.l2_constant(shape, coords, stop)
    assert c_exact <= C * (1 + 1e-12), (c_exact, C)
    if kind == "uniform":
        assert c_exact >= 0.5 * C  # the bound is not vacuous where the spacing is even
    # the budget sum_l h_l^d sum delta^2 = tol^2 / C spent on a random perturbation
    tol = 0.3
    d = rng.standard_normal(len(w))
    d *= (tol / math.sqrt(C)) / math.sqrt(float((w * d * d).sum()))
    e = R @ d
    assert math.sqrt(float(e @ M @ e)) <= tol * (1 + 1e-12)
