"""Pins of the oracle's adaptive decomposition (Sec. 4.2, Alg. 1 lines 1-16).

The estimate compares the Lorenzo predictor with the multilinear
interpolation on sampled 3^3 blocks.  Its sums are pinned by closed forms:
both predictors are exact on their own polynomial classes (Lorenzo on sums of
functions of two variables, the interpolation on piecewise multilinear
fields), and on u = x y z the Lorenzo error is the constant mixed third
difference s^3 while the interpolation is exact.  The counts are those of a
3^3 block (12 edge, 6 plane and 1 cube node).  The decisions follow the
paper's reasoning (Lorenzo wins at small tolerances on fields it predicts
well; interpolation wins when the penalties dominate), and the decomposition
that stops at the chosen level equals the fixed-level one.
"""
import numpy as np
import pytest

import dense_ref
import oracle


def grid(shape, coords=None):
    Xs = [np.arange(n, dtype=np.float64) if (coords is None or coords[k] is None) else np.asarray(coords[k])
          for k, n in enumerate(shape)]
    return np.meshgrid(*Xs, indexing="ij")


def sampled_blocks(m):
    return len(range(1, (m - 1) // 2, 4))


@pytest.mark.parametrize("shape", [(17, 17, 17), (33, 17, 65), (65, 33, 33)])
def test_counts_per_block(shape):
    L = oracle.num_levels(shape)
    u = np.zeros(shape)
    for l in range(1, L + 1):
        m = [(n - 1) // 2 ** (L - l) + 1 for n in shape]
        nb = np.prod([sampled_blocks(x) for x in m])
        sl, si, cnt = oracle.adaptive_estimate(u, l)
        assert list(cnt) == [12 * nb, 6 * nb, nb]
        assert sl == 0.0 and si == 0.0


def test_lorenzo_exact_on_two_variable_sums():
    shape = (33, 33, 33)
    z, y, x = grid(shape)
    u = np.sin(0.3 * x) * np.cos(0.2 * y) + (y * z) ** 2 / 100 + np.exp(0.05 * x) * z
    L = oracle.num_levels(shape)
    for l in range(1, L + 1):
        s = 2 ** (L - l)
        sl, si, cnt = oracle.adaptive_estimate(u, l)
        assert sl <= 1e-11 * np.abs(u).max() * cnt.sum()
        assert si > 1e-3  # the curvature defeats the interpolation


@pytest.mark.parametrize("kind", ["uniform", "random"])
def test_interpolation_exact_on_coarse_multilinear(kind):
    shape = (33, 17, 33)
    rng = np.random.default_rng(1)
    coords = None if kind == "uniform" else [np.cumsum(rng.uniform(0.5, 1.5, n)) for n in shape]
    Xs = [np.arange(n, dtype=np.float64) if coords is None else coords[k] for k, n in enumerate(shape)]
    L = oracle.num_levels(shape)
    for l in range(1, L + 1):
        coarse = rng.standard_normal(tuple((n - 1) // 2 ** (L - l + 1) + 1 for n in shape))
        u = dense_ref.interpolate(coarse, Xs, L, l - 1, L)
        sl, si, cnt = oracle.adaptive_estimate(u, l, coords)
        assert si <= 1e-12 * np.abs(coarse).max() * cnt.sum()
        assert sl > 1e-6


def test_trilinear_monomial():
    shape = (65, 33, 33)
    z, y, x = grid(shape)
    u = x * y * z
    L = oracle.num_levels(shape)
    for l in range(1, L + 1):
        s = 2 ** (L - l)
        sl, si, cnt = oracle.adaptive_estimate(u, l)
        n = cnt.sum()
        assert abs(sl - n * s ** 3) <= 1e-9 * n * s ** 3
        assert si <= 1e-9 * n * s ** 3


def test_errors_add_penalties():
    el, ei = oracle.adaptive_errors(2.0, 3.0, [12, 6, 1], 0.5)
    assert el == pytest.approx(2.0 + 1.22 * 0.5 * 19)
    assert ei == pytest.approx(3.0 + (12 * 0.369 + 6 * 0.259 + 0.182) * 0.5)


def test_decisions_and_result():
    shape = (33, 33, 33)
    z, y, x = grid(shape)
    rng = np.random.default_rng(4)
    smooth = np.sin(0.3 * x) * np.cos(0.2 * y) + (y * z) ** 2 / 100   # Lorenzo exact
    rough = rng.standard_normal(shape)
    L = oracle.num_levels(shape)
    # a field Lorenzo predicts exactly, at a small tolerance: stop at once
    v, stop = oracle.decompose_adaptive(smooth, 1e-6 * np.ptp(smooth))
    assert stop == L and np.array_equal(v, smooth)
    # white noise at a large tolerance: the penalties decide, interpolation wins everywhere
    v, stop = oracle.decompose_adaptive(rough, 10 * np.ptp(rough))
    assert stop == 0
    # the result equals the fixed-level decomposition to the chosen level
    field = smooth + 1e-3 * rough
    for tol in (1e-4, 1e-2, 1.0):
        v, stop = oracle.decompose_adaptive(field, tol * np.ptp(field))
        assert np.array_equal(v, oracle.decompose(field, None, stop)), tol


def test_adaptive_rejects_lower_dimensions():
    with pytest.raises(oracle.OracleError):
        oracle.adaptive_estimate(np.zeros((33, 33)), 1)
    with pytest.raises(oracle.OracleError):
        oracle.decompose_adaptive(np.zeros(33), 1.0)
