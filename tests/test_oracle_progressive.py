"""Pins of the oracle's progressive recomposition (the recomposition stopped
at an intermediate level, the coarse representation of data refactoring;
Sec. 1 and the analysis on decomposed representations of Sec. 6.2.2).

Recomposing up to level t must give Q_t u, the L2 projection onto the
piecewise multilinear space on N_t, whatever stop level the decomposition
went to.  It is checked against the dense brute-force projection of
``dense_ref`` (quadrature-built mass matrices, dense solves), against a
closed form (a field that is piecewise multilinear on N_t is its own
projection), and at the two ends (t = L: the full recomposition; t = stop:
the stop level's values untouched).
"""
import numpy as np
import pytest

import dense_ref
import oracle
import workloads

SHAPES = [(17,), (33,), (9, 17), (17, 9), (9, 9, 9), (5, 9, 17)]


def coords_for(shape, kind, seed=0):
    if kind == "uniform":
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


def axes(shape, coords):
    return [np.arange(n, dtype=np.float64) if (coords is None or coords[k] is None)
            else np.asarray(coords[k], dtype=np.float64) for k, n in enumerate(shape)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", ["uniform", "tanh", "random"])
def test_partial_recomposition_is_the_projection(shape, kind):
    rng = np.random.default_rng(7)
    u = rng.standard_normal(shape)
    coords = coords_for(shape, kind, seed=3)
    Xs = axes(shape, coords)
    L = oracle.num_levels(shape)
    for stop in range(0, L + 1):
        umc = oracle.decompose(u, coords, stop)
        for t in range(stop, L + 1):
            got = oracle.recompose_to(umc, t, coords, stop)
            want = dense_ref.projection(u, Xs, L, t)
            assert got.shape == want.shape
            assert np.abs(got - want).max() <= 1e-11 * (1 + np.abs(want).max()), (stop, t)


@pytest.mark.parametrize("shape", [(33,), (9, 17), (9, 9, 9)], ids=lambda s: "x".join(map(str, s)))
def test_multilinear_on_coarse_grid_is_reproduced(shape):
    """A field that is piecewise multilinear on N_t lies in V_t: Q_t u = u on N_t."""
    rng = np.random.default_rng(11)
    coords = coords_for(shape, "random", seed=5)
    Xs = axes(shape, coords)
    L = oracle.num_levels(shape)
    for t in range(0, L):
        coarse = rng.standard_normal(tuple((n - 1) // 2 ** (L - t) + 1 for n in shape))
        u = dense_ref.interpolate(coarse, Xs, L, t, L)
        got = oracle.recompose_to(oracle.decompose(u, coords, 0), t, coords, 0)
        assert np.abs(got - coarse).max() <= 1e-12 * (1 + np.abs(coarse).max()), t


def test_ends():
    rng = np.random.default_rng(3)
    shape = (9, 17, 9)
    u = rng.standard_normal(shape)
    L = oracle.num_levels(shape)
    umc = oracle.decompose(u, None, 1)
    assert np.array_equal(oracle.recompose_to(umc, L, None, 1), oracle.recompose(umc, None, 1))
    s = 2 ** (L - 1)
    assert np.array_equal(oracle.recompose_to(umc, 1, None, 1), umc[::s, ::s, ::s])
    with pytest.raises(oracle.OracleError):
        oracle.recompose_to(umc, 0, None, 1)
    with pytest.raises(oracle.OracleError):
        oracle.recompose_to(umc, L + 1, None, 1)
