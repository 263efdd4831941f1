"""Pins of the oracle on 4-D grids (the four-dimensional QMCPACK field of
Sec. 6, Table 2).

The method is the same on any number of axes (Sec. 2: tensor-product grids,
multilinear interpolation over the 2^d corners, the L2 projection one axis
after the other).  The 4-D code is pinned against things other than itself:

- a separable field f0(x0) f1(x1) f2(x2) f3(x3): the L2 projection onto a
  tensor-product space factorizes, so Q_t u is the outer product of the four
  1-D projections computed by the (separately pinned) 1-D oracle;
- a field constant along one axis: Q_t u is the 3-D oracle's Q_t g repeated
  along that axis, and its coefficients are the 3-D coefficients or zero;
- a multilinear field lies in every V_l: all coefficients vanish and the
  coarse values are the samples;
- the L-infinity constant for large uniform axes, 1 + (1 + sqrt(3)/2)^4
  (the 1-D operator norm tends to 1 + sqrt(3)/2);
- level counts and the level-centric regions of Sec. 5.1 in closed form;
- the quantization error bound of Sec. 4.1 (tau_l schedule with d = 4).
"""
import math

import numpy as np
import pytest

import oracle
import workloads


def _axes(shape, coords):
    return [np.arange(n, dtype=np.float64) if (coords is None or coords[k] is None)
            else np.asarray(coords[k], dtype=np.float64) for k, n in enumerate(shape)]


def _level_slices(shape, L, t):
    """Index of the level-t grid N_t inside the finest grid (every 2^(L-t)-th node)."""
    s = 1 << (L - t)
    return tuple(slice(None, None, s) for _ in shape)


def test_num_levels_4d():
    assert oracle.num_levels((17, 9, 33, 9)) == 2
    assert oracle.num_levels((513, 129, 129, 129)) == 6
    assert oracle.num_levels((5, 5, 5, 5)) == 1
    with pytest.raises(oracle.OracleError):
        oracle.num_levels((5, 5, 5, 5, 5))
    with pytest.raises(oracle.OracleError):
        oracle.num_levels((5, 6, 5, 5))


@pytest.mark.parametrize("kind", ["uniform", "random"])
@pytest.mark.parametrize("stop", [0, 1])
def test_separable_field_projects_axis_by_axis(kind, stop):
    """Q_t u of f0 x f1 x f2 x f3 equals the outer product of the 1-D Q_t f_k
    at every level t (each axis's 1-D hierarchy is offset by L_k - L)."""
    shape = (17, 9, 33, 9)
    L = oracle.num_levels(shape)
    coords = None if kind == "uniform" else [workloads.random_coordinates(n, 40 + k) for k, n in enumerate(shape)]
    X = _axes(shape, coords)
    rng = np.random.default_rng(5)
    fs = [np.sin(1.3 * x / x[-1] * 3.0 + rng.uniform(0, 3)) + 0.3 * rng.standard_normal(len(x)) for x in X]
    u = np.einsum("a,b,c,d->abcd", *fs)
    umc = oracle.decompose(u, coords, stop)
    for t in range(stop, L + 1):
        got = oracle.recompose_to(umc, t, coords, stop)
        parts = []
        for k, f in enumerate(fs):
            Lk = oracle.num_levels((shape[k],))
            off = Lk - L
            c1 = None if coords is None else [coords[k]]
            f_mc = oracle.decompose(f, c1, stop + off)
            parts.append(oracle.recompose_to(f_mc, t + off, c1, stop + off))
        want = np.einsum("a,b,c,d->abcd", *parts)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("axis", [0, 2, 3])
def test_field_constant_along_one_axis(axis):
    """u(x) = g(x without axis `axis`): the 4-D hierarchy is the 3-D one
    repeated along that axis; coefficients of nodes whose level comes from
    that axis alone are zero, all others are the 3-D coefficients."""
    shape3 = (9, 17, 9)
    shape = list(shape3)
    shape.insert(axis, 17)
    shape = tuple(shape)
    assert oracle.num_levels(shape) == oracle.num_levels(shape3)
    L = oracle.num_levels(shape)
    coords3 = [workloads.random_coordinates(n, 60 + k) for k, n in enumerate(shape3)]
    coords = list(coords3)
    coords.insert(axis, workloads.random_coordinates(17, 99))
    g = np.random.default_rng(11).standard_normal(shape3)
    u = np.repeat(np.expand_dims(g, axis), shape[axis], axis=axis)
    for stop in (0, 1):
        umc4 = oracle.decompose(u, coords, stop)
        umc3 = oracle.decompose(g, coords3, stop)
        lev4 = oracle.level_map(shape, stop)
        lev3 = np.expand_dims(oracle.level_map(shape3, stop), axis)
        umc3b = np.expand_dims(umc3, axis)
        want = np.where(lev4 > lev3, 0.0, umc3b)
        np.testing.assert_allclose(umc4, want, rtol=0, atol=1e-12)
        for t in range(stop, L + 1):
            q4 = oracle.recompose_to(umc4, t, coords, stop)
            q3 = np.expand_dims(oracle.recompose_to(umc3, t, coords3, stop), axis)
            np.testing.assert_allclose(q4, np.broadcast_to(q3, q4.shape), rtol=0, atol=1e-12)


def test_multilinear_field_has_no_coefficients():
    shape = (9, 5, 17, 9)
    coords = [workloads.random_coordinates(n, 70 + k) for k, n in enumerate(shape)]
    X = np.meshgrid(*coords, indexing="ij")
    u = 1.0 + 0.5 * X[0] - 0.25 * X[3] + 0.1 * X[0] * X[1] * X[2] * X[3] - 0.3 * X[1] * X[2] + 0.2 * X[0] * X[3]
    umc = oracle.decompose(u, coords, 0)
    lev = oracle.level_map(shape, 0)
    scale = np.abs(u).max()
    assert np.abs(umc[lev > 0]).max() <= 1e-12 * scale
    np.testing.assert_allclose(umc[lev == 0], u[lev == 0], rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(oracle.recompose(umc, coords, 0), u, rtol=0, atol=1e-12 * scale)


def test_linf_constant_4d_large_uniform_axes():
    c = oracle.linf_constant((65, 65, 65, 65), None, 0)
    assert abs(c - (1.0 + (1.0 + math.sqrt(3.0) / 2.0) ** 4)) < 1e-4
    # the per-level constant is the product of the four axis norms
    shape = (9, 17, 5, 9)
    X = _axes(shape, None)
    best = 1.0
    L = oracle.num_levels(shape)
    for lv in range(1, L + 1):
        prod = 1.0
        for k in range(4):
            prod *= oracle.axis_operator_norm(X[k][::1 << (L - lv)])
        best = max(best, 1.0 + prod)
    assert oracle.linf_constant(shape, None, 0) == pytest.approx(best, rel=1e-14)


@pytest.mark.parametrize("stop", [0, 1, 2])
def test_level_counts_and_regions(stop):
    shape = (17, 9, 33, 9)
    L = oracle.num_levels(shape)
    lev = oracle.level_map(shape, stop)
    m = lambda t: [(n - 1) // (1 << (L - t)) + 1 for n in shape]  # noqa: E731
    assert (lev == stop).sum() == np.prod(m(stop))
    for t in range(stop + 1, L + 1):
        c = m(t - 1)
        assert (lev == t).sum() == np.prod(m(t)) - np.prod(c)
    pos = oracle.level_centric_index(shape, stop)
    assert np.array_equal(np.sort(pos.ravel()), np.arange(pos.size))
    P = np.stack(np.unravel_index(pos, shape))  # lc coordinates of every node
    for t in range(stop + 1, L + 1):
        sel = lev == t
        inside = np.all(P[:, sel] < np.array(m(t))[:, None], axis=0)
        beyond = np.any(P[:, sel] >= np.array(m(t - 1))[:, None], axis=0)
        assert inside.all() and beyond.all()
    # the stop-level grid keeps its natural order in the corner box
    sl = _level_slices(shape, L, stop)
    idx = np.indices(shape)[(slice(None),) + sl].reshape(4, -1)
    want = np.ravel_multi_index(tuple(idx // (1 << (L - stop))), shape)
    assert np.array_equal(pos[sl].ravel(), want)


@pytest.mark.parametrize("stop", [0, 1])
def test_quantized_round_trip_within_tolerance(stop):
    shape = (9, 17, 9, 17)
    coords = [workloads.random_coordinates(n, 80 + k) for k, n in enumerate(shape)]
    u = workloads.gaussian_random_field(shape, slope=3.0, seed=21).numpy()
    np.testing.assert_allclose(oracle.recompose(oracle.decompose(u, coords, stop), coords, stop), u,
                               rtol=0, atol=1e-12)
    for rel in (1e-2, 1e-4):
        tol = rel * float(u.max() - u.min())
        umc = oracle.decompose(u, coords, stop)
        lab, code = oracle.quantize(umc, tol, coords, stop)
        assert code == 0
        back = oracle.recompose(oracle.dequantize(lab, tol, coords, stop), coords, stop)
        assert np.abs(back - u).max() <= tol
    tau = oracle.level_tolerances(shape, 1.0, coords, stop)
    np.testing.assert_allclose(tau[1:] / tau[:-1], 4.0, rtol=1e-14)  # kappa = sqrt(2^4)
