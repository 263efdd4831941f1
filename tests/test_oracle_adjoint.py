"""Pins of the oracle's adjoints (transposes) of decompose and recompose.

Neither adjoint is in the paper; both are defined as the transpose of the
oracle's forward maps, which are themselves pinned against the paper and
dense mathematics in test_oracle.py.  The pins here do not use the adjoint's
own formulas: the dot-product identity against the forward map, the
transpose of the dense matrix of the forward map built column by column on
tiny grids, and R^T = (D^T)^{-1}.
"""
import numpy as np
import pytest

import oracle
import workloads


def _coords(shape, kind, seed=0):
    if kind is None:
        return None
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


@pytest.mark.parametrize("shape", [(17,), (9, 17), (17, 9, 5), (9, 9, 17), (33, 17, 9)])
@pytest.mark.parametrize("kind", [None, "random", "tanh"])
def test_dot_product_identity(shape, kind):
    coords = _coords(shape, kind, 3)
    rng = np.random.default_rng(sum(shape))
    L = oracle.num_levels(shape)
    for stop in sorted({0, L // 2, L}):
        x = rng.standard_normal(shape)
        y = rng.standard_normal(shape)
        lhs = np.vdot(oracle.decompose(x, coords, stop), y)
        rhs = np.vdot(x, oracle.decompose_adjoint(y, coords, stop))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y) * 1e-3)
        lhs = np.vdot(oracle.recompose(x, coords, stop), y)
        rhs = np.vdot(x, oracle.recompose_adjoint(y, coords, stop))
        assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + np.linalg.norm(x) * np.linalg.norm(y) * 1e-3)


def _dense(fn, shape):
    n = int(np.prod(shape))
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = fn(e.reshape(shape)).ravel()
    return A


@pytest.mark.parametrize("shape,kind,stop", [((9,), "random", 0), ((5, 9), None, 0), ((5, 5, 9), "random", 0),
                                             ((9, 5), "random", 1)])
def test_adjoint_is_dense_transpose(shape, kind, stop):
    coords = _coords(shape, kind, 1)
    D = _dense(lambda e: oracle.decompose(e, coords, stop), shape)
    DT = _dense(lambda e: oracle.decompose_adjoint(e, coords, stop), shape)
    assert np.abs(DT - D.T).max() <= 1e-13 * np.abs(D).max()
    R = _dense(lambda e: oracle.recompose(e, coords, stop), shape)
    RT = _dense(lambda e: oracle.recompose_adjoint(e, coords, stop), shape)
    assert np.abs(RT - R.T).max() <= 1e-13 * np.abs(R).max()
    # and the forward maps are inverses of each other, so are the transposes
    assert np.abs(RT @ DT - np.eye(D.shape[0])).max() <= 1e-12


def test_recompose_adjoint_inverts_decompose_adjoint():
    shape = (17, 33, 9)
    coords = _coords(shape, "random", 7)
    g = np.random.default_rng(5).standard_normal(shape)
    for stop in (0, 1):
        back = oracle.decompose_adjoint(oracle.recompose_adjoint(g, coords, stop), coords, stop)
        assert np.abs(back - g).max() <= 1e-12 * np.abs(g).max()


def test_line_adjoint_is_transpose_of_projection():
    X = workloads.random_coordinates(17, 2)
    m, mc = 17, 9
    P = np.stack([oracle.project_line_1d(X, np.eye(m)[j]) for j in range(m)], axis=1)  # mc x m
    PT = np.stack([oracle.project_line_adjoint_1d(X, np.eye(mc)[J]) for J in range(mc)], axis=1)  # m x mc
    assert np.abs(PT - P.T).max() <= 1e-14 * np.abs(P).max()
