"""Pins of the CPU oracle against the paper and the mathematics (no GPU).

Each test checks the oracle against something other than itself: the dense
brute-force L2 projection of ``dense_ref`` (quadrature-built mass matrices,
dense solves), closed forms and constants the paper prints
(``golden/paper_constants.json``), invariants, and statistics the paper
reports.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import dense_ref
import oracle
import workloads

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def frac(s):
    return float(Fraction(s))


SHAPES = [(17,), (33,), (9, 17), (17, 9), (9, 9, 9), (5, 9, 17), (17, 5, 9)]


def coords_for(shape, kind, seed=0):
    if kind == "uniform":
        return None
    if kind == "scaled":
        return [np.arange(n) * 0.37 + 2.0 for n in shape]
    if kind == "tanh":
        return [workloads.tanh_coordinates(shape[0])] + [None] * (len(shape) - 1)
    return [workloads.random_coordinates(n, seed + k) for k, n in enumerate(shape)]


# --------------------------------------------------------------------------
# Decomposition against the dense definition (Sec. 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("kind", ["uniform", "tanh", "random"])
def test_decompose_matches_dense_projection(shape, kind):
    rng = np.random.default_rng(hash((shape, kind)) % 2**32)
    u = rng.standard_normal(shape) * 3.0 + 1.0
    c = coords_for(shape, kind, seed=7)
    L = oracle.num_levels(shape)
    for stop in range(0, L + 1):
        got = oracle.decompose(u, c, stop)
        want = dense_ref.dense_decompose(u, c, stop)
        assert np.abs(got - want).max() <= 1e-13 * np.abs(u).max(), (shape, kind, stop)


def test_num_levels_reading():
    # all axes coarsen together; the coarsest grid has 3 nodes on the shortest axis
    assert oracle.num_levels((65, 65, 65)) == 5
    assert oracle.num_levels((513, 513, 513)) == 8
    assert oracle.num_levels((257, 1025, 1025)) == 7
    assert oracle.num_levels((3,)) == 0
    for bad in [(4,), (2,), (1,), (65, 64), (0, 5)]:
        with pytest.raises(oracle.OracleError):
            oracle.num_levels(bad)


# --------------------------------------------------------------------------
# Piecewise multilinear input => zero coefficients (spec check 2)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(33,), (17, 33), (9, 17, 33), (17, 17, 17)])
@pytest.mark.parametrize("kind", ["uniform", "random"])
def test_piecewise_multilinear_has_zero_coefficients(shape, kind):
    rng = np.random.default_rng(11)
    c = coords_for(shape, kind, seed=3)
    L = oracle.num_levels(shape)
    Xs = [np.arange(n, dtype=float) if (c is None or c[k] is None) else c[k] for k, n in enumerate(shape)]
    coarse = rng.standard_normal(tuple((n - 1) // 2 ** L + 1 for n in shape)) * 10
    u = dense_ref.interpolate(coarse, Xs, L, 0, L)
    v = oracle.decompose(u, c, 0)
    lev = oracle.level_map(shape, 0)
    scale = np.abs(u).max()
    assert np.abs(v[lev > 0]).max() <= 1e-13 * scale
    # Q_0 u equals the input restricted to N_0
    s = 2 ** L
    sl = tuple(slice(0, None, s) for _ in shape)
    assert np.abs(v[sl] - coarse).max() <= 1e-13 * scale


def test_global_multilinear_is_reproduced():
    n = 17
    x = np.arange(n, dtype=float)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 1.0 + 2 * X - 3 * Y + 0.5 * Z + 0.25 * X * Y - 0.125 * X * Y * Z
    v = oracle.decompose(u)
    lev = oracle.level_map(u.shape)
    assert np.abs(v[lev > 0]).max() <= 1e-13 * np.abs(u).max()


# --------------------------------------------------------------------------
# Round trip (spec check 3) and linearity
# --------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(65,), (33, 17), (17, 33, 9), (33, 33, 33)])
@pytest.mark.parametrize("kind", ["uniform", "tanh", "random"])
def test_round_trip(shape, kind):
    rng = np.random.default_rng(5)
    u = rng.standard_normal(shape) * 100
    c = coords_for(shape, kind, seed=1)
    for stop in (0, oracle.num_levels(shape) // 2, oracle.num_levels(shape)):
        r = oracle.recompose(oracle.decompose(u, c, stop), c, stop)
        assert np.abs(r - u).max() <= 1e-12 * np.abs(u).max()


def test_linearity_and_constants():
    rng = np.random.default_rng(8)
    shape = (17, 9, 33)
    c = coords_for(shape, "random", seed=4)
    a, b = rng.standard_normal(shape), rng.standard_normal(shape)
    lhs = oracle.decompose(2.5 * a - 1.5 * b, c)
    rhs = 2.5 * oracle.decompose(a, c) - 1.5 * oracle.decompose(b, c)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()
    v = oracle.decompose(np.full(shape, 4.25), c)
    lev = oracle.level_map(shape)
    assert np.abs(v[lev > 0]).max() <= 1e-13 * 4.25
    assert np.abs(v[lev == 0] - 4.25).max() <= 1e-13 * 4.25


def test_coordinate_scale_invariance_and_axis_permutation():
    rng = np.random.default_rng(9)
    shape = (9, 17, 33)
    c = coords_for(shape, "random", seed=2)
    u = rng.standard_normal(shape)
    v = oracle.decompose(u, c)
    v_scaled = oracle.decompose(u, [x * 7.3 - 11.0 for x in c])
    assert np.abs(v - v_scaled).max() <= 1e-13 * np.abs(v).max()
    perm = (2, 0, 1)
    vp = oracle.decompose(np.transpose(u, perm), [c[p] for p in perm])
    assert np.abs(vp - np.transpose(v, perm)).max() <= 1e-13 * np.abs(v).max()


# --------------------------------------------------------------------------
# Closed forms printed in the paper
# --------------------------------------------------------------------------
def _unit_columns(fn, m):
    cols = []
    for j in range(m):
        e = np.zeros(m)
        e[j] = 1.0
        cols.append(fn(e))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("h", [1.0, 0.25, 3.0])
def test_lemma1_load_vector_rows(h):
    g = GOLDEN["lemma1_interior_row"]
    w = [frac(s) for s in g["weights"]]
    m = 17
    X = np.arange(m) * h
    RM = _unit_columns(lambda e: oracle.restrict_1d(X, oracle.mass_apply_1d(X, e)), m)
    for J in range(1, (m + 1) // 2 - 1):
        row = np.zeros(m)
        for off, wt in zip(g["offsets"], w):
            row[2 * J + off] = wt * h
        assert np.abs(RM[J] - row).max() <= 1e-15 * 8 * h
    # end rows: the same integrals with the missing neighbours removed
    # (our reading of the garbled boundary of Lemma 1), checked densely
    assert np.abs(RM - dense_ref.mixed_mass(X[::2], X)).max() <= 1e-14 * h
    assert np.allclose(RM[0, :3], np.array([5 / 12, 1 / 2, 1 / 12]) * h, rtol=0, atol=1e-15 * h)


def test_coarse_mass_matrix_matches_printed_system():
    g = GOLDEN["coarse_mass_uniform"]
    h = 0.5
    X = np.arange(17) * h
    sub, diag, sup = oracle.coarse_mass_1d(X)
    assert diag[0] == pytest.approx(frac(g["end_diagonal"]) * h, abs=1e-15)
    assert diag[-1] == pytest.approx(frac(g["end_diagonal"]) * h, abs=1e-15)
    assert np.allclose(diag[1:-1], frac(g["interior_diagonal"]) * h, atol=1e-15, rtol=0)
    assert np.allclose(sup[:-1], frac(g["off_diagonal"]) * h, atol=1e-15, rtol=0)
    assert np.allclose(sub[1:], frac(g["off_diagonal"]) * h, atol=1e-15, rtol=0)
    assert sub[0] == 0 and sup[-1] == 0
    # and equals the exact Gram matrix of the coarse hat functions
    Mc = dense_ref.mixed_mass(X[::2], X[::2])
    T = np.diag(diag) + np.diag(sup[:-1], 1) + np.diag(sub[1:], -1)
    assert np.abs(T - Mc).max() <= 1e-15


def test_multilinear_prediction_weights():
    g = GOLDEN["multilinear_prediction_weights"]
    rng = np.random.default_rng(3)
    u = rng.standard_normal((5, 5, 5))
    v = oracle.decompose(u, None, 0)  # one step: 5^3 -> 3^3 (L = 1)
    corner = lambda *idx: u[idx]
    edge = u[0, 0, 1] - frac(g["edge"]) * (u[0, 0, 0] + u[0, 0, 2])
    plane = u[0, 1, 1] - frac(g["plane"]) * (u[0, 0, 0] + u[0, 0, 2] + u[0, 2, 0] + u[0, 2, 2])
    cube = u[1, 1, 1] - frac(g["cube"]) * sum(corner(a, b, c) for a in (0, 2) for b in (0, 2) for c in (0, 2))
    assert v[0, 0, 1] == pytest.approx(edge, abs=1e-14)
    assert v[0, 1, 1] == pytest.approx(plane, abs=1e-14)
    assert v[1, 1, 1] == pytest.approx(cube, abs=1e-14)


def test_correction_identity():
    """The correction equals Q_{l-1}u - Pi_{l-1} Q_l u restricted to N_{l-1} (Sec. 2, step 4)."""
    rng = np.random.default_rng(12)
    shape = (9, 17, 9)
    c = coords_for(shape, "random", seed=6)
    u = rng.standard_normal(shape)
    L = oracle.num_levels(shape)
    Xs = [c[k] for k in range(3)]
    Q_L1 = dense_ref.projection(u, Xs, L, L - 1)
    v = oracle.decompose(u, c, L - 1)
    lev = oracle.level_map(shape, L - 1)
    z = np.where(lev == L, v, 0.0)
    y = oracle.correction(z, c)
    nodal_interp = u[::2, ::2, ::2]  # Pi_{L-1} Q_L u agrees with u on N_{L-1}
    assert np.abs(y - (Q_L1 - nodal_interp)).max() <= 1e-13 * np.abs(u).max()


# --------------------------------------------------------------------------
# Statistics the paper reports (Sec. 4.2)
# --------------------------------------------------------------------------
def test_correction_error_statistic():
    target = GOLDEN["correction_error_std"]["value"]
    rng = np.random.default_rng(20201005)
    n = 33
    vals = []
    for _ in range(8):
        z = rng.uniform(-1.0, 1.0, (n, n, n))
        z[::2, ::2, ::2] = 0.0
        y = oracle.correction(z)
        vals.append(y[2:-2, 2:-2, 2:-2].ravel())
    std = np.concatenate(vals).std()
    assert abs(std - target) < 0.005
    # "independent of the number of nodes": a 17^3 level gives the same
    small = []
    for _ in range(16):
        z = rng.uniform(-1.0, 1.0, (17, 17, 17))
        z[::2, ::2, ::2] = 0.0
        small.append(oracle.correction(z)[2:-2, 2:-2, 2:-2].ravel())
    assert abs(np.concatenate(small).std() - target) < 0.01


def test_interpolation_penalty_factors():
    """E|P| of the corner average of nodal errors = U(-1,1) quantization error plus
    the oracle's own correction error of U(-1,1) coefficient errors."""
    g = GOLDEN["interp_penalty_factors"]
    rng = np.random.default_rng(77)
    n = 33
    corr = []
    for _ in range(6):
        z = rng.uniform(-1.0, 1.0, (n, n, n))
        z[::2, ::2, ::2] = 0.0
        corr.append(oracle.correction(z)[2:-2, 2:-2, 2:-2].ravel())
    corr = np.concatenate(corr)
    N = 400000
    for name, k in (("edge", 2), ("plane", 4), ("cube", 8)):
        eps = rng.uniform(-1, 1, (N, k)) + rng.choice(corr, size=(N, k))
        est = np.abs(eps.mean(axis=1)).mean()
        assert abs(est - g[name]) < 0.004, (name, est)


# --------------------------------------------------------------------------
# L-infinity constant, level tolerances, quantizer (Sec. 4.1)
# --------------------------------------------------------------------------
def test_axis_operator_norm_against_dense():
    for m in (5, 9, 17, 33):
        X = workloads.random_coordinates(m, seed=m)
        A = dense_ref.axis_operator_dense(X)
        assert oracle.axis_operator_norm(X) == pytest.approx(np.abs(A).sum(axis=1).max(), rel=1e-13)
    # uniform limit 1 + sqrt(3)/2
    assert oracle.axis_operator_norm(np.arange(129.0)) == pytest.approx(1 + math.sqrt(3) / 2, rel=1e-12)


@pytest.mark.parametrize("shape", [(17,), (9, 17), (9, 9, 9)])
def test_linf_constant_bounds_exact_amplification(shape):
    """Dense per-level error amplification of a coefficient perturbation never exceeds C."""
    C = oracle.linf_constant(shape)
    L = oracle.num_levels(shape)
    n = int(np.prod(shape))
    lev = oracle.level_map(shape)
    worst = 0.0
    for l in range(1, L + 1):
        cols = np.flatnonzero(lev.ravel() == l)
        E = np.zeros((n, len(cols)))
        for t, idx in enumerate(cols):
            e = np.zeros(n)
            e[idx] = 1.0
            E[:, t] = oracle.recompose(e.reshape(shape)).ravel()
        worst = max(worst, np.abs(E).sum(axis=1).max())
    assert worst <= C + 1e-12
    assert C >= 1.0


def test_level_tolerances_schedule():
    shape = (65, 65, 65)
    tau = oracle.level_tolerances(shape, 1.0)
    C = oracle.linf_constant(shape)
    kappa = math.sqrt(8.0)
    assert GOLDEN["kappa_3d"]["value"] == "sqrt(8)"
    assert np.allclose(tau[1:] / tau[:-1], kappa, rtol=1e-14)
    assert tau.sum() * C == pytest.approx(1.0, rel=1e-14)
    L = 5
    closed = [(1 - kappa) * kappa ** l / (1 - kappa ** (L + 1)) / C for l in range(L + 1)]
    assert np.allclose(tau, closed, rtol=1e-13)
    tau4 = oracle.level_tolerances((513, 513, 513), 1.0, stop_level=4, c_linf=7.5)
    assert len(tau4) == 5 and tau4.sum() * 7.5 == pytest.approx(1.0, rel=1e-14)


@pytest.mark.parametrize("stop", [0, 2])
@pytest.mark.parametrize("rel", [1e-2, 1e-3, 1e-4])
def test_linf_invariant_end_to_end(stop, rel):
    u = workloads.sinusoid_field(33, seed=3)
    tol = rel * (u.max() - u.min())
    v = oracle.decompose(u, None, stop)
    labels, code = oracle.quantize(v, tol, None, stop)
    assert code == 0
    vq = oracle.dequantize(labels, tol, None, stop)
    tau = oracle.level_tolerances(u.shape, tol, None, stop)
    lev = oracle.level_map(u.shape, stop)
    assert np.all(np.abs(v - vq) <= tau[lev - stop] * (1 + 1e-15))
    ut = oracle.recompose(vq, None, stop)
    assert np.abs(u - ut).max() <= tol


def test_linf_invariant_nonuniform():
    shape = (17, 33, 33)
    c = [workloads.tanh_coordinates(17), None, workloads.random_coordinates(33, 5)]
    rng = np.random.default_rng(4)
    u = np.exp(rng.standard_normal(shape))
    tol = 1e-3 * (u.max() - u.min())
    v = oracle.decompose(u, c)
    labels, code = oracle.quantize(v, tol, c)
    assert code == 0
    ut = oracle.recompose(oracle.dequantize(labels, tol, c), c)
    assert np.abs(u - ut).max() <= tol


def test_quantizer_rounding_and_range():
    shape = (9,)
    tau = oracle.level_tolerances(shape, 1.0, c_linf=2.0)
    lev = oracle.level_map(shape)
    q = 2 * tau[lev]
    v = np.array([0.0, 0.5, -0.5, 1.5, 2.5, 1e-300, -0.49999999999, 3.0, 7.0]) * q
    labels, code = oracle.quantize(v, 1.0, c_linf=2.0)
    assert code == 0
    assert labels.tolist() == [0, 0, 0, 2, 2, 0, 0, 3, 7]  # ties to even
    huge = np.zeros(shape)
    huge[3] = 3e9 * q[3]
    _, code = oracle.quantize(huge, 1.0, c_linf=2.0)
    assert code == 6
    nan = np.zeros(shape)
    nan[2] = np.nan
    labels, code = oracle.quantize(nan, 1.0, c_linf=2.0)
    assert code == 6 and labels[2] == np.iinfo(np.int32).min


# --------------------------------------------------------------------------
# Level-centric layout (Sec. 5.1)
# --------------------------------------------------------------------------
def test_level_centric_1d_example():
    pos = oracle.level_centric_index((9,), 0)
    # nodal (even) indices of each level move to the front, coefficients follow
    assert pos.tolist() == [0, 5, 3, 6, 1, 7, 4, 8, 2]
    pos1 = oracle.level_centric_index((9,), 1)
    assert pos1.tolist() == [0, 5, 1, 6, 2, 7, 3, 8, 4]


def test_level_centric_only_reorders_the_nodal_block():
    """Sec. 5.1: each level reorders its own grid; the coefficients of a level
    stay where that level's reordering put them (9x9, two levels)."""
    pos = oracle.level_centric_index((9, 9), 0)
    def at(p):
        return divmod(int(p), 9)
    # level-2 coefficient in a nodal row (row 2 even, column 1 odd): row 2 -> 1,
    # column 1 -> 5 + 0; the level-1 reordering does not move it again
    assert at(pos[2, 1]) == (1, 5)
    assert at(pos[1, 2]) == (5, 1)
    assert at(pos[3, 3]) == (6, 6)
    # level-1 coefficient (level-1 indices (1, 2)): rows/cols of the 5x5 level-1 box
    assert at(pos[2, 4]) == (3, 1)
    # coarsest grid N_0 = {0, 4, 8}^2 in natural order in the 3x3 corner
    assert at(pos[4, 8]) == (1, 2)
    # a permutation
    assert sorted(pos.ravel().tolist()) == list(range(81))


@pytest.mark.parametrize("shape,stop", [((17, 9, 33), 0), ((33, 33), 1), ((9, 9, 9), 2)])
def test_level_centric_boxes(shape, stop):
    lev = oracle.level_map(shape, stop)
    lc = oracle.to_level_centric(lev, stop)
    L = oracle.num_levels(shape)
    for l in range(stop, L + 1):
        box = tuple(slice(0, (n - 1) // 2 ** (L - l) + 1) for n in shape)
        inside = np.zeros(shape, dtype=bool)
        inside[box] = True
        assert np.all(lc[inside] <= l) and np.all(lc[~inside] > l)
    a = np.arange(np.prod(shape)).reshape(shape)
    assert np.array_equal(oracle.from_level_centric(oracle.to_level_centric(a, stop), stop), a)


def test_input_validation():
    with pytest.raises(oracle.OracleError):
        oracle.decompose(np.zeros((6, 5)))
    with pytest.raises(oracle.OracleError):
        oracle.decompose(np.zeros((5, 5)), [np.array([0, 1, 1, 2, 3.0]), None])
    with pytest.raises(oracle.OracleError):
        oracle.decompose(np.zeros((5, 5)), None, 2)
    with pytest.raises(oracle.OracleError):
        oracle.level_tolerances((5, 5), -1.0)
