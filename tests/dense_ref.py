"""Dense brute-force L2 projections on tiny grids: an independent check of the oracle.

Nothing here reuses the oracle's formulas.  Mass matrices come from Gauss
quadrature of products of hat functions, interpolation from ``numpy.interp``,
and projections from dense ``numpy.linalg.solve``.  The definitions are those
of Sec. 2 of the paper: Q_l is the L2 projection onto the piecewise
multilinear space V_l on N_l, Pi_{l-1} interpolates from N_{l-1}, and the
multilevel coefficient of x in N*_l is ((I - Pi_{l-1}) Q_l u)(x).
"""
from __future__ import annotations

import numpy as np

_GAUSS_T = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])


def hat(nodes: np.ndarray, J: int, x: np.ndarray) -> np.ndarray:
    e = np.zeros(len(nodes))
    e[J] = 1.0
    return np.interp(x, nodes, e)


def mixed_mass(coarse: np.ndarray, fine: np.ndarray) -> np.ndarray:
    """B[J, j] = integral of phi_J^coarse * psi_j^fine, exact (2-point Gauss on fine cells)."""
    B = np.zeros((len(coarse), len(fine)))
    for i in range(len(fine) - 1):
        a, b = fine[i], fine[i + 1]
        xs = a + (b - a) * _GAUSS_T
        wq = 0.5 * (b - a)
        psi = [hat(fine, j, xs) for j in (i, i + 1)]
        for J in range(len(coarse)):
            phi = hat(coarse, J, xs)
            if not phi.any():
                continue
            for t, j in enumerate((i, i + 1)):
                B[J, j] += wq * float(np.dot(phi, psi[t]))
    return B


def tensor_apply(mats, u: np.ndarray) -> np.ndarray:
    """Apply one matrix per axis (matrix k acts on axis k)."""
    out = u
    for k, A in enumerate(mats):
        out = np.moveaxis(np.tensordot(A, out, axes=([1], [k])), 0, k)
    return out


def level_coords(X, L, l):
    return np.asarray(X)[:: 2 ** (L - l)]


def projection(u, Xs, L, l):
    """Q_l u for the fine interpolant u on N_L, as values on N_l."""
    mats = []
    for X in Xs:
        Y = level_coords(X, L, l)
        Ml = mixed_mass(Y, Y)
        B = mixed_mass(Y, np.asarray(X))
        mats.append(np.linalg.solve(Ml, B))
    return tensor_apply(mats, u)


def interpolate(vals_coarse, Xs, L, lc, lf):
    """Multilinear interpolation of values on N_lc to the nodes of N_lf."""
    mats = []
    for X in Xs:
        Yc = level_coords(X, L, lc)
        Yf = level_coords(X, L, lf)
        mats.append(np.stack([hat(Yc, J, Yf) for J in range(len(Yc))], axis=1))
    return tensor_apply(mats, vals_coarse)


def num_levels(shape):
    return min(int(np.log2(n - 1)) for n in shape) - 1


def dense_decompose(u, coords=None, stop_level=0):
    """Interleaved u_mc by the plain definition of Sec. 2."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    Xs = [np.arange(n, dtype=np.float64) if (coords is None or coords[k] is None)
          else np.asarray(coords[k], dtype=np.float64) for k, n in enumerate(shape)]
    L = num_levels(shape)
    out = np.zeros_like(u)
    for l in range(L, stop_level, -1):
        Ql = projection(u, Xs, L, l)
        nodal = Ql[tuple(slice(0, None, 2) for _ in shape)]
        interp = interpolate(nodal, Xs, L, l - 1, l)
        coeff = Ql - interp
        s = 2 ** (L - l)
        sub = out[tuple(slice(0, None, s) for _ in shape)]
        odd = np.zeros(Ql.shape, dtype=bool)
        for k in range(len(shape)):
            idx = [np.newaxis] * len(shape)
            idx[k] = slice(None)
            odd |= (np.arange(Ql.shape[k]) % 2 == 1)[tuple(idx)]
        sub[odd] = coeff[odd]
        out[tuple(slice(0, None, s) for _ in shape)] = sub
    s = 2 ** (L - stop_level)
    out[tuple(slice(0, None, s) for _ in shape)] = projection(u, Xs, L, stop_level)
    return out


def axis_operator_dense(X):
    """The 1-D correction operator Mc^{-1} R M on a line with nodes X (dense)."""
    X = np.asarray(X, dtype=np.float64)
    Y = X[::2]
    Mc = mixed_mass(Y, Y)
    B = mixed_mass(Y, X)  # equals R M: integrals of coarse hats against fine hats
    return np.linalg.solve(Mc, B)
