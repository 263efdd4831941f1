"""ctypes binding of the plain FP64 CPU oracle (``oracle/mgard_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle follows the paper (arXiv 2010.05872)
step by step: decomposition and recomposition of Sec. 2, the level-centric
reordering of Sec. 5.1, and the level-wise quantization of Sec. 4.1.  Only
the test suite, ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import this package; the product library never does.

All arrays are numpy float64 (int32 for labels), C order, interleaved layout
(indexed by the finest-grid node), unless stated otherwise.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mgard_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libmgard_oracle.so")

ERRORS = {0: "ok", 2: "shape", 3: "coords", 4: "level", 5: "tol", 6: "range", 9: "alloc"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: error {code} ({ERRORS.get(code, '?')})")
        self.code = code


def build() -> str:
    """Compile the oracle with gcc (plain C99, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
           _SRC, "-o", _LIB_PATH + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        vp = ctypes.c_void_p
        L.mgo_num_levels.argtypes = [ctypes.c_int, i64p]
        for name in ("mgo_decompose", "mgo_recompose", "mgo_decompose_adjoint", "mgo_recompose_adjoint"):
            getattr(L, name).argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.c_int]
        L.mgo_recompose_to.argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.c_int, ctypes.c_int]
        L.mgo_adaptive_estimate.argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.c_int, dp, dp, i64p]
        L.mgo_adaptive_errors.argtypes = [ctypes.c_double, ctypes.c_double, i64p, ctypes.c_double, dp, dp]
        L.mgo_adaptive_errors.restype = None
        L.mgo_decompose_adaptive.argtypes = [vp, ctypes.c_int, i64p, vp, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(ctypes.c_int)]
        L.mgo_project_line_adjoint_1d.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.mgo_correction.argtypes = [vp, vp, ctypes.c_int, i64p, vp]
        L.mgo_mass_apply_1d.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.mgo_restrict_1d.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.mgo_coarse_mass_1d.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
        L.mgo_project_line_1d.argtypes = [vp, ctypes.c_int64, vp, vp]
        L.mgo_axis_operator_norm.argtypes = [vp, ctypes.c_int64]
        L.mgo_axis_operator_norm.restype = ctypes.c_double
        L.mgo_level_map.argtypes = [vp, ctypes.c_int, i64p, ctypes.c_int]
        L.mgo_level_centric_index.argtypes = [vp, ctypes.c_int, i64p, ctypes.c_int]
        L.mgo_linf_constant.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_int]
        L.mgo_linf_constant.restype = ctypes.c_double
        L.mgo_level_tolerances.argtypes = [ctypes.c_int, i64p, vp, ctypes.c_double, ctypes.c_int,
                                           ctypes.c_double, dp]
        for name in ("mgo_quantize", "mgo_dequantize"):
            getattr(L, name).argtypes = [vp, vp, ctypes.c_int, i64p, vp, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_double]
        _lib = L
    return _lib


def _dims(shape):
    arr = (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])
    return arr


class _Coords:
    """Keeps the per-axis coordinate arrays alive for one call."""

    def __init__(self, shape, coords):
        self.keep = []
        if coords is None:
            self.ptr = None
            return
        if len(coords) != len(shape):
            raise ValueError("coords must have one entry per axis")
        ptrs = (ctypes.c_void_p * len(shape))()
        for k, c in enumerate(coords):
            if c is None:
                ptrs[k] = None
                continue
            a = np.ascontiguousarray(c, dtype=np.float64)
            if a.shape != (shape[k],):
                raise ValueError(f"coords[{k}] must have {shape[k]} entries")
            self.keep.append(a)
            ptrs[k] = a.ctypes.data
        self.keep.append(ptrs)
        self.ptr = ctypes.cast(ptrs, ctypes.c_void_p)


def _check(code, what):
    if code != 0:
        raise OracleError(code, what)


def num_levels(shape) -> int:
    r = lib().mgo_num_levels(len(shape), _dims(shape))
    if r < 0:
        raise OracleError(-r, "num_levels")
    return r


def decompose(u, coords=None, stop_level=0) -> np.ndarray:
    """Interleaved u_mc of u (float64 copy), Sec. 2 decomposition."""
    v = np.array(u, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    _check(lib().mgo_decompose(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(stop_level)), "decompose")
    return v


def recompose(u_mc, coords=None, stop_level=0) -> np.ndarray:
    v = np.array(u_mc, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    _check(lib().mgo_recompose(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(stop_level)), "recompose")
    return v


def recompose_to(u_mc, target_level, coords=None, stop_level=0) -> np.ndarray:
    """Progressive recomposition (recomposition of Sec. 2 stopped after level
    target_level): Q_target u on the level-target grid, as a compact array."""
    v = np.array(u_mc, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    _check(lib().mgo_recompose_to(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(stop_level),
                                  int(target_level)), "recompose_to")
    L = num_levels(v.shape)
    s = 2 ** (L - int(target_level))
    return np.ascontiguousarray(v[tuple(slice(None, None, s) if n > 1 else slice(None) for n in v.shape)])


def dyadic_shape(shape):
    """Every axis to the next 2^m + 1 >= n (m >= 1): the dummy-node padding of
    non-dyadic sizes (Sec. 6.2.2)."""
    out = []
    for n in shape:
        if n < 2:
            raise OracleError(2, "dyadic_shape")
        m = 1
        while 2 ** m + 1 < n:
            m += 1
        out.append(2 ** m + 1)
    return tuple(out)


def pad_to_dyadic(u):
    """Dummy nodes after the last real node of every axis, each with the value
    of the nearest real node."""
    u = np.asarray(u, dtype=np.float64)
    return np.pad(u, [(0, p - n) for n, p in zip(u.shape, dyadic_shape(u.shape))], mode="edge")


def _axis_coords(shape, coords):
    return [np.arange(n, dtype=np.float64) if (coords is None or coords[k] is None)
            else np.asarray(coords[k], dtype=np.float64) for k, n in enumerate(shape)]


def l2_constant(shape, coords=None, stop_level=0) -> float:
    """A computable C_L2 for the L2 estimator of Sec. 4.1 (the paper cites the
    constant without printing it).  The quantization error of level l lives in
    the piecewise multilinear space of N_l: its recomposed error is
    (I - Q_{l-1}) e_l for l > stop (e_l interpolating the level's coefficient
    errors, zero on N_{l-1}) and e_stop itself on the stop box.  These pieces
    are L2-orthogonal across levels and I - Q_{l-1} does not increase the L2
    norm, so ||u - u~||^2 <= sum_l ||e_l||^2 <= sum_l lambda_max(M_l) |delta_l|^2
    with M_l the level's mass matrix.  lambda_max(M_l) is bounded by the
    product over the axes of the largest row sum of the 1-D mass matrix,
    max_j (h_{j-1} + h_j) / 2, so the estimator holds with
    C = max_l prod_k rowsum_k(l) / h_l^d, h_l^d the cell volume of reading
    15 (extent / intervals per axis).  Equal to 1 on uniform grids."""
    L = num_levels(shape)
    Xs = _axis_coords(shape, coords)
    best = 0.0
    for l in range(int(stop_level), L + 1):
        ratio = 1.0
        for X, n in zip(Xs, shape):
            Y = X[:: 2 ** (L - l)]
            h = np.diff(Y)
            rows = np.concatenate(([h[0]], h[:-1] + h[1:], [h[-1]])) / 2.0
            ratio *= rows.max() / ((Y[-1] - Y[0]) / (len(Y) - 1))
        best = max(best, ratio)
    return float(best)


def level_tolerances_l2(shape, tol_l2, c_l2=0.0, coords=None, stop_level=0) -> np.ndarray:
    """L2 variant of Sec. 4.1: tau_l = tol / sqrt(C_L2 h_l^d #N_L), h_l^d the level's
    cell volume (extent / intervals per axis), levels stop_level .. L.
    c_l2 <= 0 takes l2_constant(...)."""
    L = num_levels(shape)
    Xs = _axis_coords(shape, coords)
    if c_l2 <= 0.0:
        c_l2 = l2_constant(shape, coords, stop_level)
    nL = float(np.prod(shape))
    out = []
    for l in range(int(stop_level), L + 1):
        hd = 1.0
        for X, n in zip(Xs, shape):
            m = (n - 1) // 2 ** (L - l) + 1
            hd = hd * ((X[-1] - X[0]) / (m - 1))
        out.append(tol_l2 / np.sqrt(c_l2 * hd * nL))
    return np.array(out)


def quantize_levels(u_mc, tau, stop_level=0):
    """Labels rint(c / (2 tau_l)) with caller-given per-level tolerances (FP64;
    interleaved layout in and out)."""
    v = np.asarray(u_mc, dtype=np.float64)
    lev = level_map(v.shape, stop_level)
    q = 2.0 * np.asarray(tau, dtype=np.float64)[lev - int(stop_level)]
    return np.rint(v / q).astype(np.int32)


def dequantize_levels(labels, tau, stop_level=0):
    lab = np.asarray(labels)
    lev = level_map(lab.shape, stop_level)
    return lab.astype(np.float64) * (2.0 * np.asarray(tau, dtype=np.float64)[lev - int(stop_level)])


def label_entropy(labels, stop_level=0):
    """Shannon entropy in bits per label of each level's labels (Sec. 4.1),
    interleaved layout."""
    lab = np.asarray(labels)
    lev = level_map(lab.shape, stop_level)
    L = num_levels(lab.shape)
    out = []
    for l in range(int(stop_level), L + 1):
        _, counts = np.unique(lab[lev == l], return_counts=True)
        p = counts / counts.sum()
        out.append(float(-(p * np.log2(p)).sum()))
    return np.array(out)


PENALTY = {"lorenzo": 1.22, "edge": 0.369, "plane": 0.259, "cube": 0.182}  # Sec. 4.2, units of tau


def adaptive_estimate(v, level, coords=None):
    """Sums of |u - Lorenzo| and |u - interpolant| over the coefficient nodes
    of the sampled 3^3 blocks of level `level` (cells a % 4 == 1 per axis) of
    the interleaved array v (holding Q_level u), and the sampled edge, plane
    and cube counts.  Sec. 4.2, Alg. 1 lines 4-9."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    c = _Coords(v.shape, coords)
    sl, si = ctypes.c_double(), ctypes.c_double()
    cnt = np.zeros(3, dtype=np.int64)
    _check(lib().mgo_adaptive_estimate(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(level),
                                       ctypes.byref(sl), ctypes.byref(si),
                                       cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "adaptive_estimate")
    return sl.value, si.value, cnt


def adaptive_errors(s_lorenzo, s_interp, counts, tau0):
    """(E_Lorenzo, E_interp): the sums plus the penalty factors times tau0."""
    cnt = np.ascontiguousarray(counts, dtype=np.int64)
    el, ei = ctypes.c_double(), ctypes.c_double()
    lib().mgo_adaptive_errors(float(s_lorenzo), float(s_interp), cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                              float(tau0), ctypes.byref(el), ctypes.byref(ei))
    return el.value, ei.value


def decompose_adaptive(u, tol, coords=None, c_linf=0.0):
    """Adaptive decomposition (Alg. 1 lines 1-16): (interleaved u_mc, stop level)."""
    v = np.array(u, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    stop = ctypes.c_int(-1)
    _check(lib().mgo_decompose_adaptive(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, float(tol), float(c_linf),
                                        ctypes.byref(stop)), "decompose_adaptive")
    return v, stop.value


def decompose_adjoint(g_mc, coords=None, stop_level=0) -> np.ndarray:
    """D^T applied to an interleaved coefficient-space array (transpose of
    decompose; not in the paper)."""
    v = np.array(g_mc, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    _check(lib().mgo_decompose_adjoint(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(stop_level)),
           "decompose_adjoint")
    return v


def recompose_adjoint(g_u, coords=None, stop_level=0) -> np.ndarray:
    """R^T applied to a field-space array; returns interleaved coefficient space."""
    v = np.array(g_u, dtype=np.float64, order="C", copy=True)
    c = _Coords(v.shape, coords)
    _check(lib().mgo_recompose_adjoint(v.ctypes.data, v.ndim, _dims(v.shape), c.ptr, int(stop_level)),
           "recompose_adjoint")
    return v


def project_line_adjoint_1d(X, y):
    X = np.ascontiguousarray(X, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty(len(X))
    lib().mgo_project_line_adjoint_1d(X.ctypes.data, len(X), y.ctypes.data, out.ctypes.data)
    return out


def correction(z, coords=None) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.float64)
    out_shape = tuple((n + 1) // 2 for n in z.shape)
    y = np.empty(out_shape, dtype=np.float64)
    c = _Coords(z.shape, coords)
    _check(lib().mgo_correction(z.ctypes.data, y.ctypes.data, z.ndim, _dims(z.shape), c.ptr), "correction")
    return y


def mass_apply_1d(X, g):
    X = np.ascontiguousarray(X, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.empty_like(g)
    lib().mgo_mass_apply_1d(X.ctypes.data, len(X), g.ctypes.data, out.ctypes.data)
    return out


def restrict_1d(X, g):
    X = np.ascontiguousarray(X, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    f = np.empty((len(X) + 1) // 2)
    lib().mgo_restrict_1d(X.ctypes.data, len(X), g.ctypes.data, f.ctypes.data)
    return f


def coarse_mass_1d(X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    mc = (len(X) + 1) // 2
    sub, diag, sup = np.empty(mc), np.empty(mc), np.empty(mc)
    lib().mgo_coarse_mass_1d(X.ctypes.data, len(X), sub.ctypes.data, diag.ctypes.data, sup.ctypes.data)
    return sub, diag, sup


def project_line_1d(X, z):
    X = np.ascontiguousarray(X, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64)
    y = np.empty((len(X) + 1) // 2)
    lib().mgo_project_line_1d(X.ctypes.data, len(X), z.ctypes.data, y.ctypes.data)
    return y


def axis_operator_norm(X) -> float:
    X = np.ascontiguousarray(X, dtype=np.float64)
    return lib().mgo_axis_operator_norm(X.ctypes.data, len(X))


def level_map(shape, stop_level=0) -> np.ndarray:
    lev = np.empty(shape, dtype=np.int8)
    _check(lib().mgo_level_map(lev.ctypes.data, len(shape), _dims(shape), int(stop_level)), "level_map")
    return lev


def level_centric_index(shape, stop_level=0) -> np.ndarray:
    pos = np.empty(shape, dtype=np.int64)
    _check(lib().mgo_level_centric_index(pos.ctypes.data, len(shape), _dims(shape), int(stop_level)),
           "level_centric_index")
    return pos


def to_level_centric(a, stop_level=0) -> np.ndarray:
    """Sec. 5.1 reordering of an interleaved array (any dtype)."""
    a = np.ascontiguousarray(a)
    pos = level_centric_index(a.shape, stop_level).ravel()
    out = np.empty(a.size, dtype=a.dtype)
    out[pos] = a.ravel()
    return out.reshape(a.shape)


def from_level_centric(a, stop_level=0) -> np.ndarray:
    a = np.ascontiguousarray(a)
    pos = level_centric_index(a.shape, stop_level).ravel()
    return a.ravel()[pos].reshape(a.shape)


def linf_constant(shape, coords=None, stop_level=0) -> float:
    c = _Coords(shape, coords)
    r = lib().mgo_linf_constant(len(shape), _dims(shape), c.ptr, int(stop_level))
    if r < 0:
        raise OracleError(1, "linf_constant")
    return r


def level_tolerances(shape, tol, coords=None, stop_level=0, c_linf=0.0) -> np.ndarray:
    L = num_levels(shape)
    tau = np.empty(L + 1 - stop_level, dtype=np.float64)
    c = _Coords(shape, coords)
    _check(lib().mgo_level_tolerances(len(shape), _dims(shape), c.ptr, float(tol), int(stop_level),
                                      float(c_linf), tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "level_tolerances")
    return tau


def quantize(u_mc, tol, coords=None, stop_level=0, c_linf=0.0):
    """Labels (int32, interleaved) and the status code (0 or 6 = range)."""
    v = np.ascontiguousarray(u_mc, dtype=np.float64)
    labels = np.empty(v.shape, dtype=np.int32)
    c = _Coords(v.shape, coords)
    code = lib().mgo_quantize(v.ctypes.data, labels.ctypes.data, v.ndim, _dims(v.shape), c.ptr,
                              float(tol), int(stop_level), float(c_linf))
    if code not in (0, 6):
        raise OracleError(code, "quantize")
    return labels, code


def dequantize(labels, tol, coords=None, stop_level=0, c_linf=0.0) -> np.ndarray:
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.empty(lab.shape, dtype=np.float64)
    c = _Coords(lab.shape, coords)
    _check(lib().mgo_dequantize(lab.ctypes.data, out.ctypes.data, lab.ndim, _dims(lab.shape), c.ptr,
                                float(tol), int(stop_level), float(c_linf)), "dequantize")
    return out
