"""mgx: MGARD+ multilevel decomposition on MI355X — Python binding of libmgx.

Thin ctypes layer over the C ABI of ``include/mgx.h``: it marshals torch
tensors (device memory) and the current HIP stream into the C calls and
raises ``MgxError`` on a non-zero status.  Every step of the computation runs
in the HIP kernels of ``libmgx.so``; there is no Python or CPU fallback, and
importing the compute functions fails loudly when the library is not built.

Method: "MGARD+: Optimizing Multilevel Methods for Error-bounded Scientific
Data Reduction" (arXiv 2010.05872).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmgx.so")

MGX_F32, MGX_F64 = 0, 1
MAX_LEVELS = 16

STATUS = {
    0: "MGX_OK", 1: "MGX_ERR_ARG", 2: "MGX_ERR_SHAPE", 3: "MGX_ERR_COORDS", 4: "MGX_ERR_LEVEL",
    5: "MGX_ERR_TOL", 6: "MGX_ERR_RANGE", 7: "MGX_ERR_WORKSPACE", 8: "MGX_ERR_HIP",
}


class MgxError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = lib().mgx_status_string(code).decode() if _lib is not None else ""
        super().__init__(f"{what}: {STATUS.get(code, code)} ({msg})")
        self.code = code


class QuantStats(ctypes.Structure):
    _fields_ = [
        ("first_level", ctypes.c_int32),
        ("num_levels", ctypes.c_int32),
        ("max_abs_label", ctypes.c_int32 * MAX_LEVELS),
        ("n_overflow", ctypes.c_int64),
        ("n_nonfinite", ctypes.c_int64),
    ]

    def as_dict(self):
        return {
            "first_level": self.first_level,
            "num_levels": self.num_levels,
            "max_abs_label": list(self.max_abs_label[: self.num_levels]),
            "n_overflow": self.n_overflow,
            "n_nonfinite": self.n_nonfinite,
        }


class Field(ctypes.Structure):
    """mgx_field of include/mgx.h."""
    _fields_ = [
        ("in_", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("dtype", ctypes.c_int),
        ("ndim", ctypes.c_int),
        ("dims", ctypes.c_int64 * 3),
        ("coords", ctypes.c_void_p * 3),
        ("stop_level", ctypes.c_int),
        ("tol_linf", ctypes.c_double),
        ("c_linf", ctypes.c_double),
        ("labels", ctypes.c_void_p),
        ("coef", ctypes.c_void_p),
        ("stats", ctypes.c_void_p),
    ]


class BatchInfo(ctypes.Structure):
    _fields_ = [
        ("launches", ctypes.c_int),
        ("target_blocks", ctypes.c_int),
        ("min_zchunk", ctypes.c_int),
        ("tuned_ms", ctypes.c_double),
        ("tune_source", ctypes.c_int),
    ]


class KernelTime(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 40),
        ("level", ctypes.c_int32),
        ("count", ctypes.c_int32),
        ("total_ms", ctypes.c_double),
    ]


# Every symbol declared in include/mgx.h.
EXPORTS = (
    "mgx_status_string", "mgx_num_levels", "mgx_workspace_size", "mgx_decompose", "mgx_recompose",
    "mgx_quantize", "mgx_dequantize", "mgx_linf_constant", "mgx_level_tolerances",
    "mgx_trace_enable", "mgx_trace_read", "mgx_adjoint_workspace_size", "mgx_decompose_adjoint",
    "mgx_recompose_adjoint", "mgx_batch_workspace_size", "mgx_decompose_batched", "mgx_recompose_batched",
    "mgx_batch_set_autotune", "mgx_batch_last_info", "mgx_decompose_quantize", "mgx_dequantize_recompose",
    "mgx_recompose_to", "mgx_decompose_adaptive", "mgx_adaptive_estimate", "mgx_adaptive_workspace_size",
    "mgx_dyadic_dims", "mgx_pad", "mgx_crop", "mgx_l2_constant", "mgx_level_tolerances_l2", "mgx_quantize_levels",
    "mgx_dequantize_levels", "mgx_label_entropy", "mgx_label_entropy_workspace_size", "mgx_decompose_noalloc",
    "mgx_release_cached", "mgx_label_entropy_bounded",
)

_lib = None


def lib():
    """Load libmgx.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2010_05872_amd/build.py "
                              "(or __graft_entry__.build()); there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64p, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        ci, cd, sz = ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        L.mgx_status_string.argtypes = [ci]
        L.mgx_status_string.restype = ctypes.c_char_p
        L.mgx_num_levels.argtypes = [ci, i64p]
        L.mgx_num_levels.restype = ci
        L.mgx_workspace_size.argtypes = [ci, ci, i64p, ci]
        L.mgx_workspace_size.restype = sz
        L.mgx_decompose_quantize.argtypes = [vp, vp, vp, ci, ci, i64p, vp, cd, ci, cd, vp, sz, vp, vp]
        L.mgx_decompose_quantize.restype = ci
        L.mgx_dequantize_recompose.argtypes = [vp, vp, vp, ci, ci, i64p, vp, cd, ci, cd, vp, sz, vp]
        L.mgx_dequantize_recompose.restype = ci
        L.mgx_recompose_to.argtypes = [vp, vp, ci, ci, i64p, vp, ci, ci, vp, sz, vp]
        L.mgx_recompose_to.restype = ci
        L.mgx_decompose_adaptive.argtypes = [vp, vp, ci, ci, i64p, vp, cd, cd, ctypes.POINTER(ci), vp, sz, vp]
        L.mgx_decompose_adaptive.restype = ci
        L.mgx_adaptive_estimate.argtypes = [vp, ci, ci, i64p, vp, ci, dp, i64p, vp, sz, vp]
        L.mgx_adaptive_estimate.restype = ci
        L.mgx_adaptive_workspace_size.argtypes = [ci, i64p]
        L.mgx_adaptive_workspace_size.restype = sz
        L.mgx_decompose_noalloc.argtypes = [vp, vp, ci, ci, i64p, vp, ci, vp]
        L.mgx_decompose_noalloc.restype = ci
        L.mgx_l2_constant.argtypes = [ci, i64p, vp, ci]
        L.mgx_l2_constant.restype = cd
        L.mgx_level_tolerances_l2.argtypes = [ci, i64p, vp, cd, ci, cd, dp]
        L.mgx_level_tolerances_l2.restype = ci
        L.mgx_quantize_levels.argtypes = [vp, vp, ci, ci, i64p, vp, ci, dp, vp, vp]
        L.mgx_quantize_levels.restype = ci
        L.mgx_dequantize_levels.argtypes = [vp, vp, ci, ci, i64p, vp, ci, dp, vp]
        L.mgx_dequantize_levels.restype = ci
        L.mgx_label_entropy.argtypes = [vp, ci, i64p, ci, dp, vp, sz, vp]
        L.mgx_label_entropy.restype = ci
        L.mgx_label_entropy_bounded.argtypes = [vp, ci, i64p, ci, vp, dp, vp, sz, vp]
        L.mgx_label_entropy_bounded.restype = ci
        L.mgx_label_entropy_workspace_size.argtypes = [ci, i64p, ci]
        L.mgx_label_entropy_workspace_size.restype = sz
        L.mgx_dyadic_dims.argtypes = [ci, i64p, i64p]
        L.mgx_dyadic_dims.restype = ci
        for name in ("mgx_pad", "mgx_crop"):
            getattr(L, name).argtypes = [vp, vp, ci, ci, i64p, vp]
            getattr(L, name).restype = ci
        L.mgx_adjoint_workspace_size.argtypes = [ci, ci, i64p, ci]
        L.mgx_adjoint_workspace_size.restype = sz
        for name in ("mgx_decompose", "mgx_recompose", "mgx_decompose_adjoint", "mgx_recompose_adjoint"):
            f = getattr(L, name)
            f.argtypes = [vp, vp, ci, ci, i64p, vp, ci, vp, sz, vp]
            f.restype = ci
        fp = ctypes.POINTER(Field)
        L.mgx_batch_workspace_size.argtypes = [ci, fp]
        L.mgx_batch_workspace_size.restype = sz
        for name in ("mgx_decompose_batched", "mgx_recompose_batched"):
            f = getattr(L, name)
            f.argtypes = [ci, fp, vp, sz, vp]
            f.restype = ci
        L.mgx_release_cached.argtypes = []
        L.mgx_release_cached.restype = ci
        L.mgx_batch_set_autotune.argtypes = [ci]
        L.mgx_batch_set_autotune.restype = ci
        L.mgx_batch_last_info.argtypes = [ctypes.POINTER(BatchInfo)]
        L.mgx_batch_last_info.restype = ci
        L.mgx_quantize.argtypes = [vp, vp, ci, ci, i64p, vp, cd, ci, cd, ctypes.POINTER(QuantStats), vp]
        L.mgx_quantize.restype = ci
        L.mgx_dequantize.argtypes = [vp, vp, ci, ci, i64p, vp, cd, ci, cd, vp]
        L.mgx_dequantize.restype = ci
        L.mgx_linf_constant.argtypes = [ci, i64p, vp, ci]
        L.mgx_linf_constant.restype = cd
        L.mgx_level_tolerances.argtypes = [ci, i64p, vp, cd, ci, cd, dp]
        L.mgx_level_tolerances.restype = ci
        L.mgx_trace_enable.argtypes = [ci]
        L.mgx_trace_enable.restype = ci
        L.mgx_trace_read.argtypes = [ctypes.POINTER(KernelTime), ci]
        L.mgx_trace_read.restype = ci
        _lib = L
    return _lib


def _dims(shape):
    return (ctypes.c_int64 * len(shape))(*[int(s) for s in shape])


class Coords:
    """Per-axis coordinate arrays as the ``const double *const *`` of the C ABI."""

    def __init__(self, shape, coords):
        self._keep = []
        self.ptr = None
        if coords is None:
            return
        if len(coords) != len(shape):
            raise ValueError("coords needs one entry (array or None) per axis")
        arr = (ctypes.c_void_p * len(shape))()
        for k, c in enumerate(coords):
            if c is None:
                arr[k] = None
                continue
            a = np.ascontiguousarray(np.asarray(c, dtype=np.float64))
            if a.shape != (int(shape[k]),):
                raise ValueError(f"coords[{k}] must have {shape[k]} entries")
            self._keep.append(a)
            arr[k] = a.ctypes.data
        self._keep.append(arr)
        self.ptr = ctypes.cast(arr, ctypes.c_void_p)


def _check(code, what):
    if code != 0:
        raise MgxError(code, what)


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return MGX_F32
    if t.dtype == torch.float64:
        return MGX_F64
    raise TypeError(f"unsupported dtype {t.dtype}; float32 and float64 are supported")


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _check_tensor(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


# ---------------------------------------------------------------- host utilities
def num_levels(shape) -> int:
    r = lib().mgx_num_levels(len(shape), _dims(shape))
    if r < 0:
        raise MgxError(-r, "mgx_num_levels")
    return r


def workspace_size(dtype_code: int, shape, stop_level: int = 0) -> int:
    return int(lib().mgx_workspace_size(dtype_code, len(shape), _dims(shape), int(stop_level)))


def adjoint_workspace_size(dtype_code: int, shape, stop_level: int = 0) -> int:
    return int(lib().mgx_adjoint_workspace_size(dtype_code, len(shape), _dims(shape), int(stop_level)))


def linf_constant(shape, coords=None, stop_level=0) -> float:
    c = Coords(shape, coords)
    r = lib().mgx_linf_constant(len(shape), _dims(shape), c.ptr, int(stop_level))
    if r < 0:
        raise MgxError(1, "mgx_linf_constant")
    return r


def level_tolerances(shape, tol, coords=None, stop_level=0, c_linf=0.0) -> np.ndarray:
    L = num_levels(shape)
    tau = np.zeros(L + 1 - int(stop_level), dtype=np.float64)
    c = Coords(shape, coords)
    code = lib().mgx_level_tolerances(len(shape), _dims(shape), c.ptr, float(tol), int(stop_level),
                                      float(c_linf), tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(code, "mgx_level_tolerances")
    return tau


def trace_enable(on: bool = True) -> None:
    """Bracket every library kernel launch with HIP events on its stream."""
    _check(lib().mgx_trace_enable(1 if on else 0), "mgx_trace_enable")


def trace_read(max_entries: int = 512):
    """Aggregated kernel times since the last read: list of dicts
    {name, level, count, total_ms}; waits for the recorded events."""
    buf = (KernelTime * max_entries)()
    n = lib().mgx_trace_read(buf, max_entries)
    if n < 0:
        raise MgxError(8, "mgx_trace_read")
    return [{"name": buf[i].name.decode(), "level": buf[i].level, "count": buf[i].count,
             "total_ms": buf[i].total_ms} for i in range(n)]


# ---------------------------------------------------------------- device entry points
def _workspace(t, stop_level, workspace):
    import torch
    need = workspace_size(_dtype_code(t), t.shape, stop_level)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=t.device)
    return workspace, need


def decompose(u, coords=None, stop_level=0, out=None, workspace=None):
    """u (natural order) -> u_mc (level-centric layout), on the current stream."""
    import torch
    _check_tensor(u, "u")
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out")
    ws, _ = _workspace(u, stop_level, workspace)
    c = Coords(u.shape, coords)
    code = lib().mgx_decompose(u.data_ptr(), out.data_ptr(), _dtype_code(u), u.dim(), _dims(u.shape), c.ptr,
                               int(stop_level), ws.data_ptr(), ws.numel() * ws.element_size(), _stream(u.device))
    _check(code, "mgx_decompose")
    return out


def decompose_noalloc(u, coords=None, stop_level=0, out=None):
    """decompose() through mgx_decompose_noalloc: the library's static device
    array holds the tables and the workspace (no device allocation in the
    library; out, when None, is allocated here by torch)."""
    import torch
    _check_tensor(u, "u")
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out")
    c = Coords(u.shape, coords)
    code = lib().mgx_decompose_noalloc(u.data_ptr(), out.data_ptr(), _dtype_code(u), u.dim(), _dims(u.shape), c.ptr,
                                       int(stop_level), _stream(u.device))
    _check(code, "mgx_decompose_noalloc")
    return out


def recompose(u_mc, coords=None, stop_level=0, out=None, workspace=None):
    """u_mc (level-centric layout) -> u (natural order), on the current stream."""
    import torch
    _check_tensor(u_mc, "u_mc")
    if out is None:
        out = torch.empty_like(u_mc)
    _check_tensor(out, "out")
    ws, _ = _workspace(u_mc, stop_level, workspace)
    c = Coords(u_mc.shape, coords)
    code = lib().mgx_recompose(u_mc.data_ptr(), out.data_ptr(), _dtype_code(u_mc), u_mc.dim(), _dims(u_mc.shape),
                               c.ptr, int(stop_level), ws.data_ptr(), ws.numel() * ws.element_size(),
                               _stream(u_mc.device))
    _check(code, "mgx_recompose")
    return out


def level_shape(shape, level):
    """Node counts of the level-`level` grid of a field of this shape."""
    L = num_levels(shape)
    if not 0 <= level <= L:
        raise ValueError(f"level {level} outside [0, {L}]")
    return tuple((n - 1) // 2 ** (L - level) + 1 for n in shape)


def recompose_to(u_mc, target_level, coords=None, stop_level=0, out=None, workspace=None):
    """Progressive recomposition: Q_target u on the level-target grid (natural
    order, shape level_shape(u_mc.shape, target_level)) from a decomposition
    to stop_level."""
    import torch
    _check_tensor(u_mc, "u_mc")
    shape = level_shape(u_mc.shape, target_level)
    if out is None:
        out = torch.empty(shape, dtype=u_mc.dtype, device=u_mc.device)
    _check_tensor(out, "out")
    if tuple(out.shape) != shape or out.dtype != u_mc.dtype:
        raise ValueError(f"out must be {shape} {u_mc.dtype}")
    ws, _ = _workspace(u_mc, stop_level, workspace)
    c = Coords(u_mc.shape, coords)
    code = lib().mgx_recompose_to(u_mc.data_ptr(), out.data_ptr(), _dtype_code(u_mc), u_mc.dim(),
                                  _dims(u_mc.shape), c.ptr, int(stop_level), int(target_level), ws.data_ptr(),
                                  ws.numel() * ws.element_size(), _stream(u_mc.device))
    _check(code, "mgx_recompose_to")
    return out


def dyadic_shape(shape):
    """The padded shape of a non-dyadic field: every axis to the next 2^m + 1."""
    out = (ctypes.c_int64 * len(shape))()
    _check(lib().mgx_dyadic_dims(len(shape), _dims(shape), out), "mgx_dyadic_dims")
    return tuple(int(x) for x in out)


def pad_coords(coords, shape):
    """Coordinates of the padded grid: each axis continued with its last spacing."""
    if coords is None:
        return None
    padded = dyadic_shape(shape)
    out = []
    for c, n, p in zip(coords, shape, padded):
        if c is None:
            out.append(None)
            continue
        c = np.asarray(c, dtype=np.float64)
        out.append(np.concatenate([c, c[-1] + (c[-1] - c[-2]) * np.arange(1, p - n + 1)]))
    return out


def pad(u, out=None):
    """Dummy-node padding of u to dyadic_shape(u.shape) (the nearest real node's value)."""
    import torch
    _check_tensor(u, "u")
    shape = dyadic_shape(u.shape)
    if out is None:
        out = torch.empty(shape, dtype=u.dtype, device=u.device)
    _check_tensor(out, "out")
    if tuple(out.shape) != shape or out.dtype != u.dtype:
        raise ValueError(f"out must be {shape} {u.dtype}")
    _check(lib().mgx_pad(u.data_ptr(), out.data_ptr(), _dtype_code(u), u.dim(), _dims(u.shape),
                         _stream(u.device)), "mgx_pad")
    return out


def crop(u_pad, shape, out=None):
    """The real nodes of a padded field: the inverse of pad for the shape `shape`."""
    import torch
    _check_tensor(u_pad, "u_pad")
    shape = tuple(shape)
    if tuple(u_pad.shape) != dyadic_shape(shape):
        raise ValueError(f"u_pad must have the padded shape {dyadic_shape(shape)}")
    if out is None:
        out = torch.empty(shape, dtype=u_pad.dtype, device=u_pad.device)
    _check_tensor(out, "out")
    _check(lib().mgx_crop(u_pad.data_ptr(), out.data_ptr(), _dtype_code(u_pad), len(shape), _dims(shape),
                          _stream(u_pad.device)), "mgx_crop")
    return out


def decompose_adaptive(u, tol, coords=None, c_linf=0.0, out=None, workspace=None):
    """Adaptive decomposition (Alg. 1 lines 1-16, 3-D): stops at the first
    level whose Lorenzo estimate is below the interpolation's.  Returns
    (u_mc, stop_level); u_mc is the level-centric layout of that stop."""
    import torch
    _check_tensor(u, "u")
    if out is None:
        out = torch.empty_like(u)
    _check_tensor(out, "out")
    ws, _ = _workspace(u, 0, workspace)
    c = Coords(u.shape, coords)
    stop = ctypes.c_int(-1)
    code = lib().mgx_decompose_adaptive(u.data_ptr(), out.data_ptr(), _dtype_code(u), u.dim(), _dims(u.shape), c.ptr,
                                        float(tol), float(c_linf), ctypes.byref(stop), ws.data_ptr(),
                                        ws.numel() * ws.element_size(), _stream(u.device))
    _check(code, "mgx_decompose_adaptive")
    return out, stop.value


def adaptive_estimate(v, shape, level, coords=None, workspace=None):
    """The adaptive estimate on the level box v (Q_level u of a field of
    `shape`): ((sum |u - Lorenzo|, sum |u - interpolant|), counts)."""
    import torch
    _check_tensor(v, "v")
    if tuple(v.shape) != level_shape(shape, level):
        raise ValueError(f"v must have the level-{level} shape {level_shape(shape, level)}")
    need = lib().mgx_adaptive_workspace_size(len(shape), _dims(shape))
    if workspace is None:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=v.device)
    c = Coords(shape, coords)
    sums = (ctypes.c_double * 2)()
    cnt = (ctypes.c_int64 * 3)()
    code = lib().mgx_adaptive_estimate(v.data_ptr(), _dtype_code(v), len(shape), _dims(shape), c.ptr, int(level),
                                       sums, cnt, workspace.data_ptr(), workspace.numel() * workspace.element_size(),
                                       _stream(v.device))
    _check(code, "mgx_adaptive_estimate")
    return (sums[0], sums[1]), (cnt[0], cnt[1], cnt[2])


def decompose_quantize(u, tol, coords=None, stop_level=0, c_linf=0.0, out=None, labels=None, workspace=None,
                       keep_coef=True, stats=False):
    """decompose then quantize (same labels and coefficients as the separate
    calls), the labels written by the decomposition's own kernels.  With
    keep_coef=False no u_mc is written (out is ignored) and None is returned
    in its place.  Returns (u_mc, labels); with stats=True
    (u_mc, labels, stats dict, status code), the code 6 (MGX_ERR_RANGE) when
    some coefficient was out of range."""
    import torch
    _check_tensor(u, "u")
    if not keep_coef:
        out = None
    elif out is None:
        out = torch.empty_like(u)
    if labels is None:
        labels = torch.empty(u.shape, dtype=torch.int32, device=u.device)
    if out is not None:
        _check_tensor(out, "out")
    _check_tensor(labels, "labels")
    ws, _ = _workspace(u, stop_level, workspace)
    c = Coords(u.shape, coords)
    st = QuantStats() if stats else None
    code = lib().mgx_decompose_quantize(u.data_ptr(), out.data_ptr() if out is not None else None,
                                        labels.data_ptr(), _dtype_code(u), u.dim(), _dims(u.shape), c.ptr,
                                        float(tol), int(stop_level), float(c_linf), ws.data_ptr(),
                                        ws.numel() * ws.element_size(), ctypes.byref(st) if st is not None else None,
                                        _stream(u.device))
    if stats:
        if code not in (0, 6):
            _check(code, "mgx_decompose_quantize")
        return out, labels, st.as_dict(), code
    _check(code, "mgx_decompose_quantize")
    return out, labels


def dequantize_recompose(labels, tol, dtype, coords=None, stop_level=0, c_linf=0.0, coef=None, out=None,
                         workspace=None):
    """dequantize then recompose into out (same results as the separate
    calls).  Without coef the recomposition's kernels read the coefficients
    from the labels; with coef the dequantized coefficients are also written
    there first.  Returns out."""
    import torch
    _check_tensor(labels, "labels")
    if out is None:
        out = torch.empty(labels.shape, dtype=dtype, device=labels.device)
    if coef is not None:
        _check_tensor(coef, "coef")
    _check_tensor(out, "out")
    ws, _ = _workspace(out, stop_level, workspace)
    c = Coords(labels.shape, coords)
    code = lib().mgx_dequantize_recompose(labels.data_ptr(), coef.data_ptr() if coef is not None else None,
                                          out.data_ptr(), _dtype_code(out), labels.dim(), _dims(labels.shape),
                                          c.ptr, float(tol), int(stop_level), float(c_linf), ws.data_ptr(),
                                          ws.numel() * ws.element_size(), _stream(labels.device))
    _check(code, "mgx_dequantize_recompose")
    return out


def _adjoint_call(name, src, coords, stop_level, out, workspace):
    import torch
    _check_tensor(src, "input")
    if out is None:
        out = torch.empty_like(src)
    _check_tensor(out, "out")
    need = adjoint_workspace_size(_dtype_code(src), src.shape, stop_level)
    if workspace is None:
        workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=src.device)
    c = Coords(src.shape, coords)
    code = getattr(lib(), name)(src.data_ptr(), out.data_ptr(), _dtype_code(src), src.dim(), _dims(src.shape),
                                c.ptr, int(stop_level), workspace.data_ptr(),
                                workspace.numel() * workspace.element_size(), _stream(src.device))
    _check(code, name)
    return out


def decompose_adjoint(g_mc, coords=None, stop_level=0, out=None, workspace=None):
    """D^T: coefficient-space gradient (level-centric) -> field-space gradient."""
    return _adjoint_call("mgx_decompose_adjoint", g_mc, coords, stop_level, out, workspace)


def recompose_adjoint(g_u, coords=None, stop_level=0, out=None, workspace=None):
    """R^T: field-space gradient -> coefficient-space gradient (level-centric)."""
    return _adjoint_call("mgx_recompose_adjoint", g_u, coords, stop_level, out, workspace)


# ---------------------------------------------------------------- batches of fields
class Batch:
    """A fixed list of fields for mgx_decompose_batched / mgx_recompose_batched.

    fields: list of dicts with keys
      in (tensor), out (tensor), coords (per-axis list or None), stop_level,
      tol (with labels), c_linf, labels (int32 tensor or None), coef (tensor or
      None: recompose from labels; None reads the labels in the level kernels),
      stats (decompose with labels: True asks for the field's quantization
      statistics, read back with stats() after decompose()).
    The same Batch object (same tensors) replays the captured graph; the
    workspace is allocated once per Batch.
    """

    def __init__(self, fields, workspace=None):
        import torch
        self._keep = []
        self._stats = {}
        self.code = 0
        n = len(fields)
        self.arr = (Field * n)()
        dev = None
        for i, f in enumerate(fields):
            t_in, t_out = f.get("in"), f["out"]
            ref = t_in if t_in is not None else t_out
            dev = ref.device
            x = self.arr[i]
            x.in_ = t_in.data_ptr() if t_in is not None else None
            x.out = t_out.data_ptr()
            x.dtype = _dtype_code(t_out)
            x.ndim = t_out.dim()
            for k in range(3):
                x.dims[k] = int(t_out.shape[k]) if k < t_out.dim() else 0
            c = Coords(t_out.shape, f.get("coords"))
            self._keep.append(c)
            if c.ptr is not None:
                ptrs = ctypes.cast(c.ptr, ctypes.POINTER(ctypes.c_void_p))
                for k in range(t_out.dim()):
                    x.coords[k] = ptrs[k]
            x.stop_level = int(f.get("stop_level", 0))
            x.tol_linf = float(f.get("tol", 0.0))
            x.c_linf = float(f.get("c_linf", 0.0))
            lab = f.get("labels")
            x.labels = lab.data_ptr() if lab is not None else None
            coef = f.get("coef")
            x.coef = coef.data_ptr() if coef is not None else None
            if f.get("stats"):
                st = QuantStats()
                self._stats[i] = st
                x.stats = ctypes.cast(ctypes.byref(st), ctypes.c_void_p)
            self._keep.extend([t for t in (t_in, t_out, lab, coef) if t is not None])
        self.n = n
        self.device = dev
        need = int(lib().mgx_batch_workspace_size(n, self.arr))
        if need == 0 and n > 0:
            raise MgxError(1, "mgx_batch_workspace_size")
        self.workspace = workspace if workspace is not None else torch.empty(max(need, 1), dtype=torch.uint8,
                                                                             device=dev)
        self.ws_bytes = self.workspace.numel() * self.workspace.element_size()

    def decompose(self):
        """Raises MgxError unless the status is 0, or 6 (MGX_ERR_RANGE) with
        statistics asked for (then kept in self.code; see stats())."""
        code = lib().mgx_decompose_batched(self.n, self.arr, self.workspace.data_ptr(), self.ws_bytes,
                                           _stream(self.device))
        self.code = code
        if not (code == 6 and self._stats):
            _check(code, "mgx_decompose_batched")

    def stats(self):
        """{field index: statistics dict} of the fields that asked for them."""
        return {i: st.as_dict() for i, st in self._stats.items()}

    def recompose(self):
        _check(lib().mgx_recompose_batched(self.n, self.arr, self.workspace.data_ptr(), self.ws_bytes,
                                           _stream(self.device)), "mgx_recompose_batched")


def release_cached() -> None:
    """Free the library's cached level plans and batch graphs (no other call
    of the library may be running)."""
    _check(lib().mgx_release_cached(), "mgx_release_cached")


def batch_set_autotune(on: bool) -> None:
    _check(lib().mgx_batch_set_autotune(1 if on else 0), "mgx_batch_set_autotune")


def batch_last_info() -> dict:
    info = BatchInfo()
    _check(lib().mgx_batch_last_info(ctypes.byref(info)), "mgx_batch_last_info")
    return {"launches": info.launches, "target_blocks": info.target_blocks, "min_zchunk": info.min_zchunk,
            "tuned_ms": info.tuned_ms, "tune_source": info.tune_source}


def quantize(u_mc, tol, coords=None, stop_level=0, c_linf=0.0, out=None, stats=False):
    """Level-wise labels (int32).  With stats=True returns (labels, stats dict) and
    raises MgxError(MGX_ERR_RANGE) if any label overflowed."""
    import torch
    _check_tensor(u_mc, "u_mc")
    if out is None:
        out = torch.empty(u_mc.shape, dtype=torch.int32, device=u_mc.device)
    _check_tensor(out, "labels")
    c = Coords(u_mc.shape, coords)
    st = QuantStats() if stats else None
    code = lib().mgx_quantize(u_mc.data_ptr(), out.data_ptr(), _dtype_code(u_mc), u_mc.dim(), _dims(u_mc.shape),
                              c.ptr, float(tol), int(stop_level), float(c_linf),
                              ctypes.byref(st) if st is not None else None, _stream(u_mc.device))
    if stats:
        if code not in (0, 6):
            _check(code, "mgx_quantize")
        return out, st.as_dict(), code
    _check(code, "mgx_quantize")
    return out


def dequantize(labels, tol, dtype, coords=None, stop_level=0, c_linf=0.0, out=None):
    """Labels -> coefficients of `dtype` (level-centric layout)."""
    import torch
    _check_tensor(labels, "labels")
    if labels.dtype != torch.int32:
        raise TypeError("labels must be int32")
    if out is None:
        out = torch.empty(labels.shape, dtype=dtype, device=labels.device)
    _check_tensor(out, "out")
    c = Coords(labels.shape, coords)
    code = lib().mgx_dequantize(labels.data_ptr(), out.data_ptr(), _dtype_code(out), labels.dim(),
                                _dims(labels.shape), c.ptr, float(tol), int(stop_level), float(c_linf),
                                _stream(labels.device))
    _check(code, "mgx_dequantize")
    return out


def l2_constant(shape, coords=None, stop_level=0) -> float:
    c = Coords(shape, coords)
    r = lib().mgx_l2_constant(len(shape), _dims(shape), c.ptr, int(stop_level))
    if r < 0:
        raise MgxError(1, "mgx_l2_constant")
    return r


def level_tolerances_l2(shape, tol_l2, c_l2=0.0, coords=None, stop_level=0) -> np.ndarray:
    """tau_l of the L2 variant (levels stop_level .. L); c_l2 <= 0 takes
    the library's default C_L2 (l2_constant)."""
    L = num_levels(shape)
    tau = np.zeros(L + 1 - int(stop_level), dtype=np.float64)
    c = Coords(shape, coords)
    code = lib().mgx_level_tolerances_l2(len(shape), _dims(shape), c.ptr, float(tol_l2), int(stop_level),
                                         float(c_l2), tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(code, "mgx_level_tolerances_l2")
    return tau


def _tau_arg(tau, shape, stop_level):
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    if tau.shape != (num_levels(shape) + 1 - int(stop_level),):
        raise ValueError("tau needs one entry per level stop_level .. L")
    return tau


def quantize_levels(u_mc, tau, coords=None, stop_level=0, out=None):
    """Labels with caller-given per-level tolerances tau (levels stop_level .. L)."""
    import torch
    _check_tensor(u_mc, "u_mc")
    t = _tau_arg(tau, u_mc.shape, stop_level)
    if out is None:
        out = torch.empty(u_mc.shape, dtype=torch.int32, device=u_mc.device)
    _check_tensor(out, "labels")
    c = Coords(u_mc.shape, coords)
    code = lib().mgx_quantize_levels(u_mc.data_ptr(), out.data_ptr(), _dtype_code(u_mc), u_mc.dim(),
                                     _dims(u_mc.shape), c.ptr, int(stop_level),
                                     t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), None, _stream(u_mc.device))
    _check(code, "mgx_quantize_levels")
    return out


def dequantize_levels(labels, tau, dtype, coords=None, stop_level=0, out=None):
    """Coefficients from labels with caller-given per-level tolerances."""
    import torch
    _check_tensor(labels, "labels")
    t = _tau_arg(tau, labels.shape, stop_level)
    if out is None:
        out = torch.empty(labels.shape, dtype=dtype, device=labels.device)
    _check_tensor(out, "out")
    c = Coords(labels.shape, coords)
    code = lib().mgx_dequantize_levels(labels.data_ptr(), out.data_ptr(), _dtype_code(out), labels.dim(),
                                       _dims(labels.shape), c.ptr, int(stop_level),
                                       t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(labels.device))
    _check(code, "mgx_dequantize_levels")
    return out


def label_entropy(labels, stop_level=0, workspace=None, stats=None) -> np.ndarray:
    """Shannon entropy (bits per label) of the labels of each level stop_level .. L.
    stats: the statistics dict of the quantizing call that wrote the labels
    (decompose_quantize(..., stats=True)); its per-level maxima spare the
    pass that finds them."""
    import torch
    _check_tensor(labels, "labels")
    shape = tuple(labels.shape)
    need = lib().mgx_label_entropy_workspace_size(len(shape), _dims(shape), int(stop_level))
    if workspace is None:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=labels.device)
    bits = np.zeros(num_levels(shape) + 1 - int(stop_level), dtype=np.float64)
    bp = bits.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    wb = workspace.numel() * workspace.element_size()
    if stats is None:
        code = lib().mgx_label_entropy(labels.data_ptr(), len(shape), _dims(shape), int(stop_level), bp,
                                       workspace.data_ptr(), wb, _stream(labels.device))
        _check(code, "mgx_label_entropy")
        return bits
    st = QuantStats()
    st.first_level = int(stats["first_level"])
    st.num_levels = len(stats["max_abs_label"])
    for i, m in enumerate(stats["max_abs_label"]):
        st.max_abs_label[i] = int(m)
    st.n_overflow = int(stats["n_overflow"])
    st.n_nonfinite = int(stats["n_nonfinite"])
    code = lib().mgx_label_entropy_bounded(labels.data_ptr(), len(shape), _dims(shape), int(stop_level),
                                           ctypes.byref(st), bp, workspace.data_ptr(), wb, _stream(labels.device))
    _check(code, "mgx_label_entropy_bounded")
    return bits


from .autograd import Decompose, MGXRoundTrip, QuantizeSTE, Recompose  # noqa: E402,F401
