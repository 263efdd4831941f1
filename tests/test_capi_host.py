"""The C-ABI library on a host without a GPU: it loads, exports every symbol
that include/mgx.h declares, and validates arguments (and computes the host
tables) before any launch.  No compute call reaches the device here."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import workloads

import paper_2010_05872_amd as mgx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "mgx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mgx_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mgx.lib()
    syms = header_symbols()
    assert set(syms) == set(mgx.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


def test_num_levels_and_workspace():
    assert mgx.num_levels((513, 513, 513)) == 8
    assert mgx.num_levels((257, 1025, 1025)) == 7
    assert mgx.num_levels((65,)) == 5
    for bad in [(64,), (2,), (513, 512), (5, 5, 5, 5, 5), (5, 5, 6, 5), (16385,), (2049, 2049, 1025, 3)]:
        with pytest.raises(mgx.MgxError):
            mgx.num_levels(bad)
    # 4-D (Table 2's four-axis field, padded): the shortest axis sets L
    assert mgx.num_levels((513, 129, 129, 129)) == 6
    assert mgx.num_levels((5, 5, 5, 5)) == 1
    n = 513 ** 3
    ws = mgx.workspace_size(0, (513, 513, 513), 0)
    assert 0.25 * n * 4 < ws < 0.3 * n * 4
    assert mgx.workspace_size(0, (513, 513, 513), 8) == 0
    assert mgx.workspace_size(1, (65, 65, 65), 4) > 0
    assert mgx.workspace_size(7, (65, 65, 65), 0) == 0
    # 4-D: two sweep buffers and two level-(L-1) boxes
    n4 = (17, 9, 33, 9)
    c4 = [(k - 1) // 2 + 1 for k in n4]
    want = (n4[0] * n4[1] * n4[2] * c4[3] + n4[0] * n4[1] * c4[2] * c4[3] + 2 * int(np.prod(c4))) * 4
    assert want <= mgx.workspace_size(0, n4, 0) <= want + 4 * 256
    assert mgx.workspace_size(0, n4, mgx.num_levels(n4)) == 0


def _call_decompose(u, out, dims, coords=None, stop=0, ws=0, nbytes=0, dtype=0):
    L = mgx.lib()
    d = (ctypes.c_int64 * len(dims))(*dims)
    return L.mgx_decompose(u, out, dtype, len(dims), d, coords, stop, ws, nbytes, None)


def test_validation_before_launch():
    # fake device addresses: every call below must fail validation first
    U, O, W = 0x10000000, 0x20000000, 0x30000000
    big = 1 << 40
    assert _call_decompose(U, O, [65, 65, 64], ws=W, nbytes=big) == 2
    assert _call_decompose(U, O, [65, 65], ws=W, nbytes=big, stop=9) == 4
    assert _call_decompose(0, O, [65, 65], ws=W, nbytes=big) == 1
    assert _call_decompose(U, U + 8, [65, 65], ws=W, nbytes=big) == 1  # overlap
    assert _call_decompose(U, O, [65, 65], ws=0, nbytes=0) == 7
    assert _call_decompose(U, O, [65, 65], ws=W, nbytes=16) == 7
    assert _call_decompose(U, O, [65, 65], ws=W, nbytes=big, dtype=5) == 1
    bad = mgx.Coords((5, 5), [np.array([0, 1, 1, 2, 3.0]), None])
    assert _call_decompose(U, O, [5, 5], coords=bad.ptr, ws=W, nbytes=big) == 3
    nan = mgx.Coords((5, 5), [None, np.array([0, 1, np.nan, 2, 3.0])])
    assert _call_decompose(U, O, [5, 5], coords=nan.ptr, ws=W, nbytes=big) == 3
    L = mgx.lib()
    d = (ctypes.c_int64 * 2)(65, 65)
    assert L.mgx_quantize(U, O, 0, 2, d, None, -1.0, 0, 0.0, None, None) == 5
    assert L.mgx_quantize(U, O, 0, 2, d, None, 1.0, 0, 0.5, None, None) == 5
    assert L.mgx_quantize(U, O, 0, 2, d, None, float("inf"), 0, 0.0, None, None) == 5
    assert L.mgx_quantize(U, U, 0, 2, d, None, 1.0, 0, 0.0, None, None) == 1
    assert L.mgx_dequantize(U, O, 0, 2, d, None, 1.0, 7, 0.0, None) == 4
    assert mgx.lib().mgx_status_string(6).decode().startswith("quantization")
    # 4-D fields take the same checks
    assert _call_decompose(U, O, [9, 9, 9, 10], ws=W, nbytes=big) == 2
    assert _call_decompose(U, O, [9, 9, 9, 9], ws=W, nbytes=big, stop=3) == 4
    assert _call_decompose(U, O, [9, 9, 9, 9], ws=W, nbytes=16) == 7
    assert _call_decompose(U, U + 8, [9, 9, 9, 9], ws=W, nbytes=big) == 1
    bad4 = mgx.Coords((9, 9, 9, 9), [None, None, np.array([0, 1, 2, 3, 4, 5, 6, 6, 7.0]), None])
    assert _call_decompose(U, O, [9, 9, 9, 9], coords=bad4.ptr, ws=W, nbytes=big) == 3
    d4 = (ctypes.c_int64 * 4)(9, 9, 9, 9)
    assert L.mgx_quantize(U, O, 0, 4, d4, None, -1.0, 0, 0.0, None, None) == 5
    assert L.mgx_dequantize(U, O, 0, 4, d4, None, 1.0, 3, 0.0, None) == 4
    # the entropy with the quantizer's statistics: null statistics, a bad
    # level or a short workspace are refused before any launch
    bits = (ctypes.c_double * 16)()
    st = mgx.QuantStats()
    st.num_levels = 7
    assert L.mgx_label_entropy_bounded(U, 2, d, 0, None, bits, W, big, None) == 1
    assert L.mgx_label_entropy_bounded(U, 2, d, 7, ctypes.byref(st), bits, W, big, None) == 4
    assert L.mgx_label_entropy_bounded(U, 2, d, 0, ctypes.byref(st), bits, W, 16, None) == 7
    d3 = (ctypes.c_int64 * 2)(65, 64)
    assert L.mgx_label_entropy_bounded(U, 2, d3, 0, ctypes.byref(st), bits, W, big, None) == 2


@pytest.mark.parametrize("shape,kind", [((65, 65, 65), None), ((17, 33, 65), "mixed"), ((129, 33), "random"),
                                        ((257,), None), ((17, 9, 33, 9), "random"), ((9, 9, 9, 9), None)])
def test_host_tables_match_oracle(shape, kind):
    if kind == "mixed":
        coords = [workloads.tanh_coordinates(shape[0]), None, workloads.random_coordinates(shape[2], 1)]
    elif kind == "random":
        coords = [workloads.random_coordinates(n, 4 + k) for k, n in enumerate(shape)]
    else:
        coords = None
    L = oracle.num_levels(shape)
    for stop in range(0, L + 1):
        C = mgx.linf_constant(shape, coords, stop)
        assert C == pytest.approx(oracle.linf_constant(shape, coords, stop), rel=1e-13)
        for tol in (1e-3, 0.7, 123.0):
            a = mgx.level_tolerances(shape, tol, coords, stop, c_linf=C)
            b = oracle.level_tolerances(shape, tol, coords, stop, c_linf=C)
            assert np.array_equal(a, b)  # identical FP64 operation order


def test_config3_constant():
    z = workloads.tanh_coordinates(257)
    assert mgx.linf_constant((257, 1025, 1025), [z, None, None]) == pytest.approx(7.7075, abs=1e-4)
