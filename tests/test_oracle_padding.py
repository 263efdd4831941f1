"""Non-dyadic sizes through dummy nodes (Sec. 6.2.2): the padded shape, the
padding itself, and the L-infinity bound on the real nodes after a full
decompose / quantize / dequantize / recompose of the padded field (oracle,
CPU).  The padded shape is pinned by its closed form; the bound is the
guarantee of Sec. 4.1 restricted to the real nodes."""
import numpy as np
import pytest

import oracle
import paper_2010_05872_amd as mgx


@pytest.mark.parametrize("n,p", [(2, 3), (3, 3), (4, 5), (5, 5), (6, 9), (17, 17), (18, 33), (100, 129), (500, 513)])
def test_dyadic_shape(n, p):
    assert oracle.dyadic_shape((n,)) == (p,)
    assert mgx.dyadic_shape((n,)) == (p,)      # the library's host-side count


def test_dyadic_shape_rejects_single_nodes():
    with pytest.raises(oracle.OracleError):
        oracle.dyadic_shape((1, 5))
    with pytest.raises(mgx.MgxError):
        mgx.dyadic_shape((1, 5))


def test_padding_values():
    u = np.arange(2 * 3 * 4, dtype=np.float64).reshape(2, 3, 4)
    v = oracle.pad_to_dyadic(u)
    assert v.shape == (3, 3, 5)
    assert np.array_equal(v[:2, :3, :4], u)
    assert np.array_equal(v[2], v[1]) and np.array_equal(v[:, :, 4], v[:, :, 3])


@pytest.mark.parametrize("shape", [(6, 10, 12), (100,), (7, 20)])
def test_linf_bound_on_real_nodes(shape):
    rng = np.random.default_rng(5)
    u = np.cumsum(rng.standard_normal(shape), axis=-1)
    v = oracle.pad_to_dyadic(u)
    tol = 1e-3 * np.ptp(u)
    c = oracle.decompose(v)
    labels, code = oracle.quantize(c, tol)
    assert code == 0
    r = oracle.recompose(oracle.dequantize(labels, tol))
    err = np.abs(r[tuple(slice(0, n) for n in shape)] - u).max()
    assert err <= tol
