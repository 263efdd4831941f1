"""Seeded synthetic inputs shaped like the paper's 3-D simulation fields.

This module only draws random numbers and builds test fields and grid
coordinates.  It contains none of the method's arithmetic and is shared by
the tests, the smoke check and the benchmark; both the HIP path and the CPU
oracle receive the same arrays.

The paper evaluates on SDRBench fields (Table 2: Hurricane 100x500x500,
NYX 512^3, SCALE-LETKF 98x1200x1200, QMCPACK).  Those datasets are not
available here; these generators stand in for them with the same rank,
comparable extents made dyadic (2^k+1 per axis) and turbulence-like spectra.
"""
from __future__ import annotations

import math

import numpy as np
import torch

BASE_SEED = 201005872


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def _wrap(field: torch.Tensor) -> torch.Tensor:
    """Periodic field on n^d -> (n+1)^d by repeating index 0 at the end of each axis."""
    for ax in range(field.ndim):
        first = field.narrow(ax, 0, 1)
        field = torch.cat([field, first], dim=ax)
    return field


def gaussian_random_field(shape, slope: float, seed: int, device="cpu",
                          axis_scale=None) -> torch.Tensor:
    """Periodic Gaussian random field on `shape` with power spectrum P(k) ~ k^-slope.

    White N(0,1) noise is filtered in Fourier space with amplitude k^(-slope/2)
    (k = 0 removed) and the result scaled to unit variance.  `axis_scale`
    stretches wavenumbers per axis (layered fields).  float64.
    """
    g = _gen(seed, device)
    noise = torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float64)
    spec = torch.fft.rfftn(noise)
    del noise
    ks = []
    for ax, n in enumerate(shape):
        if ax == len(shape) - 1:
            k = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
        else:
            k = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float64)
        if axis_scale is not None:
            k = k * float(axis_scale[ax])
        view = [1] * len(shape)
        view[ax] = -1
        ks.append(k.view(view))
    k2 = ks[0] ** 2
    for k in ks[1:]:
        k2 = k2 + k ** 2
    amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (-slope / 4.0), torch.zeros_like(k2))
    spec = spec * amp
    del amp, k2
    field = torch.fft.irfftn(spec, s=tuple(shape))
    del spec
    field = field - field.mean()
    field = field / field.std()
    return field


def sinusoid_field(n: int = 65, seed: int = BASE_SEED + 1) -> np.ndarray:
    """Sum of three plane waves with integer wavevectors (1 <= |k| <= 8) and
    random phases plus N(0, 1e-3^2) noise on a unit-spaced n^3 grid (float64)."""
    rng = np.random.default_rng(seed)
    x = np.arange(n, dtype=np.float64)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((n, n, n))
    period = float(n - 1)
    count = 0
    while count < 3:
        k = rng.integers(-8, 9, size=3)
        norm = math.sqrt(float((k * k).sum()))
        if not (1.0 <= norm <= 8.0):
            continue
        phase = rng.uniform(0.0, 2.0 * math.pi)
        u += np.sin(2.0 * math.pi * (k[0] * Z + k[1] * Y + k[2] * X) / period + phase)
        count += 1
    u += rng.normal(0.0, 1e-3, size=u.shape)
    return u


def turbulence_field(n: int = 513, seed: int = BASE_SEED + 2, device="cpu",
                     dtype=torch.float32) -> torch.Tensor:
    """Unit-variance Gaussian random field, P(k) ~ k^(-11/3), on an n^3 grid
    (periodic field on (n-1)^3 wrapped to n^3): the NYX-shaped workload."""
    f = gaussian_random_field((n - 1,) * 3, 11.0 / 3.0, seed, device)
    return _wrap(f).to(dtype).contiguous()


def tanh_coordinates(n: int = 257, ratio: float = 20.0) -> np.ndarray:
    """Vertical coordinates stretched by tanh: z_i = 1 + tanh(b(i/m - 1))/tanh(b),
    m = (n-1)/2, b = acosh(sqrt(ratio)); largest/smallest spacing ~= ratio."""
    b = math.acosh(math.sqrt(ratio))
    m = (n - 1) / 2.0
    i = np.arange(n, dtype=np.float64)
    return 1.0 + np.tanh(b * (i / m - 1.0)) / math.tanh(b)


def layered_lognormal_field(shape=(257, 1025, 1025), seed: int = BASE_SEED + 3, device="cpu",
                            dtype=torch.float32):
    """Weather-shaped workload: exp(G) + 4(1 - z) on a tanh-stretched vertical
    axis, G a unit-variance layered GRF (vertical wavenumbers scaled by 8).
    Returns (field, coords) with coords = [z, None, None]."""
    per = tuple(n - 1 for n in shape)
    G = _wrap(gaussian_random_field(per, 11.0 / 3.0, seed, device, axis_scale=(8.0, 1.0, 1.0)))
    z = tanh_coordinates(shape[0])
    zt = torch.as_tensor(z, device=device, dtype=torch.float64).view(-1, 1, 1)
    u = torch.exp(G) + 4.0 * (1.0 - zt)
    return u.to(dtype).contiguous(), [z, None, None]


def orbital_field(shape=(288, 115, 69, 69), seed: int = BASE_SEED + 6, device="cpu", dtype=torch.float32):
    """Four-axis workload shaped like the QMCPACK field of Table 2 (orbital
    index x three spatial axes, non-dyadic): a unit-variance Gaussian random
    field with P(k) ~ k^-4, wavenumbers along the orbital axis scaled by 4
    (neighbouring orbitals only weakly alike)."""
    G = gaussian_random_field(tuple(shape), 4.0, seed, device, axis_scale=(4.0, 1.0, 1.0, 1.0))
    return G.to(dtype).contiguous()


def batch_specs(count: int = 64, seed: int = BASE_SEED + 4):
    """Per-field shapes (each axis from {33,65,129,257}), spectral slopes in
    [2,4] and relative tolerances log-uniform in [1e-4, 1e-2]."""
    rng = np.random.default_rng(seed)
    specs = []
    for f in range(count):
        shape = tuple(int(rng.choice([33, 65, 129, 257])) for _ in range(3))
        slope = float(rng.uniform(2.0, 4.0))
        rel_tol = float(10.0 ** rng.uniform(-4.0, -2.0))
        specs.append({"shape": shape, "slope": slope, "rel_tol": rel_tol,
                      "seed": BASE_SEED + 4000 + f})
    return specs


def batch_field(spec, device="cpu", dtype=torch.float32) -> torch.Tensor:
    per = tuple(n - 1 for n in spec["shape"])
    return _wrap(gaussian_random_field(per, spec["slope"], spec["seed"], device)).to(dtype).contiguous()


def adjoint_fields(count: int = 8, n: int = 257, seed: int = BASE_SEED + 5, device="cpu",
                   dtype=torch.float32) -> torch.Tensor:
    """`count` unit-variance fields with P(k) ~ k^-3 on n^3 grids, stacked."""
    fields = [_wrap(gaussian_random_field((n - 1,) * 3, 3.0, seed + f, device)).to(dtype)
              for f in range(count)]
    return torch.stack(fields).contiguous()


def random_coordinates(n: int, seed: int, lo: float = 0.3, hi: float = 3.0) -> np.ndarray:
    """Strictly increasing coordinates with random spacings in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return np.concatenate([[0.0], np.cumsum(rng.uniform(lo, hi, n - 1))])
