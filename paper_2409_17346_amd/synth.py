"""Seeded synthetic inputs for the MSC-preserving correction stage.

The paper evaluates on real simulation fields (its Table 1) compressed by
SZ3/ZFP/SPERR/MGARD; none of those are available, so every input here is
synthetic and seeded.  This module only *draws* inputs: an original fp32 field
``f``, an absolute error bound ``xi`` and a "decompressed" field ``g_hat`` with
``|g_hat - f| <= xi`` (the precondition of the problem statement, Section 4.1).
It contains none of the correction method's arithmetic (no gradient, no floors,
no edits) and is shared by the oracle tests and the GPU path alike.

Layout: arrays are C-ordered ``(nz, ny, nx)`` (2D fields as ``(ny, nx)``), so the
linear vertex id is ``x + nx*(y + ny*z)``.

Recipes (all draws from ``numpy.random.default_rng(seed)`` in a fixed order:
centres, widths, amplitudes, noise lattices / fields, then g_hat noise or coins;
arithmetic in float64, cast to fp32 last):

* ``gauss2d_noise``  - 2D sum of isotropic Gaussians + i.i.d. uniform noise,
  normalised to [0, 1] (the small 2D climate/flow-like case, 128^2).
* ``gauss2d_value_noise`` - 2D sum of wide Gaussians + 4-octave smoothstep value
  noise, normalised to [0, 1] (the 2048^2 case).
* ``atoms3d`` - 3D molecular-density-like field: positive lognormal-amplitude
  Gaussians on a 1e-4 background floor, tails cut at 8 sigma (exact plateaus, so
  the symbolic tie-break is exercised everywhere).
* ``lognormal3d`` - exp of a Gaussian random field with P(k) ~ k^-2.5
  (cosmology-like), for the served mix.

``g_hat`` is either a 2*xi-bin quantisation of f (prediction-free SZ-like error)
or f plus uniform noise in [-xi, xi]; either way it is nudged back into the bound
by exact float64 checks.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as dc_field
from typing import Tuple

import numpy as np

__all__ = [
    "Workload", "xi_from_relative", "enforce_bound", "bin_quantize", "uniform_noise",
    "gauss2d_noise", "gauss2d_value_noise", "atoms3d", "lognormal3d",
    "config_small2d", "config_large2d", "config_atoms3d", "batch_mix", "served_job",
    "random_field", "tiny_cases",
]


@dataclass
class Workload:
    """One correction job: fields are fp32 numpy arrays shaped (nz, ny, nx) or (ny, nx)."""
    name: str
    f: np.ndarray
    g_hat: np.ndarray
    xi: float
    tier: int = 4
    q_max: int = 6
    meta: dict = dc_field(default_factory=dict)

    @property
    def dims(self) -> Tuple[int, int, int]:
        s = self.f.shape
        if len(s) == 2:
            return (s[1], s[0], 1)
        return (s[2], s[1], s[0])

    @property
    def ndim(self) -> int:
        return 2 if self.f.ndim == 2 else 3


def xi_from_relative(f: np.ndarray, rel: float) -> float:
    """Absolute bound from a relative one: fl32(rel * (max f - min f)), range in float64."""
    f64 = f.astype(np.float64)
    return float(np.float32(rel * (float(f64.max()) - float(f64.min()))))


def _two_diff_exact(a: np.ndarray, b: np.ndarray):
    """Return (a-b) in float64 and a mask telling where that float64 result is exact."""
    s = a - b
    bp = s - a
    ap = s - bp
    err = (a - ap) + (-b - bp)
    return s, err == 0.0


def enforce_bound(f: np.ndarray, g: np.ndarray, xi: float) -> np.ndarray:
    """Move each entry of g toward f one ulp at a time until |g - f| <= xi holds exactly."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.float32).copy()
    xi64 = float(np.float32(xi))
    f64 = f.astype(np.float64)
    for _ in range(64):
        d, exact = _two_diff_exact(g.astype(np.float64), f64)
        if not exact.all():
            raise ValueError("float64 difference inexact: field dynamic range too wide for the generator")
        bad = np.abs(d) > xi64
        if not bad.any():
            return g
        g[bad] = np.nextafter(g[bad], f[bad])
    raise RuntimeError("enforce_bound did not settle")


def bin_quantize(f: np.ndarray, xi: float) -> np.ndarray:
    """SZ-like prediction-free error: g = fl32(2*xi * rint(f / (2*xi))), then bound-enforced."""
    w = 2.0 * float(np.float32(xi))
    g = (w * np.rint(f.astype(np.float64) / w)).astype(np.float32)
    return enforce_bound(f, g, xi)


def uniform_noise(f: np.ndarray, xi: float, rng: np.random.Generator) -> np.ndarray:
    """Generic bounded error: g = fl32(f + U[-xi, xi]), then bound-enforced."""
    x = float(np.float32(xi))
    g = (f.astype(np.float64) + rng.uniform(-x, x, size=f.shape)).astype(np.float32)
    return enforce_bound(f, g, xi)


def _normalize01(a: np.ndarray) -> np.ndarray:
    lo, hi = float(a.min()), float(a.max())
    return (a - lo) / (hi - lo) if hi > lo else np.zeros_like(a)


def _gauss_sum_2d(side_y: int, side_x: int, cy, cx, sig, amp) -> np.ndarray:
    """Sum of isotropic 2D Gaussians, separable, as one small matrix product (float64)."""
    ys = np.arange(side_y, dtype=np.float64)
    xs = np.arange(side_x, dtype=np.float64)
    gy = np.exp(-0.5 * ((ys[None, :] - cy[:, None]) / sig[:, None]) ** 2)  # (k, ny)
    gx = np.exp(-0.5 * ((xs[None, :] - cx[:, None]) / sig[:, None]) ** 2)  # (k, nx)
    return (gy * amp[:, None]).T @ gx


def gauss2d_noise(side: int, n_gauss: int, seed: int, sig_lo=3.0, sig_hi=12.0,
                  noise=1e-3, rng: np.random.Generator | None = None) -> np.ndarray:
    """Sum of n isotropic Gaussians + U[0, noise) i.i.d. noise, normalised to [0, 1]."""
    rng = np.random.default_rng(seed) if rng is None else rng
    centres = rng.uniform(0.0, side, size=(n_gauss, 2))
    sig = rng.uniform(sig_lo, sig_hi, size=n_gauss)
    amp = rng.uniform(-1.0, 1.0, size=n_gauss)
    z = _gauss_sum_2d(side, side, centres[:, 1], centres[:, 0], sig, amp)
    z += rng.uniform(0.0, noise, size=z.shape)
    return _normalize01(z).astype(np.float32)


def _smoothstep(t):
    return t * t * (3.0 - 2.0 * t)


def _value_noise(shape, period: int, rng: np.random.Generator) -> np.ndarray:
    """Smoothstep multilinear interpolation of a U[-1,1] lattice with the given period (n-D)."""
    nd = len(shape)
    lat_shape = tuple(s // period + 2 for s in shape)
    lat = rng.uniform(-1.0, 1.0, size=lat_shape)
    out = np.zeros(shape, dtype=np.float64)
    idx = []
    wts = []
    for ax, s in enumerate(shape):
        c = np.arange(s, dtype=np.float64) / period
        i0 = np.floor(c).astype(np.int64)
        t = _smoothstep(c - i0)
        idx.append(i0)
        wts.append(t)
    for corner in range(1 << nd):
        w = np.ones(shape, dtype=np.float64)
        sl = []
        for ax in range(nd):
            bit = (corner >> ax) & 1
            t = wts[ax] if bit else 1.0 - wts[ax]
            bshape = [1] * nd
            bshape[ax] = shape[ax]
            w = w * t.reshape(bshape)
            sl.append(idx[ax] + bit)
        out += w * lat[np.ix_(*sl)]
    return out


def gauss2d_value_noise(side: int, n_gauss: int, seed: int, rng: np.random.Generator | None = None,
                        octaves: int = 4, amp0: float = 0.05, falloff: float = 0.5) -> np.ndarray:
    """Wide Gaussians (sigma ~ U[3,12]*side/128) + octave value noise, normalised to [0, 1]."""
    rng = np.random.default_rng(seed) if rng is None else rng
    centres = rng.uniform(0.0, side, size=(n_gauss, 2))
    scale = side / 128.0
    sig = rng.uniform(3.0 * scale, 12.0 * scale, size=n_gauss)
    amp = rng.uniform(-1.0, 1.0, size=n_gauss)
    z = _gauss_sum_2d(side, side, centres[:, 1], centres[:, 0], sig, amp)
    for o in range(octaves):
        period = max(2, side // 8 // (2 ** o))
        z += amp0 * (falloff ** o) * _value_noise((side, side), period, rng)
    return _normalize01(z).astype(np.float32)


def atoms3d(side: int, n_atoms: int, seed: int, rng: np.random.Generator | None = None,
            floor: float = 1e-4, sig_lo: float = 1.5, sig_hi: float = 4.0, cut: float = 8.0) -> np.ndarray:
    """1e-4 floor + sum of atom-centred Gaussians (lognormal(0,0.5) amplitudes), cut at 8 sigma."""
    rng = np.random.default_rng(seed) if rng is None else rng
    centres = rng.uniform(0.0, side, size=(n_atoms, 3))
    sig = rng.uniform(sig_lo, sig_hi, size=n_atoms)
    amp = rng.lognormal(0.0, 0.5, size=n_atoms)
    acc = np.zeros((side, side, side), dtype=np.float64)
    for (cx, cy, cz), s, a in zip(centres, sig, amp):
        r = cut * s
        lo = [max(0, int(math.floor(c - r))) for c in (cz, cy, cx)]
        hi = [min(side, int(math.ceil(c + r)) + 1) for c in (cz, cy, cx)]
        z = np.arange(lo[0], hi[0], dtype=np.float64)[:, None, None] - cz
        y = np.arange(lo[1], hi[1], dtype=np.float64)[None, :, None] - cy
        x = np.arange(lo[2], hi[2], dtype=np.float64)[None, None, :] - cx
        r2 = z * z + y * y + x * x
        v = a * np.exp(-0.5 * r2 / (s * s))
        v[r2 > r * r] = 0.0
        acc[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += v
    return (floor + acc).astype(np.float32)


def lognormal3d(side: int, seed: int, rng: np.random.Generator | None = None,
                slope: float = -2.5) -> np.ndarray:
    """exp of a standardised Gaussian random field with power spectrum P(k) ~ k^slope."""
    rng = np.random.default_rng(seed) if rng is None else rng
    white = rng.standard_normal((side, side, side))
    spec = np.fft.rfftn(white)
    kz = np.fft.fftfreq(side) * side
    ky = np.fft.fftfreq(side) * side
    kx = np.fft.rfftfreq(side) * side
    k = np.sqrt(kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = k[nz] ** (slope / 2.0)
    field = np.fft.irfftn(spec * amp, s=(side, side, side), axes=(0, 1, 2))
    field = (field - field.mean()) / field.std()
    return np.exp(field).astype(np.float32)


# ---------------------------------------------------------------------------------------------
# The workloads

def config_small2d(seed: int = 1) -> Workload:
    """2D 128x128: 16 Gaussians + 1e-3 noise; g_hat = 2*xi bins, xi = 1e-3 * range; tier 4."""
    rng = np.random.default_rng(seed)
    f = gauss2d_noise(128, 16, seed, rng=rng)
    xi = xi_from_relative(f, 1e-3)
    return Workload("2d-128-gauss16-bin-1e-3", f, bin_quantize(f, xi), xi, 4, 6,
                    {"rel": 1e-3, "ghat": "bin", "seed": seed})


def config_large2d(seed: int = 2, side: int = 2048) -> Workload:
    """2D 2048x2048: 256 Gaussians + 4-octave value noise; g_hat = f + U[-xi,xi], xi = 1e-4 * range."""
    rng = np.random.default_rng(seed)
    f = gauss2d_value_noise(side, 256 * (side * side) // (2048 * 2048) or 1, seed, rng=rng)
    xi = xi_from_relative(f, 1e-4)
    return Workload(f"2d-{side}-gauss256-valuenoise-noise-1e-4", f, uniform_noise(f, xi, rng), xi, 4, 6,
                    {"rel": 1e-4, "ghat": "noise", "seed": seed})


def config_atoms3d(seed: int = 3, side: int = 256, n_atoms: int = 512) -> Workload:
    """3D 256^3 density: 512 atoms on a 1e-4 floor; g_hat = 2*xi bins, xi = 1e-4 * range."""
    rng = np.random.default_rng(seed)
    f = atoms3d(side, n_atoms, seed, rng=rng)
    xi = xi_from_relative(f, 1e-4)
    return Workload(f"3d-{side}-atoms{n_atoms}-bin-1e-4", f, bin_quantize(f, xi), xi, 4, 6,
                    {"rel": 1e-4, "ghat": "bin", "seed": seed})


def lognormal_case(side: int, seed: int, rel: float = 1e-4) -> Workload:
    """3D lognormal field (the served mix's large requests) at any side; g_hat = 2*xi bins."""
    rng = np.random.default_rng(seed)
    f = lognormal3d(side, seed, rng=rng)
    xi = xi_from_relative(f, rel)
    return Workload(f"3d-{side}-lognormal-bin-{rel:g}", f, bin_quantize(f, xi), xi, 4, 6,
                    {"rel": rel, "ghat": "bin", "seed": seed})


def _mix_field(rng: np.random.Generator, dim: int, side: int, seed: int) -> np.ndarray:
    """n-D field from the 2D generators: coin picks Gaussians+noise or Gaussians+value noise."""
    kind = int(rng.integers(0, 2))
    shape = (side,) * dim
    # Gaussian count scaled from the 128^2 (16 Gaussians) and 2048^2 (256 Gaussians) fields by
    # cross-section area, at least 2 resp. 4.
    n_small = max(2, int(round(16 * (side / 128.0) ** 2)))
    n_large = max(4, int(round(256 * (side / 2048.0) ** 2)))
    n = n_small if kind == 0 else n_large
    centres = rng.uniform(0.0, side, size=(n, dim))
    scale = 1.0 if kind == 0 else side / 128.0
    sig = rng.uniform(3.0 * scale, 12.0 * scale, size=n)
    amp = rng.uniform(-1.0, 1.0, size=n)
    z = np.zeros(shape, dtype=np.float64)
    axes = [np.arange(side, dtype=np.float64)] * dim
    for c, s, a in zip(centres, sig, amp):
        g = None
        for ax in range(dim):
            gg = np.exp(-0.5 * ((axes[ax] - c[dim - 1 - ax]) / s) ** 2)
            bshape = [1] * dim
            bshape[ax] = side
            gg = gg.reshape(bshape)
            g = gg if g is None else g * gg
        z += a * g
    if kind == 0:
        z += rng.uniform(0.0, 1e-3, size=shape)
    else:
        for o in range(4):
            period = max(2, side // 8 // (2 ** o))
            z += 0.05 * (0.5 ** o) * _value_noise(shape, period, rng)
    return _normalize01(z).astype(np.float32)


def batch_field(batch: int, i: int, n_fields: int = 64) -> Workload:
    """Field i of batch `batch`: 2D (side log-uniform [256,1024]) for the first half, else 3D
    (side log-uniform [64,160]); each field draws from its own generator."""
    rng = np.random.default_rng([4000 + batch, i])
    dim = 2 if i < n_fields // 2 else 3
    lo, hi = (256, 1024) if dim == 2 else (64, 160)
    side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    f = _mix_field(rng, dim, side, 4000 + batch)
    rel = 1e-3 if rng.integers(0, 2) == 0 else 1e-4
    xi = xi_from_relative(f, rel)
    g = bin_quantize(f, xi) if rng.integers(0, 2) == 0 else uniform_noise(f, xi, rng)
    return Workload(f"batch{batch}-{i}-{dim}d-{side}", f, g, xi, 4, 6, {"rel": rel, "batch": batch, "index": i})


def batch_mix(batch: int = 0, n_fields: int = 64) -> list:
    """Batch of uneven fields: half 2D (side log-uniform [256,1024]), half 3D (side log-uniform [64,160])."""
    return [batch_field(batch, i, n_fields) for i in range(n_fields)]


def served_job(j: int, big_side: int = 384) -> Workload:
    """One request of the served stream: 5% are 3D lognormal fields (384^3), the rest like the batch mix."""
    rng = np.random.default_rng(5000 + j)
    if rng.uniform() < 0.05:
        f = lognormal3d(big_side, 5000 + j, rng=rng)
        xi = xi_from_relative(f, 1e-4)
        g = bin_quantize(f, xi) if rng.integers(0, 2) == 0 else uniform_noise(f, xi, rng)
        return Workload(f"serve{j}-3d-{big_side}-lognormal", f, g, xi, 4, 6, {"rel": 1e-4})
    dim = 2 if rng.integers(0, 2) == 0 else 3
    lo, hi = (256, 1024) if dim == 2 else (64, 160)
    side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    f = _mix_field(rng, dim, side, 5000 + j)
    xi = xi_from_relative(f, 1e-4)
    g = bin_quantize(f, xi) if rng.integers(0, 2) == 0 else uniform_noise(f, xi, rng)
    return Workload(f"serve{j}-{dim}d-{side}", f, g, xi, 4, 6, {"rel": 1e-4})


# ---------------------------------------------------------------------------------------------
# Small random cases for tests

def flow2d(ny: int, nx: int, seed: int, rel: float = 1e-4, ghat: str = "bin") -> Workload:
    """2D ny x nx field from the 2048^2 generator (Gaussians of width ~ side/128 * U[3,12] plus
    4-octave value noise) on a square of side max(ny, nx), cropped; the stand-in for the paper's
    2D climate and flow fields in the q_max sweep (150 x 450, Heated Flow's shape) and the tier
    study (361 x 576, IVT's shape).  g_hat = 2*xi bins or f + U[-xi, xi]."""
    rng = np.random.default_rng([seed, ny, nx])
    side = max(ny, nx)
    f = gauss2d_value_noise(side, max(4, int(round(256 * side * side / 2048 ** 2))), seed, rng=rng)
    f = _normalize01(f[:ny, :nx].astype(np.float64)).astype(np.float32)
    xi = xi_from_relative(f, rel)
    g = bin_quantize(f, xi) if ghat == "bin" else uniform_noise(f, xi, rng)
    return Workload(f"2d-{ny}x{nx}-flow-{ghat}-{rel:g}", f, g, xi, 4, 6, {"rel": rel, "ghat": ghat, "seed": seed})


def extreme_noise2d(side: int, seed: int, xi: float = 1e-4) -> Workload:
    """The paper's extreme case (Section 5.9): i.i.d. noise f ~ U[0, xi) with the absolute bound xi,
    so the 2*xi-bin quantizer returns an exactly flat g_hat = 0 and destroys every local order."""
    rng = np.random.default_rng([seed, side])
    xi32 = float(np.float32(xi))
    f = (rng.uniform(0.0, xi32, size=(side, side))).astype(np.float32)
    f = np.minimum(f, np.nextafter(np.float32(xi32), np.float32(0)))
    return Workload(f"2d-{side}-noise-flat-xi{xi:g}", f, bin_quantize(f, xi32), xi32, 4, 6,
                    {"abs": xi32, "ghat": "bin", "seed": seed})


def random_field(shape, kind: str, seed: int) -> np.ndarray:
    """Small test fields: 'uniform' U[0,1), 'plateau' (few distinct values, many ties),
    'perm' (a random permutation of 0..N-1), 'const' (all equal), 'smooth' (few Gaussians)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    if kind == "uniform":
        a = rng.uniform(0.0, 1.0, size=shape)
    elif kind == "plateau":
        a = rng.integers(0, 4, size=shape).astype(np.float64) * 0.25
    elif kind == "perm":
        a = rng.permutation(n).reshape(shape).astype(np.float64)
    elif kind == "const":
        a = np.full(shape, 0.5)
    elif kind == "smooth":
        grids = np.meshgrid(*[np.arange(s, dtype=np.float64) for s in shape], indexing="ij")
        a = np.zeros(shape)
        for _ in range(4):
            c = [rng.uniform(0, s) for s in shape]
            s = rng.uniform(1.0, max(shape) / 2.0)
            r2 = sum((g - cc) ** 2 for g, cc in zip(grids, c))
            a += rng.uniform(-1, 1) * np.exp(-0.5 * r2 / (s * s))
        a += rng.uniform(0, 1e-3, size=shape)
    else:
        raise ValueError(kind)
    return a.astype(np.float32)


def tiny_cases(seed: int, shape, rel: float = 0.05, kind: str = "uniform", ghat: str = "noise") -> Workload:
    """A small random job (for parity sweeps): field of the given kind, g_hat by noise or bins."""
    rng = np.random.default_rng([seed, 77])
    f = random_field(shape, kind, seed)
    xi = xi_from_relative(f, rel) if float(f.max()) > float(f.min()) else float(np.float32(rel))
    g = uniform_noise(f, xi, rng) if ghat == "noise" else bin_quantize(f, xi)
    return Workload(f"tiny-{kind}-{ghat}-{'x'.join(map(str, shape))}-{seed}", f, g, xi, 4, 6,
                    {"rel": rel})
