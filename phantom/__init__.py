"""Seeded synthetic brain phantoms: the inputs that both sides of every check consume.

The paper evaluates on a simulated brain phantom with four classes (white
matter, grey matter, cerebrospinal fluid and background, Sec. 5.2) at 1 byte
per pixel (Sec. 4.2, Sec. 5.3).  Those data are not available here, so this
module draws stand-ins of the same shape and structure:

* labels: 0 background, 1 CSF, 2 GM, 3 WM, as nested ellipses (2-D) or
  ellipsoids (3-D) centred in the field of view; the CSF ellipse holds the GM
  ellipse, which holds the WM core;
* intensity ``I = clip(rint(mu[label] * b + sigma * n), 0, 255)`` as uint8,
  with class means ``mu``, a smooth multiplicative bias field
  ``b = 1 + A * s / max|s|``, ``s = prod_d cos(pi * u_d / 2 + phi_d)`` over the
  normalised coordinates ``u_d`` in (-1, 1), and standard normal noise ``n``;
* every random number comes from a counter-based generator (the SplitMix64
  output function applied to ``key + (k + 1) * 0x9E3779B97F4A7C15`` for draw
  ``k``), so a voxel's value depends only on (seed, voxel index), never on
  chunking or call order.  Normals use the Box-Muller transform on draws
  ``2i`` and ``2i + 1``.

This module contains no clustering arithmetic.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "PhantomParams",
    "phantom",
    "phantom_2d",
    "phantom_3d",
    "counter_u64",
    "uniform01",
    "uniform24",
    "normal01",
    "jittered_params",
    "batch_instances",
    "sha256",
]

_GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_U64 = (1 << 64) - 1

# Stream salts: one independent stream per use.
_SALT_NOISE = 0x6E6F6973
_SALT_PHASE = 0x70686173
_SALT_JITTER = 0x6A697474
_SALT_BATCH = 0x62617463

MEANS = (0.0, 40.0, 110.0, 150.0)
# Semi-axes as fractions of the half-extent, per class, ordered (x, y, z).
AXES = {
    1: (0.90, 0.80, 0.85),  # CSF (outer)
    2: (0.80, 0.70, 0.75),  # GM
    3: (0.55, 0.45, 0.50),  # WM (core)
}


def _mix_int(z: int) -> int:
    z &= _U64
    z = ((z ^ (z >> 30)) * _M1) & _U64
    z = ((z ^ (z >> 27)) * _M2) & _U64
    return z ^ (z >> 31)


def _key(seed: int, salt: int) -> int:
    return _mix_int((seed & _U64) ^ (salt * _GAMMA & _U64))


def counter_u64(key: int, idx: np.ndarray) -> np.ndarray:
    """64-bit draw number ``idx`` of the stream ``key`` (vectorised)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(key & _U64) + (idx + np.uint64(1)) * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(key: int, idx: np.ndarray) -> np.ndarray:
    """Uniform doubles in (0, 1] with 53 random bits."""
    h = counter_u64(key, idx)
    return ((h >> np.uint64(11)).astype(np.float64) + 1.0) * (1.0 / 9007199254740992.0)


def uniform24(key: int, idx: np.ndarray) -> np.ndarray:
    """Uniform values in (0, 1] with 24 random bits, (top 24 bits + 1) / 2^24:
    exact in FP32 and FP64 alike."""
    h = counter_u64(key, idx)
    return ((h >> np.uint64(40)).astype(np.float64) + 1.0) * (1.0 / 16777216.0)


def normal01(key: int, idx: np.ndarray) -> np.ndarray:
    """Standard normals by Box-Muller on draws (2i, 2i+1)."""
    idx = np.asarray(idx, dtype=np.uint64)
    u1 = uniform01(key, idx * np.uint64(2))
    u2 = uniform01(key, idx * np.uint64(2) + np.uint64(1))
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


@dataclasses.dataclass(frozen=True)
class PhantomParams:
    shape: tuple            # (H, W) or (D, H, W), row-major, x fastest
    seed: int = 1
    sigma: float = 8.0      # noise standard deviation, intensity units
    bias: float = 0.10      # amplitude A of the multiplicative bias field
    means: tuple = MEANS    # class means (bg, CSF, GM, WM)
    axes: tuple = (AXES[1], AXES[2], AXES[3])  # semi-axis fractions (x, y, z) per class 1..3

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))


def _coords(length: int) -> np.ndarray:
    i = np.arange(length, dtype=np.float64)
    return 2.0 * (i + 0.5) / length - 1.0


def _phases(p: PhantomParams, ndim: int) -> np.ndarray:
    # phi_d ~ U[-1/2, 1/2], ordered (x, y, z)
    return uniform01(_key(p.seed, _SALT_PHASE), np.arange(ndim)) - 0.5


def phantom(p: PhantomParams, with_labels: bool = False, chunk_voxels: int = 1 << 22):
    """Generate the phantom; returns ``img`` (uint8, shape p.shape) and optionally labels."""
    shape = tuple(int(s) for s in p.shape)
    if len(shape) not in (2, 3) or min(shape) < 1:
        raise ValueError("shape must be (H, W) or (D, H, W) with positive sizes")
    ndim = len(shape)
    # axis order in the array is (z,) y, x; coordinates in (x, y, z) order
    ux = _coords(shape[-1])
    uy = _coords(shape[-2])
    uz = _coords(shape[0]) if ndim == 3 else None
    phi = _phases(p, ndim)
    cx = np.cos(np.pi * ux / 2.0 + phi[0])
    cy = np.cos(np.pi * uy / 2.0 + phi[1])
    smax = np.max(np.abs(cx)) * np.max(np.abs(cy))
    if ndim == 3:
        cz = np.cos(np.pi * uz / 2.0 + phi[2])
        smax *= np.max(np.abs(cz))
    means = np.asarray(p.means, dtype=np.float64)
    noise_key = _key(p.seed, _SALT_NOISE)

    n = p.n
    img = np.empty(n, dtype=np.uint8)
    lab = np.empty(n, dtype=np.uint8) if with_labels else None
    rows_per_chunk = max(1, chunk_voxels // shape[-1])
    # iterate over flattened rows (z*H + y) in chunks
    n_rows = n // shape[-1]
    for r0 in range(0, n_rows, rows_per_chunk):
        r1 = min(n_rows, r0 + rows_per_chunk)
        rows = np.arange(r0, r1)
        yi = rows % shape[-2]
        gy = uy[yi][:, None]
        gx = ux[None, :]
        s = cy[yi][:, None] * cx[None, :]
        if ndim == 3:
            zi = rows // shape[-2]
            gz = uz[zi][:, None]
            s = s * cz[zi][:, None]
        label = np.zeros((r1 - r0, shape[-1]), dtype=np.uint8)
        for cls in (1, 2, 3):
            a = p.axes[cls - 1]
            r2 = (gx / a[0]) ** 2 + (gy / a[1]) ** 2
            if ndim == 3:
                r2 = r2 + (gz / a[2]) ** 2
            label[r2 <= 1.0] = cls
        b = 1.0 + p.bias * (s / smax)
        idx = np.arange(r0 * shape[-1], r1 * shape[-1], dtype=np.uint64)
        val = means[label] * b + p.sigma * normal01(noise_key, idx).reshape(label.shape)
        img[r0 * shape[-1]: r1 * shape[-1]] = np.clip(np.rint(val), 0, 255).astype(np.uint8).ravel()
        if with_labels:
            lab[r0 * shape[-1]: r1 * shape[-1]] = label.ravel()
    img = img.reshape(shape)
    if with_labels:
        return img, lab.reshape(shape)
    return img


def phantom_2d(h: int, w: int, seed: int = 1, with_labels: bool = False, **kw):
    return phantom(PhantomParams(shape=(h, w), seed=seed, **kw), with_labels=with_labels)


def phantom_3d(d: int, h: int, w: int, seed: int = 2, with_labels: bool = False, **kw):
    return phantom(PhantomParams(shape=(d, h, w), seed=seed, **kw), with_labels=with_labels)


def jittered_params(shape, seed: int) -> PhantomParams:
    """Per-phantom parameter draw for training/evaluation sets of the warm start.

    Class means jittered by up to +-15 % (order kept, background stays 0),
    sigma ~ U[3, 10], bias amplitude ~ U[0, 0.2], semi-axes scaled by up to +-10 %.
    """
    key = _key(seed, _SALT_JITTER)
    u = uniform01(key, np.arange(16))
    m = [0.0]
    for k, base in enumerate(MEANS[1:]):
        m.append(base * (1.0 + 0.30 * (u[k] - 0.5)))
    m = sorted(m)
    sigma = 3.0 + 7.0 * u[4]
    bias = 0.2 * u[5]
    scale = 1.0 + 0.20 * (u[6:9] - 0.5)
    axes = tuple(tuple(float(a * s) for a, s in zip(AXES[c], scale)) for c in (1, 2, 3))
    return PhantomParams(shape=tuple(shape), seed=seed, sigma=float(sigma), bias=float(bias),
                         means=tuple(float(x) for x in m), axes=axes)


def batch_instances(count_2d: int = 496, count_3d: int = 16, seed: int = 4000):
    """Instance list of the batched workload: square slices with side ~ U{64..512}
    and cubes with side ~ U{96..160}; cluster count C_i ~ U{3..8}.

    Returns a list of (PhantomParams, C_i)."""
    key = _key(seed, _SALT_BATCH)
    out = []
    total = count_2d + count_3d
    u = uniform01(key, np.arange(2 * total))
    for i in range(total):
        c = 3 + min(5, int(u[2 * i + 1] * 6))
        if i < count_2d:
            side = 64 + min(448, int(u[2 * i] * 449))
            shape = (side, side)
        else:
            side = 96 + min(64, int(u[2 * i] * 65))
            shape = (side, side, side)
        out.append((PhantomParams(shape=shape, seed=seed + i), c))
    return out


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()
