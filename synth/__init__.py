"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws phantoms and noise only. It contains none of the
reconstruction method's arithmetic (no projector, no Krylov step, no
regularisation), so that both sides of a parity test can take their inputs
from here without sharing any computation.

Conventions (the paper specifies none of these; they are choices of this package):

* Random streams: ``numpy.random.default_rng([cfg_id, idx, stream])`` (PCG64),
  with stream 0 = phantom, 1 = noise vector, 2 = noise level.
* 2D pixel (i, j) has its centre at X_j = j - (nx-1)/2, Y_i = i - (ny-1)/2,
  unit pixel size, image stored row-major ``[ny][nx]``.
* 3D voxel (k, i, j) has its centre at (X_j, Y_i, Z_k) with the same rule,
  stored ``[nz][ny][nx]``.
* Phantoms are sums of uniform ellipses (2D) or ellipsoids (3D) with
  intensities in U[0.1, 1], 5 to 10 of them, semi-axes U[0.05, 0.25]*N, each
  lying inside the inscribed circle/sphere of radius 0.45*N.  Pixel values are
  the mean over s x s sub-samples (4x4 in 2D, 2x2x2 in 3D).
* Noise follows the usual relative-noise model of CT experiments: e is a
  Gaussian direction scaled so that ||e|| = eta * ||b_true||.
"""
from __future__ import annotations

import math

import numpy as np

STREAM_PHANTOM = 0
STREAM_NOISE = 1
STREAM_LEVEL = 2


def rng_for(cfg_id: int, idx: int, stream: int) -> np.random.Generator:
    """The generator for (configuration, sample index, stream)."""
    return np.random.default_rng([int(cfg_id), int(idx), int(stream)])


# --------------------------------------------------------------------------
# 2D ellipse phantoms
# --------------------------------------------------------------------------

def ellipse_params(rng: np.random.Generator, n: int, count=None) -> np.ndarray:
    """Random ellipses for an n x n image.

    Returns an array of rows (cx, cy, a, b, phi, rho): centre, semi-axes,
    rotation angle of the ``a`` axis from the x axis, and density.
    """
    if count is None:
        count = int(rng.integers(5, 11))
    rows = []
    for _ in range(count):
        rho = rng.uniform(0.1, 1.0)
        a = rng.uniform(0.05, 0.25) * n
        b = rng.uniform(0.05, 0.25) * n
        phi = rng.uniform(0.0, math.pi)
        rmax = 0.45 * n - max(a, b)
        # uniform point in a disk of radius rmax
        r = rmax * math.sqrt(rng.uniform(0.0, 1.0))
        t = rng.uniform(0.0, 2.0 * math.pi)
        rows.append((r * math.cos(t), r * math.sin(t), a, b, phi, rho))
    return np.asarray(rows, dtype=np.float64)


def rasterize_ellipses(params: np.ndarray, nx: int, ny: int | None = None,
                       sub: int = 4, device=None) -> np.ndarray:
    """Mean of sub x sub point samples per pixel of a sum of uniform ellipses.

    With ``device`` set (a torch device), the work runs in torch on that
    device in float64 and a torch tensor is returned; otherwise numpy.
    """
    ny = nx if ny is None else ny
    if device is not None:
        return _rasterize_ellipses_torch(params, nx, ny, sub, device)
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    xs = (np.arange(nx) - (nx - 1) / 2.0)[None, :, None] + offs[None, None, :]
    ys = (np.arange(ny) - (ny - 1) / 2.0)[:, None, None] + offs[None, None, :]
    img = np.zeros((ny, nx), dtype=np.float64)
    # sample grid: [ny, sub, nx, sub]
    X = xs[:, None, :, :].reshape(1, 1, nx, sub)
    Y = ys.reshape(ny, sub, 1, 1)
    for cx, cy, a, b, phi, rho in params:
        c, s = math.cos(phi), math.sin(phi)
        dx = X - cx
        dy = Y - cy
        u = dx * c + dy * s
        v = -dx * s + dy * c
        inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0
        img += rho * inside.mean(axis=(1, 3))
    return img


def _rasterize_ellipses_torch(params, nx, ny, sub, device):
    import torch
    offs = (torch.arange(sub, dtype=torch.float64, device=device) + 0.5) / sub - 0.5
    xs = (torch.arange(nx, dtype=torch.float64, device=device) - (nx - 1) / 2.0)
    ys = (torch.arange(ny, dtype=torch.float64, device=device) - (ny - 1) / 2.0)
    X = (xs[:, None] + offs[None, :]).reshape(1, 1, nx, sub)
    Y = (ys[:, None] + offs[None, :]).reshape(ny, sub, 1, 1)
    img = torch.zeros((ny, nx), dtype=torch.float64, device=device)
    for cx, cy, a, b, phi, rho in np.asarray(params).tolist():
        c, s = math.cos(phi), math.sin(phi)
        dx = X - cx
        dy = Y - cy
        u = dx * c + dy * s
        v = -dx * s + dy * c
        inside = ((u / a) ** 2 + (v / b) ** 2 <= 1.0).to(torch.float64)
        img += rho * inside.mean(dim=(1, 3))
    return img


def phantom2d(cfg_id: int, idx: int, n: int, sub: int = 4, device=None):
    """Seeded random-ellipse phantom (and its ellipse parameters)."""
    params = ellipse_params(rng_for(cfg_id, idx, STREAM_PHANTOM), n)
    return rasterize_ellipses(params, n, n, sub=sub, device=device), params


# --------------------------------------------------------------------------
# 3D ellipsoid phantoms
# --------------------------------------------------------------------------

def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation from a unit quaternion (Shoemake's method)."""
    u1, u2, u3 = rng.uniform(0.0, 1.0, size=3)
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2),
                  math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3),
                  math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    x, y, z, w = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_params(rng: np.random.Generator, n: int, count=None):
    """Random ellipsoids: list of (centre[3], semi-axes[3], rotation[3x3], rho)."""
    if count is None:
        count = int(rng.integers(5, 11))
    out = []
    for _ in range(count):
        rho = rng.uniform(0.1, 1.0)
        axes = rng.uniform(0.05, 0.25, size=3) * n
        rot = _random_rotation(rng)
        rmax = 0.45 * n - float(axes.max())
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        r = rmax * rng.uniform(0.0, 1.0) ** (1.0 / 3.0)
        out.append((d * r, axes, rot, rho))
    return out


def rasterize_ellipsoids(params, n: int, sub: int = 2, device=None):
    """Mean of sub^3 point samples per voxel of a sum of uniform ellipsoids.

    Returns a float64 array ``[n][n][n]`` (z, y, x).  Runs in torch when
    ``device`` is given (the 256^3 case is too slow in numpy).
    """
    import torch
    dev = torch.device("cpu") if device is None else device
    offs = (torch.arange(sub, dtype=torch.float64, device=dev) + 0.5) / sub - 0.5
    c = torch.arange(n, dtype=torch.float64, device=dev) - (n - 1) / 2.0
    vol = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    for centre, axes, rot, rho in params:
        R = torch.tensor(rot, dtype=torch.float64, device=dev)
        ctr = torch.tensor(centre, dtype=torch.float64, device=dev)
        ax = torch.tensor(axes, dtype=torch.float64, device=dev)
        # bounding box in voxel indices
        ext = float(np.max(axes)) + 1.0
        lo = [max(0, int(math.floor(centre[d] - ext + (n - 1) / 2.0))) for d in range(3)]
        hi = [min(n, int(math.ceil(centre[d] + ext + (n - 1) / 2.0)) + 1) for d in range(3)]
        acc = None
        for oz in offs:
            for oy in offs:
                for ox in offs:
                    X = c[lo[0]:hi[0]] + ox
                    Y = c[lo[1]:hi[1]] + oy
                    Z = c[lo[2]:hi[2]] + oz
                    pz, py, px = torch.meshgrid(Z - ctr[2], Y - ctr[1], X - ctr[0], indexing="ij")
                    p = torch.stack([px, py, pz], dim=-1)      # world xyz offsets
                    q = p @ R                                   # body coords: R^T p
                    ins = ((q / ax) ** 2).sum(-1) <= 1.0
                    acc = ins.to(torch.float64) if acc is None else acc + ins
        vol[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += rho * acc / float(sub ** 3)
    return vol if device is not None else vol.numpy()


def phantom3d(cfg_id: int, idx: int, n: int, sub: int = 2, device=None):
    params = ellipsoid_params(rng_for(cfg_id, idx, STREAM_PHANTOM), n)
    return rasterize_ellipsoids(params, n, sub=sub, device=device), params


# --------------------------------------------------------------------------
# Noise
# --------------------------------------------------------------------------

def noise_direction(cfg_id: int, idx: int, m: int) -> np.ndarray:
    """Standard normal vector g in R^m from the noise stream."""
    return rng_for(cfg_id, idx, STREAM_NOISE).standard_normal(m)


def noise_level(cfg_id: int, idx: int, lo: float, hi: float) -> float:
    """Per-sample noise level eta, log-uniform in [lo, hi]."""
    u = rng_for(cfg_id, idx, STREAM_LEVEL).uniform(math.log10(lo), math.log10(hi))
    return float(10.0 ** u)


def add_relative_noise(b_true: np.ndarray, g: np.ndarray, eta: float):
    """b = b_true + e with e = eta * ||b_true|| * g / ||g||.  Returns (b, ||e||)."""
    nb = float(np.linalg.norm(b_true))
    e = (eta * nb / float(np.linalg.norm(g))) * g
    return b_true + e, eta * nb


def default_ndet(n: int) -> int:
    """Detector bins covering the image diagonal: D = ceil(N*sqrt(2)) (odd-rounded)."""
    d = int(math.ceil(n * math.sqrt(2.0)))
    return d


# --------------------------------------------------------------------------
# Initial weights of the learned-rule network (64 -> 128 -> 128 -> 128 -> 2)
# --------------------------------------------------------------------------

MLP_LAYERS = [(128, 64), (128, 128), (128, 128), (2, 128)]


def mlp_init(seed: int) -> np.ndarray:
    """Flat float32 parameters [W1, b1, W2, b2, W3, b3, W4, b4]: He-normal
    weights (standard deviation sqrt(2 / fan_in)), zero biases."""
    r = np.random.default_rng([7, int(seed)])
    parts = []
    for o, i in MLP_LAYERS:
        parts.append(r.standard_normal(o * i) * math.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)
