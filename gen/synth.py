"""Seeded synthetic float images with the structure of the paper's workloads.

The paper measures on natural photographs and microCT volumes that are not
available here (Evaluation and Results section, dataset paragraph). These
generators stand in for them with images whose gradients carry the same
structure: smooth regions whose quantised gradients form plateaux, sharp edges
and noise that create many small catchment basins.

Arrays are numpy C-order with x fastest: 2D arrays are (ny, nx), 3D arrays are
(nz, ny, nx), so the linear pixel index is x + nx*(y + ny*z) (row-major order,
as in the Step I description of the paper).

Every draw comes from numpy's PCG64 (`default_rng(seed)`) in a fixed order, so a
(recipe, seed) pair always gives the same bytes on every machine.
"""
from __future__ import annotations

import math

import numpy as np

# Workload table. `kind` names the generator, `sigma` is the Gaussian blur of
# the gradient pre-processing (0 = none), `dtype` the quantised gradient type.
CONFIGS = {
    # 256x256 u8, 32 blobs + 1 % salt, Sobel only, 4-conn, NL = 3.
    "blobs256": dict(kind="blobs2d", shape=(256, 256), seed=0, sigma=0.0, dtype="u8", conn=4, NL=3),
    # 4096x4096 u16, 2000 ellipses + N(0, 500^2), blur sigma 1 + Sobel, 8-conn, NL = 6.
    "ellipses4096": dict(kind="ellipses2d", shape=(4096, 4096), seed=1, sigma=1.0, dtype="u16", conn=8, NL=6),
    # 928^3 u8, 5000 blobs + N(0, 2^2), 3D Sobel, 6-conn, NL = 6.
    "blobs928": dict(kind="blobs3d", shape=(928, 928, 928), seed=2, sigma=0.0, dtype="u8", conn=6, NL=6),
}


def _rng(seed_or_rng):
    if isinstance(seed_or_rng, np.random.Generator):
        return seed_or_rng
    return np.random.default_rng(seed_or_rng)


def blobs2d(ny: int, nx: int, seed=0, n_blobs: int = 32, sigma=(8.0, 24.0),
            amp=(0.2, 1.0), salt: float = 0.01) -> np.ndarray:
    """Sum of isotropic Gaussian blobs plus salt pixels, float32 (ny, nx).

    Draw order: centres x, centres y, sigmas, amplitudes (n_blobs each), then
    the salt positions (without replacement). Each blob is evaluated inside its
    4-sigma box only. Salt pixels are set to the maximum of the blob sum.
    """
    rng = _rng(seed)
    cx = rng.uniform(0.0, nx, n_blobs)
    cy = rng.uniform(0.0, ny, n_blobs)
    sg = rng.uniform(sigma[0], sigma[1], n_blobs)
    am = rng.uniform(amp[0], amp[1], n_blobs)
    f = np.zeros((ny, nx), dtype=np.float64)
    for i in range(n_blobs):
        r = 4.0 * sg[i]
        x0, x1 = max(0, int(math.floor(cx[i] - r))), min(nx, int(math.ceil(cx[i] + r)) + 1)
        y0, y1 = max(0, int(math.floor(cy[i] - r))), min(ny, int(math.ceil(cy[i] + r)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        xs = np.arange(x0, x1, dtype=np.float64)[None, :] - cx[i]
        ys = np.arange(y0, y1, dtype=np.float64)[:, None] - cy[i]
        f[y0:y1, x0:x1] += am[i] * np.exp(-(xs * xs + ys * ys) / (2.0 * sg[i] * sg[i]))
    n_salt = int(round(salt * nx * ny))
    if n_salt > 0:
        idx = rng.choice(nx * ny, size=n_salt, replace=False)
        f.reshape(-1)[idx] = f.max()
    return f.astype(np.float32)


def ellipses2d(ny: int, nx: int, seed=1, n_ellipses: int = 2000, axes=(4.0, 128.0),
               intensity=(0.0, 65535.0), noise: float = 500.0) -> np.ndarray:
    """Filled ellipses painted in order onto 0, plus Gaussian noise, float32.

    Per ellipse, in this order: centre x, centre y ~ U[0, n); semi-axes a, b
    log-uniform in `axes`; angle ~ U[0, pi); intensity ~ U(intensity). Later
    ellipses overwrite earlier ones. Then N(0, noise^2) is added (not clipped).
    """
    rng = _rng(seed)
    f = np.zeros((ny, nx), dtype=np.float64)
    la, lb = math.log(axes[0]), math.log(axes[1])
    for _ in range(n_ellipses):
        cx = rng.uniform(0.0, nx)
        cy = rng.uniform(0.0, ny)
        a = math.exp(rng.uniform(la, lb))
        b = math.exp(rng.uniform(la, lb))
        th = rng.uniform(0.0, math.pi)
        v = rng.uniform(intensity[0], intensity[1])
        r = max(a, b)
        x0, x1 = max(0, int(math.floor(cx - r))), min(nx, int(math.ceil(cx + r)) + 1)
        y0, y1 = max(0, int(math.floor(cy - r))), min(ny, int(math.ceil(cy + r)) + 1)
        if x0 >= x1 or y0 >= y1:
            continue
        dx = np.arange(x0, x1, dtype=np.float64)[None, :] - cx
        dy = np.arange(y0, y1, dtype=np.float64)[:, None] - cy
        c, s = math.cos(th), math.sin(th)
        u = (dx * c + dy * s) / a
        w = (-dx * s + dy * c) / b
        inside = (u * u + w * w) <= 1.0
        f[y0:y1, x0:x1][inside] = v
    if noise > 0:
        f += rng.normal(0.0, noise, size=f.shape)
    return f.astype(np.float32)


def blobs3d(nz: int, ny: int, nx: int, seed=2, n_blobs: int = 5000, sigma=(4.0, 32.0),
            amp=(0.2, 1.0), scale: float = 255.0, noise: float = 2.0) -> np.ndarray:
    """Sum of isotropic 3D Gaussian blobs plus Gaussian noise, float32 (nz, ny, nx).

    Draw order: centres x, y, z, sigmas, amplitude factors (n_blobs each), then
    the noise field. Amplitude = scale * U(amp). Each blob is evaluated inside
    its 4-sigma box only (as a separable product of 1D Gaussians).
    """
    rng = _rng(seed)
    cx = rng.uniform(0.0, nx, n_blobs)
    cy = rng.uniform(0.0, ny, n_blobs)
    cz = rng.uniform(0.0, nz, n_blobs)
    sg = rng.uniform(sigma[0], sigma[1], n_blobs)
    am = scale * rng.uniform(amp[0], amp[1], n_blobs)
    f = np.zeros((nz, ny, nx), dtype=np.float64)
    for i in range(n_blobs):
        r = 4.0 * sg[i]
        lo = [max(0, int(math.floor(c - r))) for c in (cx[i], cy[i], cz[i])]
        hi = [min(n, int(math.ceil(c + r)) + 1) for c, n in ((cx[i], nx), (cy[i], ny), (cz[i], nz))]
        if any(a >= b for a, b in zip(lo, hi)):
            continue
        k = -1.0 / (2.0 * sg[i] * sg[i])
        gx = np.exp(k * (np.arange(lo[0], hi[0]) - cx[i]) ** 2)
        gy = np.exp(k * (np.arange(lo[1], hi[1]) - cy[i]) ** 2)
        gz = np.exp(k * (np.arange(lo[2], hi[2]) - cz[i]) ** 2)
        f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += am[i] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
    if noise > 0:
        f += rng.normal(0.0, noise, size=f.shape)
    return f.astype(np.float32)


def config_image(name: str) -> np.ndarray:
    """The float image of a named workload (blobs256, ellipses4096; blobs928 is too large for numpy here)."""
    c = CONFIGS[name]
    if c["kind"] == "blobs2d":
        return blobs2d(*c["shape"], seed=c["seed"])
    if c["kind"] == "ellipses2d":
        return ellipses2d(*c["shape"], seed=c["seed"])
    if c["kind"] == "blobs3d":
        return blobs3d(*c["shape"], seed=c["seed"])
    raise KeyError(name)


def batch_sizes(n_images: int = 512, base_seed: int = 3000, lo: int = 128, hi: int = 2048):
    """(ny, nx) of the uneven batch: each side round(exp(U[ln lo, ln hi])), seed base+i."""
    out = []
    for i in range(n_images):
        rng = np.random.default_rng(base_seed + i)
        ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append((ny, nx))
    return out


def batch_image(i: int, base_seed: int = 3000, lo: int = 128, hi: int = 2048) -> np.ndarray:
    """Image i of the uneven batch: sizes as in `batch_sizes`, then blobs2d content."""
    rng = np.random.default_rng(base_seed + i)
    ny = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    nx = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
    return blobs2d(ny, nx, seed=rng)


def paper_row(n: int, lo_left: int = 75, plateau: int = 89, lo_right: int = 81) -> np.ndarray:
    """The (2n+2) x 1 worst-case row of the Step II discussion: 75, 89 x 2n, 81."""
    row = np.full((1, 2 * n + 2), plateau, dtype=np.uint16)
    row[0, 0] = lo_left
    row[0, -1] = lo_right
    return row


def serpentine(ny: int, nx: int, wall: int = 9, corridor: int = 5, exit_value: int = 0) -> np.ndarray:
    """A one-pixel-wide serpentine corridor (a single non-minimal plateau).

    Odd rows are open corridor; even rows are wall except one gap that joins
    consecutive corridor rows at alternating ends. The only pixel lower than the
    corridor sits above its start, so geodesic distances grow to about nx*ny/2.
    """
    img = np.full((ny, nx), wall, dtype=np.uint16)
    rows = list(range(1, ny - 1, 2))
    for k, y in enumerate(rows):
        img[y, 1:nx - 1] = corridor
        if k + 1 < len(rows) and y + 1 < ny - 1:
            gx = nx - 2 if k % 2 == 0 else 1
            img[y + 1, gx] = corridor
    img[0, 1] = exit_value
    return img


def blobs_device(shape, seed, n_blobs, sigma, amp=(0.2, 1.0), scale=1.0, noise=0.0, salt=0.0, device="cuda:0"):
    """The blob recipe evaluated on a torch device in float32 (pools of large
    serving inputs). Parameters are drawn with PCG64 in the order of
    blobs2d / blobs3d (centres x, y[, z], sigmas, amplitudes, then salt
    positions or the noise field); each blob covers its 4-sigma box."""
    import torch
    rng = _rng(seed)
    nd = len(shape)
    dims = list(reversed(shape))  # x, y[, z]
    cs = [rng.uniform(0.0, dims[a], n_blobs) for a in range(nd)]
    sg = rng.uniform(sigma[0], sigma[1], n_blobs)
    am = scale * rng.uniform(amp[0], amp[1], n_blobs)
    f = torch.zeros(shape, dtype=torch.float32, device=device)
    for i in range(n_blobs):
        r = 4.0 * sg[i]
        lo = [max(0, int(math.floor(cs[a][i] - r))) for a in range(nd)]
        hi = [min(dims[a], int(math.ceil(cs[a][i] + r)) + 1) for a in range(nd)]
        if any(l >= h for l, h in zip(lo, hi)):
            continue
        k = -1.0 / (2.0 * sg[i] * sg[i])
        g1 = [torch.exp(k * (torch.arange(lo[a], hi[a], device=device, dtype=torch.float32) - float(cs[a][i])) ** 2)
              for a in range(nd)]
        if nd == 2:
            f[lo[1]:hi[1], lo[0]:hi[0]] += float(am[i]) * g1[1][:, None] * g1[0][None, :]
        else:
            f[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += float(am[i]) * (g1[2][:, None, None] * g1[1][None, :, None]
                                                                          * g1[0][None, None, :])
    n = f.numel()
    if salt > 0:
        idx = rng.choice(n, size=int(round(salt * n)), replace=False)
        f.view(-1)[torch.from_numpy(idx).to(device)] = f.max()
    if noise > 0:
        f += torch.from_numpy(rng.normal(0.0, noise, size=shape).astype(np.float32)).to(device)
    return f


def blobs3d_device(shape=(928, 928, 928), seed: int = 2, n_blobs=None, sigma=(4.0, 32.0), amp=(0.2, 1.0),
                   scale: float = 255.0, noise: float = 2.0, device="cuda:0"):
    """The 928^3 volume recipe (blobs3d's parameters) evaluated on a torch
    device in float32, for volumes too large for numpy. Blob centres, sigmas and
    amplitudes are drawn with PCG64 in blobs3d's order; n_blobs defaults to
    5000 scaled by volume / 928^3 (the 928^3 density). The N(0, noise^2) field
    comes from torch's seeded device generator (Philox), so it differs from
    blobs3d's host noise but is fixed by (seed, shape)."""
    import torch
    if n_blobs is None:
        n_blobs = max(1, int(round(5000 * float(np.prod(shape)) / 928.0 ** 3)))
    f = blobs_device(shape, seed, n_blobs, sigma, amp=amp, scale=scale, noise=0.0, device=device)
    if noise > 0:
        g = torch.Generator(device=device)
        g.manual_seed(int(seed) * 1_000_003 + 17)
        f += noise * torch.randn(tuple(shape), generator=g, device=device, dtype=torch.float32)
    return f


def serving_pool_specs(n2d: int = 24, n3d: int = 8, seed: int = 4):
    """Job shapes of the serving mix: square 2D sides log-uniform in
    [512, 4096] (8-connectivity), cubic 3D sides log-uniform in [128, 512]
    (6-connectivity); 3D blob count at the 928^3 recipe's density."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n2d):
        s = int(round(math.exp(rng.uniform(math.log(512), math.log(4096)))))
        specs.append(dict(shape=(s, s), conn=8, seed=4_000_000 + i, n_blobs=32, sigma=(8.0, 24.0), salt=0.01,
                          noise=0.0, scale=1.0))
    for i in range(n3d):
        s = int(round(math.exp(rng.uniform(math.log(128), math.log(512)))))
        nb = max(1, int(round(5000 * (s / 928.0) ** 3)))
        specs.append(dict(shape=(s, s, s), conn=6, seed=4_100_000 + i, n_blobs=nb, sigma=(4.0, 32.0), salt=0.0,
                          noise=2.0, scale=255.0))
    return specs
