"""Seeded synthetic inputs for the primal-dual image sweep.

This module only draws random test scenes; it holds none of the solver's
arithmetic.  Both the FP64 oracle tests and the GPU path take their inputs from
here, so that the two sides start from the same float32 data.

Scenes are piecewise constant: a zero background painted (in draw order) with
random discs / axis-aligned rectangles (2D) or randomly rotated ellipsoids (3D),
each of intensity U[0, 1], followed by i.i.d. Gaussian noise.  No clipping.
Everything is generated in float64 with ``numpy.random.default_rng(seed)``;
callers cast to float32 for the device.

Pixel (y, x) has its centre at (y + 0.5, x + 0.5) in image coordinates.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "scene2d",
    "scene3d",
    "batch_sides",
    "batch_scenes",
    "phantom2d",
    "phantom_sinogram",
    "tomo_scene",
    "WORKLOADS",
]


def _paint_disc(img, cy, cx, r, val):
    H, W = img.shape
    y0 = max(int(math.floor(cy - r - 0.5)), 0)
    y1 = min(int(math.ceil(cy + r + 0.5)), H)
    x0 = max(int(math.floor(cx - r - 0.5)), 0)
    x1 = min(int(math.ceil(cx + r + 0.5)), W)
    if y0 >= y1 or x0 >= x1:
        return
    yy = np.arange(y0, y1)[:, None] + 0.5
    xx = np.arange(x0, x1)[None, :] + 0.5
    m = (yy - cy) ** 2 + (xx - cx) ** 2 <= r * r
    sub = img[y0:y1, x0:x1]
    sub[m] = val


def _paint_rect(img, ya, yb, xa, xb, val):
    H, W = img.shape
    # pixels whose centre lies inside [ya, yb] x [xa, xb]
    y0 = max(int(math.ceil(ya - 0.5)), 0)
    y1 = min(int(math.floor(yb - 0.5)) + 1, H)
    x0 = max(int(math.ceil(xa - 0.5)), 0)
    x1 = min(int(math.floor(xb - 0.5)) + 1, W)
    if y0 < y1 and x0 < x1:
        img[y0:y1, x0:x1] = val


def scene2d(H: int, W: int, n_shapes: int = 20, noise: float = 0.1,
            seed: int = 0):
    """Return ``(clean, noisy)`` float64 arrays of shape (H, W).

    Each shape is a disc or a rectangle with probability 1/2.  Disc centres are
    uniform over the image and radii U[0.02, 0.15] * min(H, W); rectangle
    corners are two uniform points, sorted per axis.
    """
    rng = np.random.default_rng(seed)
    img = np.zeros((H, W), dtype=np.float64)
    m = min(H, W)
    for _ in range(n_shapes):
        kind = rng.integers(0, 2)
        val = rng.uniform(0.0, 1.0)
        if kind == 0:
            cy = rng.uniform(0.0, H)
            cx = rng.uniform(0.0, W)
            r = rng.uniform(0.02, 0.15) * m
            _paint_disc(img, cy, cx, r, val)
        else:
            ys = np.sort(rng.uniform(0.0, H, size=2))
            xs = np.sort(rng.uniform(0.0, W, size=2))
            _paint_rect(img, ys[0], ys[1], xs[0], xs[1], val)
    noisy = img + rng.normal(0.0, noise, size=img.shape)
    return img, noisy


def _random_rotation(rng):
    # uniform random rotation from a unit quaternion (Shoemake's method)
    u1, u2, u3 = rng.uniform(0.0, 1.0, size=3)
    a = math.sqrt(1 - u1)
    b = math.sqrt(u1)
    w, x, y, z = (a * math.sin(2 * math.pi * u2), a * math.cos(2 * math.pi * u2),
                  b * math.sin(2 * math.pi * u3), b * math.cos(2 * math.pi * u3))
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def scene3d(D: int, H: int, W: int, n_shapes: int = 32, noise: float = 0.1,
            seed: int = 0):
    """Return ``(clean, noisy)`` float64 volumes of shape (D, H, W).

    Randomly rotated ellipsoids, centres uniform over the volume, semi-axes
    U[0.05, 0.25] * min(D, H, W), intensity U[0, 1], painter's order.
    """
    rng = np.random.default_rng(seed)
    vol = np.zeros((D, H, W), dtype=np.float64)
    m = min(D, H, W)
    dims = np.array([D, H, W], dtype=np.float64)
    for _ in range(n_shapes):
        c = rng.uniform(0.0, 1.0, size=3) * dims
        ax = rng.uniform(0.05, 0.25, size=3) * m
        Rm = _random_rotation(rng)
        val = rng.uniform(0.0, 1.0)
        rmax = float(ax.max())
        lo = np.maximum(np.floor(c - rmax - 0.5).astype(int), 0)
        hi = np.minimum(np.ceil(c + rmax + 0.5).astype(int), [D, H, W])
        if np.any(lo >= hi):
            continue
        zz = np.arange(lo[0], hi[0])[:, None, None] + 0.5 - c[0]
        yy = np.arange(lo[1], hi[1])[None, :, None] + 0.5 - c[1]
        xx = np.arange(lo[2], hi[2])[None, None, :] + 0.5 - c[2]
        # coordinates in the ellipsoid frame: Rm^T (v - c)
        e0 = Rm[0, 0] * zz + Rm[1, 0] * yy + Rm[2, 0] * xx
        e1 = Rm[0, 1] * zz + Rm[1, 1] * yy + Rm[2, 1] * xx
        e2 = Rm[0, 2] * zz + Rm[1, 2] * yy + Rm[2, 2] * xx
        m_in = (e0 / ax[0]) ** 2 + (e1 / ax[1]) ** 2 + (e2 / ax[2]) ** 2 <= 1.0
        sub = vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        sub[m_in] = val
    noisy = vol + rng.normal(0.0, noise, size=vol.shape)
    return vol, noisy


def batch_sides(n: int, seed: int, lo: int = 128, hi: int = 1024):
    """Image sides (H, W), each i.i.d. round(exp(U[ln lo, ln hi]))."""
    rng = np.random.default_rng(seed)
    s = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=(n, 2))))
    return [(int(h), int(w)) for h, w in s]


def batch_scenes(n: int = 64, seed: int = 3000, n_shapes: int = 20,
                 lo: int = 128, hi: int = 1024):
    """Uneven batch: sides from :func:`batch_sides` (seed ``seed``), image i
    drawn by :func:`scene2d` with seed ``seed + 1 + i`` and noise level
    U[0.05, 0.2] drawn from the side generator's stream."""
    sides = batch_sides(n, seed, lo, hi)
    rng = np.random.default_rng(seed + 100000)
    noises = rng.uniform(0.05, 0.2, size=n)
    out = []
    for i, (h, w) in enumerate(sides):
        clean, noisy = scene2d(h, w, n_shapes, float(noises[i]), seed + 1 + i)
        out.append((clean, noisy, float(noises[i])))
    return out


def phantom2d(H: int, W: int, n_ellipses: int = 32, seed: int = 0):
    """Random ellipse phantom inside the disc inscribed in the image.

    Returns ``(image, ellipses)``.  Each ellipse is a tuple
    ``(cx, cy, a, b, phi, rho)``: centre relative to the image centre (x along
    columns, y along rows, pixel units), semi-axes a, b of U[0.02, 0.15] * m
    (m = min(H, W)), rotation phi of its a-axis from the x-axis, U[0, pi), and
    intensity rho of U[0.1, 1].  Centres lie within 0.3 m of the image centre,
    so every ellipse stays inside radius 0.45 m.  Intensities add where
    ellipses overlap; the image samples the phantom at pixel centres
    (b + 1/2 - W/2, a + 1/2 - H/2).
    """
    rng = np.random.default_rng(seed)
    m = float(min(H, W))
    ell = []
    for _ in range(n_ellipses):
        rc = 0.3 * m * math.sqrt(rng.uniform(0.0, 1.0))
        ac = rng.uniform(0.0, 2.0 * math.pi)
        a, b = rng.uniform(0.02, 0.15, size=2) * m
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.1, 1.0)
        ell.append((rc * math.cos(ac), rc * math.sin(ac), float(a), float(b),
                    float(phi), float(rho)))
    x = (np.arange(W) + 0.5 - W / 2.0)[None, :]
    y = (np.arange(H) + 0.5 - H / 2.0)[:, None]
    img = np.zeros((H, W), dtype=np.float64)
    for cx, cy, a, b, phi, rho in ell:
        c, s = math.cos(phi), math.sin(phi)
        u = (x - cx) * c + (y - cy) * s
        v = -(x - cx) * s + (y - cy) * c
        img += rho * ((u / a) ** 2 + (v / b) ** 2 <= 1.0)
    return img, ell


def phantom_sinogram(ellipses, n_angles: int, n_det: int, noise: float = 0.0,
                     seed: int = 0):
    """Synthetic measurements of a :func:`phantom2d` phantom.

    Exact line integrals of the continuous phantom (sum over ellipses of
    rho times the chord length) along the lines {X . (cos theta, sin theta) =
    t}, theta_k = k pi / n_angles, t_i = i + 1/2 - n_det / 2, plus Gaussian
    noise of standard deviation ``noise`` times the largest clean value.
    Returns ``(clean, noisy)`` of shape (n_angles, n_det).
    """
    th = (np.arange(n_angles) * (math.pi / n_angles))[:, None]
    t = (np.arange(n_det) + 0.5 - n_det / 2.0)[None, :]
    out = np.zeros((n_angles, n_det), dtype=np.float64)
    for cx, cy, a, b, phi, rho in ellipses:
        ct = cx * np.cos(th) + cy * np.sin(th)          # centre's offset
        h2 = (a * np.cos(th - phi)) ** 2 + (b * np.sin(th - phi)) ** 2
        d2 = h2 - (t - ct) ** 2
        out += np.where(d2 > 0.0,
                        rho * 2.0 * a * b * np.sqrt(np.maximum(d2, 0.0)) / h2,
                        0.0)
    rng = np.random.default_rng(seed + 1)
    noisy = out + rng.normal(0.0, noise * float(out.max(initial=0.0)),
                             size=out.shape)
    return out, noisy


def tomo_scene(H: int, W: int, n_angles: int, n_det: int,
               n_ellipses: int = 32, noise: float = 0.01, seed: int = 0):
    """``(image, clean sinogram, noisy sinogram)`` of one phantom."""
    img, ell = phantom2d(H, W, n_ellipses, seed)
    clean, noisy = phantom_sinogram(ell, n_angles, n_det, noise, seed)
    return img, clean, noisy


# The six workloads, by what they are.
WORKLOADS = {
    "denoise_256": dict(kind="2d", H=256, W=256, n_shapes=20, noise=0.1,
                        seed=1000, lam=0.1, iters=1000),
    "denoise_4096": dict(kind="2d", H=4096, W=4096, n_shapes=200, noise=0.1,
                         seed=2000, lam=0.1, iters=2000),
    "batch64_uneven": dict(kind="batch", n=64, seed=3000, n_shapes=20,
                           lam=0.1, gap_tol=1e-4, check_every=10,
                           max_iter=20000),
    "unrolled_32x512": dict(kind="unrolled2d", B=32, H=512, W=512,
                            n_shapes=20, noise=0.1, seed=4000, K=20),
    "unrolled_256cube": dict(kind="unrolled3d", D=256, H=256, W=256,
                             n_shapes=32, noise=0.1, seed=5000, K=100,
                             ckpt_every=10),
    # a 2048^2 slice from 1000 projections of 2048 rays: the size of the
    # paper's measured sinograms (Section 7)
    "tomo_2048x1000": dict(kind="tomo", H=2048, W=2048, n_angles=1000,
                           n_det=2048, n_ellipses=32, noise=0.01, seed=6000,
                           lam=10.0, iters=20),
}
