"""Post-process passes of the frame (section 2.1: the engine's compute system
runs a screen-space roughness approximation and fast approximate
anti-aliasing on the traced image) -- TEST INFRASTRUCTURE ONLY, plain NumPy
in FP64, vectorised over pixels and nothing else.

The paper names the two passes and gives no detail; the readings written out
here are:

roughness_blur
    A material-aware Gaussian blur whose width follows the roughness of the
    material seen at each pixel (the primary hit's material; sky pixels and
    materials with roughness below 1/256 are left as they are).  Two 1-D
    passes, along x then along y, each over the taps k = -R..R of the window
    `radius` R, with weights exp(-k^2 / (2 sigma^2)), sigma = r R / 3 (r the
    centre pixel's roughness, clamped to [0, 1]); a tap counts only if it lies
    inside the image and shows the centre pixel's material, and the weights
    are normalised over the taps that count.  Both passes use the centre
    pixel's sigma and material.

fxaa
    Lottes' fast approximate anti-aliasing (NVIDIA whitepaper, 2009; the
    "quality" variant), restated: perceptual luma L = sqrt(clamp(0.299 R +
    0.587 G + 0.114 B, 0, 1)); a pixel whose 4-neighbourhood luma range is
    below max(T_MIN, T_REL * max luma) is left as it is; otherwise the edge
    is horizontal if the weighted second differences across rows are at
    least those across columns; the steeper of the two neighbours across the
    edge picks the side; from the point half a pixel towards that side the
    edge is followed both ways with the steps STEPS, sampling the luma image
    bilinearly (clamped at the borders), until the luma departs from the
    average of the pixel and that neighbour by a quarter of the gradient;
    the nearer end gives an offset 0.5 - distance / span if the luma there
    moves away from the pixel's, else 0; a sub-pixel offset grows with how
    far the pixel's luma is from its 3x3 low-pass (smoothstep squared, times
    SUBPIX); the pixel becomes the bilinear sample of the image at the larger
    offset towards that side.  Addressing is clamp-to-edge throughout.

Every comparison that float32 could decide otherwise than FP64 (the
contrast test, the edge orientation, the steeper side, each end test, the
sign tests) contributes |a - b| to a per-pixel margin; a pixel whose margin is
below DECIDE_EPS is ambiguous.  Ties of the two search distances are exact in
both precisions (multiples of 1/2) and are reported separately.
"""
from __future__ import annotations

import numpy as np

MISS = 0xFFFFFFFF
ROUGH_MIN = 1.0 / 256.0
T_REL = 0.125
T_MIN = 0.0625
SUBPIX = 0.75
STEPS = (1.0, 1.0, 1.0, 1.0, 1.0, 1.5, 2.0, 2.0, 2.0, 2.0, 4.0, 8.0)
DECIDE_EPS = 1e-5


def roughness_blur(img: np.ndarray, mat: np.ndarray, rough: np.ndarray, radius: int) -> np.ndarray:
    """img f[H,W,3]; mat u32[H,W] (MISS = sky); rough f[n_mats]; radius >= 0."""
    img = np.asarray(img, np.float64)
    mat = np.asarray(mat, np.uint32)
    rough = np.asarray(rough, np.float64).reshape(-1)
    H, W = mat.shape
    n = rough.shape[0]
    known = (mat != MISS) & (mat < n)
    r = np.where(known, np.clip(rough[np.minimum(mat, n - 1)], 0.0, 1.0), 0.0)
    active = known & (r >= ROUGH_MIN) & (radius > 0)
    sigma = r * radius / 3.0
    inv = np.where(active, 1.0 / (2.0 * np.where(active, sigma, 1.0) ** 2), 0.0)
    yy, xx = np.mgrid[0:H, 0:W]

    def one_pass(src, along_x):
        num = np.zeros_like(src)
        den = np.zeros((H, W))
        for k in range(-radius, radius + 1):
            if along_x:
                qx, qy = xx + k, yy
            else:
                qx, qy = xx, yy + k
            inside = (qx >= 0) & (qx < W) & (qy >= 0) & (qy < H)
            cx, cy = np.clip(qx, 0, W - 1), np.clip(qy, 0, H - 1)
            same = inside & (mat[cy, cx] == mat)
            w = np.where(same, np.exp(-(k * k) * inv), 0.0)
            num += w[..., None] * src[cy, cx]
            den += w
        return np.where(active[..., None], num / np.maximum(den, 1e-300)[..., None], src)

    return one_pass(one_pass(img, True), False)


def luma(img: np.ndarray) -> np.ndarray:
    img = np.asarray(img, np.float64)
    y = 0.299 * img[..., 0] + 0.587 * img[..., 1] + 0.114 * img[..., 2]
    return np.sqrt(np.clip(y, 0.0, 1.0))


def _bilinear(L, px, py):
    H, W = L.shape
    x0, y0 = np.floor(px), np.floor(py)
    fx, fy = px - x0, py - y0
    x0i, y0i = x0.astype(np.int64), y0.astype(np.int64)
    xa, xb = np.clip(x0i, 0, W - 1), np.clip(x0i + 1, 0, W - 1)
    ya, yb = np.clip(y0i, 0, H - 1), np.clip(y0i + 1, 0, H - 1)
    top = (1.0 - fx) * L[ya, xa] + fx * L[ya, xb]
    bot = (1.0 - fx) * L[yb, xa] + fx * L[yb, xb]
    return (1.0 - fy) * top + fy * bot


def fxaa(img: np.ndarray) -> dict:
    """img f[H,W,3].  Returns rgb f64[H,W,3], amb (margin below DECIDE_EPS),
    tie (equal search distances), active (the pixel passed the contrast
    test), offset (the blend weight) and the neighbour blended in (nx, ny)."""
    img = np.asarray(img, np.float64)
    H, W = img.shape[:2]
    L = luma(img)
    yy, xx = np.mgrid[0:H, 0:W]

    def at(dx, dy):
        return L[np.clip(yy + dy, 0, H - 1), np.clip(xx + dx, 0, W - 1)]

    m, n, s, w, e = L, at(0, -1), at(0, 1), at(-1, 0), at(1, 0)
    hi = np.maximum.reduce([m, n, s, w, e])
    lo = np.minimum.reduce([m, n, s, w, e])
    rng = hi - lo
    thr = np.maximum(T_MIN, hi * T_REL)
    active = rng >= thr
    margin = np.abs(rng - thr)

    nw, ne, sw, se = at(-1, -1), at(1, -1), at(-1, 1), at(1, 1)
    edge_h = np.abs(nw - 2.0 * w + sw) + 2.0 * np.abs(n - 2.0 * m + s) + np.abs(ne - 2.0 * e + se)
    edge_v = np.abs(nw - 2.0 * n + ne) + 2.0 * np.abs(w - 2.0 * m + e) + np.abs(sw - 2.0 * s + se)
    horiz = edge_h >= edge_v
    l1, l2 = np.where(horiz, n, w), np.where(horiz, s, e)
    g1, g2 = np.abs(l1 - m), np.abs(l2 - m)
    first = g1 >= g2
    sign = np.where(first, -1.0, 1.0)
    lavg = np.where(first, 0.5 * (l1 + m), 0.5 * (l2 + m))
    gscaled = 0.25 * np.maximum(g1, g2)
    dec = [np.abs(edge_h - edge_v), np.abs(g1 - g2), np.abs(m - lavg)]

    ex, ey = np.where(horiz, 1.0, 0.0), np.where(horiz, 0.0, 1.0)   # along the edge
    px, py = 1.0 - ex, 1.0 - ey                                        # across it
    cx, cy = xx + 0.5 * sign * px, yy + 0.5 * sign * py
    dist, dend = [], []
    for dirn in (-1.0, 1.0):
        t = np.zeros((H, W))
        done = np.zeros((H, W), bool)
        last = np.zeros((H, W))
        for step in STEPS:
            run = ~done
            t = np.where(run, t + step, t)
            d = _bilinear(L, cx + dirn * t * ex, cy + dirn * t * ey) - lavg
            last = np.where(run, d, last)
            dec.append(np.where(run, np.abs(np.abs(d) - gscaled), np.inf))
            done = done | (np.abs(d) >= gscaled)
        dist.append(t)
        dend.append(last)
    near_neg = dist[0] < dist[1]
    tie = dist[0] == dist[1]
    dmin = np.where(near_neg, dist[0], dist[1])
    d_end = np.where(near_neg, dend[0], dend[1])
    dec.append(np.abs(d_end))
    span = dist[0] + dist[1]
    good = (d_end < 0.0) != ((m - lavg) < 0.0)
    off_edge = np.where(good, 0.5 - dmin / span, 0.0)
    avg = (2.0 * (n + s + w + e) + (nw + ne + sw + se)) / 12.0
    sub1 = np.clip(np.abs(avg - m) / np.where(active, rng, 1.0), 0.0, 1.0)
    sub2 = (-2.0 * sub1 + 3.0) * sub1 * sub1
    off = np.maximum(off_edge, sub2 * sub2 * SUBPIX)

    margin = np.where(active, np.minimum(margin, np.minimum.reduce(dec)), margin)
    nx = np.clip(xx + (sign * px).astype(np.int64), 0, W - 1)
    ny = np.clip(yy + (sign * py).astype(np.int64), 0, H - 1)
    out = np.where(active[..., None], (1.0 - off)[..., None] * img + off[..., None] * img[ny, nx], img)
    return dict(rgb=out, amb=margin < DECIDE_EPS, tie=active & tie, active=active,
                offset=np.where(active, off, 0.0), nx=nx, ny=ny)
