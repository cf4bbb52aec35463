"""A float32 model of the traversal's ray/triangle arithmetic, for checking
the oracle's float32 error bands (beta, delta) against what float32 actually
does.  Test infrastructure: it imports neither the oracle nor the HIP
library, and shares no code with either.

It evaluates, with numpy in IEEE float32 (round to nearest even, no fused
multiply-add), the steps a float32 traversal takes for one instance and one
triangle: the world ray is mapped into object space in double with the
world->object matrix stored in float32 (its inverse computed in double and
rounded), the object-space origin is slid to where the ray enters the mesh's
box, and the triangle is tested in the ray-space shear of Woop, Benthin &
Wald (JCGT 2013): three 2-D edge functions U, V, W of the sheared vertices,
their sum det, and T with t = T * (1 / det) measured from the slid origin.
"""
import numpy as np

f32 = np.float32


def _inv3(m):
    """Inverse of the 3x3 linear parts m[..., 3, 3] in float64 (adjugate)."""
    a, b, c = m[..., 0, 0], m[..., 0, 1], m[..., 0, 2]
    d, e, f = m[..., 1, 0], m[..., 1, 1], m[..., 1, 2]
    g, h, k = m[..., 2, 0], m[..., 2, 1], m[..., 2, 2]
    A, B, C = e * k - f * h, -(d * k - f * g), d * h - e * g
    det = a * A + b * B + c * C
    rows = [[A, -(b * k - c * h), b * f - c * e],
            [B, a * k - c * g, -(a * f - c * d)],
            [C, -(a * h - b * g), a * e - b * d]]
    return np.stack([np.stack(r, -1) for r in rows], -2) * (1.0 / det)[..., None, None]  # as the GPU: one division


def trace_tri(xform, box_lo, box_hi, o, d, tmin, tmax, tri):
    """Vectorised over a leading axis n.  xform f32[n,3,4] object->world;
    box_lo/hi f32[n,3] the mesh's object-space box; o, d f32[n,3] the world
    ray; tmin, tmax f32[n]; tri f32[n,3,3] object-space vertices.
    Returns dict: hit (bool: inside by the edge-function signs, det != 0),
    t (world t = t0 + T/det, float32), u, v (float32), det."""
    xform = np.asarray(xform, f32)
    o, d = np.asarray(o, f32), np.asarray(d, f32)
    tmin, tmax = np.asarray(tmin, f32), np.asarray(tmax, f32)
    tri = np.asarray(tri, f32)
    inv = _inv3(xform[:, :, :3].astype(np.float64)).astype(f32).astype(np.float64)
    q = o.astype(np.float64) - xform[:, :, 3].astype(np.float64)
    od = np.einsum("nij,nj->ni", inv, q)
    dd = np.einsum("nij,nj->ni", inv, d.astype(np.float64))
    # slide to the box entry, in float32
    of, df = od.astype(f32), dd.astype(f32)
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        rr = f32(1.0) / np.where(np.abs(df) < f32(1e-30), np.copysign(f32(1e-30), df), df)
        a = (np.asarray(box_lo, f32) - of) * rr
        b = (np.asarray(box_hi, f32) - of) * rr
    ten = np.minimum(a, b).max(axis=1)
    tex = np.maximum(a, b).min(axis=1)
    ts = np.where((ten <= tex) & (ten > tmin), ten, tmin).astype(np.float64)
    ts = np.minimum(ts, tmax.astype(np.float64))
    t0 = ts.astype(f32)
    ox = (od + t0.astype(np.float64)[:, None] * dd).astype(f32)
    ld = dd.astype(f32)
    # shear constants: kz the largest |d| axis, (kx, ky) the next two in
    # cyclic order, swapped when d[kz] < 0 so the sheared frame keeps its
    # handedness
    ax, ay, az = np.abs(ld[:, 0]), np.abs(ld[:, 1]), np.abs(ld[:, 2])
    kz = np.where(ax > ay, np.where(ax > az, 0, 2), np.where(ay > az, 1, 2))
    kx = np.where(kz == 2, 0, kz + 1)
    ky = np.where(kx == 2, 0, kx + 1)
    n = o.shape[0]
    ii = np.arange(n)
    neg = ld[ii, kz] < 0
    kx, ky = np.where(neg, ky, kx), np.where(neg, kx, ky)
    rz = f32(1.0) / ld[ii, kz]
    sx, sy, sz = ld[ii, kx] * rz, ld[ii, ky] * rz, rz
    rel = tri - ox[:, None, :]                      # a', b', c' in float32
    pz = rel[ii, :, kz]                             # [n, 3]
    px = rel[ii, :, kx] - sx[:, None] * pz
    py = rel[ii, :, ky] - sy[:, None] * pz
    Ax, Bx, Cx = px[:, 0], px[:, 1], px[:, 2]
    Ay, By, Cy = py[:, 0], py[:, 1], py[:, 2]
    U = Cx * By - Cy * Bx
    V = Ax * Cy - Ay * Cx
    W = Bx * Ay - By * Ax
    det = U + V + W
    T = U * (sz * pz[:, 0]) + V * (sz * pz[:, 1]) + W * (sz * pz[:, 2])
    negs = (U < 0) | (V < 0) | (W < 0)
    poss = (U > 0) | (V > 0) | (W > 0)
    hit = ~(negs & poss) & (det != 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        tl = T * (f32(1.0) / det)            # the GPU's reciprocal, then a product
        u = V / det
        v = W / det
    return dict(hit=hit, t=t0 + tl, u=u, v=v, det=det)
