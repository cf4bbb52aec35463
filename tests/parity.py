"""Comparison of GPU results with the oracle, per the tolerance rules:

closest hit, for every ray the oracle does not flag as ambiguous:
  hit/miss agree; the GPU's (inst, prim) is in the oracle's tie set (exact
  ties within 1e-6 t*, and both triangles of a covered edge crossing, each
  within 1e-5 t*); against that member's FP64 values (u, v clamped to
  [0, 1] as the library reports them), |t - t*| <= 1e-5 t* and
  |u - u*|, |v - v*| <= 1e-4.  The trace calls report t, u, v recomputed in
  double for the triangle the float32 traversal chose.
  With t_band=True (hits a render pass keeps internally, whose t is the
  float32 traversal's): |t - t*| <= max(1e-5 t*, delta), delta the float32
  error band of that triangle's t; u, v are not compared.
any hit: occluded agrees on every non-ambiguous ray.
render: RMSE over non-ambiguous pixels and all channels <= 1e-4, and by
  default over all pixels as well.
Allowed ambiguous fractions (max_amb) are the measured ones with a margin of
about 2x, stated per call.
"""
import numpy as np

T_REL = 1e-5
UV_ABS = 1e-4
RMSE_MAX = 1e-4


def check_closest(g, o, max_amb: float = 0.003, label: str = "", t_band: bool = False, orc=None, rays=None):
    """g: dict of numpy arrays from the GPU (t, inst, prim, u, v; u, v not
    needed with t_band); o: oracle.  With the oracle scene `orc` and the
    float32 rays, the hits of ambiguous rays are checked too: each must be a
    near candidate of its ray (check_candidates)."""
    n = o["t"].shape[0]
    ok = o["amb"] == 0
    amb_frac = 1.0 - ok.mean() if n else 0.0
    assert amb_frac <= max_amb, f"{label}: ambiguous fraction {amb_frac:.4f} > {max_amb}"
    ghit = g["inst"].astype(np.uint32) != 0xFFFFFFFF
    ohit = o["hit"] == 1
    bad = np.nonzero(ok & (ghit != ohit))[0]
    assert bad.size == 0, f"{label}: hit/miss differ on {bad.size} rays, e.g. {bad[:5]}"
    miss = ok & ~ohit
    assert np.isinf(g["t"][miss]).all()
    assert (g["prim"][miss].astype(np.uint32) == 0xFFFFFFFF).all()
    idx = np.nonzero(ok & ohit)[0]
    worst_t = 0.0
    worst_uv = 0.0
    loose = 0
    ratio_uv = 0.0   # observed error / band: how much of the band the GPU uses
    ratio_t = 0.0
    for i in idx:
        gi, gp = np.uint32(g["inst"][i]), np.uint32(g["prim"][i])
        k = o["nties"][i]
        ties = o["ties"][i, :k]
        sel = np.nonzero((ties[:, 0] == gi) & (ties[:, 1] == gp))[0]
        assert sel.size > 0, (f"{label}: ray {i}: GPU hit ({gi},{gp}) t={g['t'][i]} not in the tie set "
                              f"{ties.tolist()} (oracle ({o['inst'][i]},{o['prim'][i]}) t={o['t'][i]})")
        tt, tu, tv = o["ties_tuv"][i, sel[0]]
        dt = abs(float(g["t"][i]) - tt)
        t_tol = max(T_REL * tt, o["delta"][i]) if t_band else T_REL * tt
        loose += t_tol > T_REL * tt
        assert dt <= t_tol, f"{label}: ray {i}: t {g['t'][i]} vs {tt} (tol {t_tol:.3g})"
        worst_t = max(worst_t, dt / max(o["t"][i], 1e-30))
        ratio_t = max(ratio_t, dt / max(o["delta"][i], 1e-300))
        if t_band:
            continue
        tu, tv = min(max(tu, 0.0), 1.0), min(max(tv, 0.0), 1.0)
        du = max(abs(float(g["u"][i]) - tu), abs(float(g["v"][i]) - tv))
        assert du <= UV_ABS, f"{label}: ray {i}: uv ({g['u'][i]},{g['v'][i]}) vs ({tu},{tv}), tol {UV_ABS}"
        worst_uv = max(worst_uv, du)
        ratio_uv = max(ratio_uv, du / max(o["beta"][i], 1e-300))
    amb_checked = check_candidates(g, o, orc, rays, label) if orc is not None else None
    return dict(band_use_uv=float(ratio_uv), band_use_t=float(ratio_t), n=n, amb_frac=float(amb_frac),
                hits=int(idx.size), worst_t_rel=worst_t, worst_uv=worst_uv, t_band_used=int(loose),
                amb_hits_checked=amb_checked)


def check_candidates(g, o, orc, rays, label: str = ""):
    """For the ambiguous rays on which the GPU reports a hit: the reported
    triangle must be one float32 could choose, i.e. its FP64 evaluation
    (orc.eval_hits) lies inside it up to its band (least barycentric weight
    >= -beta), at t within [tmin - delta, tmax + delta], and no farther than
    the exact closest hit plus both t bands.  So a wrong hit cannot hide
    behind the ambiguity flag."""
    rays = np.asarray(rays, np.float32).reshape(-1, 8)
    gi = g["inst"].astype(np.uint32)
    sel = np.nonzero((o["amb"] != 0) & (gi != 0xFFFFFFFF))[0]
    if sel.size == 0:
        return 0
    ev = orc.eval_hits(rays[sel], gi[sel], g["prim"].astype(np.uint32)[sel])
    assert np.isfinite(ev["t"]).all(), f"{label}: an ambiguous ray's hit is parallel to it or out of range"
    bad = ev["m"] < -ev["beta"]
    assert not bad.any(), f"{label}: {bad.sum()} ambiguous rays report a triangle they miss, e.g. {sel[bad][:5]}"
    tmin, tmax = rays[sel, 6].astype(np.float64), rays[sel, 7].astype(np.float64)
    bad = (ev["t"] < tmin - ev["delta"]) | (ev["t"] > tmax + ev["delta"])
    assert not bad.any(), f"{label}: {bad.sum()} ambiguous rays report a hit outside [tmin, tmax]"
    oh = o["hit"][sel] == 1
    far = oh & (ev["t"] > o["t"][sel] + ev["delta"] + o["delta"][sel] + 1e-6 * np.abs(o["t"][sel]))
    assert not far.any(), f"{label}: {far.sum()} ambiguous rays report a hit beyond the closest one"
    return int(sel.size)


def check_any(occ, o, max_amb: float = 0.003, label: str = ""):
    ok = o["amb"] == 0
    amb_frac = 1.0 - ok.mean()
    assert amb_frac <= max_amb, f"{label}: ambiguous fraction {amb_frac:.4f}"
    bad = np.nonzero(ok & ((occ != 0) != (o["hit"] == 1)))[0]
    assert bad.size == 0, f"{label}: occlusion differs on {bad.size} rays, e.g. {bad[:5]}"
    return dict(n=int(occ.shape[0]), amb_frac=float(amb_frac), occluded=int((o["hit"] == 1).sum()))


def check_found(found, occ, rays, orc, oa, label: str = ""):
    """The any-hit call's reported hit: for every occluded ray that the
    oracle's any-hit result `oa` does not flag, the reported (inst, prim) must
    be a genuine hit of the ray (paper section 1: any hit; several answers are
    correct, so this checks validity, not equality): the FP64 evaluation of
    that triangle (orc.eval_hits) is inside it (least barycentric weight
    >= -beta) with t in [tmin - delta, tmax + delta], and the reported t, u, v
    are that triangle's within 1e-5 relative / 1e-4.  Rays not occluded
    report a miss."""
    rays = np.asarray(rays, np.float32).reshape(-1, 8)
    gi = found["inst"].astype(np.uint32)
    occ = occ != 0
    assert np.array_equal(occ, gi != 0xFFFFFFFF), f"{label}: found hit and occluded disagree"
    assert np.isinf(found["t"][~occ]).all()
    sel = np.nonzero(occ & (oa["amb"] == 0))[0]
    ev = orc.eval_hits(rays[sel], gi[sel], found["prim"].astype(np.uint32)[sel])
    tmin, tmax = rays[sel, 6].astype(np.float64), rays[sel, 7].astype(np.float64)
    assert np.isfinite(ev["t"]).all(), f"{label}: reported hit is parallel to its ray or out of range"
    bad = ev["m"] < -ev["beta"]
    assert not bad.any(), f"{label}: {bad.sum()} reported hits lie outside their triangle, e.g. {sel[bad][:5]}"
    bad = (ev["t"] < tmin - ev["delta"]) | (ev["t"] > tmax + ev["delta"])
    assert not bad.any(), f"{label}: {bad.sum()} reported hits lie outside [tmin, tmax]"
    gt = found["t"][sel].astype(np.float64)
    bad = np.abs(gt - ev["t"]) > T_REL * np.abs(ev["t"]) + 1e-30
    assert not bad.any(), f"{label}: t of {bad.sum()} reported hits, e.g. {gt[bad][:3]} vs {ev['t'][bad][:3]}"
    du = np.maximum(np.abs(found["u"][sel] - np.clip(ev["u"], 0, 1)), np.abs(found["v"][sel] - np.clip(ev["v"], 0, 1)))
    assert (du <= UV_ABS).all(), f"{label}: u, v of reported hits off by up to {du.max():.3g}"
    return dict(checked=int(sel.size), worst_t_rel=float(np.max(np.abs(gt - ev["t"]) / np.abs(ev["t"]))) if sel.size else 0.0)


def check_image(img, o, max_amb: float = 0.01, label: str = "", unmasked: bool = True):
    """img: float [n,3] GPU pixels for the sampled pixels; o: oracle render.
    RMSE over the non-ambiguous pixels <= 1e-4; with `unmasked`, over all
    pixels too (an ambiguous pixel may legitimately differ, but on these
    seeded frames none does by enough to matter, so a wrong pixel cannot hide
    behind the mask)."""
    ok = o["amb"] == 0
    amb_frac = 1.0 - ok.mean()
    assert amb_frac <= max_amb, f"{label}: ambiguous pixel fraction {amb_frac:.4f}"
    diff = img[ok].astype(np.float64) - o["rgb"][ok]
    rmse = float(np.sqrt(np.mean(diff ** 2))) if diff.size else 0.0
    full = float(np.sqrt(np.mean((img.astype(np.float64) - o["rgb"]) ** 2)))
    assert rmse <= RMSE_MAX, f"{label}: masked RMSE {rmse:.3g} > {RMSE_MAX} (unmasked {full:.3g})"
    if unmasked:
        assert full <= RMSE_MAX, f"{label}: unmasked RMSE {full:.3g} > {RMSE_MAX} (masked {rmse:.3g})"
    return dict(n=int(img.shape[0]), amb_frac=float(amb_frac), rmse=rmse, rmse_unmasked=full,
                max_abs=float(np.abs(diff).max()) if diff.size else 0.0)


def hits_to_numpy(h):
    return {k: v.cpu().numpy() for k, v in h.items()}
