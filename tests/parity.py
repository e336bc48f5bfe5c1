"""Comparison of device hits with the oracle's (test helper).

Bar (from the project's parity contract):
  - hit id bit-exact on every ray whose oracle id margin is >= 1e-6 (the id
    margin holds only the gaps that can change which leaf is hit);
  - id mismatch rate over all rays reported (configs require <= 1e-4);
  - on rays whose id matches: t within 1e-5 relative to the ray's FP32
    scale max(t, S), S = max(|o|inf, |o + t d|inf, 1) / |d|inf -- FP32 plane
    crossings and frame maps carry an absolute error that grows with the
    coordinates, not with t, so a hit right next to a far-away origin is
    held to the coordinate scale (the same scale the grazing margin uses);
    for rays from a distant camera t ~ S and this is plain relative error;
  - slot equal, and on rays whose normal margin (the id margin and the
    entry-face gaps) is >= 1e-6 the normal within 1e-5 per component.
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF
GRAZING = 1e-6
T_REL = 1e-5
N_ABS = 1e-5


def to_numpy(h):
    return (h.id.cpu().numpy().view(np.uint32), h.inst.cpu().numpy().view(np.uint32),
            h.t.cpu().numpy().astype(np.float64), h.normal.cpu().numpy().astype(np.float64))


def ray_scale(rays, t):
    """S = max(|o|inf, |o + t d|inf, 1) / |d|inf per ray (t = +inf: origin only)."""
    r = np.asarray(rays, np.float32).astype(np.float64)
    o, d = r[:, 0:3], r[:, 4:7]
    tt = np.where(np.isfinite(t), t, 0.0)
    m = np.maximum(np.maximum(np.abs(o).max(1), np.abs(o + tt[:, None] * d).max(1)), 1.0)
    return m / np.maximum(np.abs(d).max(1), 1e-300)


def compare(gpu, ref, margin=None, rays=None):
    """margin: the oracle's id margin per ray (default ref.margin); the
    normal check takes ref.margin_n when the oracle computed it."""
    gid, ginst, gt, gn = gpu
    if margin is None:
        margin = ref.margin
    margin_n = ref.margin_n if getattr(ref, "margin_n", None) is not None else margin
    ok = margin >= GRAZING
    ok_n = np.minimum(margin, margin_n) >= GRAZING
    idm = gid != ref.id
    same = ~idm
    both_hit = same & (ref.id != NONE)
    with np.errstate(invalid="ignore"):
        dt = np.abs(gt - ref.t)
    scale = np.maximum(np.abs(np.where(np.isfinite(ref.t), ref.t, 0.0)), 1.0)
    if rays is not None:
        scale = np.maximum(scale, ray_scale(rays, ref.t))
    tol = T_REL * scale
    t_bad = both_hit & ~(dt <= tol)
    t_rel_pure = both_hit & ~(dt <= T_REL * np.maximum(np.abs(np.where(np.isfinite(ref.t), ref.t, 0.0)), 1.0))
    inst_bad = same & (ginst != ref.inst)
    n_bad = both_hit & ok_n & (np.abs(gn - ref.normal).max(axis=1) > N_ABS)
    miss_bad = same & (ref.id == NONE) & ~(np.isinf(gt) & (gt > 0))
    n = gid.shape[0]
    worst = None
    if both_hit.any():
        rel = np.where(both_hit, dt / scale, -1.0)
        j = int(np.argmax(rel))
        worst = dict(ray=j, t_gpu=float(gt[j]), t_ref=float(ref.t[j]), inst=int(ref.inst[j]), id=int(ref.id[j]))
    return dict(worst_t=worst, n=n, mismatch=int(idm.sum()), mismatch_rate=float(idm.mean()) if n else 0.0,
                nongrazing_mismatch=int((idm & ok).sum()), grazing=int((~ok).sum()),
                grazing_normal=int((~ok_n).sum()), t_bad=int(t_bad.sum()),
                inst_bad=int(inst_bad.sum()), normal_bad=int(n_bad.sum()), miss_bad=int(miss_bad.sum()),
                max_t_rel=float((dt[both_hit] / scale[both_hit]).max()) if both_hit.any() else 0.0,
                t_rel_to_t_only=int(t_rel_pure.sum()),
                hits=int((ref.id != NONE).sum()))


def assert_parity(stats, max_rate=None):
    msg = repr(stats)
    assert stats["nongrazing_mismatch"] == 0, msg
    assert stats["t_bad"] == 0, msg
    assert stats["inst_bad"] == 0, msg
    assert stats["normal_bad"] == 0, msg
    assert stats["miss_bad"] == 0, msg
    if max_rate is not None:
        assert stats["mismatch_rate"] <= max_rate, msg
