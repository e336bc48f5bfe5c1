"""Comparison of device hits with the oracle's (test helper).

Bar (from the project's parity contract):
  - hit id bit-exact on every ray whose oracle grazing margin is >= 1e-6;
  - id mismatch rate over all rays reported (configs require <= 1e-4);
  - on rays whose id matches: t within 1e-5 relative (absolute floor of
    1e-5 for t < 1), slot equal, and on non-grazing rays the normal within
    1e-5 per component.
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


def compare(gpu, ref, margin):
    gid, ginst, gt, gn = gpu
    ok = margin >= GRAZING
    idm = gid != ref.id
    same = ~idm
    both_hit = same & (ref.id != NONE)
    dt = np.abs(gt - ref.t)
    tol = T_REL * np.maximum(np.abs(ref.t), 1.0)
    t_bad = both_hit & ~(dt <= tol)
    inst_bad = same & (ginst != ref.inst)
    n_bad = both_hit & ok & (np.abs(gn - ref.normal).max(axis=1) > N_ABS)
    miss_bad = same & (ref.id == NONE) & ~(np.isinf(gt) & (gt > 0))
    n = gid.shape[0]
    return dict(n=n, mismatch=int(idm.sum()), mismatch_rate=float(idm.mean()) if n else 0.0,
                nongrazing_mismatch=int((idm & ok).sum()), grazing=int((~ok).sum()), t_bad=int(t_bad.sum()),
                inst_bad=int(inst_bad.sum()), normal_bad=int(n_bad.sum()), miss_bad=int(miss_bad.sum()),
                max_t_rel=float((dt[both_hit] / np.maximum(np.abs(ref.t[both_hit]), 1.0)).max()) if both_hit.any() else 0.0,
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
