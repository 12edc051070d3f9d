"""Per-ray comparison of GPU renders with the oracle.

Rule (tolerances of the method's stated FP32 bar):
  1. The GPU's blended id list is compared with the oracle's. Allowed differences:
     (i)   ids whose FP64 alpha is within 1e-5 of alpha_min may be present or absent;
     (ii)  adjacent hits whose key distances differ by < 1e-5 may swap;
     (iii) the last hit may be extra or missing when the oracle's transmittance after
           that hit is within 1e-6 of T_min;
     (iv)  for a ray bounded by a surface at t_far, hits whose key is within 1e-5 of
           t_far may be present or absent.
  2. Identical lists: |rgb - oracle| <= 1e-4 per channel and |depth - oracle| <= 1e-4.
  3. Lists that differ only by allowed exceptions: the same bound against the oracle's
     re-composition of the GPU's own list (from the ray's starting transmittance).
  4. At most a fraction 1e-3 of the compared rays (and at least one) may need an exception.
"""
from __future__ import annotations

import numpy as np

import oracle

TOL = 1e-4
ALPHA_BAND = 1e-5
T_SWAP = 1e-5
T_ERT = 1e-6


def lists_match_with_exceptions(g, o, hits, scene, origin, direction, amin, T_min, tafter, t_far=np.inf):
    # `hits` holds the oracle's alpha and key distance of every hit on this ray
    """True if GPU list g and oracle list o differ only by the allowed exceptions."""
    alpha = dict(zip(hits["ids"].tolist(), hits["alpha"].tolist()))
    tkey = dict(zip(hits["ids"].tolist(), hits["t"].tolist()))
    if np.isfinite(t_far):
        # (iv) hits at the bounding surface
        near = {i for i, t in tkey.items() if abs(t - t_far) < T_SWAP}
        g = [i for i in g if i not in near]
        o = [i for i in o if i not in near]

    def a_of(i):
        if i in alpha:
            return alpha[i]
        return oracle.composite_list(scene, origin, direction, [i], amin)["opacity"]

    g2 = [i for i in g if abs(a_of(i) - amin) >= ALPHA_BAND]
    o2 = [i for i in o if abs(a_of(i) - amin) >= ALPHA_BAND]
    # (iii) early termination may move by one hit when the transmittance at the
    # crossing is within T_ERT of T_min, or, after an allowed (i) difference, within the
    # relative change such a near-threshold hit makes (below 1% of T_min)
    if len(g2) != len(o2):
        if abs(len(g2) - len(o2)) != 1:
            return False
        band = max(T_ERT, 0.01 * T_min) if len(g2) + len(o2) < len(g) + len(o) else T_ERT
        near_ert = any(abs(tafter[i] - T_min) < band for i in (len(o) - 1, len(o) - 2) if 0 <= i < len(tafter))
        if not near_ert:
            return False
        n = min(len(g2), len(o2))
        g2, o2 = g2[:n], o2[:n]
    j = 0
    while j < len(g2):
        if g2[j] == o2[j]:
            j += 1
            continue
        # (ii) near-equal keys may come in either order: an adjacent swap, or a tie cut
        # by early termination right there (the last blended hit is the other one)
        if abs(tkey.get(g2[j], np.inf) - tkey.get(o2[j], -np.inf)) < T_SWAP:
            if j + 1 == len(g2):
                j += 1
                continue
            if g2[j] == o2[j + 1] and g2[j + 1] == o2[j]:
                j += 2
                continue
        return False
    return True


def _describe(g, o, hits, tafter, T_min):
    """First difference of two id lists with the oracle's alpha and key of the ids there."""
    j = next((i for i in range(min(len(g), len(o))) if g[i] != o[i]), min(len(g), len(o)))
    alpha = dict(zip(hits["ids"].tolist(), hits["alpha"].tolist()))
    tkey = dict(zip(hits["ids"].tolist(), hits["t"].tolist()))
    win = lambda L: [(i, round(alpha.get(i, float("nan")), 7), round(tkey.get(i, float("nan")), 7))
                     for i in L[max(0, j - 2):j + 3]]
    return dict(first_diff=j, len_gpu=len(g), len_oracle=len(o), gpu=win(g), oracle=win(o),
                T_after_last=float(tafter[-1]) if len(tafter) else None, T_min=T_min)


def compare_render(scene, origins, dirs, gpu, ref, amin, T_min, max_exception_frac=1e-3, label="", key_mode=0,
                   t_far=None, trans0=None, bg=(0.0, 0.0, 0.0)):
    """Compare GPU outputs (numpy dict: rgb, depth, hit_ids, hit_counts) with an oracle
    render (with cap) of the same rays, which may be bounded (t_far) and start with a
    transmittance (trans0). Returns a summary dict; asserts the rule."""
    R = origins.shape[0]
    tf = np.full(R, np.inf) if t_far is None else np.asarray(t_far, np.float64)
    t0 = np.ones(R) if trans0 is None else np.asarray(trans0, np.float64)
    cap = gpu["hit_ids"].shape[1]
    n_exact = n_exc = 0
    worst = 0.0
    bad = []
    for r in range(R):
        gcount = int(gpu["hit_counts"][r])
        ocount = int(ref["nblend"][r])
        assert gcount <= cap and ocount <= ref["ids"].shape[1], (label, r, gcount, ocount, "raise hit capacity")
        g = gpu["hit_ids"][r, :gcount].tolist()
        o = ref["ids"][r, :ocount].tolist()
        if g == o:
            err = max(np.abs(gpu["rgb"][r] - ref["rgb"][r]).max(), abs(gpu["depth"][r] - ref["depth"][r]))
            worst = max(worst, err)
            if err > TOL:
                bad.append((r, "exact-list", float(err), g[:8]))
            n_exact += 1
            continue
        hits = oracle.ray_hits(scene, origins[r], dirs[r], amin, key_mode=key_mode)
        if not lists_match_with_exceptions(g, o, hits, scene, origins[r], dirs[r], amin, T_min,
                                           ref["tafter"][r, :ocount], tf[r]):
            bad.append((r, "list", _describe(g, o, hits, ref["tafter"][r, :ocount], T_min)))
            continue
        c = oracle.composite_list(scene, origins[r], dirs[r], g, amin, bg=bg if np.isinf(tf[r]) else (0, 0, 0),
                                  trans0=t0[r])
        err = max(np.abs(gpu["rgb"][r] - c["rgb"]).max(), abs(gpu["depth"][r] - c["depth"]))
        worst = max(worst, err)
        if err > TOL:
            bad.append((r, "exception-list", float(err), g[:8]))
        n_exc += 1
    summary = dict(rays=R, exact=n_exact, exceptions=n_exc, bad=len(bad), worst=worst)
    assert not bad, (label, summary, bad[:5])
    assert n_exc <= max_exception_frac * R + 1, (label, summary)
    return summary
