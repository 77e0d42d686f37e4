"""Shared helpers of the GPU parity tests: layout conversion between the device
store and the oracle's plain store, and the comparison rules.

Tolerances (derived in the design notes):
  * verification decisions (info words, first-invalid index, queue): bit-exact,
    except paths the oracle flags within 1e-6 of a decision boundary;
  * photon positions after re-tracing: 1e-5 scene units plus four times the
    first-order FP32 error bound propagated along the path, capped at 1e-4;
    a photon whose bound exceeds the cap and whose difference lies between
    the cap and the bound (a grazing hit) is flagged; once a path's bound
    exceeds the cap the two sides may part (another hit, or an earlier end)
    and such a path is flagged too; flagged paths are counted and reported,
    at most 0.5% of the compared paths; hit ids exact up to that point,
    energies 1e-5 relative;
  * paths whose traced rays pass within 1e-5 of a triangle edge, of eps_end,
    of another surface or of eps_close are excluded and counted (at most 5%
    of the paths of a frame; for a full trace, where every path casts all of
    its rays, the rate the oracle itself shows on an independent sample of the
    scene plus three binomial standard deviations of the compared sample).
    The oracle alone decides what is excluded, so a budget bounds how much of
    a frame is left uncompared, never how far the kernels may be off.

Every comparison is recorded in REPORT (label -> list of records); the test
session writes it as JSON (conftest.py).
"""
import numpy as np

import oracle as O

POS_TOL = 1e-5
POS_CAP = 1e-4     # largest position tolerance applied
FLAG_FRAC = 0.005  # largest fraction of compared paths with a flagged (grazing) photon
EXCL_FRAC = 0.05   # largest fraction of a frame's paths inside a decision band
E_RTOL = 1e-5
EPS_POS = 2e-7   # FP32 rounding of a computed position (coordinates within [-1, 1])
EPS_DIR = 4e-7   # FP32 error of a sampled or normalised unit direction


def photon_tolerance(ora, verts9, before=None):
    """Per-photon position tolerance: first-order bound of |FP32 - FP64|.

    A ray whose origin is off by e and whose direction is off by EPS_DIR hits a
    surface at incidence cosine c with an error of at most (e + d EPS_DIR) / c,
    d being the ray length; the bound is propagated along the path from the
    light sample and the tolerance is 1e-5 plus four times it.

    With 'before' (the store as the frame found it), a vertex that the frame
    hit anew may start a segment aimed at the old next photon (Algorithm 1
    checks, then traces, the segment from the new vertex to the old photon):
    that direction is the difference of two points a distance l apart, so the
    new vertex's error e tilts it by up to e / l on top of EPS_DIR."""
    V = verts9.reshape(-1, 3, 3).astype(np.float64)
    B, N = ora.hit.shape
    n = (ora.info >> 22) & 15
    tol = np.full((B, N), POS_TOL)
    err = np.full(N, EPS_POS)
    prev = ora.origin.astype(np.float64)
    if before is not None:
        prev_old = before.origin.astype(np.float64)
        n_old = (before.info >> 22) & 15
        # vertices the re-trace may hit anew: photons k.. of a replaced path
        # (their FP32 value can even equal the old one on one side only)
        rep = ((before.info >> 30) & 1).astype(bool)
        k_old = ((before.info >> 26) & 15).astype(np.int64)
    for r in range(B):
        valid = r < n
        p = ora.pos[r].astype(np.float64)
        h = np.where(valid, ora.hit[r], 0).astype(np.int64)
        h = np.minimum(h, V.shape[0] - 1)
        tri = V[h]
        nrm = np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0])
        nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-300)
        d = p - prev
        dist = np.linalg.norm(d, axis=1)
        c = np.abs(np.einsum("ij,ij->i", d, nrm)) / np.maximum(dist, 1e-300)
        eps_d = np.full(N, EPS_DIR)
        if before is not None:
            # the vertex this segment starts from was hit anew and an old
            # photon r existed: the segment may have been aimed at it
            moved = (np.any(prev != prev_old, axis=1) | (rep & (r - 1 >= k_old))) & (r < n_old)
            target = before.pos[r].astype(np.float64)
            ell = np.linalg.norm(target - prev, axis=1)
            eps_d = np.where(moved & (ell > 0), eps_d + err / np.maximum(ell, 1e-300), eps_d)
            prev_old = np.where((r < n_old)[:, None], target, prev_old)
        err = np.where(valid, (err + dist * eps_d) / np.maximum(c, 1e-3) + EPS_POS, err)
        tol[r] = POS_TOL + 4.0 * err
        prev = np.where(valid[:, None], p, prev)
    return tol


REPORT = {}


def record(label, **fields):
    """Keep one comparison's counts for the session report."""
    REPORT.setdefault(label, []).append({k: (float(v) if isinstance(v, (float, np.floating)) else
                                             int(v) if isinstance(v, (bool, int, np.integer, np.bool_)) else v)
                                         for k, v in fields.items()})


def sampled_budget(rate, n):
    """Exclusion budget of n compared paths when the oracle flags a fraction
    'rate' of the scene's paths: rate plus three binomial standard deviations."""
    return rate + 3.0 * np.sqrt(rate * (1.0 - rate) / max(n, 1))


# Oracle-flagged share of full 7-ray traces of the paper-scale scene: 1279 of
# 20000 independent paths (seed 5), 6.4%, almost all within 1e-5 of an edge of
# its finely tessellated walls (about 0.94% per traced ray).
PAPER_FULL_TRACE_RATE = 0.064

# The same share for the paper-scale rooms scene lit by two moving spotlights
# (kind 1, cone cosine 0.8) or two cameras (kind 2, near plane 0.6 x 0.4):
# 1386 and 1356 of 20000 independent paths (seed 99), 6.9% and 6.8%.
PAPER_FULL_EMITTER_TRACE_RATE = {1: 0.069, 2: 0.068}


def check_excluded(excluded, total, label, frac=EXCL_FRAC):
    """Assert and record the paths left out of an element-wise comparison."""
    record(label + " [exclusions]", excluded=int(excluded), paths=int(total), budget=float(frac))
    assert excluded <= frac * total, "%s: %d of %d paths inside a decision band" % (label, excluded, total)


def to_oracle(d):
    return O.Store(pos=d["pos"].astype(np.float32).copy(), hit=d["hit"].astype(np.uint32).copy(),
                   energy=d["energy"].astype(np.float32).copy(), radius=d["radius"].astype(np.float32).copy(),
                   origin=d["origin"].astype(np.float32).copy(), info=d["info"].astype(np.uint32).copy())


def from_oracle(st):
    return dict(pos=st.pos, hit=st.hit, energy=st.energy, radius=st.radius, origin=st.origin, info=st.info)


def compare_stores(gpu, ora, mask, label="", verts9=None, excluded=None, before=None):
    """Element-wise comparison of the columns selected by mask (bool [N]).

    Positions use the per-photon tolerance, capped at POS_CAP, when the
    frame's vertices are given; a photon between the cap and its bound is
    flagged.  From the first photon of a path whose bound exceeds the cap on
    (a grazing chain: the bound only grows along a path), the FP32 and FP64
    rays may differ by more than the oracle's 1e-5 decision bands assume, so
    the two sides may part there (another triangle hit, or one path ending):
    hits, positions and energies are compared up to that point, and a path
    that parts is flagged.  Flagged paths are counted, at most FLAG_FRAC of
    the compared paths.  Returns the counts it also records: paths compared,
    paths excluded (when given), largest position difference, largest
    tolerance applied, photons and paths flagged, paths parted."""
    idx = np.flatnonzero(mask)
    g_info, o_info = gpu["info"][idx], ora.info[idx]
    B = ora.B
    n = (o_info >> 22) & 15
    n_g = (g_info >> 22) & 15
    rows = np.arange(B)[:, None] < n[None, :]
    dp = np.abs(gpu["pos"][:, idx] - ora.pos[:, idx]).max(axis=-1)
    bound = photon_tolerance(ora, verts9, before)[:, idx] if verts9 is not None else np.full(dp.shape, POS_TOL)
    tol = np.minimum(bound, POS_CAP)
    # the grazing suffix of each path and where it starts (n when none)
    suffix = rows & (bound > POS_CAP)
    start = np.where(suffix.any(0), np.argmax(suffix, axis=0), n)
    head = np.arange(B)[:, None] < start[None, :]
    # information words: exact, except the segment count of a path with a
    # grazing suffix, which must still cover the compared head
    nmask = np.uint32(15 << 22)
    same_info = (g_info == o_info) | (suffix.any(0) & ((g_info & ~nmask) == (o_info & ~nmask)) &
                                      (np.minimum(n, n_g) >= start))
    bad = np.flatnonzero(~same_info)
    assert bad.size == 0, "%s info differs at %d paths, e.g. path %d: gpu %08x oracle %08x" % (
        label, bad.size, idx[bad[0]], g_info[bad[0]], o_info[bad[0]])
    gh, oh = gpu["hit"][:, idx], ora.hit[:, idx]
    ar = np.arange(B)[:, None]
    # the first row where the two sides part (another hit, or one side ended)
    parted = rows & ((gh != oh) | (ar >= n_g[None, :]))
    part = np.where(parted.any(0), np.argmax(parted, axis=0), n)
    assert (part >= start).all(), "%s hit ids differ at %d photons (first path %d)" % (
        label, int((parted & head).sum()), idx[np.flatnonzero(part < start)[0]])
    checked = ar < part[None, :]           # same hits: positions within their bounds
    over = rows & checked & (dp > bound)
    assert not over.any(), "%s positions differ at %d photons: worst %g (tolerance %g)" % (
        label, over.sum(), dp[over].max(), bound[over][np.argmax(dp[over])])
    ge, oe = gpu["energy"][:, idx], ora.energy[:, idx]
    rel = np.abs(ge - oe) / np.maximum(np.abs(oe), 1e-30)
    e_rows = rows & (ar <= part[None, :]) & (ar < n_g[None, :])  # an energy depends on the hits before it
    assert (rel[e_rows] <= E_RTOL).all(), "%s energies differ by up to %g rel" % (label, rel[e_rows].max())
    # flagged: a photon between the cap and its bound, or a grazing suffix
    # whose paths part
    flagged_ph = rows & checked & (dp > tol)
    flagged_paths = flagged_ph.any(0) | (part < n) | (n != n_g)
    n_flag_paths = int(flagged_paths.sum())
    assert n_flag_paths <= FLAG_FRAC * max(idx.size, 1), "%s: %d flagged paths (grazing chains)" % (
        label, n_flag_paths)
    # rows beyond each side's own path end are cleared
    g_rows = np.arange(B)[:, None] < n_g[None, :]
    assert (gh[~g_rows] == O.HIT_NONE).all() and (oh[~rows] == O.HIT_NONE).all()
    do = np.abs(gpu["origin"][idx] - ora.origin[idx]).max() if idx.size else 0.0
    assert do <= POS_TOL, "%s origins differ by %g" % (label, do)
    cmp_rows = rows & checked
    counts = dict(compared=idx.size, photons=int(rows.sum()),
                  max_pos_diff=float(dp[cmp_rows].max()) if cmp_rows.any() else 0.0,
                  max_tol_applied=float(tol[cmp_rows].max()) if cmp_rows.any() else 0.0,
                  max_energy_rel=float(rel[e_rows].max()) if e_rows.any() else 0.0,
                  flagged_photons=int(flagged_ph.sum()), flagged_paths=n_flag_paths,
                  parted_paths=int((part < n).sum() + ((part >= n) & (n != n_g)).sum()),
                  grazing_suffix_photons=int(suffix.sum()))
    if excluded is not None:
        counts["excluded"] = int(excluded)
    record(label, **counts)
    return counts
