"""Shared helpers of the GPU parity tests: layout conversion between the device
store and the oracle's plain store, and the comparison rules.

Tolerances (derived in the design notes):
  * verification decisions (info words, first-invalid index, queue): bit-exact,
    except paths the oracle flags within 1e-6 of a decision boundary;
  * photon positions after re-tracing: 1e-5 scene units (FP32 rounding along
    up to 15 traced bounces), hit ids exact, energies 1e-5 relative;
  * paths whose traced rays pass within 1e-5 of a triangle edge, of eps_end,
    of another surface or of eps_close are excluded and counted.
"""
import numpy as np

import oracle as O

POS_TOL = 1e-5
E_RTOL = 1e-5


def to_oracle(d):
    return O.Store(pos=d["pos"].astype(np.float32).copy(), hit=d["hit"].astype(np.uint32).copy(),
                   energy=d["energy"].astype(np.float32).copy(), radius=d["radius"].astype(np.float32).copy(),
                   origin=d["origin"].astype(np.float32).copy(), info=d["info"].astype(np.uint32).copy())


def from_oracle(st):
    return dict(pos=st.pos, hit=st.hit, energy=st.energy, radius=st.radius, origin=st.origin, info=st.info)


def compare_stores(gpu, ora, mask, label=""):
    """Element-wise comparison of the columns selected by mask (bool [N])."""
    idx = np.flatnonzero(mask)
    g_info, o_info = gpu["info"][idx], ora.info[idx]
    bad = np.flatnonzero(g_info != o_info)
    assert bad.size == 0, "%s info differs at %d paths, e.g. path %d: gpu %08x oracle %08x" % (
        label, bad.size, idx[bad[0]], g_info[bad[0]], o_info[bad[0]])
    n = (o_info >> 22) & 15
    B = ora.B
    rows = np.arange(B)[:, None] < n[None, :]
    gh, oh = gpu["hit"][:, idx], ora.hit[:, idx]
    diff = rows & (gh != oh)
    assert not diff.any(), "%s hit ids differ at %d photons (first path %d)" % (
        label, diff.sum(), idx[np.flatnonzero(diff.any(0))[0]])
    dp = np.abs(gpu["pos"][:, idx] - ora.pos[:, idx]).max(axis=-1)
    assert (dp[rows] <= POS_TOL).all(), "%s positions differ by up to %g" % (label, dp[rows].max())
    ge, oe = gpu["energy"][:, idx], ora.energy[:, idx]
    rel = np.abs(ge - oe) / np.maximum(np.abs(oe), 1e-30)
    assert (rel[rows] <= E_RTOL).all(), "%s energies differ by up to %g rel" % (label, rel[rows].max())
    # rows beyond the path end are cleared on both sides
    assert (gh[~rows] == O.HIT_NONE).all() and (oh[~rows] == O.HIT_NONE).all()
    do = np.abs(gpu["origin"][idx] - ora.origin[idx]).max() if idx.size else 0.0
    assert do <= POS_TOL, "%s origins differ by %g" % (label, do)
