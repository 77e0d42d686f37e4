"""Brute-force geometric queries in numpy, FP64, for the oracle pins.

A different formulation from the oracle's Moller-Trumbore test: the ray is
intersected with each triangle's plane (t = n.(v0 - o) / n.w) and the crossing
point is tested against the three edge functions n.((v_{i+1} - v_i) x (p - v_i)),
all of which are non-negative inside the triangle whatever its winding (n
comes from the same winding).  Every triangle of the scene is tested.
"""
import numpy as np


def _planes(V):
    V = np.asarray(V, np.float64).reshape(-1, 3, 3)
    n = np.cross(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0])
    return V, n


def ray_crossings(V, o, w):
    """Distances t along o + t w (w need not be unit) at which the line crosses
    each triangle's interior or boundary; inf where it does not."""
    V, n = _planes(V)
    o = np.asarray(o, np.float64)
    w = np.asarray(w, np.float64)
    den = n @ w
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.einsum("ij,ij->i", n, V[:, 0] - o) / den
    p = o + t[:, None] * w
    inside = np.ones(V.shape[0], bool)
    for i in range(3):
        a, b = V[:, i], V[:, (i + 1) % 3]
        inside &= np.einsum("ij,ij->i", n, np.cross(b - a, p - a)) >= 0.0
    ok = (den != 0.0) & inside & np.isfinite(t)
    return np.where(ok, t, np.inf)


def closest_hit(V, o, w, eps):
    """(triangle id, t) of the nearest crossing with t > eps along unit w
    (lowest id among equal t), or (-1, inf)."""
    t = ray_crossings(V, o, w)
    t = np.where(t > eps, t, np.inf)
    if not np.isfinite(t).any():
        return -1, np.inf
    tmin = t.min()
    return int(np.flatnonzero(t == tmin)[0]), float(tmin)


def segment_blocked(V, a, b, eps, tri_ids=None):
    """Whether a triangle (of tri_ids, default all) crosses segment a->b
    strictly inside (eps, L - eps) of its length L."""
    V = np.asarray(V, np.float64).reshape(-1, 3, 3)
    if tri_ids is not None:
        V = V[np.asarray(tri_ids)]
    if V.shape[0] == 0:
        return False
    a = np.asarray(a, np.float64)
    d = np.asarray(b, np.float64) - a
    L = np.linalg.norm(d)
    if L == 0.0:
        return False
    t = ray_crossings(V, a, d / L)
    return bool(np.any((t > eps) & (t < L - eps)))
