"""Seeded synthetic scenes and per-frame motion for photon-path verification.

This module is the one input source shared by the HIP path and the CPU oracle.
It builds triangle soups, materials, area lights and the per-frame rigid
transforms of dynamic objects and lights.  It performs none of the method's
arithmetic: no transform is applied to a vertex here, no ray is traced, no
energy is computed.  Every array it returns is float32 / uint32, exactly what
both sides consume.

Conventions (shared data format, not code):

* A transform is a row-major 3x4 float32 matrix ``[R | t]`` (12 floats); the
  world position of a local point ``p`` is ``R p + t``.
* A light is a rectangle in its local ``z = 0`` plane, ``|u| <= half[0]``,
  ``|v| <= half[1]``, emitting into local ``+z``; its transform is rigid.
* Object 0 is the static world (world-space vertices); objects ``1..D`` are
  rigid dynamic objects given in local space.
* Paths ``[base_l, base_{l+1})`` belong to light ``l``.

Workload recipes (the paper measures on its own Conference / Villa scenes,
whose assets are not available; these procedural scenes stand in, with the
paper's path counts, bounce limit and thresholds):

* ``tiny``: open box of 5 quads (10 triangles, albedo 0.7), one 12-triangle
  cube of side 0.2 (albedo 0.5) moving +0.05 along x per frame, one 0.2x0.2
  ceiling light, 16384 paths, 3 bounces.
* ``rooms``: a grid of rooms with doorways in ``[-1,1] x [-0.25,0.25] x
  [-1,1]``, tessellated walls and clutter boxes up to a triangle budget,
  32 grey materials with albedo ~ U(0.3, 0.8), torus-shaped rigid dynamic
  objects on a random walk (at most 0.5% of the scene extent and 1 degree per
  frame), 0.1x0.1 ceiling lights that optionally translate and tilt.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

F32 = np.float32
U32 = np.uint32


@dataclass
class Scene:
    name: str
    static_verts: np.ndarray          # float32 [S, 3, 3] world space
    static_mat: np.ndarray            # uint32  [S]
    obj_local: List[np.ndarray]       # per dynamic object float32 [n_o, 3, 3]
    obj_mat: List[np.ndarray]         # per dynamic object uint32 [n_o]
    obj_xforms: np.ndarray            # float32 [F, D, 12]
    albedo: np.ndarray                # float32 [M, 3]
    light_half: np.ndarray            # float32 [L, 2]
    light_power: np.ndarray           # float32 [L, 3]
    light_xforms: np.ndarray          # float32 [F, L, 12]
    light_paths: np.ndarray           # int64 [L] paths per light
    max_bounces: int
    threshold: float                  # energy-error threshold T (fraction); < 0 = naive
    seed: int
    eps_end: float = 1e-4
    eps_close: float = 1e-4
    photon_radius: float = 0.01
    meta: dict = field(default_factory=dict)
    light_kind: object = None         # None (every light a rectangle / point), or int32 [L]: 0, 1 spot, 2 camera
    light_param: object = None        # float32 [L, 2]: spot (cos of the cone half-angle, 0); camera (tan u, tan v)

    @property
    def n_frames(self) -> int:
        return int(self.obj_xforms.shape[0])

    @property
    def n_dynamic(self) -> int:
        return len(self.obj_local)

    @property
    def n_static(self) -> int:
        return int(self.static_verts.shape[0])

    @property
    def n_paths(self) -> int:
        return int(self.light_paths.sum())

    @property
    def light_base(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.light_paths)]).astype(np.int64)

    def n_dynamic_tris(self) -> int:
        return int(sum(o.shape[0] for o in self.obj_local))

    def tri_layout(self):
        """Global triangle numbering: static first, then each object in order.

        Returns (tri_obj uint32[T], tri_mat uint32[T], obj_begin int64[D+2]).
        """
        counts = [self.n_static] + [o.shape[0] for o in self.obj_local]
        begin = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        tri_obj = np.concatenate([np.full(c, i, U32) for i, c in enumerate(counts)])
        tri_mat = np.concatenate([self.static_mat] + list(self.obj_mat)).astype(U32)
        return tri_obj, tri_mat, begin

    def frames(self, n: int) -> "Scene":
        """Same scene with at least ``n`` frames of motion (extends the walk)."""
        if n <= self.n_frames:
            return self
        raise ValueError("scene was generated with %d frames" % self.n_frames)


# ----------------------------------------------------------------------------
# small geometry helpers (mesh construction only)

def _quad(p0, p1, p2, p3):
    """Two triangles of the planar quad p0-p1-p2-p3 (in order around it)."""
    return [(p0, p1, p2), (p0, p2, p3)]


def _tess_quad(origin, eu, ev, nu, nv):
    """Quad origin + s*eu + t*ev, s,t in [0,1], cut into nu x nv cells."""
    o = np.asarray(origin, np.float64)
    eu = np.asarray(eu, np.float64)
    ev = np.asarray(ev, np.float64)
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i, j = i.reshape(-1, 1), j.reshape(-1, 1)
    a = o + eu * (i / nu) + ev * (j / nv)
    b = o + eu * ((i + 1) / nu) + ev * (j / nv)
    c = o + eu * ((i + 1) / nu) + ev * ((j + 1) / nv)
    d = o + eu * (i / nu) + ev * ((j + 1) / nv)
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    return list(np.stack([t1, t2], axis=1).reshape(-1, 3, 3))


def _box(lo, hi, h=None):
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    ext = hi - lo
    faces = [
        (lo, [ext[0], 0, 0], [0, 0, ext[2]]),                        # bottom
        (lo + [0, ext[1], 0], [0, 0, ext[2]], [ext[0], 0, 0]),       # top
        (lo, [0, ext[1], 0], [ext[0], 0, 0]),                        # z = lo
        (lo + [0, 0, ext[2]], [ext[0], 0, 0], [0, ext[1], 0]),       # z = hi
        (lo, [0, 0, ext[2]], [0, ext[1], 0]),                        # x = lo
        (lo + [ext[0], 0, 0], [0, ext[1], 0], [0, 0, ext[2]]),       # x = hi
    ]
    tris = []
    for o, eu, ev in faces:
        if h is None:
            nu = nv = 1
        else:
            nu = max(1, int(math.ceil(np.linalg.norm(eu) / h)))
            nv = max(1, int(math.ceil(np.linalg.norm(ev) / h)))
        tris += _tess_quad(o, eu, ev, nu, nv)
    return tris


def _torus(R, r, n_major, n_minor):
    """Torus about the local z axis: 2 * n_major * n_minor triangles."""
    tris = []

    def pt(i, j):
        u = 2 * math.pi * (i % n_major) / n_major
        v = 2 * math.pi * (j % n_minor) / n_minor
        return np.array([(R + r * math.cos(v)) * math.cos(u),
                         (R + r * math.cos(v)) * math.sin(u),
                         r * math.sin(v)])

    for i in range(n_major):
        for j in range(n_minor):
            tris += _quad(pt(i, j), pt(i + 1, j), pt(i + 1, j + 1), pt(i, j + 1))
    return tris


def _as_f32_tris(tris):
    return np.asarray(tris, np.float64).reshape(-1, 3, 3).astype(F32)


def _rot_axis_angle(axis, ang):
    axis = np.asarray(axis, np.float64)
    axis = axis / np.linalg.norm(axis)
    x, y, z = axis
    c, s = math.cos(ang), math.sin(ang)
    C = 1 - c
    return np.array([[c + x * x * C, x * y * C - z * s, x * z * C + y * s],
                     [y * x * C + z * s, c + y * y * C, y * z * C - x * s],
                     [z * x * C - y * s, z * y * C + x * s, c + z * z * C]])


def _xf(R, t):
    m = np.zeros((3, 4), np.float64)
    m[:, :3] = R
    m[:, 3] = t
    return m.astype(F32).reshape(12)


# A light facing world -y (down): local x -> world x, local y -> world +z,
# local z (the emitting normal) -> world -y.
R_DOWN = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])


# ----------------------------------------------------------------------------
# the tiny configuration

def make_tiny(n_paths=16384, max_bounces=3, frames=2, threshold=-1.0, seed=1):
    walls = []
    walls += _quad([0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1])      # floor y=0
    walls += _quad([0, 1, 0], [0, 1, 1], [1, 1, 1], [1, 1, 0])      # ceiling y=1
    walls += _quad([0, 0, 0], [0, 0, 1], [0, 1, 1], [0, 1, 0])      # left x=0
    walls += _quad([1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1])      # right x=1
    walls += _quad([0, 0, 0], [0, 1, 0], [1, 1, 0], [1, 0, 0])      # back z=0
    static = _as_f32_tris(walls)
    cube = _as_f32_tris(_box([-0.1, -0.1, -0.1], [0.1, 0.1, 0.1]))
    albedo = np.array([[0.7, 0.7, 0.7], [0.5, 0.5, 0.5]], F32)
    xf = np.stack([_xf(np.eye(3), [0.3 + 0.05 * f, 0.5, 0.5])[None] for f in range(frames)])
    lxf = np.stack([_xf(R_DOWN, [0.5, 0.999, 0.5])[None] for _ in range(frames)])
    return Scene(
        name="tiny", static_verts=static, static_mat=np.zeros(10, U32),
        obj_local=[cube], obj_mat=[np.ones(12, U32)], obj_xforms=xf.astype(F32),
        albedo=albedo, light_half=np.array([[0.1, 0.1]], F32),
        light_power=np.ones((1, 3), F32), light_xforms=lxf.astype(F32),
        light_paths=np.array([n_paths], np.int64), max_bounces=max_bounces,
        threshold=threshold, seed=seed,
        meta={"static_tris": 10, "dynamic_tris": 12})


def make_objects_only(n_paths=4096, max_bounces=4, frames=3, threshold=-1.0, seed=5):
    """The tiny box as a rigid object that never moves (no static triangles),
    with the tiny configuration's cube moving inside it."""
    walls = []
    walls += _quad([0, 0, 0], [1, 0, 0], [1, 0, 1], [0, 0, 1])      # floor y=0
    walls += _quad([0, 1, 0], [0, 1, 1], [1, 1, 1], [1, 1, 0])      # ceiling y=1
    walls += _quad([0, 0, 0], [0, 0, 1], [0, 1, 1], [0, 1, 0])      # left x=0
    walls += _quad([1, 0, 0], [1, 1, 0], [1, 1, 1], [1, 0, 1])      # right x=1
    walls += _quad([0, 0, 0], [0, 1, 0], [1, 1, 0], [1, 0, 0])      # back z=0
    box = _as_f32_tris(walls)
    cube = _as_f32_tris(_box([-0.1, -0.1, -0.1], [0.1, 0.1, 0.1]))
    albedo = np.array([[0.7, 0.7, 0.7], [0.5, 0.5, 0.5]], F32)
    xf = np.stack([np.stack([_xf(np.eye(3), [0, 0, 0]), _xf(np.eye(3), [0.3 + 0.05 * f, 0.5, 0.5])])
                   for f in range(frames)])
    lxf = np.stack([_xf(R_DOWN, [0.5, 0.999, 0.5])[None] for _ in range(frames)])
    return Scene(
        name="objects_only", static_verts=np.zeros((0, 3, 3), F32), static_mat=np.zeros(0, U32),
        obj_local=[box, cube], obj_mat=[np.zeros(10, U32), np.ones(12, U32)], obj_xforms=xf.astype(F32),
        albedo=albedo, light_half=np.array([[0.1, 0.1]], F32),
        light_power=np.ones((1, 3), F32), light_xforms=lxf.astype(F32),
        light_paths=np.array([n_paths], np.int64), max_bounces=max_bounces,
        threshold=threshold, seed=seed,
        meta={"static_tris": 0, "dynamic_tris": 22})


# ----------------------------------------------------------------------------
# procedural room grids

def _room_panels(nx, nz, rng):
    """Planar panels (origin, eu, ev) of a room grid with doorways."""
    y0, y1 = -0.25, 0.25
    H = y1 - y0
    wx, wz = 2.0 / nx, 2.0 / nz
    panels = []
    for i in range(nx):
        for k in range(nz):
            x0, z0 = -1 + i * wx, -1 + k * wz
            panels.append(([x0, y0, z0], [wx, 0, 0], [0, 0, wz]))   # floor
            panels.append(([x0, y1, z0], [0, 0, wz], [wx, 0, 0]))   # ceiling
    door_h = 0.6 * H

    def wall(p0, along, length, inner):
        # a wall from p0 along unit 'along' of given length, full height
        p0 = np.asarray(p0, np.float64)
        a = np.asarray(along, np.float64)
        up = np.array([0, H, 0])
        if not inner:
            panels.append((p0, a * length, up))
            return
        dw = 0.3 * length
        s0 = 0.5 * (length - dw)
        panels.append((p0, a * s0, up))                                    # left
        panels.append((p0 + a * (s0 + dw), a * (length - s0 - dw), up))    # right
        panels.append((p0 + a * s0 + [0, door_h, 0], a * dw, [0, H - door_h, 0]))  # lintel

    for i in range(nx + 1):                 # walls x = const
        for k in range(nz):
            wall([-1 + i * wx, y0, -1 + k * wz], [0, 0, 1], wz, 0 < i < nx)
    for k in range(nz + 1):                 # walls z = const
        for i in range(nx):
            wall([-1 + i * wx, y0, -1 + k * wz], [1, 0, 0], wx, 0 < k < nz)
    return panels, wx, wz


def _clutter(nx, nz, per_room, rng):
    wx, wz = 2.0 / nx, 2.0 / nz
    boxes = []
    for i in range(nx):
        for k in range(nz):
            for _ in range(per_room):
                sx, sz = rng.uniform(0.08, 0.25) * wx, rng.uniform(0.08, 0.25) * wz
                sy = rng.uniform(0.05, 0.35) * 0.5
                cx = -1 + (i + rng.uniform(0.2, 0.8)) * wx
                cz = -1 + (k + rng.uniform(0.2, 0.8)) * wz
                boxes.append(([cx - sx / 2, -0.25, cz - sz / 2], [cx + sx / 2, -0.25 + sy, cz + sz / 2]))
    return boxes


def _tess_count(panels, boxes, h):
    n = 0
    for o, eu, ev in panels:
        n += 2 * max(1, int(math.ceil(np.linalg.norm(eu) / h))) * max(1, int(math.ceil(np.linalg.norm(ev) / h)))
    for lo, hi in boxes:
        e = np.asarray(hi) - np.asarray(lo)
        nx_, ny_, nz_ = [max(1, int(math.ceil(v / h))) for v in e]
        n += 4 * (nx_ * nz_ + nx_ * ny_ + ny_ * nz_)
    return n


def make_rooms(name, nx, nz, static_target, n_dyn, torus_segs, n_paths, max_bounces,
               frames, threshold, seed, n_lights=2, lights_move=False,
               torus_size=(0.16, 0.055), clutter_per_room=2, point_lights=False, light_kind=0,
               light_param=(0.0, 0.0)):
    rng = np.random.default_rng(seed)
    panels, wx, wz = _room_panels(nx, nz, rng)
    boxes = _clutter(nx, nz, clutter_per_room, rng)
    # cell size h so that the tessellated count is close to the budget
    lo_h, hi_h = 1e-3, 2.0
    for _ in range(60):
        mid = math.sqrt(lo_h * hi_h)
        if _tess_count(panels, boxes, mid) > static_target:
            lo_h = mid
        else:
            hi_h = mid
    h = hi_h
    n_mat = 32
    albedo_grey = rng.uniform(0.3, 0.8, n_mat)
    albedo = np.repeat(albedo_grey[:, None], 3, axis=1).astype(F32)
    tris, mats = [], []
    for o, eu, ev in panels:
        nu = max(1, int(math.ceil(np.linalg.norm(eu) / h)))
        nv = max(1, int(math.ceil(np.linalg.norm(ev) / h)))
        t = _tess_quad(o, eu, ev, nu, nv)
        tris += t
        mats += [int(rng.integers(n_mat))] * len(t)
    for lo, hi in boxes:
        t = _box(lo, hi, h)
        tris += t
        mats += [int(rng.integers(n_mat))] * len(t)
    static = _as_f32_tris(tris)
    static_mat = np.asarray(mats, U32)

    # lights: in distinct rooms, just below the ceiling, facing down
    rooms = [(i, k) for i in range(nx) for k in range(nz)]
    order = rng.permutation(len(rooms))
    light_rooms = [rooms[j] for j in order[:n_lights]]
    y_light = 0.25 - (0.02 if lights_move else 0.001)
    # rectangles of 0.1 x 0.1, or points (both half extents 0); spot lights
    # and cameras (light_kind 1, 2) are points with a cone / near plane
    point_lights = point_lights or light_kind != 0
    light_half = np.full((n_lights, 2), 0.0 if point_lights else 0.05, F32)
    light_power = np.ones((n_lights, 3), F32)
    lpos = np.array([[-1 + (i + 0.5) * wx, y_light, -1 + (k + 0.5) * wz] for i, k in light_rooms])
    ltilt = np.zeros((n_lights, 2))
    lxf = np.zeros((frames, n_lights, 12), F32)
    for f in range(frames):
        for l in range(n_lights):
            R = R_DOWN @ _rot_axis_angle([1, 0, 0], ltilt[l, 0]) @ _rot_axis_angle([0, 1, 0], ltilt[l, 1])
            lxf[f, l] = _xf(R, lpos[l])
            if lights_move:
                i, k = light_rooms[l]
                step = rng.normal(size=2)
                step *= rng.uniform(0, 0.01) / max(1e-12, np.linalg.norm(step))
                nxp, nzp = lpos[l, 0] + step[0], lpos[l, 2] + step[1]
                xlo, xhi = -1 + (i + 0.25) * wx, -1 + (i + 0.75) * wx
                zlo, zhi = -1 + (k + 0.25) * wz, -1 + (k + 0.75) * wz
                lpos[l, 0] = nxp if xlo < nxp < xhi else lpos[l, 0] - step[0]
                lpos[l, 2] = nzp if zlo < nzp < zhi else lpos[l, 2] - step[1]
                dt = rng.uniform(-1, 1, 2) * math.radians(1.0)
                ltilt[l] = np.clip(ltilt[l] + dt, -math.radians(10), math.radians(10))

    # dynamic tori: in the lit rooms first, then their neighbours
    near = list(light_rooms)
    for (i, k) in light_rooms:
        for di, dk in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            if 0 <= i + di < nx and 0 <= k + dk < nz and (i + di, k + dk) not in near:
                near.append((i + di, k + dk))
    obj_local, obj_mat = [], []
    Rt, rt = torus_size[0] * min(wx, wz), torus_size[1] * min(wx, wz)
    pos, rot, homes = [], [], []
    for d in range(n_dyn):
        room = near[d % len(near)]
        homes.append(room)
        obj_local.append(_as_f32_tris(_torus(Rt, rt, torus_segs[0], torus_segs[1])))
        obj_mat.append(np.full(2 * torus_segs[0] * torus_segs[1], int(rng.integers(n_mat)), U32))
        i, k = room
        pos.append(np.array([-1 + (i + rng.uniform(0.3, 0.7)) * wx, rng.uniform(-0.1, 0.1),
                             -1 + (k + rng.uniform(0.3, 0.7)) * wz]))
        rot.append(_rot_axis_angle(rng.normal(size=3), rng.uniform(0, 2 * math.pi)))
    oxf = np.zeros((frames, n_dyn, 12), F32)
    for f in range(frames):
        for d in range(n_dyn):
            oxf[f, d] = _xf(rot[d], pos[d])
            step = rng.normal(size=3)
            step *= rng.uniform(0, 0.01) / max(1e-12, np.linalg.norm(step))
            i, k = homes[d]
            lo = np.array([-1 + i * wx + 1.1 * (Rt + rt), -0.25 + 1.1 * (Rt + rt), -1 + k * wz + 1.1 * (Rt + rt)])
            hi = np.array([-1 + (i + 1) * wx - 1.1 * (Rt + rt), 0.25 - 1.1 * (Rt + rt), -1 + (k + 1) * wz - 1.1 * (Rt + rt)])
            newp = pos[d] + step
            bad = (newp < lo) | (newp > hi)
            step[bad] = -step[bad]
            pos[d] = np.clip(pos[d] + step, np.minimum(lo, hi), np.maximum(lo, hi))
            rot[d] = _rot_axis_angle(rng.normal(size=3), rng.uniform(0, math.radians(1.0))) @ rot[d]

    per_light = np.full(n_lights, n_paths // n_lights, np.int64)
    per_light[: n_paths - per_light.sum()] += 1
    return Scene(
        name=name, static_verts=static, static_mat=static_mat, obj_local=obj_local,
        obj_mat=obj_mat, obj_xforms=oxf, albedo=albedo, light_half=light_half,
        light_power=light_power, light_xforms=lxf, light_paths=per_light,
        max_bounces=max_bounces, threshold=threshold, seed=seed,
        meta={"static_tris": int(static.shape[0]), "dynamic_tris": int(sum(o.shape[0] for o in obj_local)),
              "rooms": [nx, nz], "lights_move": bool(lights_move), "cell": h},
        light_kind=None if light_kind == 0 else np.full(n_lights, light_kind, np.int32),
        light_param=None if light_kind == 0 else np.tile(np.asarray(light_param, F32), (n_lights, 1)))


def make_mid(n_paths=1_000_000, frames=10, threshold=-1.0, seed=2, static_target=50_000):
    """4x4 rooms, ~50k static triangles, 3 tori of 2000 triangles, 2 static lights."""
    return make_rooms("mid", 4, 4, static_target, 3, (50, 20), n_paths, 7, frames,
                      threshold, seed, n_lights=2, lights_move=False)


def make_paper(n_paths=3_000_000, frames=30, threshold=0.01, seed=3, static_target=300_000):
    """6x6 rooms, ~300k static triangles, 8 tori of 10000 triangles, 2 moving lights."""
    return make_rooms("paper", 6, 6, static_target, 8, (100, 50), n_paths, 7, frames,
                      threshold, seed, n_lights=2, lights_move=True, torus_size=(0.2, 0.07))


def make_batch(n_scenes=64, frames=10, seed=4, path_range=(10_000, 2_000_000),
               tri_range=(5_000, 200_000), threshold=0.01):
    """Uneven scenes: triangle budgets and path counts log-uniform, 1..8 tori, B in 2..7."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(n_scenes):
        budget = int(math.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1]))))
        n_paths = int(math.exp(rng.uniform(math.log(path_range[0]), math.log(path_range[1]))))
        n_dyn = int(rng.integers(1, 9))
        B = int(rng.integers(2, 8))
        # dynamic share of the budget: at most 20%, split over the tori
        dyn_tris = max(200, int(0.2 * budget / n_dyn))
        nmaj = max(8, int(math.sqrt(dyn_tris / 2 * 2.5)))
        nmin = max(4, int(dyn_tris / (2 * nmaj)))
        side = 2 if budget < 20_000 else (3 if budget < 60_000 else 4)
        sc = make_rooms("batch%02d" % s, side, side, max(1000, budget - n_dyn * 2 * nmaj * nmin),
                        n_dyn, (nmaj, nmin), n_paths, B, frames, threshold,
                        seed * 1000 + s, n_lights=1 + int(rng.integers(0, 2)),
                        lights_move=bool(rng.integers(0, 2)))
        out.append(sc)
    return out


CONFIGS = {
    "tiny": make_tiny,
    "mid": make_mid,
    "paper": make_paper,
}
