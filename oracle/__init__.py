"""CPU oracle for photon-path verification -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It wraps ``liboracle.so`` (plain C, FP64, brute force) with
numpy marshalling and shares no code with the HIP library; the only thing the
two sides have in common is the seeded scene generator, which holds none of
the method's arithmetic.

Store layout used here (plain numpy):
    pos [B,N,3] f32, hit [B,N] u32, energy [B,N,3] f32, radius [B,N] f32,
    origin [N,3] f32, info [N] u32.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

HIT_NONE = 0xFFFFFFFF
AMB_EDGE, AMB_END, AMB_LIGHT, AMB_TIE, AMB_HEMI, AMB_CLOSE, AMB_BOX, AMB_CELL, AMB_EQ2 = 1, 2, 4, 8, 16, 32, 64, 128, 256

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("PV_ORACLE_LIB", _build.LIB)  # mutation tests load planted variants
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
        _declare(_lib)
    return _lib


class CScene(C.Structure):
    _fields_ = [
        ("n_tris", C.c_int64), ("verts", C.c_void_p), ("tri_obj", C.c_void_p),
        ("tri_mat", C.c_void_p), ("n_obj", C.c_int32), ("obj_moved", C.c_void_p),
        ("albedo", C.c_void_p), ("n_lights", C.c_int32), ("light_xf", C.c_void_p),
        ("light_half", C.c_void_p), ("light_power", C.c_void_p), ("light_moved", C.c_void_p),
        ("light_base", C.c_void_p), ("eps_end", C.c_double), ("eps_close", C.c_double),
        ("band_verify", C.c_double), ("band_trace", C.c_double), ("radius", C.c_float),
        ("verify_boxes", C.c_int32), ("band_box", C.c_double), ("dm", C.c_void_p),
        ("light_kind", C.c_void_p), ("light_param", C.c_void_p), ("energy_test", C.c_int32),
    ]


class CStore(C.Structure):
    _fields_ = [
        ("n_paths", C.c_int64), ("B", C.c_int32), ("pos", C.c_void_p), ("hit", C.c_void_p),
        ("energy", C.c_void_p), ("radius", C.c_void_p), ("origin", C.c_void_p), ("info", C.c_void_p),
    ]


def _declare(L):
    P = C.c_void_p
    L.or_transform.argtypes = [C.c_int64, P, P, P]
    L.or_xf_moved.argtypes = [P, P]
    L.or_xf_moved.restype = C.c_int
    L.or_philox4x64.argtypes = [P, P, P]
    L.or_cosine_local.argtypes = [C.c_double, C.c_double, P]
    L.or_cosine_dir.argtypes = [C.c_double, C.c_double, P, P]
    L.or_onb.argtypes = [P, P, P]
    L.or_segment_blocked_tri.argtypes = [P, P, P, C.c_double]
    L.or_segment_blocked_tri.restype = C.c_int
    L.or_segseg_dist.argtypes = [P, P, P, P]
    L.or_segseg_dist.restype = C.c_double
    L.or_light_update.argtypes = [P, P, C.c_int32, P, P, P, C.c_double, C.c_double, P, P]
    L.or_light_update.restype = C.c_int
    L.or_light_sample.argtypes = [P, P, C.c_int32, P, C.c_uint64, C.c_uint64, C.c_uint64, P, P]
    L.or_eq2.argtypes = [P, P, C.c_float]
    L.or_eq2.restype = C.c_int
    L.or_verify.argtypes = [P, P, P, P]
    L.or_verify_list.argtypes = [P, P, P, C.c_int64, P, P]
    L.or_segment_query.argtypes = [P, P, P, P]
    L.or_segment_query.restype = C.c_int
    L.or_closest_query.argtypes = [P, P, P, P, P]
    L.or_closest_query.restype = C.c_int64
    L.or_retrace.argtypes = [P, P, C.c_float, C.c_uint64, C.c_uint64, P, P]
    L.or_retrace_list.argtypes = [P, P, C.c_float, C.c_uint64, C.c_uint64, P, C.c_int64, P, P]
    L.or_energy_forward.argtypes = [P, C.c_int64, C.c_int32, P, P, P, P, P]
    L.or_energy_backward.argtypes = [P, C.c_int64, C.c_int32, P, P, P, P, P, C.c_int32, P, P]
    L.or_info_make.argtypes = [C.c_uint32] * 5
    L.or_info_make.restype = C.c_uint32
    L.or_dm_cells.argtypes = [P, C.c_int32, P]
    L.or_dm_cells.restype = C.c_int64
    L.or_dm_target.argtypes = [C.c_int64, C.c_int64, P]
    L.or_dm_cell.argtypes = [P, P, C.c_int32, P, P, P, P, C.c_double, P]
    L.or_dm_cell.restype = C.c_int64
    L.or_dm_sample.argtypes = [P, P, C.c_int32, P, P, C.c_int64, C.c_uint64, C.c_uint64, C.c_uint64, P, P]
    L.or_dm_update.argtypes = [P, P, C.c_uint64, C.c_uint64, P, P, P]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


# ---------------------------------------------------------------------------
# info word helpers (Section 4 layout: 22 | 4 | 4 | 1 | 1)

def info_make(cell, nseg, start, replace, reuse):
    return int(lib().or_info_make(cell, nseg, start, replace, reuse))


def info_fields(info):
    info = np.asarray(info, np.uint32)
    return {"cell": info & 0x3FFFFF, "nseg": (info >> 22) & 15, "start": (info >> 26) & 15,
            "replace": (info >> 30) & 1, "reuse": (info >> 31) & 1}


# ---------------------------------------------------------------------------
# scene state at one frame

@dataclass
class FrameScene:
    """Geometry and light state of one frame, as the oracle consumes it."""
    verts: np.ndarray       # [T,9] f32 world vertices
    tri_obj: np.ndarray     # [T] u32
    tri_mat: np.ndarray     # [T] u32
    obj_moved: np.ndarray   # [D+1] u8
    albedo: np.ndarray      # [M,3] f32
    light_xf: np.ndarray    # [L,12] f32
    light_half: np.ndarray  # [L,2] f32
    light_power: np.ndarray # [L,3] f32
    light_moved: np.ndarray # [L] u8
    light_base: np.ndarray  # [L+1] i64
    eps_end: float = 1e-4
    eps_close: float = 1e-4
    band_verify: float = 1e-6
    band_trace: float = 1e-5
    radius: float = 0.01
    verify_boxes: int = 0     # 1: Section 3.2's box test instead of the triangles
    band_box: float = 1e-5    # ambiguity band of the box test (covers the kernels' box padding)
    dm: object = None         # None, or the distribution-map grid (gu, gv, rings, sectors)
    light_kind: object = None   # None (all 0), or [L] i32: 0 rectangle / point, 1 spot, 2 camera
    light_param: object = None  # [L,2] f32: spot (cos of the half-angle, 0); camera (tan u, tan v)
    energy_test: int = 0        # Equation 2's E_N: 0 albedo (arrival side), 1 also the cosine ratio

    def cstruct(self):
        self._keep = [_c(self.verts, np.float32), _c(self.tri_obj, np.uint32), _c(self.tri_mat, np.uint32),
                      _c(self.obj_moved, np.uint8), _c(self.albedo, np.float32), _c(self.light_xf, np.float32),
                      _c(self.light_half, np.float32), _c(self.light_power, np.float32),
                      _c(self.light_moved, np.uint8), _c(self.light_base, np.int64),
                      None if self.dm is None else _c(self.dm, np.int32),
                      None if self.light_kind is None else _c(self.light_kind, np.int32),
                      None if self.light_param is None else _c(self.light_param, np.float32)]
        k = self._keep
        opt = [None if a is None else _p(a) for a in k[10:13]]
        return CScene(k[0].shape[0], _p(k[0]), _p(k[1]), _p(k[2]), k[3].shape[0], _p(k[3]), _p(k[4]),
                      k[5].shape[0], _p(k[5]), _p(k[6]), _p(k[7]), _p(k[8]), _p(k[9]),
                      self.eps_end, self.eps_close, self.band_verify, self.band_trace, self.radius,
                      int(self.verify_boxes), self.band_box, *opt, int(self.energy_test))

    def kind(self, l):
        return 0 if self.light_kind is None else int(self.light_kind[l])

    def param(self, l):
        return np.zeros(2, np.float32) if self.light_param is None else np.asarray(self.light_param[l], np.float32)

    def dm_offsets(self):
        """First cell of each light in the maps of all lights, and the total."""
        sizes = [dm_cells(self.light_half[l], self.dm, self.kind(l)) for l in range(self.light_half.shape[0])]
        return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def transform(local_verts, m12):
    """World vertices of a rigid object: FP64 fma chain rounded to FP32."""
    loc = _c(local_verts, np.float32).reshape(-1, 3)
    out = np.empty_like(loc)
    lib().or_transform(loc.shape[0], _p(loc), _p(_c(m12, np.float32)), _p(out))
    return out


def xf_moved(a, b):
    return bool(lib().or_xf_moved(_p(_c(a, np.float32)), _p(_c(b, np.float32))))


def frame_scene(scene, frame, prev_frame=None, band_verify=1e-6, band_trace=1e-5):
    """Oracle view of ``scene`` at ``frame``; moved flags relative to ``prev_frame``."""
    tri_obj, tri_mat, _ = scene.tri_layout()
    parts = [scene.static_verts.reshape(-1, 9)]
    for d, loc in enumerate(scene.obj_local):
        parts.append(transform(loc.reshape(-1, 3), scene.obj_xforms[frame, d]).reshape(-1, 9))
    verts = np.concatenate(parts).astype(np.float32)
    D = scene.n_dynamic
    L = scene.light_half.shape[0]
    obj_moved = np.zeros(D + 1, np.uint8)
    light_moved = np.zeros(L, np.uint8)
    if prev_frame is not None:
        for d in range(D):
            obj_moved[d + 1] = xf_moved(scene.obj_xforms[frame, d], scene.obj_xforms[prev_frame, d])
        for l in range(L):
            light_moved[l] = xf_moved(scene.light_xforms[frame, l], scene.light_xforms[prev_frame, l])
    return FrameScene(verts=verts, tri_obj=tri_obj, tri_mat=tri_mat, obj_moved=obj_moved,
                      albedo=scene.albedo, light_xf=scene.light_xforms[frame], light_half=scene.light_half,
                      light_power=scene.light_power, light_moved=light_moved, light_base=scene.light_base,
                      eps_end=scene.eps_end, eps_close=scene.eps_close, band_verify=band_verify,
                      band_trace=band_trace, radius=scene.photon_radius,
                      light_kind=getattr(scene, "light_kind", None), light_param=getattr(scene, "light_param", None))


# ---------------------------------------------------------------------------
# path store

@dataclass
class Store:
    pos: np.ndarray
    hit: np.ndarray
    energy: np.ndarray
    radius: np.ndarray
    origin: np.ndarray
    info: np.ndarray

    @property
    def n_paths(self):
        return int(self.info.shape[0])

    @property
    def B(self):
        return int(self.hit.shape[0])

    @staticmethod
    def empty(n_paths, B):
        return Store(pos=np.zeros((B, n_paths, 3), np.float32),
                     hit=np.full((B, n_paths), HIT_NONE, np.uint32),
                     energy=np.zeros((B, n_paths, 3), np.float32),
                     radius=np.zeros((B, n_paths), np.float32),
                     origin=np.zeros((n_paths, 3), np.float32),
                     info=np.zeros(n_paths, np.uint32))

    def copy(self):
        return Store(*(np.array(a, copy=True) for a in
                       (self.pos, self.hit, self.energy, self.radius, self.origin, self.info)))

    def cstruct(self):
        for a, dt in ((self.pos, np.float32), (self.hit, np.uint32), (self.energy, np.float32),
                      (self.radius, np.float32), (self.origin, np.float32), (self.info, np.uint32)):
            assert a.dtype == dt and a.flags.c_contiguous
        return CStore(self.n_paths, self.B, _p(self.pos), _p(self.hit), _p(self.energy),
                      _p(self.radius), _p(self.origin), _p(self.info))

    def select(self, idx):
        idx = np.asarray(idx)
        return Store(pos=np.ascontiguousarray(self.pos[:, idx]), hit=np.ascontiguousarray(self.hit[:, idx]),
                     energy=np.ascontiguousarray(self.energy[:, idx]),
                     radius=np.ascontiguousarray(self.radius[:, idx]),
                     origin=np.ascontiguousarray(self.origin[idx]), info=np.ascontiguousarray(self.info[idx]))


# ---------------------------------------------------------------------------
# the method's steps

def verify(fs: FrameScene, store: Store, paths=None):
    """Origin update + dynamic occlusions (Sections 3.1, 3.2), in place.

    Returns (amb flags, examined segment counts) per path (or per listed path).
    """
    cs, st = fs.cstruct(), store.cstruct()
    if paths is None:
        amb = np.zeros(store.n_paths, np.uint32)
        ex = np.zeros(store.n_paths, np.int32)
        lib().or_verify(C.byref(cs), C.byref(st), _p(amb), _p(ex))
    else:
        lst = _c(paths, np.int64)
        amb = np.zeros(lst.shape[0], np.uint32)
        ex = np.zeros(lst.shape[0], np.int32)
        lib().or_verify_list(C.byref(cs), C.byref(st), _p(lst), lst.shape[0], _p(amb), _p(ex))
    return amb, ex


def retrace(fs: FrameScene, store: Store, T, seed, frame, paths=None):
    """Re-trace paths with the replace bit (naive for T < 0, Algorithm 1 otherwise)."""
    cs, st = fs.cstruct(), store.cstruct()
    if paths is None:
        amb = np.zeros(store.n_paths, np.uint32)
        tr = np.zeros(store.n_paths, np.int32)
        lib().or_retrace(C.byref(cs), C.byref(st), C.c_float(T), seed, frame, _p(amb), _p(tr))
    else:
        lst = _c(paths, np.int64)
        amb = np.zeros(lst.shape[0], np.uint32)
        tr = np.zeros(lst.shape[0], np.int32)
        lib().or_retrace_list(C.byref(cs), C.byref(st), C.c_float(T), seed, frame, _p(lst), lst.shape[0],
                              _p(amb), _p(tr))
    return amb, tr


def initial_trace(fs: FrameScene, n_paths, B, seed, frame=0, paths=None):
    """Frame-0 photon paths: every path a new light sample traced to B photons
    (with distribution maps, the fill first gives every path its cell)."""
    st = Store.empty(n_paths, B)
    st.info[:] = info_make(0, 0, 0, 1, 0)
    if fs.dm is not None:
        dm_update(fs, st, seed, frame)
    amb, tr = retrace(fs, st, -1.0, seed, frame, paths)
    return st, amb, tr


# ---------------------------------------------------------------------------
# distribution maps (Section 3.1)

def dm_cells(half, dm, kind=0):
    return int(lib().or_dm_cells(_p(_c(half, np.float32)), int(kind), _p(_c(dm, np.int32))))


def dm_target(n_cells, n_paths):
    out = np.zeros(n_cells, np.uint32)
    lib().or_dm_target(n_cells, n_paths, _p(out))
    return out


def dm_cell(xf, half, dm, x0, w, band=1e-6, kind=0, param=(0.0, 0.0)):
    """(cell or -1, ambiguity flags) of a light sample."""
    amb = np.zeros(1, np.uint32)
    c = lib().or_dm_cell(_p(_c(xf, np.float32)), _p(_c(half, np.float32)), int(kind), _p(_c(param, np.float32)),
                         _p(_c(dm, np.int32)), _p(_c(x0, np.float64)), _p(_c(w, np.float64)), band, _p(amb))
    return int(c), int(amb[0])


def dm_sample(xf, half, dm, cell, seed, path, frame, kind=0, param=(0.0, 0.0)):
    x0 = np.zeros(3)
    w = np.zeros(3)
    lib().or_dm_sample(_p(_c(xf, np.float32)), _p(_c(half, np.float32)), int(kind), _p(_c(param, np.float32)),
                       _p(_c(dm, np.int32)), int(cell), seed, path, frame, _p(x0), _p(w))
    return x0, w


def dm_update(fs: FrameScene, store: Store, seed, frame):
    """Compute DM_C, prune (Equation 1), fill, in place; returns (DM_C before
    pruning, pruned per cell, ambiguity flags per path)."""
    total = int(fs.dm_offsets()[-1])
    dm_c = np.zeros(total, np.uint32)
    pruned = np.zeros(total, np.uint32)
    amb = np.zeros(store.n_paths, np.uint32)
    lib().or_dm_update(C.byref(fs.cstruct()), C.byref(store.cstruct()), seed, frame, _p(dm_c), _p(pruned),
                       _p(amb))
    return dm_c, pruned, amb


def queue(info):
    """Retrace work list: ascending ids of paths with the replace bit."""
    return np.flatnonzero((np.asarray(info, np.uint32) >> 30) & 1).astype(np.uint32)


def compact_photons(store: Store):
    """Existing photons in (row, path) order: positions and energies."""
    n = info_fields(store.info)["nseg"].astype(np.int64)
    mask = np.arange(store.B)[:, None] < n[None, :]
    return store.pos[mask], store.energy[mask]


def segment_query(fs: FrameScene, a, b):
    amb = np.zeros(1, np.uint32)
    r = lib().or_segment_query(C.byref(fs.cstruct()), _p(_c(a, np.float64)), _p(_c(b, np.float64)), _p(amb))
    return bool(r), int(amb[0])


def closest_query(fs: FrameScene, o, w):
    amb = np.zeros(1, np.uint32)
    t = np.zeros(1, np.float64)
    tri = lib().or_closest_query(C.byref(fs.cstruct()), _p(_c(o, np.float64)), _p(_c(w, np.float64)), _p(t),
                                 _p(amb))
    return int(tri), float(t[0]), int(amb[0])


def light_update(xf, half, x0, x1, eps=1e-4, band=1e-6, kind=0, param=(0.0, 0.0)):
    out = np.zeros(3, np.float64)
    amb = np.zeros(1, np.uint32)
    ok = lib().or_light_update(_p(_c(xf, np.float32)), _p(_c(half, np.float32)), int(kind),
                               _p(_c(param, np.float32)), _p(_c(x0, np.float64)), _p(_c(x1, np.float64)), eps,
                               band, _p(out), _p(amb))
    return bool(ok), out, int(amb[0])


def light_sample(xf, half, seed, path, frame, kind=0, param=(0.0, 0.0)):
    x0 = np.zeros(3)
    w = np.zeros(3)
    lib().or_light_sample(_p(_c(xf, np.float32)), _p(_c(half, np.float32)), int(kind), _p(_c(param, np.float32)),
                          seed, path, frame, _p(x0), _p(w))
    return x0, w


def philox4x64(ctr, key):
    out = np.zeros(4, np.uint64)
    lib().or_philox4x64(_p(_c(ctr, np.uint64)), _p(_c(key, np.uint64)), _p(out))
    return out


def cosine_local(u1, u2):
    out = np.zeros(3)
    lib().or_cosine_local(u1, u2, _p(out))
    return out


def cosine_dir(u1, u2, n):
    out = np.zeros(3)
    lib().or_cosine_dir(u1, u2, _p(_c(n, np.float64)), _p(out))
    return out


def onb(n):
    t, b = np.zeros(3), np.zeros(3)
    lib().or_onb(_p(_c(n, np.float64)), _p(t), _p(b))
    return t, b


def segment_blocked_tri(a, b, tri9, eps):
    return bool(lib().or_segment_blocked_tri(_p(_c(a, np.float64)), _p(_c(b, np.float64)),
                                             _p(_c(tri9, np.float64)), eps))


def segseg_dist(p0, p1, q0, q1):
    return float(lib().or_segseg_dist(*[_p(_c(x, np.float64)) for x in (p0, p1, q0, q1)]))


def eq2(en, eo, T):
    return bool(lib().or_eq2(_p(_c(en, np.float32)), _p(_c(eo, np.float32)), C.c_float(T)))


def energy_forward(fs: FrameScene, store: Store, albedo, power):
    N, B = store.n_paths, store.B
    E = np.zeros((B, N, 3), np.float64)
    lib().or_energy_forward(C.byref(fs.cstruct()), N, B, _p(store.hit), _p(store.info),
                            _p(_c(albedo, np.float64)), _p(_c(power, np.float64)), _p(E))
    return E


def energy_backward(fs: FrameScene, store: Store, albedo, power, gE):
    N, B = store.n_paths, store.B
    alb = _c(albedo, np.float64)
    pw = _c(power, np.float64)
    ga = np.zeros_like(alb)
    gp = np.zeros_like(pw)
    lib().or_energy_backward(C.byref(fs.cstruct()), N, B, _p(store.hit), _p(store.info), _p(alb), _p(pw),
                             _p(_c(gE, np.float64)), alb.shape[0], _p(ga), _p(gp))
    return ga, gp
