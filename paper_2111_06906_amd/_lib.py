"""ctypes binding of libpv.so (the C-ABI declared in include/pv.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpv.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pv.h")

PV_OK, PV_ERR_ARG, PV_ERR_OOM, PV_ERR_HIP, PV_ERR_CAPACITY, PV_ERR_STATE = 0, -1, -2, -3, -4, -5
PV_MAX_BOUNCES, PV_MAX_OBJECTS, PV_MAX_LIGHTS = 15, 64, 8
HIT_NONE = 0xFFFFFFFF
_NAMES = {0: "PV_OK", -1: "PV_ERR_ARG", -2: "PV_ERR_OOM", -3: "PV_ERR_HIP", -4: "PV_ERR_CAPACITY",
          -5: "PV_ERR_STATE"}


class PVError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (_NAMES.get(code, str(code)), msg))
        self.code = code


class PathStore(C.Structure):
    _fields_ = [("n_paths", C.c_uint32), ("max_bounces", C.c_uint32), ("stride", C.c_uint32),
                ("d_pos_hit", C.c_void_p), ("d_energy", C.c_void_p), ("d_origin", C.c_void_p),
                ("d_info", C.c_void_p)]


class SceneDesc(C.Structure):
    _fields_ = [("n_static", C.c_uint32), ("h_static_verts", C.c_void_p), ("h_static_mat", C.c_void_p),
                ("n_objects", C.c_uint32), ("h_obj_tris", C.c_void_p), ("h_obj_verts", C.c_void_p),
                ("h_obj_mat", C.c_void_p), ("n_materials", C.c_uint32), ("h_albedo", C.c_void_p),
                ("n_lights", C.c_uint32), ("h_light_half", C.c_void_p), ("h_light_power", C.c_void_p),
                ("eps_end", C.c_float), ("eps_close", C.c_float), ("photon_radius", C.c_float),
                ("h_light_kind", C.c_void_p), ("h_light_param", C.c_void_p)]


STAT_FIELDS = ["segments_examined", "paths_invalid", "paths_light_lost", "rays_traced", "photons_written",
               "reuse_accepted", "paths_truncated", "verify_box_hits"]


class Config(C.Structure):
    _fields_ = [("max_paths", C.c_uint32), ("max_bounces", C.c_uint32), ("verify_mode", C.c_int32),
                ("object_rebuild", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [(n, C.c_ulonglong) for n in STAT_FIELDS]


_lib = None


def lib():
    """The loaded library; raises if it was not built (no CPU fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpv.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    try:
        import torch  # noqa: F401  -- load torch's HIP runtime first so both share it
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    P, U32, I32, U64, F = C.c_void_p, C.c_uint32, C.c_int32, C.c_uint64, C.c_float
    sig = {
        "pv_create": ([C.POINTER(P), P], I32),
        "pv_destroy": ([P], None),
        "pv_last_error": ([P], C.c_char_p),
        "pv_upload_scene": ([P, C.POINTER(SceneDesc)], I32),
        "pv_set_light_paths": ([P, P], I32),
        "pv_reserve": ([P, U32, U32], I32),
        "pv_create_config": ([C.POINTER(P), C.POINTER(Config), P], I32),
        "pv_frame_begin": ([P, P, P], I32),
        "pv_update_transforms": ([P, U32, P, P], I32),
        "pv_update_lights": ([P, U32, P, P], I32),
        "pv_verify_paths": ([P, C.POINTER(PathStore), P], I32),
        "pv_build_queue": ([P, C.POINTER(PathStore)], I32),
        "pv_queue_all": ([P, C.POINTER(PathStore)], I32),
        "pv_copy_queue": ([P, P, U32, P], I32),
        "pv_retrace_paths": ([P, C.POINTER(PathStore), F, U64, U32, P], I32),
        "pv_compact_photons": ([P, C.POINTER(PathStore), P, P, U32, P], I32),
        "pv_compact_photons_async": ([P, C.POINTER(PathStore), P, P, U32, P, P], I32),
        "pv_compact_photons_noalloc": ([P, C.POINTER(PathStore), P, P, U32, P], I32),
        "pv_energy_forward": ([P, C.POINTER(PathStore), P, P, P], I32),
        "pv_energy_backward": ([P, C.POINTER(PathStore), P, P, P, P, P], I32),
        "pv_store_bytes": ([U64, U32], U64),
        "pv_info_pack": ([U32, U32, U32, U32, U32], U32),
        "pv_info_unpack": ([U32, P, P, P, P, P], None),
        "pv_version": ([], C.c_char_p),
        "pv_hierarchy_info": ([P, U32, I32, P], I32),
        "pv_object_hierarchy_info": ([P, U32, P], I32),
        "pv_set_tuning": ([P, I32, I32], I32),
        "pv_set_verify_mode": ([P, I32], I32),
        "pv_get_tuning": ([P, I32, P], I32),
        "pv_autotune": ([P, C.POINTER(PathStore), F, U64, U32, P], I32),
        "pv_autotune_report": ([P, P], I32),
        "pv_set_distribution_map": ([P, P], I32),
        "pv_set_energy_test": ([P, I32], I32),
        "pv_distribution_cells": ([P], U32),
        "pv_update_distribution": ([P, C.POINTER(PathStore), U64, U32, P, P], I32),
    }
    optional = {}
    sig.update({
        "pv_batch_create": ([C.POINTER(P), P, P, U32, P, P, F, U64], I32),
        "pv_batch_destroy": ([P], None),
        "pv_batch_frame": ([P, U32, P], I32),
        "pv_batch_frames": ([P, U32, U32, P, P, P], I32),
        "pv_batch_copy_photons": ([P, P, P, U32, P], I32),
        "pv_batch_set_transforms": ([P, P, P], I32),
    })
    for name, (args, res) in list(sig.items()) + list(optional.items()):
        if not hasattr(L, name):
            if name in optional:
                continue
            raise RuntimeError("libpv.so lacks %s" % name)
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def declared_symbols():
    """Function names declared in include/pv.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pv_[a-z_]+)\s*\(", txt)))


def check(code, ctx=None):
    if code != PV_OK:
        msg = lib().pv_last_error(ctx)
        raise PVError(code, msg.decode() if msg else "")
    return code


def create(stream=None):
    ctx = C.c_void_p()
    check(lib().pv_create(C.byref(ctx), stream))
    return ctx


def create_config(max_paths=0, max_bounces=1, verify_mode=0, object_rebuild=0, stream=None):
    ctx = C.c_void_p()
    cfg = Config(max_paths, max_bounces, verify_mode, object_rebuild)
    check(lib().pv_create_config(C.byref(ctx), C.byref(cfg), stream))
    return ctx


def update_transforms(ctx, n, d_ids, d_m3x4):
    return check(lib().pv_update_transforms(ctx, n, d_ids, d_m3x4), ctx)


def update_lights(ctx, n, d_ids, d_m3x4):
    return check(lib().pv_update_lights(ctx, n, d_ids, d_m3x4), ctx)


def destroy(ctx):
    lib().pv_destroy(ctx)


def upload_scene(ctx, desc):
    check(lib().pv_upload_scene(ctx, C.byref(desc)), ctx)


def set_light_paths(ctx, counts_ptr):
    check(lib().pv_set_light_paths(ctx, counts_ptr), ctx)


def reserve(ctx, max_paths, max_bounces):
    check(lib().pv_reserve(ctx, max_paths, max_bounces), ctx)


def frame_begin(ctx, d_obj_xf, d_light_xf):
    check(lib().pv_frame_begin(ctx, d_obj_xf, d_light_xf), ctx)


def verify_paths(ctx, store, d_stats=None):
    check(lib().pv_verify_paths(ctx, C.byref(store), d_stats), ctx)


def build_queue(ctx, store):
    check(lib().pv_build_queue(ctx, C.byref(store)), ctx)


def queue_all(ctx, store):
    check(lib().pv_queue_all(ctx, C.byref(store)), ctx)


def copy_queue(ctx, d_out, capacity, d_count):
    check(lib().pv_copy_queue(ctx, d_out, capacity, d_count), ctx)


def retrace_paths(ctx, store, threshold, seed, frame, d_stats=None):
    check(lib().pv_retrace_paths(ctx, C.byref(store), C.c_float(threshold), seed, frame, d_stats), ctx)


def compact_photons(ctx, store, d_pos, d_energy, capacity, d_count):
    check(lib().pv_compact_photons(ctx, C.byref(store), d_pos, d_energy, capacity, d_count), ctx)


PV_NOALLOC_MAX_COUNTS = 131008  # path blocks x bounce rows the fixed scratch of the no-allocation form holds


def compact_photons_noalloc(ctx, store, d_pos, d_energy, capacity, d_count):
    check(lib().pv_compact_photons_noalloc(ctx, C.byref(store), d_pos, d_energy, capacity, d_count), ctx)


def compact_photons_async(ctx, store, d_pos, d_energy, capacity, d_count, stream):
    check(lib().pv_compact_photons_async(ctx, C.byref(store), d_pos, d_energy, capacity, d_count, stream), ctx)


def energy_forward(ctx, store, d_albedo, d_power, d_E):
    check(lib().pv_energy_forward(ctx, C.byref(store), d_albedo, d_power, d_E), ctx)


def energy_backward(ctx, store, d_albedo, d_power, d_gE, d_g_albedo, d_g_power):
    check(lib().pv_energy_backward(ctx, C.byref(store), d_albedo, d_power, d_gE, d_g_albedo, d_g_power), ctx)


def store_bytes(n_paths, max_bounces):
    return int(lib().pv_store_bytes(n_paths, max_bounces))


def info_pack(cell, nseg, start, replace, reuse):
    return int(lib().pv_info_pack(cell, nseg, start, replace, reuse))


def hierarchy_info(verts9, kind):
    import numpy as np
    v = np.ascontiguousarray(verts9, np.float32).reshape(-1, 9)
    out = (C.c_uint32 * 4)()
    check(lib().pv_hierarchy_info(v.ctypes.data_as(C.c_void_p), v.shape[0], kind, out))
    return {"nodes": out[0], "leaves": out[1], "depth": out[2], "valid": bool(out[3])}


def info_unpack(w):
    out = [C.c_uint32() for _ in range(5)]
    lib().pv_info_unpack(w, *[C.byref(o) for o in out])
    return tuple(o.value for o in out)


def batch_create(ctxs, stores, d_obj_xf, d_light_xf, threshold, seed):
    n = len(ctxs)
    carr = (C.c_void_p * n)(*[c.value for c in ctxs])
    sarr = (PathStore * n)(*stores)
    oarr = (C.c_void_p * n)(*d_obj_xf)
    larr = (C.c_void_p * n)(*d_light_xf)
    b = C.c_void_p()
    code = lib().pv_batch_create(C.byref(b), carr, sarr, n, oarr, larr, C.c_float(threshold), seed)
    check(code, ctxs[0])
    return b


def batch_destroy(b):
    lib().pv_batch_destroy(b)


def batch_frame(b, frame, d_stats=None, owner=None):
    check(lib().pv_batch_frame(b, frame, d_stats), owner)


def batch_frames(b, first_frame, k, d_obj_xf, d_light_xf, d_stats=None, owner=None):
    """d_obj_xf / d_light_xf: k * n device pointers, frame-major."""
    oarr = (C.c_void_p * len(d_obj_xf))(*d_obj_xf)
    larr = (C.c_void_p * len(d_light_xf))(*d_light_xf)
    check(lib().pv_batch_frames(b, first_frame, k, oarr, larr, d_stats), owner)


def batch_copy_photons(b, d_pos, d_energy, capacity, d_base, owner=None):
    check(lib().pv_batch_copy_photons(b, d_pos, d_energy, capacity, d_base), owner)


def batch_set_transforms(b, d_obj_xf, d_light_xf, owner=None):
    n = len(d_obj_xf)
    oarr = (C.c_void_p * n)(*d_obj_xf)
    larr = (C.c_void_p * n)(*d_light_xf)
    check(lib().pv_batch_set_transforms(b, oarr, larr), owner)


(PV_TUNE_RETRACE_VARIANT, PV_TUNE_RETRACE_BLOCKS_PER_CU, PV_TUNE_WALK_MIN_ACTIVE, PV_TUNE_VERIFY_BLOCKS_PER_CU,
 PV_TUNE_VERIFY_MIN_ACTIVE, PV_TUNE_OBJECT_REBUILD) = 0, 1, 2, 3, 4, 5


def object_hierarchy_info(ctx, obj):
    out = (C.c_uint32 * 5)()
    check(lib().pv_object_hierarchy_info(ctx, obj, out), ctx)
    return {"nodes": out[0], "leaves": out[1], "depth": out[2], "valid": bool(out[3]), "rebuilt": bool(out[4])}


def set_tuning(ctx, key, value):
    check(lib().pv_set_tuning(ctx, key, value), ctx)


PV_VERIFY_TRIANGLES, PV_VERIFY_BOXES = 0, 1
PV_LIGHT_AREA, PV_LIGHT_SPOT, PV_LIGHT_CAMERA = 0, 1, 2
PV_ENERGY_ALBEDO, PV_ENERGY_COSINE_RATIO = 0, 1


def set_energy_test(ctx, mode):
    check(lib().pv_set_energy_test(ctx, mode), ctx)


def set_verify_mode(ctx, mode):
    check(lib().pv_set_verify_mode(ctx, mode), ctx)


def get_tuning(ctx, key):
    v = C.c_int32()
    check(lib().pv_get_tuning(ctx, key, C.byref(v)), ctx)
    return v.value


def autotune(ctx, store, threshold, seed, frame):
    ms = C.c_float()
    check(lib().pv_autotune(ctx, C.byref(store), C.c_float(threshold), seed, frame, C.byref(ms)), ctx)
    return ms.value


AUTOTUNE_REPORT = ["verify_ms", "verify_spread", "verify_max_spread", "retrace_ms", "retrace_spread",
                   "retrace_max_spread", "trials"]


def autotune_report(ctx):
    out = (C.c_float * len(AUTOTUNE_REPORT))()
    check(lib().pv_autotune_report(ctx, out), ctx)
    return dict(zip(AUTOTUNE_REPORT, [float(x) for x in out]))


def set_distribution_map(ctx, grid):
    """grid: (gu, gv, rings, sectors), or None to disable the maps."""
    if grid is None:
        check(lib().pv_set_distribution_map(ctx, None), ctx)
    else:
        g = (C.c_int32 * 4)(*[int(x) for x in grid])
        check(lib().pv_set_distribution_map(ctx, g), ctx)


def distribution_cells(ctx):
    return int(lib().pv_distribution_cells(ctx))


def update_distribution(ctx, store, seed, frame, d_dm_c=None, d_pruned=None):
    check(lib().pv_update_distribution(ctx, C.byref(store), seed, frame, d_dm_c, d_pruned), ctx)
