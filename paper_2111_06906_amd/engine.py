"""Python-side owner of a scene context and its device path store.

PyTorch only provides device memory and the stream; every computation is a
call into libpv.so through the ctypes binding.  On a machine without a HIP
device, constructing a Context raises.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .scenes import Scene

F32 = torch.float32
I32 = torch.int32


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class Store:
    """Device path store (layout of include/pv.h)."""

    def __init__(self, n_paths, max_bounces, device="cuda"):
        if not 1 <= max_bounces <= L.PV_MAX_BOUNCES:
            raise ValueError("max_bounces out of range")
        self.n_paths = int(n_paths)
        self.B = int(max_bounces)
        self.stride = max(64, (self.n_paths + 63) // 64 * 64)
        self.pos_hit = torch.zeros((self.B, self.stride, 4), dtype=F32, device=device)
        self.pos_hit.view(I32)[:, :, 3] = -1  # hit = 0xFFFFFFFF
        self.energy = torch.zeros((self.B, self.stride, 4), dtype=F32, device=device)
        self.origin = torch.zeros((3, self.stride), dtype=F32, device=device)
        self.info = torch.zeros((self.stride,), dtype=I32, device=device)

    def cstruct(self):
        return L.PathStore(self.n_paths, self.B, self.stride, self.pos_hit.data_ptr(), self.energy.data_ptr(),
                           self.origin.data_ptr(), self.info.data_ptr())

    # plain layout used by the tests: pos [B,N,3], hit [B,N], energy [B,N,3],
    # radius [B,N], origin [N,3], info [N] (layout conversion only)
    def to_numpy(self, cols=None):
        n = self.n_paths
        ph = self.pos_hit[:, :n].cpu().numpy()
        en = self.energy[:, :n].cpu().numpy()
        d = dict(pos=np.ascontiguousarray(ph[..., :3]),
                 hit=np.ascontiguousarray(ph[..., 3]).view(np.uint32),
                 energy=np.ascontiguousarray(en[..., :3]), radius=np.ascontiguousarray(en[..., 3]),
                 origin=np.ascontiguousarray(self.origin[:, :n].cpu().numpy().T),
                 info=self.info[:n].cpu().numpy().view(np.uint32).copy())
        if cols is not None:
            cols = np.asarray(cols)
            d = {k: (np.ascontiguousarray(v[:, cols]) if k in ("pos", "hit", "energy", "radius")
                     else np.ascontiguousarray(v[cols])) for k, v in d.items()}
        return d

    def load_numpy(self, d, cols=None):
        """Write plain-layout arrays into all columns, or into the given ones."""
        dev = self.pos_hit.device
        ph = np.concatenate([d["pos"], d["hit"].view(np.float32)[..., None]], axis=-1).astype(np.float32)
        en = np.concatenate([d["energy"], d["radius"][..., None]], axis=-1).astype(np.float32)
        idx = torch.arange(self.n_paths, device=dev) if cols is None else torch.as_tensor(
            np.asarray(cols, np.int64), device=dev)
        self.pos_hit[:, idx] = torch.from_numpy(ph).to(dev)
        self.energy[:, idx] = torch.from_numpy(en).to(dev)
        self.origin[:, idx] = torch.from_numpy(np.ascontiguousarray(d["origin"].T)).to(dev)
        self.info[idx] = torch.from_numpy(d["info"].astype(np.uint32).view(np.int32)).to(dev)


class Context:
    """One scene on the device: upload, per-frame transforms, the method's calls."""

    def __init__(self, scene: Scene, max_paths=None, max_bounces=None, stream=None, config=None):
        """config: None, or a dict of pv_config fields other than the sizes
        (verify_mode, object_rebuild): the context is then made by
        pv_create_config, which also reserves the scratch."""
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.scene = scene
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.max_paths = int(max_paths or scene.n_paths)
        self.max_bounces = int(max_bounces or scene.max_bounces)
        if config is None:
            self.ctx = L.create(C.c_void_p(self.stream.cuda_stream))
        else:
            self.ctx = L.create_config(self.max_paths, self.max_bounces, int(config.get("verify_mode", 0)),
                                       int(config.get("object_rebuild", 0)), C.c_void_p(self.stream.cuda_stream))
        self._upload(scene)
        counts = np.ascontiguousarray(scene.light_paths, np.uint32)
        L.set_light_paths(self.ctx, _np_ptr(counts))
        if config is None:
            L.reserve(self.ctx, self.max_paths, self.max_bounces)
        self.obj_xf = torch.from_numpy(np.ascontiguousarray(scene.obj_xforms, np.float32)).cuda()
        self.light_xf = torch.from_numpy(np.ascontiguousarray(scene.light_xforms, np.float32)).cuda()
        if self.obj_xf.numel() == 0:
            self.obj_xf = torch.zeros((scene.n_frames, 1, 12), dtype=F32, device="cuda")

    def _upload(self, sc: Scene):
        sv = np.ascontiguousarray(sc.static_verts.reshape(-1, 9), np.float32)
        sm = np.ascontiguousarray(sc.static_mat, np.uint32)
        ot = np.ascontiguousarray([o.shape[0] for o in sc.obj_local] or [0], np.uint32)
        ov = np.ascontiguousarray(np.concatenate([o.reshape(-1, 9) for o in sc.obj_local]) if sc.obj_local
                                  else np.zeros((1, 9)), np.float32)
        om = np.ascontiguousarray(np.concatenate(sc.obj_mat) if sc.obj_mat else np.zeros(1), np.uint32)
        alb = np.ascontiguousarray(sc.albedo, np.float32)
        lh = np.ascontiguousarray(sc.light_half, np.float32)
        lp = np.ascontiguousarray(sc.light_power, np.float32)
        lk = None if sc.light_kind is None else np.ascontiguousarray(sc.light_kind, np.int32)
        lq = None if sc.light_param is None else np.ascontiguousarray(sc.light_param, np.float32)
        self._keep = (sv, sm, ot, ov, om, alb, lh, lp, lk, lq)
        desc = L.SceneDesc(sv.shape[0], _np_ptr(sv), _np_ptr(sm), len(sc.obj_local), _np_ptr(ot), _np_ptr(ov),
                           _np_ptr(om), alb.shape[0], _np_ptr(alb), lh.shape[0], _np_ptr(lh), _np_ptr(lp),
                           sc.eps_end, sc.eps_close, sc.photon_radius,
                           None if lk is None else _np_ptr(lk), None if lq is None else _np_ptr(lq))
        L.upload_scene(self.ctx, desc)

    def close(self):
        if getattr(self, "ctx", None):
            L.destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def new_store(self, n_paths=None):
        return Store(n_paths or self.scene.n_paths, self.scene.max_bounces)

    def new_stats(self):
        return torch.zeros(len(L.STAT_FIELDS), dtype=torch.int64, device="cuda")

    @staticmethod
    def stats_dict(t):
        return dict(zip(L.STAT_FIELDS, t.cpu().tolist()))

    # --- the method's calls ---------------------------------------------
    def frame_begin(self, frame):
        L.frame_begin(self.ctx, _ptr(self.obj_xf[frame]), _ptr(self.light_xf[frame]))

    def frame_begin_staged(self):
        """Begin a frame with the staged transforms (pv_frame_begin(ctx, NULL, NULL))."""
        L.frame_begin(self.ctx, None, None)

    def update_transforms(self, ids, m3x4):
        """Stage transforms of the objects 'ids' (pv_update_transforms); returns
        the device arrays, which must live until the stream has used them."""
        d_ids = torch.as_tensor(np.asarray(ids, np.int64).astype(np.int32), device="cuda")
        d_m = torch.as_tensor(np.asarray(m3x4, np.float32).reshape(-1, 12), device="cuda").contiguous()
        L.update_transforms(self.ctx, int(d_ids.numel()), _ptr(d_ids), _ptr(d_m))
        return d_ids, d_m

    def update_lights(self, ids, m3x4):
        """Stage transforms of the lights 'ids' (pv_update_lights)."""
        d_ids = torch.as_tensor(np.asarray(ids, np.int64).astype(np.int32), device="cuda")
        d_m = torch.as_tensor(np.asarray(m3x4, np.float32).reshape(-1, 12), device="cuda").contiguous()
        L.update_lights(self.ctx, int(d_ids.numel()), _ptr(d_ids), _ptr(d_m))
        return d_ids, d_m

    def verify(self, store, stats=None, build_queue=True):
        L.verify_paths(self.ctx, store.cstruct(), _ptr(stats))
        if build_queue:
            L.build_queue(self.ctx, store.cstruct())

    def build_queue(self, store):
        L.build_queue(self.ctx, store.cstruct())

    def queue_all(self, store):
        L.queue_all(self.ctx, store.cstruct())

    def queue(self):
        out = torch.zeros(self.max_paths, dtype=I32, device="cuda")
        cnt = torch.zeros(1, dtype=I32, device="cuda")
        L.copy_queue(self.ctx, _ptr(out), self.max_paths, _ptr(cnt))
        n = int(cnt.item())
        return out[:n].cpu().numpy().view(np.uint32)

    def retrace(self, store, threshold, seed, frame, stats=None):
        L.retrace_paths(self.ctx, store.cstruct(), float(threshold), int(seed), int(frame), _ptr(stats))

    def compact_photons(self, store, capacity=None):
        cap = store.n_paths * store.B if capacity is None else int(capacity)
        pos = torch.zeros((max(cap, 1), 3), dtype=F32, device="cuda")
        en = torch.zeros((max(cap, 1), 3), dtype=F32, device="cuda")
        cnt = torch.zeros(1, dtype=I32, device="cuda")
        L.compact_photons(self.ctx, store.cstruct(), _ptr(pos), _ptr(en), cap, _ptr(cnt))
        n = int(cnt.item())
        return pos[:min(n, cap)], en[:min(n, cap)], n

    def compact_photons_into(self, store, pos, en, cnt, stream=None):
        """Compaction into preallocated outputs; no host synchronisation.  With
        a torch stream, the overlap form: it runs there beside the next frame's
        begin and verification, and the next re-trace waits for it."""
        if stream is None:
            L.compact_photons(self.ctx, store.cstruct(), _ptr(pos), _ptr(en), pos.shape[0], _ptr(cnt))
        else:
            L.compact_photons_async(self.ctx, store.cstruct(), _ptr(pos), _ptr(en), pos.shape[0], _ptr(cnt),
                                    stream.cuda_stream)

    def energy_forward(self, store, albedo, power):
        E = torch.empty((store.B, store.n_paths, 3), dtype=F32, device="cuda")
        L.energy_forward(self.ctx, store.cstruct(), _ptr(albedo.contiguous()), _ptr(power.contiguous()), _ptr(E))
        return E

    def energy_backward(self, store, albedo, power, gE):
        ga = torch.empty_like(albedo)
        gp = torch.empty_like(power)
        L.energy_backward(self.ctx, store.cstruct(), _ptr(albedo.contiguous()), _ptr(power.contiguous()),
                          _ptr(gE.contiguous()), _ptr(ga), _ptr(gp))
        return ga, gp

    def autotune(self, store, threshold, seed, frame):
        """Pick the fastest verification and re-trace grids, thresholds and variant on this workload."""
        ms = L.autotune(self.ctx, store.cstruct(), float(threshold), int(seed), int(frame))
        return {"retrace_variant": L.get_tuning(self.ctx, L.PV_TUNE_RETRACE_VARIANT),
                "retrace_blocks_per_cu": L.get_tuning(self.ctx, L.PV_TUNE_RETRACE_BLOCKS_PER_CU),
                "walk_min_active": L.get_tuning(self.ctx, L.PV_TUNE_WALK_MIN_ACTIVE),
                "verify_blocks_per_cu": L.get_tuning(self.ctx, L.PV_TUNE_VERIFY_BLOCKS_PER_CU),
                "verify_min_active": L.get_tuning(self.ctx, L.PV_TUNE_VERIFY_MIN_ACTIVE),
                "retrace_ms": ms, "report": L.autotune_report(self.ctx)}

    def set_tuning(self, variant=None, blocks_per_cu=None, walk_min_active=None, verify_blocks_per_cu=None,
                   verify_min_active=None, object_rebuild=None):
        for key, v in ((L.PV_TUNE_RETRACE_VARIANT, variant), (L.PV_TUNE_RETRACE_BLOCKS_PER_CU, blocks_per_cu),
                       (L.PV_TUNE_WALK_MIN_ACTIVE, walk_min_active),
                       (L.PV_TUNE_VERIFY_BLOCKS_PER_CU, verify_blocks_per_cu),
                       (L.PV_TUNE_VERIFY_MIN_ACTIVE, verify_min_active),
                       (L.PV_TUNE_OBJECT_REBUILD, object_rebuild)):
            if v is not None:
                L.set_tuning(self.ctx, key, int(v))

    def set_verify_mode(self, boxes):
        """Section 3.2's conservative box test (True) or the triangle test (False)."""
        L.set_verify_mode(self.ctx, L.PV_VERIFY_BOXES if boxes else L.PV_VERIFY_TRIANGLES)

    def set_energy_test(self, cosine_ratio):
        """Equation 2's E_N: the albedo test (False) or the cosine-ratio test (True)."""
        L.set_energy_test(self.ctx, L.PV_ENERGY_COSINE_RATIO if cosine_ratio else L.PV_ENERGY_ALBEDO)

    def set_distribution_map(self, grid):
        """Section 3.1's distribution maps with grid (gu, gv, rings, sectors), or None."""
        L.set_distribution_map(self.ctx, grid)

    def update_distribution(self, store, seed, frame):
        """Compute DM_C, prune (Equation 1), fill; returns (DM_C before pruning,
        pruned per cell) as device tensors over all lights' cells."""
        n = L.distribution_cells(self.ctx)
        dm_c = torch.zeros(max(n, 1), dtype=I32, device="cuda")
        pruned = torch.zeros(max(n, 1), dtype=I32, device="cuda")
        L.update_distribution(self.ctx, store.cstruct(), int(seed), int(frame), _ptr(dm_c), _ptr(pruned))
        return dm_c[:n], pruned[:n]

    def object_hierarchy_info(self, obj):
        """Check of dynamic object obj's current device hierarchy (synchronises)."""
        return L.object_hierarchy_info(self.ctx, int(obj))

    def initial_trace(self, store, seed, frame=0, stats=None):
        """Frame-0 photon paths (every path a new light sample; with
        distribution maps, the fill first gives every path its cell)."""
        self.queue_all(store)
        if L.distribution_cells(self.ctx):
            self.update_distribution(store, seed, frame)
        self.retrace(store, -1.0, seed, frame, stats)


class Batch:
    """Several scene contexts run as one frame: one launch per phase, the whole
    frame captured in a HIP graph (batched form)."""

    def __init__(self, contexts, stores, threshold, seed):
        self.contexts = list(contexts)
        self.stores = list(stores)
        self._cs = [s.cstruct() for s in self.stores]
        self.b = L.batch_create([c.ctx for c in self.contexts], self._cs,
                                [c.obj_xf[0].data_ptr() for c in self.contexts],
                                [c.light_xf[0].data_ptr() for c in self.contexts], float(threshold), int(seed))

    def frame(self, f, stats=None):
        owner = self.contexts[0].ctx
        L.batch_set_transforms(self.b, [c.obj_xf[f].data_ptr() for c in self.contexts],
                               [c.light_xf[f].data_ptr() for c in self.contexts], owner)
        L.batch_frame(self.b, int(f), _ptr(stats), owner)

    def frames(self, first, k, stats=None):
        """Frames first .. first + k - 1 of every scene in one graph launch."""
        owner = self.contexts[0].ctx
        obj, light = [], []
        for f in range(first, first + k):
            obj += [c.obj_xf[f].data_ptr() for c in self.contexts]
            light += [c.light_xf[f].data_ptr() for c in self.contexts]
        L.batch_frames(self.b, int(first), int(k), obj, light, _ptr(stats), owner)

    def photons(self):
        """(positions [cap,3], energies [cap,3], per-scene first photon [n+1]) of the last frame."""
        cap = sum(s.n_paths * s.B for s in self.stores)
        pos = torch.empty((max(cap, 1), 3), dtype=F32, device="cuda")
        en = torch.empty((max(cap, 1), 3), dtype=F32, device="cuda")
        base = torch.empty(len(self.contexts) + 1, dtype=I32, device="cuda")
        L.batch_copy_photons(self.b, _ptr(pos), _ptr(en), cap, _ptr(base), self.contexts[0].ctx)
        return pos, en, base

    def close(self):
        if getattr(self, "b", None):
            L.batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
