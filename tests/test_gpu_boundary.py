"""The boundary's own names drive a frame: a context made by pv_create_config,
transforms given per object and light id (pv_update_transforms /
pv_update_lights), then pv_verify_paths, pv_retrace_paths (which builds the
work queue itself) and pv_compact_photons.  The result must equal the dense
form (pv_frame_begin with whole transform arrays, pv_build_queue) bit for bit
and the oracle element by element.
"""
import numpy as np
import pytest

import oracle as O
from paper_2111_06906_amd import scenes
from tests import harness as H

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_06906_amd import engine
    return engine


def _scene():
    # objects 1, 2 and 5 never move and object 7 stops in frame 2; both lights move
    sc = scenes.make_paper(n_paths=4096 + 13, frames=3)
    for o in (1, 2, 5):
        sc.obj_xforms[:, o] = sc.obj_xforms[0, o]
    sc.obj_xforms[2, 7] = sc.obj_xforms[1, 7]
    return sc


def _changed(a, b):
    return [i for i in range(a.shape[0]) if not np.array_equal(a[i].view(np.uint32), b[i].view(np.uint32))]


def test_frame_through_the_boundary_names(E):
    import torch
    sc = _scene()
    T, seed = 0.01, sc.seed
    ora, _ = O.initial_trace(O.frame_scene(sc, 0), sc.n_paths, sc.max_bounces, seed)[:2]
    # sparse form: pv_create_config, pv_update_*, verify, retrace, compaction
    a = E.Context(sc, config={"verify_mode": 0})
    sa = a.new_store()
    keep = [a.update_transforms(range(sc.n_dynamic), sc.obj_xforms[0]), a.update_lights([0, 1], sc.light_xforms[0])]
    a.queue_all(sa)
    a.retrace(sa, -1.0, seed, 0)        # begins frame 0 with the staged transforms
    # dense form
    b = E.Context(sc)
    sb = b.new_store()
    b.frame_begin(0)
    for f in (1, 2):
        sa.load_numpy(H.from_oracle(ora))
        sb.load_numpy(H.from_oracle(ora))
        moved = _changed(sc.obj_xforms[f], sc.obj_xforms[f - 1])
        log("frame %d: objects updated by id %s" % (f, moved))
        # a repeated id takes its last matrix: stage a wrong one first
        ids = [moved[0]] + moved
        mats = np.concatenate([sc.obj_xforms[f - 1][moved[:1]], sc.obj_xforms[f][moved]])
        keep.append(a.update_transforms(ids, mats))
        keep.append(a.update_lights([1, 0], sc.light_xforms[f][[1, 0]]))
        stats = a.new_stats()
        a.verify(sa, stats, build_queue=False)
        a.retrace(sa, T, seed, f, stats)
        pa, ea, na = a.compact_photons(sa)
        b.frame_begin(f)
        b.verify(sb)
        b.retrace(sb, T, seed, f)
        pb, eb, nb = b.compact_photons(sb)
        torch.cuda.synchronize()
        da, db = sa.to_numpy(), sb.to_numpy()
        for k in da:
            assert np.array_equal(da[k].view(np.uint32), db[k].view(np.uint32)), (f, k)
        assert na == nb and torch.equal(pa, pb) and torch.equal(ea, eb)
        # against the oracle
        fs = O.frame_scene(sc, f, f - 1)
        ambv, _ = O.verify(fs, ora)
        ambr, _ = O.retrace(fs, ora, T, seed, f)
        ok = (ambv == 0) & (ambr == 0)
        H.check_excluded((~ok).sum(), sc.n_paths, "boundary names frame %d" % f)
        H.compare_stores(da, ora, ok, "boundary names frame %d" % f, fs.verts, (~ok).sum())
        s = a.stats_dict(stats)
        assert s["paths_invalid"] > 0 and s["rays_traced"] > 0
        assert na == int(((da["info"] >> 22) & 15).sum())
    a.close()
    b.close()


def test_boundary_argument_errors(E):
    import ctypes as C
    import torch
    from paper_2111_06906_amd import _lib as L
    sc = scenes.make_tiny(n_paths=256)
    # a bad option returns no context
    with pytest.raises(L.PVError) as e:
        L.create_config(256, 3, 7, 0)
    assert e.value.code == L.PV_ERR_ARG
    with pytest.raises(L.PVError) as e:
        L.create_config(256, 16, 0, 0)
    assert e.value.code == L.PV_ERR_ARG
    ctx = E.Context(sc, config={})
    ids = torch.zeros(65, dtype=torch.int32, device="cuda")
    m = torch.zeros((65, 12), dtype=torch.float32, device="cuda")
    for fn in (L.update_transforms, L.update_lights):
        with pytest.raises(L.PVError) as e:
            fn(ctx.ctx, 65, C.c_void_p(ids.data_ptr()), C.c_void_p(m.data_ptr()))
        assert e.value.code == L.PV_ERR_ARG
        with pytest.raises(L.PVError) as e:
            fn(ctx.ctx, 1, None, C.c_void_p(m.data_ptr()))
        assert e.value.code == L.PV_ERR_ARG
    with pytest.raises(L.PVError) as e:
        L.update_lights(ctx.ctx, 9, C.c_void_p(ids.data_ptr()), C.c_void_p(m.data_ptr()))
    assert e.value.code == L.PV_ERR_ARG
    # an id beyond the scene's objects is skipped; the rest is taken
    ctx.update_transforms([0, 5], np.stack([sc.obj_xforms[0, 0], sc.obj_xforms[0, 0]]))
    ctx.update_lights([0], sc.light_xforms[0])
    st = ctx.new_store()
    ctx.initial_trace(st, sc.seed, 0)
    ctx.frame_begin(0)           # the dense arrays of frame 0: nothing moved
    ctx.verify(st)
    assert ctx.queue().size == 0
    ctx.close()


def test_boundary_call_order_and_store_errors(E):
    # calls out of order return PV_ERR_STATE, malformed stores PV_ERR_ARG, a
    # store beyond the reservation PV_ERR_CAPACITY; each before anything is
    # enqueued, and the context stays usable: a frame run afterwards matches
    # the same frame on a fresh context bit for bit
    import ctypes as C
    import torch
    from paper_2111_06906_amd import _lib as L
    sc = scenes.make_tiny(n_paths=512)
    lib = L.lib()

    def code(fn, *args):
        return fn(*args)

    # a context without a scene
    bare = L.create(C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert code(lib.pv_frame_begin, bare, None, None) == L.PV_ERR_STATE
    out = (C.c_uint32 * 4)()
    assert code(lib.pv_object_hierarchy_info, bare, 0, out) == L.PV_ERR_STATE
    L.destroy(bare)

    ctx = E.Context(sc)
    st = ctx.new_store()
    good = st.cstruct()
    # verification before any transforms; the queue before any verification
    assert code(lib.pv_verify_paths, ctx.ctx, C.byref(good), None) == L.PV_ERR_STATE
    assert code(lib.pv_build_queue, ctx.ctx, C.byref(good)) == L.PV_ERR_STATE
    # the distribution-map update without maps
    assert code(lib.pv_update_distribution, ctx.ctx, C.byref(good), 1, 1, None, None) == L.PV_ERR_STATE
    # malformed stores
    bad = []
    s1 = st.cstruct(); s1.stride = st.stride + 1; bad.append((s1, L.PV_ERR_ARG))          # stride not a multiple of 64
    s2 = st.cstruct(); s2.max_bounces = 0; bad.append((s2, L.PV_ERR_ARG))                  # no rows
    s3 = st.cstruct(); s3.d_info = None; bad.append((s3, L.PV_ERR_ARG))                    # a NULL array
    s4 = st.cstruct(); s4.d_pos_hit = st.pos_hit.data_ptr() + 4; bad.append((s4, L.PV_ERR_ARG))  # misaligned rows
    s5 = st.cstruct(); s5.n_paths = st.n_paths - 64; bad.append((s5, L.PV_ERR_ARG))       # light ranges do not add up
    s6 = st.cstruct(); s6.n_paths = ctx.max_paths + 64; s6.stride = ((ctx.max_paths + 64 + 63) // 64) * 64
    bad.append((s6, L.PV_ERR_CAPACITY))                                                    # beyond the reservation
    ctx.frame_begin(0)
    for sv, want in bad:
        assert code(lib.pv_verify_paths, ctx.ctx, C.byref(sv), None) == want, (sv.n_paths, sv.stride, want)
        assert code(lib.pv_retrace_paths, ctx.ctx, C.byref(sv), 0.01, 1, 1, None) == want
    # still usable: the same two frames as on a fresh context
    ref = E.Context(sc)
    sr = ref.new_store()
    for c, x in ((ctx, st), (ref, sr)):
        c.frame_begin(0)
        c.initial_trace(x, sc.seed, 0)
        c.frame_begin(1)
        c.verify(x)
        c.retrace(x, 0.01, sc.seed, 1)
    torch.cuda.synchronize()
    da, db = st.to_numpy(), sr.to_numpy()
    for k in da:
        assert np.array_equal(da[k].view(np.uint32), db[k].view(np.uint32)), k
    ctx.close()
    ref.close()
