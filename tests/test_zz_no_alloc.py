"""The compaction entry point that allocates nothing (pv_compact_photons_noalloc,
fixed scratch of the library) against pv_compact_photons, through the C-ABI.

Two calls in a row on one device share the fixed scratch: a 1M-path store
(more counts than one scan tile: the multi-tile scan path) and then a smaller
one; each must equal the context-scratch compaction of the same store bit for
bit.  A store beyond the fixed limit is rejected before anything is enqueued.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2111_06906_amd import scenes

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_06906_amd import engine
    return engine


def _outputs(torch, cap):
    return (torch.full((cap, 3), -7.0, dtype=torch.float32, device="cuda"),
            torch.full((cap, 3), -7.0, dtype=torch.float32, device="cuda"),
            torch.full((1,), -1, dtype=torch.int32, device="cuda"))


def _both(E, L, torch, ctx, st, cap):
    """(count, positions, energies) of the context-scratch and the fixed-scratch
    compaction of the same store."""
    res = []
    for fn in (L.compact_photons, L.compact_photons_noalloc):
        pos, en, cnt = _outputs(torch, cap)
        fn(ctx.ctx, st.cstruct(), C.c_void_p(pos.data_ptr()), C.c_void_p(en.data_ptr()), cap,
           C.c_void_p(cnt.data_ptr()))
        torch.cuda.synchronize()
        res.append((int(cnt.item()), pos.cpu().numpy(), en.cpu().numpy()))
    return res


def _traced(E, sc, frames):
    ctx = E.Context(sc)
    st = ctx.new_store()
    ctx.frame_begin(0)
    ctx.initial_trace(st, sc.seed, 0)
    for f in range(1, frames):
        ctx.frame_begin(f)
        ctx.verify(st)
        ctx.retrace(st, 0.01, sc.seed, f)
    return ctx, st


def test_noalloc_compaction_matches_reserved_scratch_twice(E):
    import torch
    from paper_2111_06906_amd import _lib as L
    cases = [("mid, 1M paths, 7 rows", scenes.make_mid(n_paths=1_000_000 + 77, frames=3, threshold=0.01)),
             ("tiny, 16k paths, 3 rows", scenes.make_tiny(n_paths=16384 + 5, frames=2))]
    for label, sc in cases:
        log("no-alloc compaction: %s" % label)
        ctx, st = _traced(E, sc, sc.n_frames)
        nb = (st.n_paths + 255) // 256
        assert nb * st.B <= L.PV_NOALLOC_MAX_COUNTS
        full = st.n_paths * st.B
        for cap in (full, full // 3):
            (n0, p0, e0), (n1, p1, e1) = _both(E, L, torch, ctx, st, cap)
            info = st.info[:st.n_paths].cpu().numpy().view(np.uint32)
            assert n0 == n1 == int(((info >> 22) & 15).sum())
            # every written photon bit for bit, untouched slots alike
            assert np.array_equal(p0.view(np.uint32), p1.view(np.uint32))
            assert np.array_equal(e0.view(np.uint32), e1.view(np.uint32))
            log("  capacity %d: %d photons, outputs identical" % (cap, n1))
        ctx.close()


def test_noalloc_compaction_rejects_a_store_beyond_its_limit(E):
    import torch
    from paper_2111_06906_amd import _lib as L
    sc = scenes.make_tiny(n_paths=4096, frames=2)
    ctx = E.Context(sc)
    st = ctx.new_store()
    pos, en, cnt = _outputs(torch, 16)
    # a store descriptor one block beyond the limit (B = 1): rejected by the
    # size check, which runs before the store is bound or read
    big = L.PathStore((L.PV_NOALLOC_MAX_COUNTS + 1) * 256, 1, (L.PV_NOALLOC_MAX_COUNTS + 1) * 256,
                      st.pos_hit.data_ptr(), st.energy.data_ptr(), st.origin.data_ptr(), st.info.data_ptr())
    with pytest.raises(L.PVError) as e:
        L.compact_photons_noalloc(ctx.ctx, big, C.c_void_p(pos.data_ptr()), C.c_void_p(en.data_ptr()), 16,
                                  C.c_void_p(cnt.data_ptr()))
    assert e.value.code == L.PV_ERR_CAPACITY and "fixed compaction scratch" in str(e.value)
    torch.cuda.synchronize()
    assert int(cnt.item()) == -1  # nothing was enqueued
    ctx.close()
