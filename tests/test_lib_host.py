"""The C-ABI library loads and exports every declared symbol; host-only
utilities and argument checks run without a GPU."""
import ctypes as C

import numpy as np
import pytest

import oracle as O
from paper_2111_06906_amd import _lib as L


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = L.declared_symbols()
    assert "pv_verify_paths" in declared and "pv_retrace_paths" in declared
    missing = [s for s in declared if not hasattr(lib, s)]
    assert missing == []


def test_store_bytes_reproduce_table1():
    # Table 1: 5 million paths of at most 7 photons, 32 B per photon
    MiB = 1024.0 * 1024.0
    n, B = 5_000_000, 7
    total = L.store_bytes(n, B)
    photon_map = n * B * 32
    assert round(photon_map / MiB) == 1068
    assert round(n * 4 / MiB, 2) == 19.07          # path information
    assert round(n * 12 / MiB, 2) == 57.22         # path origin position
    assert round((total - photon_map) / MiB, 2) == 76.29   # sub-total, reuse with objects
    assert round(total / MiB) == 1144               # total, reuse with objects


def test_info_word_round_trip_and_limits():
    rng = np.random.default_rng(0)
    for _ in range(500):
        cell = int(rng.integers(0, 1 << 22))
        nseg, start = int(rng.integers(0, 16)), int(rng.integers(0, 16))
        rep, reuse = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        w = L.info_pack(cell, nseg, start, rep, reuse)
        assert L.info_unpack(w) == (cell, nseg, start, rep, reuse)
        assert w == O.info_make(cell, nseg, start, rep, reuse)
    # 22 + 4 + 4 + 1 + 1 = 32 bits: the top bit is the reuse-light flag
    assert L.info_pack(0, 0, 0, 0, 1) == 1 << 31
    assert L.info_pack((1 << 22) - 1, 15, 15, 1, 1) == 0xFFFFFFFF


def test_argument_errors_without_device():
    lib = L.lib()
    # NULL context
    assert lib.pv_upload_scene(None, None) == L.PV_ERR_ARG
    assert lib.pv_verify_paths(None, None, None) == L.PV_ERR_ARG
    assert lib.pv_set_verify_mode(None, L.PV_VERIFY_BOXES) == L.PV_ERR_ARG
    out = C.c_void_p()
    code = lib.pv_create(C.byref(out), None)
    import torch
    if torch.cuda.is_available():
        assert code == L.PV_OK
        lib.pv_destroy(out)
    else:
        assert code == L.PV_ERR_HIP
        assert b"HIP" in lib.pv_last_error(None) or b"device" in lib.pv_last_error(None)


def test_every_entry_point_rejects_a_null_handle():
    # every call that takes a context or a batch returns PV_ERR_ARG for a NULL
    # one (nothing is enqueued, no device is touched); the out-parameter
    # constructors reject a NULL out pointer; the destructors accept NULL
    lib = L.lib()
    skip = {"pv_store_bytes", "pv_info_pack", "pv_info_unpack", "pv_version", "pv_last_error"}
    checked = []
    for name in sorted(L.declared_symbols()):
        if name in skip:
            continue
        fn = getattr(lib, name)
        args = []
        for t in fn.argtypes:
            if t in (C.c_uint32, C.c_int32, C.c_uint64):
                args.append(0)
            elif t is C.c_float:
                args.append(0.0)
            else:
                args.append(None)
        res = fn(*args)
        if fn.restype is None:
            continue  # pv_destroy / pv_batch_destroy: no crash is the check
        if name == "pv_distribution_cells":
            assert res == 0, name
        else:
            assert res == L.PV_ERR_ARG, (name, res)
        checked.append(name)
    assert {"pv_verify_paths", "pv_retrace_paths", "pv_compact_photons", "pv_batch_frames",
            "pv_compact_photons_noalloc", "pv_update_distribution"} <= set(checked)
    assert lib.pv_last_error(None) is not None


def test_declared_symbols_parse():
    names = L.declared_symbols()
    for n in ("pv_create", "pv_upload_scene", "pv_frame_begin", "pv_verify_paths", "pv_retrace_paths",
              "pv_compact_photons", "pv_energy_forward", "pv_energy_backward"):
        assert n in names


# traversal stack: 40 entries per lane hold a top-level tree of depth 7 plus
# a hierarchy of depth 31 (one entry per internal ancestor, the sentinel and
# the slot above the top)
MAX_DEPTH = 31


def _degenerate(kind, n, rng):
    """Triangle sets that unbalance a surface-area split."""
    if kind == "identical":
        t = np.tile(np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32), (n, 1, 1))
    elif kind == "exponential":
        # centres spread over many orders of magnitude along x
        x = np.exp(np.linspace(0, 40, n)).astype(np.float64)
        t = np.zeros((n, 3, 3))
        t[:, :, 0] = x[:, None]
        t[:, 1, 1] = 1e-3 * x
        t[:, 2, 2] = 1e-3 * x
    else:  # one big triangle among many tiny ones
        t = rng.uniform(0, 1e-3, (n, 3, 3))
        t[0] = [[0, 0, 0], [1e3, 0, 0], [0, 1e3, 0]]
    return np.ascontiguousarray(t, np.float32)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("dist", ["identical", "exponential", "one_big"])
def test_hierarchy_depth_bound_on_degenerate_inputs(kind, dist):
    info = L.hierarchy_info(_degenerate(dist, 20000, np.random.default_rng(3)), kind)
    assert info["valid"]
    assert info["depth"] <= MAX_DEPTH


@pytest.mark.parametrize("make,kind", [("tiny", 0), ("mid", 0), ("mid_obj", 1), ("paper", 0), ("paper_obj", 1)])
def test_hierarchy_invariants(make, kind):
    from paper_2111_06906_amd import scenes
    if make == "tiny":
        v = scenes.make_tiny().static_verts
    elif make.startswith("mid"):
        sc = scenes.make_mid(n_paths=10, frames=2)
        v = sc.static_verts if kind == 0 else sc.obj_local[0]
    else:
        sc = scenes.make_paper(n_paths=10, frames=2)
        v = sc.static_verts if kind == 0 else sc.obj_local[0]
    info = L.hierarchy_info(v, kind)
    n = v.shape[0]
    assert info["valid"]
    assert info["nodes"] == info["leaves"] - 1          # full binary tree
    assert info["depth"] <= MAX_DEPTH
    if kind == 1:
        assert info["leaves"] >= n // 2                  # leaves of at most 2 triangles


def test_bench_refuses_more_than_one_gpu():
    # the benchmark measures one GPU; another count is refused with a message
    # before anything touches a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""
