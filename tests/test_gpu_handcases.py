"""The oracle's hand-built cases run through the C-ABI on the device.

Each case is the open unit box with hand-placed photon paths and blockers
(tests/handscenes.py): a blocker on a known segment, the three scenarios of
Figure 1, the box test's box-without-triangle case (Section 3.3: no ray),
moved area and point lights, and decisions that graze a triangle edge.  The
device verifies and re-traces the same store as the oracle; outside the
oracle's decision bands the results are compared element by element, and the
outcome each case is built for is asserted on the device's result as well.
"""
import numpy as np
import pytest

import oracle as O
from tests import handscenes as HS
from tests import harness as H


def log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def E():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2111_06906_amd import engine
    return engine


def _worked_path():
    # light origin -> floor -> right wall -> left wall
    return ([0.5, 0.999, 0.5], [([0.5, 0, 0.5], 0), ([1, 0.5, 0.5], 7), ([0, 0.5, 0.25], 4)])


def _path_off_diagonal():
    return ([0.52, 0.999, 0.47], [([0.52, 0, 0.47], 0), ([1, 0.5, 0.5], 7), ([0, 0.5, 0.25], 4)])


def _fig1_path():
    # light -> floor -> right wall -> back wall
    return ([0.5, 0.999, 0.5], [([0.5, 0.0, 0.5], 0), ([1.0, 0.4, 0.5], 7), ([0.6, 0.5, 0.0], 8)])


# a tilted triangle whose box segment 1 of the worked path crosses while its
# plane is crossed outside the triangle
TRI_NEAR_SEG1 = [[0.75, 0.28, 0.45], [0.85, 0.28, 0.45], [0.75, 0.32, 0.53]]
# the same for segment 0 of the off-diagonal path
TRI_NEAR_SEG0 = [[0.47, 0.5, 0.42], [0.57, 0.5, 0.42], [0.47, 0.6, 0.50]]


def _light_shift(dx, dy=0.0):
    xf = HS.LIGHT_DOWN.copy()
    xf[3] += np.float32(dx)
    xf[7] += np.float32(dy)
    return xf


def run_case(E, label, paths, T=None, boxes=False, energy_test=0, **scene_kw):
    """Verify (and re-trace with threshold T, unless None) the hand-built paths
    on the device and in the oracle; compare outside the decision bands.
    Returns (oracle store after verify, oracle store at the end, device store
    as numpy, oracle flags of verify and re-trace, device statistics)."""
    B = scene_kw.pop("max_bounces", 3)
    sc = HS.device_scene(n_paths=len(paths), max_bounces=B, **scene_kw)
    fs = O.frame_scene(sc, 1, 0)
    fs.verify_boxes = int(boxes)
    fs.energy_test = int(energy_test)
    ora = HS.store_from_paths(paths, B)
    ctx = E.Context(sc)
    ctx.set_verify_mode(boxes)
    ctx.set_energy_test(bool(energy_test))
    ctx.frame_begin(0)
    st = ctx.new_store()
    st.load_numpy(H.from_oracle(ora))
    ctx.frame_begin(1)
    stats = ctx.new_stats()
    ctx.verify(st, stats)
    gv = st.to_numpy()
    ambv, _ = O.verify(fs, ora)
    ok = ambv == 0
    assert np.array_equal(gv["info"][ok], ora.info[ok]), label
    assert np.abs(gv["origin"][ok] - ora.origin[ok]).max(initial=0) <= H.POS_TOL, label
    after_verify = ora.copy()
    ambr = np.zeros_like(ambv)
    if T is not None:
        ctx.retrace(st, T, 1, 1, stats)
        ambr, _ = O.retrace(fs, ora, T, 1, 1)
        ok &= ambr == 0
        H.compare_stores(st.to_numpy(), ora, ok, "hand: " + label, fs.verts, (~ok).sum())
    else:
        H.record("hand: " + label, compared=int(ok.sum()), excluded=int((~ok).sum()))
    out = st.to_numpy()
    s = ctx.stats_dict(stats)
    ctx.close()
    log("%s: gpu info %08x, oracle %08x, flags %x/%x, rays %d" % (
        label, out["info"][0], ora.info[0], ambv[0], ambr[0], s["rays_traced"]))
    return after_verify, ora, out, ambv, ambr, s


def _fields(info):
    f = O.info_fields(np.asarray(info, np.uint32))
    return tuple(int(f[k][0]) for k in ("replace", "start", "reuse", "nseg"))


@pytest.mark.gpu
def test_worked_case_blocker_on_second_segment(E):
    for T in (-1.0, 0.001):
        v, o, g, av, ar, s = run_case(E, "worked case T=%g" % T, [_worked_path()], T,
                                      blockers=[((0.76, 0.25, 0.5), 0.1)])
        assert av[0] == 0 and ar[0] == 0
        assert _fields(v.info) == (1, 1, 1, 3)
        assert s["paths_invalid"] == 1 and s["segments_examined"] == 2


@pytest.mark.gpu
@pytest.mark.parametrize("j", [0, 1, 2])
def test_blocker_on_known_segment_invalidates_exactly_it(E, j):
    orig, photons = _worked_path()
    pts = [np.array(orig, float)] + [np.array(p, float) for p, _ in photons]
    mid = 0.5 * (pts[j] + pts[j + 1]) + np.array([0.0031, 0.0017, -0.0043])
    for T in (-1.0, 0.01):
        v, o, g, av, ar, s = run_case(E, "blocker on segment %d T=%g" % (j, T), [(orig, photons)], T,
                                      blockers=[(tuple(mid), 0.04)])
        assert av[0] == 0
        assert _fields(v.info)[:2] == (1, j)
        assert s["segments_examined"] == j + 1


@pytest.mark.gpu
def test_unmoved_blocker_and_photon_on_moved_object(E):
    v, o, g, av, _, s = run_case(E, "unmoved blocker", [_worked_path()], 0.01,
                                 blockers=[((0.75, 0.25, 0.5), 0.1)], moved=False)
    assert _fields(g["info"])[0] == 0 and s["rays_traced"] == 0
    orig, photons = _worked_path()
    photons = list(photons)
    photons[1] = (photons[1][0], 10)   # second photon recorded on the moved cube (first object triangle)
    v, o, g, av, _, s = run_case(E, "photon on moved object", [(orig, photons)], None,
                                 blockers=[((0.2, 0.8, 0.8), 0.05)])
    assert _fields(g["info"])[:2] == (1, 1)


@pytest.mark.gpu
def test_figure1_last_segment_only_new_hit(E):
    v, o, g, av, ar, s = run_case(E, "figure 1: last segment", [_fig1_path()], 0.001,
                                  blockers=[((0.7, 0.47, 0.15), 0.1)], albedo_blocker=0.7)
    assert _fields(v.info)[:2] == (1, 2)
    assert s["rays_traced"] == 1                               # only the new end point
    assert np.array_equal(g["pos"][:2], v.pos[:2])
    assert 10 <= g["hit"][2, 0] < 22                           # lands on the blocker
    assert np.array_equal(g["energy"], v.energy)               # energies untouched


@pytest.mark.gpu
def test_figure1_first_segment_resampled_when_energy_differs(E):
    v, o, g, av, ar, s = run_case(E, "figure 1: resampled", [_fig1_path()], 0.001,
                                  blockers=[((0.503, 0.5, 0.498), 0.1)], albedo_blocker=0.3)
    assert _fields(v.info)[:2] == (1, 0)
    assert 10 <= g["hit"][0, 0] < 22
    assert not np.array_equal(g["pos"][1], v.pos[1])
    assert g["energy"][1, 0, 0] == np.float32(g["energy"][0, 0, 0] * np.float32(0.3))


@pytest.mark.gpu
def test_figure1_first_segment_kept_tail_when_energy_close(E):
    v, o, g, av, ar, s = run_case(E, "figure 1: kept tail", [_fig1_path()], 0.001,
                                  blockers=[((0.503, 0.3, 0.498), 0.1)], albedo_blocker=0.7)
    assert 10 <= g["hit"][0, 0] < 22
    assert g["hit"][1, 0] in (6, 7)
    assert np.linalg.norm(g["pos"][1, 0] - v.pos[1, 0]) < 1e-4
    assert np.array_equal(g["pos"][2], v.pos[2])
    assert np.array_equal(g["energy"], v.energy)


@pytest.mark.gpu
def test_walk_close_rehit_then_next_segment_blocked(E):
    # kept-tail case plus a moved cube across segment 2: the close re-hit is
    # written and segment 2 traced again, ending on the cube at (0.82, 0.445, 0.275)
    blockers = [((0.503, 0.3, 0.498), 0.1), ((0.8, 0.45, 0.25), 0.05)]
    v, o, g, av, ar, s = run_case(E, "close re-hit, next segment blocked", [_fig1_path()], 0.001,
                                  blockers=blockers, albedo_blocker=0.7)
    assert av[0] == 0 and ar[0] == 0 and s["rays_traced"] == 3
    assert 10 <= g["hit"][0, 0] < 22 and g["hit"][1, 0] == 7 and 22 <= g["hit"][2, 0] < 34
    assert np.linalg.norm(g["pos"][1, 0] - v.pos[1, 0]) < 1e-5
    assert np.abs(g["pos"][2, 0] - np.array([0.82, 0.445, 0.275])).max() < 1e-5
    assert np.array_equal(g["energy"], v.energy)


@pytest.mark.gpu
def test_walk_accepted_far_hit_continues_from_it(E):
    # kept-tail case plus a same-albedo cube across the new segment 1: the far
    # new hit is written and the walk goes on from it to the old third photon
    blockers = [((0.503, 0.3, 0.498), 0.1), ((0.75, 0.375, 0.5), 0.05)]
    v, o, g, av, ar, s = run_case(E, "accepted far hit, walk continues", [_fig1_path()], 0.001,
                                  blockers=blockers, albedo_blocker=0.7)
    assert av[0] == 0 and ar[0] == 0 and s["rays_traced"] == 3
    expect = np.array([[0.5, 0.35, 0.5], [0.725, 0.3725, 0.5], [0.6, 0.5, 0.0]])
    assert np.abs(g["pos"][:, 0] - expect).max() < 1e-5
    assert 10 <= g["hit"][0, 0] < 22 and 22 <= g["hit"][1, 0] < 34
    assert np.array_equal(g["energy"], v.energy)


@pytest.mark.gpu
def test_walk_energy_differs_after_an_accepted_segment(E):
    # the first cube accepted at segment 0, Equation 2 fails at segment 1 on
    # the darker second cube: its hit is kept and one bounce re-sampled from it
    blockers = [((0.503, 0.3, 0.498), 0.1), ((0.75, 0.375, 0.5), 0.05)]
    v, o, g, av, ar, s = run_case(E, "energy differs after an accepted segment", [_fig1_path()], 0.001,
                                  blockers=blockers, blocker_albedos=[0.7, 0.3])
    assert av[0] == 0 and ar[0] == 0 and s["rays_traced"] == 3
    assert np.abs(g["pos"][:2, 0] - np.array([[0.5, 0.35, 0.5], [0.725, 0.3725, 0.5]])).max() < 1e-5
    assert 22 <= g["hit"][1, 0] < 34
    assert np.all(g["energy"][2, 0] == np.float32(np.float32(0.7) * np.float32(0.3)))


@pytest.mark.gpu
def test_box_test_box_without_triangle_casts_no_ray(E):
    # triangle test: the path stays valid
    v, o, g, av, ar, s = run_case(E, "box without triangle, triangle test", [_worked_path()], 0.001,
                                  tri_blockers=[TRI_NEAR_SEG1])
    assert _fields(v.info)[0] == 0 and s["verify_box_hits"] == 1
    # box test: segment 1 is invalid; the error-based walk checks it against
    # the triangles first and traces nothing (Section 3.3)
    v, o, g, av, ar, s = run_case(E, "box without triangle, box test", [_worked_path()], 0.001, boxes=True,
                                  tri_blockers=[TRI_NEAR_SEG1])
    assert _fields(v.info)[:3] == (1, 1, 1) and av[0] == 0 and ar[0] == 0
    assert s["rays_traced"] == 0 and _fields(g["info"]) == (0, 0, 0, 3)
    # the naive method re-traces from segment 1 regardless: two rays
    v, o, g, av, ar, s = run_case(E, "box without triangle, box test, naive", [_worked_path()], -1.0,
                                  boxes=True, tri_blockers=[TRI_NEAR_SEG1])
    assert s["rays_traced"] == 2
    # through segment 0 with the light still: no ray either
    v, o, g, av, ar, s = run_case(E, "box without triangle on segment 0", [_path_off_diagonal()], 0.001,
                                  boxes=True, tri_blockers=[TRI_NEAR_SEG0])
    assert _fields(v.info)[:3] == (1, 0, 1) and s["rays_traced"] == 0 and _fields(g["info"])[0] == 0


@pytest.mark.gpu
def test_box_test_traces_a_segment_whose_origin_moved(E):
    # the light translates in its plane: segment 0's origin counts as moved and
    # is traced (one ray); the new hit coincides with the old photon
    v, o, g, av, ar, s = run_case(E, "box test, light moved", [_path_off_diagonal()], 0.001, boxes=True,
                                  tri_blockers=[TRI_NEAR_SEG0], light_moved=True, light_xf=_light_shift(0.01))
    assert _fields(v.info)[:3] == (1, 0, 1) and av[0] == 0 and ar[0] == 0
    assert s["rays_traced"] == 1 and _fields(g["info"])[0] == 0
    assert np.array_equal(g["hit"], v.hit)


@pytest.mark.gpu
def test_area_light_moves_out_of_reach_and_point_light_visibility(E):
    # area light shifted so far that the re-aimed origin leaves the rectangle:
    # the path is lost (replace, start 0, reuse-light 0) and re-sampled
    v, o, g, av, ar, s = run_case(E, "area light lost", [_worked_path()], 0.01,
                                  light_moved=True, light_xf=_light_shift(0.2))
    assert _fields(v.info)[:3] == (1, 0, 0) and s["paths_light_lost"] == 1
    # point light moved +0.05 in x with an unmoved occluder across the new
    # segment 0: the visibility segment is tested against every triangle
    occ = [((0.53, 0.5, 0.5), 0.1)]
    v, o, g, av, ar, s = run_case(E, "point light occluded", [_worked_path()], 0.01, blockers=occ, moved=False,
                                  light_moved=True, light_xf=_light_shift(0.05), light_half=(0.0, 0.0))
    assert _fields(v.info)[:3] == (1, 0, 1) and abs(v.origin[0, 0] - 0.55) < 1e-7
    v, o, g, av, ar, s = run_case(E, "point light clear", [_worked_path()], 0.01,
                                  light_moved=True, light_xf=_light_shift(0.05), light_half=(0.0, 0.0))
    assert _fields(v.info)[0] == 0
    # an area light moved the same way ignores the static occluder
    v, o, g, av, ar, s = run_case(E, "area light, static occluder", [_worked_path()], 0.01, blockers=occ,
                                  moved=False, light_moved=True, light_xf=_light_shift(0.05))
    assert _fields(v.info)[0] == 0


@pytest.mark.gpu
def test_grazing_edges(E):
    # through the cube's edges (centred exactly at (0.75, 0.25, 0.5)): the
    # oracle flags the decision; the device must take one of the two outcomes
    v, o, g, av, ar, s = run_case(E, "through cube edges", [_worked_path()], None,
                                  blockers=[((0.75, 0.25, 0.5), 0.1)])
    assert av[0] & O.AMB_EDGE
    assert _fields(g["info"])[:2] in ((1, 1), (0, 0))
    # one-segment paths 1e-7 below a cube's top face (through the side faces
    # next to their top edges), 1e-3 above it and 1e-3 below it
    paths = [([0.1, 0.6 - 1e-7, 0.5], [([0.9, 0.6 - 1e-7, 0.5], 0)]),
             ([0.1, 0.6 + 1e-3, 0.5], [([0.9, 0.6 + 1e-3, 0.5], 0)]),
             ([0.1, 0.6 - 1e-3, 0.5], [([0.9, 0.6 - 1e-3, 0.5], 0)])]
    v, o, g, av, ar, s = run_case(E, "grazing a top edge", paths, None, max_bounces=1,
                                  blockers=[((0.5, 0.5, 0.5), 0.2)])
    assert av[0] & O.AMB_EDGE and av[1] == 0 and av[2] == 0
    f = O.info_fields(g["info"])
    assert f["replace"][1] == 0 and f["replace"][2] == 1


def test_device_scene_equals_oracle_hand_scene():
    # the two-frame device scene seen by the oracle at frame 1 is the hand scene
    cases = [dict(blockers=[((0.76, 0.25, 0.5), 0.1)]), dict(tri_blockers=[TRI_NEAR_SEG1], moved=False),
             dict(blockers=[((0.53, 0.5, 0.5), 0.1)], moved=False, light_moved=True,
                  light_xf=_light_shift(0.05), light_half=(0.0, 0.0))]
    for kw in cases:
        a = HS.box_scene(**kw)
        b = O.frame_scene(HS.device_scene(**kw), 1, 0)
        for k in ("verts", "tri_obj", "tri_mat", "obj_moved", "albedo", "light_xf", "light_half",
                  "light_power", "light_moved", "light_base"):
            assert np.array_equal(np.asarray(getattr(a, k)), np.asarray(getattr(b, k))), k


@pytest.mark.gpu
def test_cosine_ratio_energy_test_closed_form(E):
    # first segment blocked by a slab 0.02 above the floor, albedo 0.72
    # against the floor's 0.7: with T = 0.5% the albedo test resamples the
    # tail, while the cosine ratio (0.968) keeps it and re-aims the second
    # photon from the new first one
    path = _fig1_path()
    blk = [((0.503, -0.03, 0.498), 0.1)]
    v, o, g, av, ar, s = run_case(E, "cosine ratio: kept", [path], 0.005, energy_test=1, blockers=blk,
                                  albedo_blocker=0.72)
    assert av[0] == 0 and ar[0] == 0
    assert 10 <= g["hit"][0, 0] < 22 and np.linalg.norm(g["pos"][1, 0] - np.array(path[1][1][0])) < 1e-5
    v, o, g, av, ar, s = run_case(E, "cosine ratio: albedo test resamples", [path], 0.005, energy_test=0,
                                  blockers=blk, albedo_blocker=0.72)
    assert np.linalg.norm(g["pos"][1, 0] - np.array(path[1][1][0])) > 1e-3
