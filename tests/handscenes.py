"""Hand-built scenes for the oracle pins (plain data, no method arithmetic)."""
import numpy as np

import oracle as O

# open box [0,1]^3 in the triangle order of the tiny configuration:
# floor 0-1, ceiling 2-3, left 4-5, right 6-7, back 8-9
BOX = np.array([
    [[0, 0, 0], [1, 0, 0], [1, 0, 1]], [[0, 0, 0], [1, 0, 1], [0, 0, 1]],
    [[0, 1, 0], [0, 1, 1], [1, 1, 1]], [[0, 1, 0], [1, 1, 1], [1, 1, 0]],
    [[0, 0, 0], [0, 0, 1], [0, 1, 1]], [[0, 0, 0], [0, 1, 1], [0, 1, 0]],
    [[1, 0, 0], [1, 1, 0], [1, 1, 1]], [[1, 0, 0], [1, 1, 1], [1, 0, 1]],
    [[0, 0, 0], [0, 1, 0], [1, 1, 0]], [[0, 0, 0], [1, 1, 0], [1, 0, 0]],
], np.float32)


def cube_tris(center, side):
    c = np.asarray(center, np.float64)
    h = side / 2.0
    lo, hi = c - h, c + h
    x0, y0, z0 = lo
    x1, y1, z1 = hi
    P = lambda x, y, z: [x, y, z]
    q = [
        (P(x0, y0, z0), P(x1, y0, z0), P(x1, y0, z1), P(x0, y0, z1)),
        (P(x0, y1, z0), P(x0, y1, z1), P(x1, y1, z1), P(x1, y1, z0)),
        (P(x0, y0, z0), P(x0, y1, z0), P(x1, y1, z0), P(x1, y0, z0)),
        (P(x0, y0, z1), P(x1, y0, z1), P(x1, y1, z1), P(x0, y1, z1)),
        (P(x0, y0, z0), P(x0, y0, z1), P(x0, y1, z1), P(x0, y1, z0)),
        (P(x1, y0, z0), P(x1, y1, z0), P(x1, y1, z1), P(x1, y0, z1)),
    ]
    tris = []
    for a, b, c_, d in q:
        tris += [(a, b, c_), (a, c_, d)]
    return np.asarray(tris, np.float32)


# light 0.2 x 0.2 just under the ceiling, facing -y
LIGHT_DOWN = np.array([1, 0, 0, 0.5, 0, 0, -1, 0.999, 0, 1, 0, 0.5], np.float32)


def _blocker_materials(n_parts, albedo_box, albedo_blocker, blocker_albedos):
    """(material of each blocker, albedo table): every blocker takes material 1
    (albedo_blocker), or blocker i material 1 + i with blocker_albedos[i]."""
    if blocker_albedos is None:
        return [1] * n_parts, np.array([[albedo_box] * 3, [albedo_blocker] * 3], np.float32)
    assert len(blocker_albedos) == n_parts
    return [1 + i for i in range(n_parts)], np.array([[albedo_box] * 3] + [[a] * 3 for a in blocker_albedos],
                                                     np.float32)


def box_scene(blockers=(), moved=True, albedo_box=0.7, albedo_blocker=0.5, n_paths=1, light_moved=False,
              light_xf=LIGHT_DOWN, tri_blockers=(), light_half=(0.1, 0.1), blocker_albedos=None):
    """Box plus optional cube blockers and single-triangle blockers (each its
    own object, cubes first), as a FrameScene."""
    tris = [BOX]
    obj = [np.zeros(10, np.uint32)]
    mat = [np.zeros(10, np.uint32)]
    parts = [cube_tris(center, side) for center, side in blockers]
    parts += [np.asarray(t, np.float32).reshape(1, 3, 3) for t in tri_blockers]
    mats, albedo = _blocker_materials(len(parts), albedo_box, albedo_blocker, blocker_albedos)
    for i, t in enumerate(parts):
        tris.append(t)
        obj.append(np.full(t.shape[0], i + 1, np.uint32))
        mat.append(np.full(t.shape[0], mats[i], np.uint32))
    verts = np.concatenate(tris).reshape(-1, 9)
    return O.FrameScene(
        verts=verts, tri_obj=np.concatenate(obj), tri_mat=np.concatenate(mat),
        obj_moved=np.array([0] + [1 if moved else 0] * len(parts), np.uint8),
        albedo=albedo,
        light_xf=np.asarray(light_xf, np.float32)[None], light_half=np.array([light_half], np.float32),
        light_power=np.ones((1, 3), np.float32), light_moved=np.array([1 if light_moved else 0], np.uint8),
        light_base=np.array([0, n_paths], np.int64))


def store_from_paths(paths, B):
    """paths: list of (origin, [(pos, hit_tri), ...]) -> oracle Store with energies 1/N * 0.7^j."""
    N = len(paths)
    st = O.Store.empty(N, B)
    for p, (orig, photons) in enumerate(paths):
        st.origin[p] = orig
        e = np.float32(1.0) / np.float32(N)
        for r, (pos, hit) in enumerate(photons):
            st.pos[r, p] = pos
            st.hit[r, p] = hit
            st.energy[r, p] = e
            e = np.float32(e * np.float32(0.7))
        st.info[p] = O.info_make(0, len(photons), 0, 0, 0)
    return st


IDENTITY = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], np.float32)
PARKED = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 5], np.float32)   # frame-0 place of a moved blocker


def device_scene(blockers=(), moved=True, albedo_box=0.7, albedo_blocker=0.5, n_paths=1, light_moved=False,
                 light_xf=LIGHT_DOWN, tri_blockers=(), light_half=(0.1, 0.1), max_bounces=3, blocker_albedos=None):
    """The scene of box_scene(...) with the same arguments as a two-frame
    Scene for the device context: frame 1 holds the blockers at their world
    positions (identity transforms, so the world vertices are the given ones
    bit for bit); in frame 0 a moved blocker is parked elsewhere and a moved
    light holds LIGHT_DOWN.  O.frame_scene(scene, 1, 0) equals box_scene(...)."""
    from paper_2111_06906_amd import scenes
    parts = [cube_tris(center, side) for center, side in blockers]
    parts += [np.asarray(t, np.float32).reshape(1, 3, 3) for t in tri_blockers]
    D = len(parts)
    mats, albedo = _blocker_materials(D, albedo_box, albedo_blocker, blocker_albedos)
    xf1 = np.tile(IDENTITY, (D, 1))
    xf0 = np.tile(PARKED if moved else IDENTITY, (D, 1))
    lxf1 = np.asarray(light_xf, np.float32)[None]
    lxf0 = LIGHT_DOWN[None] if light_moved else lxf1
    if light_moved:
        assert not np.array_equal(lxf0, lxf1), "a moved light needs a transform other than LIGHT_DOWN"
    return scenes.Scene(
        name="hand", static_verts=BOX.copy(), static_mat=np.zeros(10, np.uint32),
        obj_local=parts, obj_mat=[np.full(p.shape[0], m, np.uint32) for p, m in zip(parts, mats)],
        obj_xforms=np.stack([xf0, xf1]).reshape(2, D, 12).astype(np.float32),
        albedo=albedo,
        light_half=np.array([light_half], np.float32), light_power=np.ones((1, 3), np.float32),
        light_xforms=np.stack([lxf0, lxf1]).astype(np.float32),
        light_paths=np.array([n_paths], np.int64), max_bounces=max_bounces, threshold=-1.0, seed=1)
