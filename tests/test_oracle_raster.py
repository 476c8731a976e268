"""Pins of the oracle's raster against facts that do not come from it:
the float64 ray caster in bruteforce.py, exact tessellation coverage,
analytic projected areas, the road-plane closed form, and invariants."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g

from bruteforce import raycast


def _check_vs_bruteforce(scene, cam, pal, ego, k, max_amb_frac=0.06):
    rgb, depth, prim, amb = raycast(scene, cam, pal, ego, k)
    v = oracle.render_scene_view(scene, cam, pal, ego, k)
    ok = ~amb
    assert amb.mean() <= max_amb_frac, f"too many ambiguous pixels: {amb.mean():.3f}"
    assert np.array_equal(v.primid[ok], prim[ok]), np.argwhere((v.primid != prim) & ok)[:5]
    assert np.array_equal(v.rgb[ok], rgb[ok].astype(np.uint8))
    fin = ok & np.isfinite(depth)
    assert np.array_equal(np.isinf(v.depth[ok]), np.isinf(depth[ok]))
    rel = np.abs(v.depth[fin].astype(np.float64) - depth[fin]) / depth[fin]
    assert rel.size == 0 or rel.max() <= 1e-5, rel.max()
    return v


# ------------------------------------------------------------------ fill rule

def test_tessellation_covers_every_sample_exactly_once():
    """Triangulated jittered grid spanning past the screen: every sample is
    covered exactly once.  A third of the vertices sit exactly on sample
    coordinates so that E == 0 occurs on edges of every direction."""
    W = H = 24
    rng = np.random.default_rng(7)
    nx = ny = 7
    step = 256 * (W + 8) // (nx - 1)
    gx = -4 * 256 + step * np.arange(nx)
    gy = -4 * 256 + step * np.arange(ny)
    X = np.add.outer(np.zeros(ny, int), gx) + rng.integers(-300, 300, (ny, nx))
    Y = np.add.outer(gy, np.zeros(nx, int)) + rng.integers(-300, 300, (ny, nx))
    snap = rng.random((ny, nx)) < 0.35
    X = np.where(snap, (X // 256) * 256 + 128, X)
    Y = np.where(snap, (Y // 256) * 256 + 128, Y)
    # keep the outer ring on the grid lines so the union is the whole rectangle
    X[:, 0], X[:, -1], Y[0, :], Y[-1, :] = gx[0], gx[-1], gy[0], gy[-1]
    count = np.zeros((H, W), dtype=np.uint8)
    for r in range(ny - 1):
        for c in range(nx - 1):
            a, b, d, e = (r, c), (r, c + 1), (r + 1, c + 1), (r + 1, c)
            diag = rng.random() < 0.5
            tris = [(a, b, d), (a, d, e)] if diag else [(a, b, e), (b, d, e)]
            for t in tris:
                oracle.cover_tri([X[p] for p in t], [Y[p] for p in t], W, H, count)
    assert np.all(count == 1), np.argwhere(count != 1)[:10]


def test_fill_rule_axis_aligned_edges_through_samples():
    # square with corners on samples: top and left edges are in, bottom and right out
    W = H = 8
    x0, x1, y0, y1 = 256 * 2 + 128, 256 * 5 + 128, 256 * 1 + 128, 256 * 4 + 128
    c = np.zeros((H, W), np.uint8)
    oracle.cover_tri([x0, x1, x1], [y0, y0, y1], W, H, c)
    oracle.cover_tri([x0, x1, x0], [y0, y1, y1], W, H, c)
    expect = np.zeros((H, W), np.uint8)
    expect[1:4, 2:5] = 1
    assert np.array_equal(c, expect)


def test_zero_area_and_orientation():
    W = H = 8
    c = oracle.cover_tri([128, 1000, 1800], [128, 1000, 1800], W, H)      # collinear
    assert c.sum() == 0
    c1 = oracle.cover_tri([0, 2000, 0], [0, 0, 2000], W, H)
    c2 = oracle.cover_tri([0, 0, 2000], [0, 2000, 0], W, H)              # reversed winding
    assert np.array_equal(c1, c2) and c1.sum() > 0


# ------------------------------------------------------------ brute force

@pytest.mark.parametrize("ego", range(8))
def test_small_workload_vs_bruteforce(ego):
    w = g.workload("small")
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    for k in range(3):
        _check_vs_bruteforce(w.scenes[0], cam, g.default_palette(), ego, k)


@pytest.mark.parametrize("seed", range(8))
def test_crowded_vs_bruteforce(seed):
    s = g.crowded_scene(seed)
    cam = g.camera_for(48, cams=g.FRONT_AND_SIDES)
    for k in range(3):
        _check_vs_bruteforce(s, cam, g.mixed_palette(), 0, k)


def test_crowded_nonsquare_vs_bruteforce():
    s = g.crowded_scene(11)
    cam = g.Camera(width=56, height=34, focal_px=28.0, cam_dirs=g.FRONT_AND_SIDES)
    for k in range(3):
        _check_vs_bruteforce(s, cam, g.mixed_palette(), 0, k)


# ------------------------------------------------------------ analytic

def _two_box_scene(boxes, roads=None):
    """Ego at the origin heading +x plus the given (x, y, psi, L, W, H) boxes."""
    st = [[0.0, 0.0, 0.0, 0.0]] + [[b[0], b[1], b[2], 0.0] for b in boxes]
    dm = [[4.0, 2.0, 1.5]] + [[b[3], b[4], b[5]] for b in boxes]
    n = len(st)
    rx = np.zeros((0, 4, 2), np.float32) if roads is None else np.asarray(roads, np.float32)
    return g.Scene(agent_state=np.array(st, np.float32), agent_dims=np.array(dm, np.float32),
                   agent_color=np.array([2] + [3 + (i % 3) for i in range(n - 1)], np.uint8),
                   road_xy=rx, road_color=np.full(rx.shape[0], 1, np.uint8))


@pytest.mark.parametrize("D,L,W,H,res", [(12.0, 4.4, 2.1, 1.9, 64), (20.5, 5.0, 1.9, 1.75, 128),
                                         (7.25, 4.0, 2.2, 2.0, 96), (33.0, 4.6, 2.0, 1.8, 256)])
def test_axis_facing_box_projected_area(D, L, W, H, res):
    """A box straight ahead, taller than the camera: only its near face shows,
    the rectangle u in cx -+ f (W/2)/z0, v in [cy - f (H-1.6)/z0, cy + f 1.6/z0].
    The covered count is N_u * N_v with half-open sample intervals (left and
    top edges in, right and bottom out)."""
    cam = g.camera_for(res)
    f, cx, cy = res / 2.0, res / 2.0, res / 2.0
    L32, W32, H32 = (float(np.float32(v)) for v in (L, W, H))
    z0 = D - L32 / 2.0
    uL, uR = cx - f * (W32 / 2) / z0, cx + f * (W32 / 2) / z0
    vT, vB = cy - f * (H32 - 1.6) / z0, cy + f * 1.6 / z0
    samples = np.arange(res) + 0.5
    # the parameters keep every edge > 0.01 px away from a sample
    for e in (uL, uR, vT, vB):
        assert np.min(np.abs(samples - e)) > 0.01
    n_u = int(np.sum((samples >= uL) & (samples < uR)))
    n_v = int(np.sum((samples >= vT) & (samples < vB)))
    s = _two_box_scene([(D, 0.0, 0.0, L, W, H)])
    v = oracle.render_scene_view(s, cam, g.mixed_palette(), 0)
    covered = v.primid >= 0
    assert covered.sum() == n_u * n_v
    assert set(np.unique(v.primid[covered])) == {6 * 1 + 2}       # back face of box 1
    # continuous area within the perimeter bound
    area = (uR - uL) * (vB - vT)
    assert abs(covered.sum() - area) <= 2 * ((uR - uL) + (vB - vT)) + 4
    # depth of a face parallel to the image plane is z0 everywhere
    assert np.allclose(v.depth[covered], z0, rtol=1e-5, atol=0)


def test_low_box_shows_top_face_trapezoid():
    """Box lower than the camera: the near face plus the top face; each top-face
    row j covers the samples between the projected side edges at that row's depth."""
    res, D, L, W, H = 64, 9.0, 4.0, 2.0, 1.2
    cam = g.camera_for(res)
    s = _two_box_scene([(D, 0.0, 0.0, L, W, H)])
    v = oracle.render_scene_view(s, cam, g.mixed_palette(), 0)
    f = c = res / 2.0
    top = v.primid == 6 + 4
    near = v.primid == 6 + 2
    assert top.any() and near.any()
    for j in range(res):
        if not top[j].any():
            continue
        dv = j + 0.5 - c
        z = f * (1.6 - H) / dv               # depth of the top plane on this row
        assert D - L / 2 - 1e-3 <= z <= D + L / 2 + 1e-3
        half = f * (W / 2) / z
        expect = np.abs(np.arange(res) + 0.5 - c) < half
        got = top[j]
        border = np.abs(np.abs(np.arange(res) + 0.5 - c) - half) < 0.02
        assert np.array_equal(got[~border], expect[~border])
        assert np.allclose(v.depth[j][got], z, rtol=1e-5)


def test_road_plane_closed_form():
    """A 400 m square under the camera covers exactly the rows whose sample
    lies below the far line v = cy + 1.6 f / 100; depth = 1.6 f / (j + 0.5 - cy)."""
    for res in (64, 128, 512):
        cam = g.camera_for(res)
        quad = [[[-200, -200], [200, -200], [200, 200], [-200, 200]]]
        s = _two_box_scene([], roads=quad)
        v = oracle.render_scene_view(s, cam, g.default_palette(), 0)
        f = cy = res / 2.0
        v_far = cy + 1.6 * f / 100.0
        rows = (np.arange(res) + 0.5) >= v_far
        assert np.all(v.primid[rows] == 6) and np.all(v.primid[~rows] == -1)
        j = np.arange(res)[rows]
        expect = 1.6 * f / (j + 0.5 - cy)
        assert np.allclose(v.depth[rows], expect[:, None], rtol=1e-5, atol=0)
        assert np.all(v.rgb[rows] == (128, 128, 128)) and np.all(v.rgb[~rows] == 0)
    # at 128 x 128 the horizon rows 0..64 are background
    assert not rows[:65].any() if res == 128 else True


def test_guard_band_huge_quad():
    """A 200 km quad still renders as the road plane (the guard band keeps the
    snapped coordinates in range) and equals the 400 m result on screen."""
    cam = g.camera_for(128)
    big = [[[-1e5, -1e5], [1e5, -1e5], [1e5, 1e5], [-1e5, 1e5]]]
    small = [[[-200, -200], [200, -200], [200, 200], [-200, 200]]]
    vb = oracle.render_scene_view(_two_box_scene([], roads=big), cam, g.default_palette(), 0)
    vs = oracle.render_scene_view(_two_box_scene([], roads=small), cam, g.default_palette(), 0)
    assert np.array_equal(vb.primid, vs.primid)
    assert np.array_equal(vb.depth, vs.depth)


def test_empty_scene_and_everything_behind():
    cam = g.camera_for(32)
    s = _two_box_scene([])
    v = oracle.render_scene_view(s, cam, g.default_palette(), 0)
    assert np.all(v.rgb == 0) and np.all(np.isinf(v.depth)) and np.all(v.primid == -1)
    behind = _two_box_scene([(-10.0, 0.0, 0.3, 4.0, 2.0, 1.8), (-3.0, 2.0, 1.0, 4.0, 2.0, 1.5)],
                            roads=[[[-50, -2], [-1, -2], [-1, 2], [-50, 2]]])
    v = oracle.render_scene_view(behind, cam, g.default_palette(), 0)
    assert np.all(v.primid == -1) and np.all(np.isinf(v.depth))


def test_occlusion_nearer_box_wins():
    cam = g.camera_for(64)
    s = _two_box_scene([(10.0, 0.0, 0.0, 4.0, 2.0, 1.8), (18.0, 0.3, 0.0, 4.0, 3.0, 2.5)])
    v = oracle.render_scene_view(s, cam, g.mixed_palette(), 0)
    ids = set(np.unique(v.primid)) - {-1}
    assert 6 + 2 in ids and 12 + 2 in ids
    # the nearer box's face region shows box 1 only; box 2 is visible around it
    near = v.primid == 8
    alone = oracle.render_scene_view(_two_box_scene([(10.0, 0.0, 0.0, 4.0, 2.0, 1.8)]), cam,
                                     g.mixed_palette(), 0)
    assert np.array_equal(near, alone.primid == 8)
    assert np.array_equal(v.depth[near], alone.depth[near])


def test_permutation_invariance():
    s = g.crowded_scene(3)
    cam = g.camera_for(48)
    pal = g.default_palette()
    s.agent_color[:] = 2
    s.road_color[:] = 1
    base = oracle.render_scene_view(s, cam, pal, 0)
    rng = np.random.default_rng(0)
    pa = np.concatenate([[0], 1 + rng.permutation(s.n_agents - 1)])
    pr = rng.permutation(s.n_roads)
    t = g.Scene(agent_state=s.agent_state[pa], agent_dims=s.agent_dims[pa],
                agent_color=s.agent_color[pa], road_xy=s.road_xy[pr], road_color=s.road_color[pr])
    v = oracle.render_scene_view(t, cam, pal, 0)
    assert np.array_equal(v.rgb, base.rgb)
    assert np.array_equal(v.depth, base.depth)


def test_ego_box_excluded_and_others_present():
    s = g.crowded_scene(5)
    cam = g.camera_for(48, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    seen = set()
    for ego in range(6):
        for k in range(3):
            v = oracle.render_scene_view(s, cam, pal, ego, k)
            assert not np.any((v.primid >= 6 * ego) & (v.primid < 6 * ego + 6))
            seen |= set((v.primid[(v.primid >= 0) & (v.primid < 6 * s.n_agents)] // 6).tolist())
    assert len(seen) >= 5


def test_flat_box_on_road_ties_go_to_the_agent():
    """A box of zero height lying on a road strip has its top face in the road
    plane, so both fragments have identical 1/z: the reading 'agents above
    roads' decides, and the box colour shows."""
    cam = g.camera_for(64)
    road = [[[2, -4], [40, -4], [40, 4], [2, 4]]]
    s = _two_box_scene([(8.0, 0.0, 0.2, 8.0, 3.0, 0.0)], roads=road)
    v = oracle.render_scene_view(s, cam, g.mixed_palette(), 0)
    top = v.primid == 6 + 4
    assert top.sum() > 20
    assert np.all(v.rgb[top] == g.mixed_palette()[3])
    # the same pixels without the box are road at the same depth
    r = oracle.render_scene_view(_two_box_scene([], roads=road), cam, g.mixed_palette(), 0)
    assert np.all(r.primid[top] == 6) and np.array_equal(r.depth[top], v.depth[top])


@pytest.mark.parametrize("frac,covered", [(0.7, True), (0.3, False), (-0.3, False), (-0.7, False)])
def test_vertex_snap_rounds_to_nearest_subpixel(frac, covered):
    """The right edge of an axis-facing face projects to u = (S + frac)/256 px
    where S is a sample column's subpixel coordinate.  Rounding to the nearest
    1/256 px moves it to S + 1 (frac 0.7: sample in, right edges exclude only
    samples on them), to S (frac +-0.3: sample on the edge, excluded) or to
    S - 1 (frac -0.7: sample outside)."""
    res, z0 = 64, 10.0
    f = cx = res / 2.0
    i = 40
    S = 256 * i + 128
    u_right = (S + frac) / 256.0
    W = 2.0 * z0 * (u_right - cx) / f
    L = 4.0
    s = _two_box_scene([(z0 + L / 2, 0.0, 0.0, L, W, 1.9)])
    # the float32 box width must still put the edge within 0.1 subpixel of the target
    W32 = float(np.float32(W))
    got = 256 * (cx + f * (W32 / 2) / z0)
    assert abs(got - (S + frac)) < 0.1
    v = oracle.render_scene_view(s, g.camera_for(res), g.mixed_palette(), 0)
    row = res // 2
    assert bool(v.primid[row, i] >= 0) == covered
    assert v.primid[row, i - 1] >= 0


# ------------------------------------------------------------------ compositing

_FAR = 1.0e5     # a position no camera of these scenes sees (beyond the far plane)


def _only(scene, ego, box=None, road=None):
    """The scene with one primitive group kept: the ego, box `box` and road
    strip `road` where they are given; every other agent is moved far away
    and every other strip collapsed to a far point, so that the numbering of
    what is kept (6 box + face, 6 n_agents + strip) is unchanged."""
    st = scene.agent_state.copy()
    keep = {ego} | ({box} if box is not None else set())
    for a in range(scene.n_agents):
        if a not in keep:
            st[a, 0] = _FAR
            st[a, 1] = _FAR
    rx = np.full_like(scene.road_xy, _FAR)
    if road is not None:
        rx[road] = scene.road_xy[road]
    return g.Scene(agent_state=st, agent_dims=scene.agent_dims, agent_color=scene.agent_color,
                   road_xy=rx, road_color=scene.road_color)


@pytest.mark.parametrize("which", ["small", "crowded"])
def test_render_is_the_per_pixel_max_of_single_primitive_renders(which):
    """The depth test composes: every pixel's key in the full render is the
    largest of its keys over renders that hold one box (its faces) or one
    road strip each, and a pixel no single render covers is background.  A
    depth test that lets a later primitive win regardless of depth, a key
    that depends on what else was drawn, or coverage lost or added through
    other primitives breaks the identity."""
    if which == "small":
        w = g.workload("small")
        scene, cam, views = w.scenes[0], w.camera, [(0, 0), (5, 0)]
    else:
        scene, cam = g.crowded_scene(11, n_agents=12, n_roads=40), g.camera_for(48, cams=g.FRONT_AND_SIDES)
        views = [(0, 0), (3, 1), (7, 2)]
    pal = g.mixed_palette()
    for ego, k in views:
        full = oracle.render_scene_view(scene, cam, pal, ego, k)
        comp = np.zeros_like(full.key)
        drawn = 0
        for b in range(scene.n_agents):
            if b == ego:
                continue
            v = oracle.render_scene_view(_only(scene, ego, box=b), cam, pal, ego, k)
            drawn += int((v.key != 0).any())
            comp = np.maximum(comp, v.key)
        for r in range(scene.n_roads):
            v = oracle.render_scene_view(_only(scene, ego, road=r), cam, pal, ego, k)
            drawn += int((v.key != 0).any())
            comp = np.maximum(comp, v.key)
        assert drawn >= 3, "too few primitives in view for the check to mean anything"
        assert (full.key != 0).any() and (full.key == 0).any()
        assert np.array_equal(comp, full.key), np.argwhere(comp != full.key)[:5]
        empty = oracle.render_scene_view(_only(scene, ego), cam, pal, ego, k)
        assert not empty.key.any()
