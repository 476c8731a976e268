"""Oracle pins for static obstacles (Sec. 3.1 / App. A: static objects are
cuboids like the vehicles, coloured per instance).

A static obstacle is a box that never moves and owns no view.  The pins
reduce it to the agent path, which the brute-force ray caster and the
closed-form raster tests pin: a scene with statics renders and checks exactly
like the same scene with the statics appended as extra (view-less) agents,
primitive indices included; plus closed-form collision cases."""
import numpy as np

import oracle
from paper_2606_19641_amd import scenegen as g


def _as_agents(sc):
    k = sc.n_static
    st = np.concatenate([sc.agent_state, np.column_stack([sc.static_xyp, np.zeros(k, np.float32)])])
    return g.Scene(agent_state=st.astype(np.float32), agent_dims=np.concatenate([sc.agent_dims, sc.static_dims]),
                   agent_color=np.concatenate([sc.agent_color, sc.static_color]), road_xy=sc.road_xy,
                   road_color=sc.road_color)


def _scene_with_statics():
    sc = g.make_scene(0x5EED0003, 2, 14, 500, n_static=40)
    sc.static_color[::3] = 4
    return sc


def test_statics_render_as_viewless_agents():
    sc = _scene_with_statics()
    ref = _as_agents(sc)
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    shown = set()
    for ego in range(sc.n_agents):
        for c in range(3):
            a = oracle.render_scene_view(sc, cam, pal, ego, c)
            b = oracle.render_scene_view(ref, cam, pal, ego, c)
            assert np.array_equal(a.rgb, b.rgb) and np.array_equal(a.primid, b.primid)
            assert np.array_equal(a.depth, b.depth)
            p = a.primid[(a.primid >= 6 * sc.n_agents) & (a.primid < 6 * (sc.n_agents + sc.n_static))]
            shown.update((p // 6).tolist())
            lit = oracle.render_scene_view(sc, cam, pal, ego, c, light=(0.6, 0.0, 0.8, 0.3))
            assert np.array_equal(lit.rgb, oracle.render_scene_view(ref, cam, pal, ego, c,
                                                                    light=(0.6, 0.0, 0.8, 0.3)).rgb)
    assert len(shown) >= 10                       # many obstacles are actually seen
    # roads are numbered after every box
    v = oracle.render_scene_view(sc, cam, pal, 0, 0)
    roads = v.primid[v.primid >= 6 * (sc.n_agents + sc.n_static)]
    assert roads.size and roads.max() < 6 * (sc.n_agents + sc.n_static) + sc.n_roads


def test_statics_collide_like_agents_and_are_never_flagged():
    sc = _scene_with_statics()
    rng = np.random.default_rng(9)
    state = sc.agent_state.copy()
    # move half the agents onto obstacles
    for i in range(0, sc.n_agents, 2):
        k = int(rng.integers(0, sc.n_static))
        state[i, :2] = sc.static_xyp[k, :2] + rng.uniform(-0.5, 0.5, 2)
    z = np.zeros(sc.n_agents, np.uint8)
    st, hl, fl = oracle.infractions(state, sc.agent_dims, sc.road_xy, z, sc.static_xyp, sc.static_dims)
    ref = _as_agents(sc)
    ref_state = ref.agent_state.copy()
    ref_state[:sc.n_agents] = state
    st2, hl2, fl2 = oracle.infractions(ref_state, ref.agent_dims, sc.road_xy, np.zeros(ref.n_agents, np.uint8))
    assert np.array_equal(fl & 1, fl2[:sc.n_agents] & 1)          # same collisions
    assert np.all(fl[::2] & 1)
    assert fl.shape == (sc.n_agents,)


def test_static_collision_closed_forms():
    road = np.array([[[-100, -10], [100, -10], [100, 10], [-100, 10]]], np.float32)
    dims = np.array([[4.0, 2.0, 1.5]], np.float32)
    sdims = np.array([[2.0, 1.0, 1.0]], np.float32)
    z = np.zeros(1, np.uint8)
    for dx, hit in ((2.9, True), (3.0, False), (3.1, False), (0.0, True)):
        st = np.array([[0.0, 0.0, 0.0, 5.0]], np.float32)
        sx = np.array([[dx, 0.0, 0.0]], np.float32)              # obstacle ahead, 1 m half length
        _, hl, fl = oracle.infractions(st, dims, road, z, sx, sdims)
        assert bool(fl[0] & 1) == hit, dx
        assert bool(hl[0]) == hit
    # no obstacles: as before
    _, _, fl = oracle.infractions(np.array([[0.0, 0.0, 0.0, 5.0]], np.float32), dims, road, z)
    assert fl[0] == 0


def test_generated_obstacles_sit_beside_the_lanes():
    sc = g.make_scene(0x5EED0002, 1, 8, 800, n_static=64)
    assert sc.n_static == 64 and sc.static_dims.min() > 0.4
    # on lane edges (the road's edge or the line between its two 3.5 m lanes):
    # away from intersections no centreline passes within 1 m
    q = sc.road_xy.astype(np.float64)
    back, front = 0.5 * (q[:, 0] + q[:, 3]), 0.5 * (q[:, 1] + q[:, 2])
    far = 0
    for p in sc.static_xyp[:, :2].astype(np.float64):
        d = front - back
        t = np.clip(((p - back) * d).sum(1) / (d * d).sum(1), 0, 1)
        dist = np.hypot(*(back + t[:, None] * d - p).T)
        far += dist.min() > 1.0
    assert far >= 0.75 * sc.n_static
