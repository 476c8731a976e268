"""Oracle pins for the ray-cast backend (App. A: Gigapixel renders either by
rasterisation or by ray tracing, the same scene).

The binary32 caster is checked against the float64 brute-force caster
(tests/bruteforce.py, written from the geometry) on every pixel that caster
does not flag as ambiguous; static obstacles by reduction to view-less agents;
traffic lights against the raster's identical sphere test; and the whole
image against the raster, which renders the same scene definition."""
import sys
import os

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g

sys.path.insert(0, os.path.dirname(__file__))
import bruteforce  # noqa: E402


def _views():
    w = g.workload("small")
    crowded = g.crowded_scene(17, n_agents=16, n_roads=40, radius=12.0)
    return [(w.scenes[0], g.camera_for(64, cams=g.FRONT_AND_SIDES)), (crowded, g.camera_for(48, cams=g.FRONT_AND_SIDES))]


@pytest.mark.parametrize("k", range(2))
def test_raycast_matches_float64_caster(k):
    sc, cam = _views()[k]
    pal = g.mixed_palette()
    checked = 0
    for ego in range(0, sc.n_agents, 2):
        for c in range(3):
            v = oracle.render_scene_view(sc, cam, pal, ego, c, backend="raycast")
            _, depth, prim, amb = bruteforce.raycast(sc, cam, pal, ego, c)
            ok = ~amb
            assert np.array_equal(v.primid[ok], prim[ok]), (ego, c)
            hit = ok & (prim >= 0)
            assert np.allclose(v.depth[hit], depth[hit], rtol=1e-5, atol=0)
            assert np.all(np.isinf(v.depth[ok & (prim < 0)]))
            checked += int(ok.sum())
    assert checked > 0.9 * sc.n_agents // 2 * 3 * cam.width * cam.height


def test_raycast_agrees_with_the_raster():
    pal = g.mixed_palette()
    same = total = 0
    for sc, cam in _views():
        for ego in range(sc.n_agents):
            for c in range(3):
                a = oracle.render_scene_view(sc, cam, pal, ego, c)
                b = oracle.render_scene_view(sc, cam, pal, ego, c, backend="raycast")
                same += int((a.primid == b.primid).sum())
                total += a.primid.size
                lit_a = oracle.render_scene_view(sc, cam, pal, ego, c, light=(0.48, 0.0, 0.8773, 0.2))
                lit_b = oracle.render_scene_view(sc, cam, pal, ego, c, light=(0.48, 0.0, 0.8773, 0.2),
                                                 backend="raycast")
                m = a.primid == b.primid
                assert np.array_equal(lit_a.rgb[m], lit_b.rgb[m])     # one resolve for both backends
    assert same / total > 0.995


def test_statics_reduce_to_agents_and_lights_match_the_raster():
    sc = g.make_scene(0x5EED0003, 2, 12, 500, n_static=30, n_signals=30)
    as_agents = g.Scene(agent_state=np.concatenate([sc.agent_state, np.column_stack(
                            [sc.static_xyp, np.zeros(sc.n_static, np.float32)])]).astype(np.float32),
                        agent_dims=np.concatenate([sc.agent_dims, sc.static_dims]),
                        agent_color=np.concatenate([sc.agent_color, sc.static_color]), road_xy=sc.road_xy,
                        road_color=sc.road_color, signal_xyzr=sc.signal_xyzr, signal_color=sc.signal_color)
    lights_only = g.Scene(agent_state=sc.agent_state, agent_dims=sc.agent_dims, agent_color=sc.agent_color,
                          road_xy=np.zeros((0, 4, 2), np.float32), road_color=np.zeros(0, np.uint8),
                          signal_xyzr=sc.signal_xyzr, signal_color=sc.signal_color)
    lights_only.agent_state = sc.agent_state.copy()
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.default_palette()
    seen = 0
    for ego in range(sc.n_agents):
        for c in range(3):
            a = oracle.render_scene_view(sc, cam, pal, ego, c, backend="raycast")
            b = oracle.render_scene_view(as_agents, cam, pal, ego, c, backend="raycast")
            assert np.array_equal(a.primid, b.primid) and np.array_equal(a.rgb, b.rgb)
            # only the ego's own box is excluded, every other agent box is in the way of
            # the lights; with the agents pushed far away, rays see lights alone
            far = g.Scene(agent_state=lights_only.agent_state.copy(), agent_dims=sc.agent_dims,
                          agent_color=sc.agent_color, road_xy=lights_only.road_xy, road_color=lights_only.road_color,
                          signal_xyzr=sc.signal_xyzr, signal_color=sc.signal_color)
            far.agent_state[np.arange(sc.n_agents) != ego, 0] += 1e4
            r1 = oracle.render_scene_view(far, cam, pal, ego, c)
            r2 = oracle.render_scene_view(far, cam, pal, ego, c, backend="raycast")
            assert np.array_equal(r1.primid, r2.primid) and np.array_equal(r1.depth, r2.depth)
            seen += int((r1.primid >= 0).sum())
    assert seen > 100
