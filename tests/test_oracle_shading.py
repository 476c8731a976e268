"""Oracle pins for directional-light shading (App. A: one directional light per
world, a colour per instance).

The expected colour of every pixel is rebuilt in float64 from the geometry:
the face the pixel shows (the primitive id, pinned by the raster tests), that
face's outward normal from math.cos / math.sin of the box heading, and the
shading law s = a + (1 - a) max(0, n . l) with level round(255 s) and channel
round(c q / 255).  binary32 rounding may move a level by one where 255 s lies
next to a half-integer, so a channel may differ by one there; everywhere else
it is exact."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g


def _normal(state, face):
    if face == 4:
        return (0.0, 0.0, 1.0)
    if face == 5:
        return (0.0, 0.0, -1.0)
    c, s = math.cos(float(state[2])), math.sin(float(state[2]))
    return [(c, s, 0.0), (-s, c, 0.0), (-c, -s, 0.0), (s, -c, 0.0)][face]


def _expected(scene, pal, prim, light):
    lx, ly, lz, a = (float(np.float32(x)) for x in light)
    H, W = prim.shape
    out = np.zeros((H, W, 3), np.int64)
    near = np.zeros((H, W), bool)
    n_a = scene.n_agents
    for j in range(H):
        for i in range(W):
            p = int(prim[j, i])
            if p < 0:
                out[j, i] = pal[0]
                continue
            if p < 6 * n_a:
                n = _normal(scene.agent_state[p // 6], p % 6)
                col = pal[scene.agent_color[p // 6]]
            else:
                n = (0.0, 0.0, 1.0)
                col = pal[scene.road_color[p - 6 * n_a]]
            s = a + (1 - a) * max(0.0, n[0] * lx + n[1] * ly + n[2] * lz)
            x = 255 * s + 0.5
            q = math.floor(x)
            near[j, i] = abs(x - round(x)) < 1e-4
            out[j, i] = [(int(c) * q + 127) // 255 for c in col]
    return out, near


def _scenes():
    return [g.crowded_scene(s, n_agents=20, n_roads=30, radius=15.0) for s in (5, 6)] + \
        [g.make_scene(0x5EED0002, 3, 16, 500)]


@pytest.mark.parametrize("light", [(0.3, -0.5, 0.8124, 0.25), (-0.8, 0.2, 0.5657, 0.0),
                                   (0.0, 0.0, 1.0, 0.4), (0.6, 0.8, 0.0, 0.1)])
def test_shaded_colours_follow_the_float64_lighting_law(light):
    cam = g.camera_for(48)
    pal = g.mixed_palette()
    n = math.sqrt(sum(x * x for x in light[:3]))
    light = tuple(x / n for x in light[:3]) + (light[3],)
    checked = exact = 0
    for sc in _scenes():
        for ego in range(0, sc.n_agents, 4):
            flat = oracle.render_scene_view(sc, cam, pal, ego)
            lit = oracle.render_scene_view(sc, cam, pal, ego, light=light)
            assert np.array_equal(flat.primid, lit.primid) and np.array_equal(flat.depth, lit.depth)
            exp, near = _expected(sc, pal, lit.primid, light)
            diff = np.abs(lit.rgb.astype(np.int64) - exp)
            assert np.all(diff[~near] == 0), (ego, light)
            assert np.all(diff <= 1)
            checked += diff.size
            exact += int((diff == 0).sum())
    assert exact / checked > 0.999


def test_overhead_light_closed_forms():
    sc = g.crowded_scene(7, n_agents=20, n_roads=30, radius=15.0)
    cam = g.camera_for(48)
    pal = g.mixed_palette()
    for ego in range(0, 20, 5):
        flat = oracle.render_scene_view(sc, cam, pal, ego)
        top = oracle.render_scene_view(sc, cam, pal, ego, light=(0.0, 0.0, 1.0, 0.0))
        below = oracle.render_scene_view(sc, cam, pal, ego, light=(0.0, 0.0, -1.0, 0.0))
        amb = oracle.render_scene_view(sc, cam, pal, ego, light=(0.0, 0.0, -1.0, 1.0))
        face = np.where(flat.primid >= 0, flat.primid % 6, -1)
        box = (flat.primid >= 0) & (flat.primid < 6 * sc.n_agents)
        road = flat.primid >= 6 * sc.n_agents
        bg = flat.primid < 0
        # light from straight above, no ambient: tops and roads keep their colour, sides go black
        assert np.array_equal(top.rgb[road], flat.rgb[road])
        assert np.array_equal(top.rgb[box & (face == 4)], flat.rgb[box & (face == 4)])
        assert not top.rgb[box & (face < 4)].any()
        # from below: everything lit goes black but bottoms (never visible above ground)
        assert not below.rgb[road].any() and not below.rgb[box & (face != 5)].any()
        # full ambient: the flat image; the background is never lit
        assert np.array_equal(amb.rgb, flat.rgb)
        assert np.array_equal(top.rgb[bg], flat.rgb[bg]) and np.array_equal(below.rgb[bg], flat.rgb[bg])
