"""Directional-light shading on the GPU vs the oracle (App. A: one directional
light per world, a colour per instance): lit frames bit-identical to the
oracle's through the plain render, the step + render graph and the batched
serving launch, as the agents turn; switching the light off gives the flat
frames back; bad lights are refused."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LIGHT = (0.36, -0.48, 0.8, 0.2)       # unit direction, ambient


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp
    gp.lib()


def _scenes(uniform_roads):
    scenes = [g.crowded_scene(71, n_agents=18, n_roads=40, radius=14.0),
              g.crowded_scene(72, n_agents=9, n_roads=25, radius=10.0), g.make_scene(0x5EED0003, 6, 20, 600)]
    if uniform_roads:
        for s in scenes:
            s.road_color[:] = 1
    return scenes


def _check_views(rgb, scenes, state, cam, pal, light, stride=3):
    got = rgb.cpu().numpy()
    o = 0
    for sc in scenes:
        cur = g.Scene(agent_state=state[o:o + sc.n_agents], agent_dims=sc.agent_dims,
                      agent_color=sc.agent_color, road_xy=sc.road_xy, road_color=sc.road_color)
        for a in range(0, sc.n_agents, stride):
            for c in range(len(cam.cam_dirs)):
                v = (o + a) * len(cam.cam_dirs) + c
                ref = oracle.render_scene_view(cur, cam, pal, a, c, light=light).rgb
                assert np.array_equal(got[v], ref), (o, a, c)
        o += sc.n_agents


@pytest.mark.parametrize("uniform_roads", [True, False])
def test_lit_frames_match_oracle_as_agents_turn(uniform_roads):
    from paper_2606_19641_amd import gp
    scenes = _scenes(uniform_roads)
    cam = g.camera_for(56, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    sim = gp.Sim(scenes, cam, pal)
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    dims = np.concatenate([s.agent_dims for s in scenes])
    sim.set_light(LIGHT)
    for k in range(3):
        rgb, _, _ = sim.render()
        torch.cuda.synchronize()
        print(f"lit render step {k}", flush=True)
        _check_views(rgb, scenes, state, cam, pal, LIGHT)
        # depth / primid requested: same colours
        rgb2, d, p = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        assert torch.equal(rgb, rgb2)
        a = g.batch_actions(0xF00D, k, scenes)
        a[:, 1] = 0.4                                      # turn hard: the lit sides change
        sim.step(torch.from_numpy(a).cuda())
        state, _ = oracle.step(state, dims, a, 0.1)
    # light off: the flat frames (the rgb kernel again where the roads allow it)
    sim.set_light(None)
    rgb, _, _ = sim.render()
    torch.cuda.synchronize()
    _check_views(rgb, scenes, state, cam, pal, None, stride=4)


def test_graph_and_batched_launches_are_lit_too():
    from paper_2606_19641_amd import gp
    scenes = _scenes(True)
    cam = g.camera_for(48)
    pal = g.mixed_palette()
    a_sim, b_sim = gp.Sim(scenes, cam, pal), gp.Sim(scenes, cam, pal)
    act = torch.from_numpy(g.batch_actions(0xF00E, 0, scenes)).cuda()
    ra, rb = a_sim.new_rgb(), b_sim.new_rgb()
    a_sim.step_render_graph(act, ra)                      # captured unlit
    a_sim.set_light(LIGHT)                                # drops the graph
    b_sim.set_light(LIGHT)
    a_sim.step_render_graph(act, ra)
    b_sim.step(act)
    b_sim.step(act)
    b_sim.render(rgb=rb)
    torch.cuda.synchronize()
    assert torch.equal(a_sim.get_state(), b_sim.get_state())
    assert torch.equal(ra, rb)
    flat = b_sim.new_rgb()
    b_sim.set_light(None)
    b_sim.render(rgb=flat)
    torch.cuda.synchronize()
    assert not torch.equal(flat, rb)
    # batched serving launch, one sim lit and one not
    sims = [gp.Sim([s], cam, pal) for s in scenes[:2]]
    alone = [gp.Sim([s], cam, pal) for s in scenes[:2]]
    sims[0].set_light(LIGHT)
    alone[0].set_light(LIGHT)
    nb = gp.batch_required_bytes(sims)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    staging = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
    acts = [g.actions(3, 0, np.full(s.n_agents, i), np.arange(s.n_agents)) for i, s in enumerate(scenes[:2])]
    out_b = [x.new_rgb() for x in sims]
    gp.batch_step_render(sims, acts, out_b, ws, staging)
    torch.cuda.synchronize()
    for x, a, r in zip(alone, acts, out_b):
        x.step(torch.from_numpy(a).cuda())
        ref = x.new_rgb()
        x.render(rgb=ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, r)


def test_bad_lights_are_refused():
    from paper_2606_19641_amd import gp
    sim = gp.Sim(_scenes(True)[:1], g.camera_for(32), g.mixed_palette())
    for bad in [(1.0, 1.0, 0.0, 0.2), (0.0, 0.0, 1.0, 1.5), (0.0, 0.0, 1.0, -0.1), (math.nan, 0.0, 1.0, 0.2)]:
        with pytest.raises(gp.GpError):
            sim.set_light(bad)
