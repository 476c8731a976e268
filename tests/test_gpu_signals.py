"""Traffic lights on the GPU vs the oracle (Sec. 3.1: traffic lights are small
spheres): rgb, depth and primitive ids bit-identical, with boxes, obstacles,
roads and the directional light around them, as the agents move and the
lights change state; the batched launch and fork carry them; bad lights are
refused."""
import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp
    gp.lib()


def _scenes():
    a = g.make_scene(0x5EED0003, 5, 16, 600, n_static=20, n_signals=40)
    b = g.make_scene(0x5EED0002, 6, 9, 300)                        # no lights in this one
    c = g.crowded_scene(44, n_agents=10, n_roads=30, radius=12.0)
    rng = np.random.default_rng(5)                                  # big, close, cut by the near plane
    xy = rng.uniform(-12, 12, (30, 2))
    c.signal_xyzr = np.column_stack([xy, rng.uniform(0.2, 4.0, 30), rng.uniform(0.2, 3.0, 30)]).astype(np.float32)
    c.signal_color = rng.choice([6, 7, 8], 30).astype(np.uint8)
    return [a, b, c]


def _cur(sc, st, colors=None):
    return g.Scene(agent_state=st, agent_dims=sc.agent_dims, agent_color=sc.agent_color, road_xy=sc.road_xy,
                   road_color=sc.road_color, static_xyp=sc.static_xyp, static_dims=sc.static_dims,
                   static_color=sc.static_color, signal_xyzr=sc.signal_xyzr,
                   signal_color=sc.signal_color if colors is None else colors)


def _compare(rgb, d, p, scenes, state, colors, cam, pal, light=None, stride=2):
    got = rgb.cpu().numpy()
    gd = None if d is None else d.cpu().numpy()
    gp_ = None if p is None else p.cpu().numpy()
    o = go = 0
    for sc in scenes:
        cur = _cur(sc, state[o:o + sc.n_agents], colors[go:go + sc.n_signals])
        for a in range(0, sc.n_agents, stride):
            for c in range(len(cam.cam_dirs)):
                v = (o + a) * len(cam.cam_dirs) + c
                ref = oracle.render_scene_view(cur, cam, pal, a, c, light=light)
                assert np.array_equal(got[v], ref.rgb), (o, a, c)
                if gp_ is not None:
                    assert np.array_equal(gp_[v], ref.primid), (o, a, c)
                    fin = np.isfinite(ref.depth)
                    assert np.array_equal(np.isfinite(gd[v]), fin)
                    assert np.allclose(gd[v][fin], ref.depth[fin], rtol=1e-5, atol=0)
        o += sc.n_agents
        go += sc.n_signals


def test_lights_match_oracle_through_steps_state_changes_and_light():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    for s in scenes:
        s.road_color[:] = 1                      # would take the rgb kernel without lights
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    pal[6:9] = g.default_palette()[6:9]
    sim = gp.Sim(scenes, cam, pal)
    assert sim.n_signals == sum(s.n_signals for s in scenes)
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    dims = np.concatenate([s.agent_dims for s in scenes])
    colors = np.concatenate([s.signal_color for s in scenes])
    seen = 0
    for k in range(3):
        print(f"lights step {k}", flush=True)
        rgb, _, _ = sim.render()
        torch.cuda.synchronize()
        _compare(rgb, None, None, scenes, state, colors, cam, pal)
        rgb2, d, p = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        assert torch.equal(rgb, rgb2)
        _compare(rgb2, d, p, scenes, state, colors, cam, pal, stride=4)
        sig0 = np.concatenate([np.full(s.n_agents * 3, 6 * (s.n_agents + s.n_static) + s.n_roads)
                               for s in scenes])
        seen += int((p.cpu().numpy() >= sig0[:, None, None]).sum())
        a = g.batch_actions(0xD1CE, k, scenes)
        sim.step(torch.from_numpy(a).cuda())
        state, _ = oracle.step(state, dims, a, 0.1)
        colors = np.roll(colors, 1)                # the lights change state
        sim.set_signal_colors(torch.from_numpy(colors).cuda())
    assert seen > 200
    sim.set_light((0.0, -0.6, 0.8, 0.3))
    rgb, _, _ = sim.render()
    torch.cuda.synchronize()
    _compare(rgb, None, None, scenes, state, colors, cam, pal, light=(0.0, -0.6, 0.8, 0.3), stride=3)


def test_batched_launch_and_fork_carry_the_lights():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    cam = g.camera_for(48)
    pal = g.default_palette()
    sims = [gp.Sim([s], cam, pal) for s in scenes]
    alone = [gp.Sim([s], cam, pal) for s in scenes]
    new = torch.from_numpy(np.full(scenes[0].n_signals, 8, np.uint8)).cuda()
    sims[0].set_signal_colors(new)
    alone[0].set_signal_colors(new)
    nb = gp.batch_required_bytes(sims)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    staging = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
    acts = [g.actions(5, 0, np.full(s.n_agents, i), np.arange(s.n_agents)) for i, s in enumerate(scenes)]
    out = [x.new_rgb() for x in sims]
    gp.batch_step_render(sims, acts, out, ws, staging)
    torch.cuda.synchronize()
    for x, a, r in zip(alone, acts, out):
        x.step(torch.from_numpy(a).cuda())
        ref = x.new_rgb()
        x.render(rgb=ref)
        torch.cuda.synchronize()
        assert torch.equal(ref, r)
    # fork copies the light states
    f = gp.Sim([scenes[0]], cam, pal)
    f.fork_from(alone[0])
    ra, rf = alone[0].new_rgb(), f.new_rgb()
    alone[0].render(rgb=ra)
    f.render(rgb=rf)
    torch.cuda.synchronize()
    assert torch.equal(ra, rf)


def test_bad_lights_are_refused():
    from paper_2606_19641_amd import gp
    sc = _scenes()[0]
    for bad_r in (0.0, -1.0, np.nan, 1e4):
        b = _cur(sc, sc.agent_state)
        b.signal_xyzr = sc.signal_xyzr.copy()
        b.signal_xyzr[2, 3] = bad_r
        with pytest.raises(gp.GpError):
            gp.Sim([b], g.camera_for(32), g.default_palette())
    sim = gp.Sim([sc], g.camera_for(32), g.default_palette())
    with pytest.raises(ValueError):
        sim.set_signal_colors(torch.zeros(sc.n_signals + 1, dtype=torch.uint8, device="cuda"))


def test_graph_replays_with_lights_and_state_changes():
    """step + render captured once as a graph on a sim with lights (the
    general kernel's lights instances): replays follow light-state changes and
    equal the eager step + render."""
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    cam = g.camera_for(48)
    pal = g.default_palette()
    a, b = gp.Sim(scenes, cam, pal), gp.Sim(scenes, cam, pal)
    ra, rb = a.new_rgb(), b.new_rgb()
    act = torch.empty((a.n_agents, 2), dtype=torch.float32, device="cuda")
    colors = np.concatenate([s.signal_color for s in scenes])
    for k in range(4):
        act.copy_(torch.from_numpy(g.batch_actions(0xB0B, k, scenes)))
        colors = np.roll(colors, 3)
        c = torch.from_numpy(colors).cuda()
        a.set_signal_colors(c)
        b.set_signal_colors(c)
        a.step_render_graph(act, ra)
        b.step(act)
        b.render(rgb=rb)
        torch.cuda.synchronize()
        assert torch.equal(a.get_state(), b.get_state()), k
        assert torch.equal(ra, rb), k
