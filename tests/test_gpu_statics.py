"""Static obstacles on the GPU vs the oracle (Sec. 3.1: static objects are
cuboids like the vehicles): rgb, depth and primitive ids bit-identical through
both kernels and under the light, unchanged by steps; collisions with
obstacles flagged as the oracle flags them; bad obstacles refused."""
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
    a = g.make_scene(0x5EED0003, 3, 20, 600, n_static=50)
    a.static_color[::4] = 3
    b = g.make_scene(0x5EED0002, 4, 9, 300, n_static=0)          # none in this one
    c = g.crowded_scene(33, n_agents=12, n_roads=30, radius=12.0)
    c.static_xyp, c.static_dims = g.place_statics(7, 0, c.road_xy, 25)
    c.static_color = np.full(25, 5, np.uint8)
    return [a, b, c]


def _cur(sc, st):
    return g.Scene(agent_state=st, agent_dims=sc.agent_dims, agent_color=sc.agent_color, road_xy=sc.road_xy,
                   road_color=sc.road_color, static_xyp=sc.static_xyp, static_dims=sc.static_dims,
                   static_color=sc.static_color)


def _compare(sim, scenes, state, cam, pal, light=None, depth=False, stride=2):
    rgb, d, p = sim.render(depth=depth, primid=depth)
    torch.cuda.synchronize()
    got = rgb.cpu().numpy()
    gd = d.cpu().numpy() if depth else None
    gpid = p.cpu().numpy() if depth else None
    o = 0
    for sc in scenes:
        cur = _cur(sc, state[o:o + sc.n_agents])
        for a in range(0, sc.n_agents, stride):
            for c in range(len(cam.cam_dirs)):
                v = (o + a) * len(cam.cam_dirs) + c
                ref = oracle.render_scene_view(cur, cam, pal, a, c, light=light)
                assert np.array_equal(got[v], ref.rgb), (o, a, c)
                if depth:
                    assert np.array_equal(gpid[v], ref.primid), (o, a, c)
                    fin = np.isfinite(ref.depth)
                    assert np.array_equal(np.isfinite(gd[v]), fin)
                    assert np.allclose(gd[v][fin], ref.depth[fin], rtol=1e-5, atol=0)
        o += sc.n_agents


@pytest.mark.parametrize("uniform_roads", [True, False])
def test_obstacles_render_like_the_oracle_and_stay_put(uniform_roads):
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    if uniform_roads:
        for s in scenes:
            s.road_color[:] = 1
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    sim = gp.Sim(scenes, cam, pal)
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    dims = np.concatenate([s.agent_dims for s in scenes])
    for k in range(3):
        print(f"statics step {k}", flush=True)
        _compare(sim, scenes, state, cam, pal)
        _compare(sim, scenes, state, cam, pal, depth=True, stride=5)
        a = g.batch_actions(0xABC, k, scenes)
        sim.step(torch.from_numpy(a).cuda())
        state, _ = oracle.step(state, dims, a, 0.1)
    assert sim.get_state().shape[0] == sum(s.n_agents for s in scenes)
    sim.set_light((0.0, 0.6, 0.8, 0.25))
    _compare(sim, scenes, state, cam, pal, light=(0.0, 0.6, 0.8, 0.25), stride=3)


def test_collisions_with_obstacles_match_oracle():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    sim = gp.Sim(scenes, g.camera_for(32), g.mixed_palette())
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    rng = np.random.default_rng(12)
    o = 0
    for sc in scenes:                     # park some agents on obstacles
        for i in range(0, sc.n_agents, 3):
            if sc.n_static:
                kk = int(rng.integers(0, sc.n_static))
                state[o + i, :2] = sc.static_xyp[kk, :2] + rng.uniform(-0.8, 0.8, 2)
        o += sc.n_agents
    sim.set_state(torch.from_numpy(state).cuda())
    flags = sim.check_infractions().cpu().numpy()
    ref = []
    o = 0
    for sc in scenes:
        _, hl, fl = oracle.scene_infractions(sc, state[o:o + sc.n_agents], np.zeros(sc.n_agents, np.uint8))
        ref.append(fl | (hl << 2))
        o += sc.n_agents
    ref = np.concatenate(ref)
    assert np.array_equal(flags, ref)
    assert (ref & 1).sum() >= 8


def test_bad_obstacles_are_refused():
    from paper_2606_19641_amd import gp
    sc = _scenes()[0]
    bad = _cur(sc, sc.agent_state)
    bad.static_xyp = sc.static_xyp.copy()
    bad.static_xyp[3, 0] = np.nan
    with pytest.raises(gp.GpError):
        gp.Sim([bad], g.camera_for(32), g.mixed_palette())
    bad.static_xyp = sc.static_xyp[:, :2].copy()
    with pytest.raises(ValueError):
        gp.Sim([bad], g.camera_for(32), g.mixed_palette())
    a = gp.Sim([sc], g.camera_for(32), g.mixed_palette())
    fewer = _cur(sc, sc.agent_state)
    fewer.static_xyp, fewer.static_dims, fewer.static_color = sc.static_xyp[:5], sc.static_dims[:5], sc.static_color[:5]
    b = gp.Sim([fewer], g.camera_for(32), g.mixed_palette())
    with pytest.raises(gp.GpError):
        b.fork_from(a)
