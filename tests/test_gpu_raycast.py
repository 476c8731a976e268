"""Ray-cast backend on the GPU vs the oracle's ray caster (App. A: the
renderer rasterises or ray-traces the same scene): rgb, depth and primitive
ids bit-identical on every view of small and crowded scenes with obstacles,
lights and the directional light, and on sampled views of the full uniform
workload, whose images agree with the raster's except at primitive edges."""
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


def _check(sim, scenes, cam, pal, light=None, stride=1, depth=True):
    rgb, d, p = sim.render_raycast(depth=depth, primid=depth)
    torch.cuda.synchronize()
    got = rgb.cpu().numpy()
    gd = d.cpu().numpy() if depth else None
    gpid = p.cpu().numpy() if depth else None
    o = 0
    for sc in scenes:
        for a in range(0, sc.n_agents, stride):
            for c in range(len(cam.cam_dirs)):
                v = (o + a) * len(cam.cam_dirs) + c
                ref = oracle.render_scene_view(sc, cam, pal, a, c, light=light, backend="raycast")
                assert np.array_equal(got[v], ref.rgb), (o, a, c)
                if depth:
                    assert np.array_equal(gpid[v], ref.primid), (o, a, c)
                    assert np.array_equal(gd[v].view(np.uint32), ref.depth.view(np.uint32)), (o, a, c)
        o += sc.n_agents
    return rgb


def _scenes():
    a = g.make_scene(0x5EED0003, 7, 14, 700, n_static=25, n_signals=30)
    b = g.crowded_scene(55, n_agents=12, n_roads=40, radius=12.0)
    c = g.workload("small").scenes[0]
    return [a, b, c]


def test_raycast_matches_oracle_on_every_view():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    cam = g.camera_for(56, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    pal[6:9] = g.default_palette()[6:9]
    sim = gp.Sim(scenes, cam, pal)
    print("raycast: unlit", flush=True)
    _check(sim, scenes, cam, pal)
    print("raycast: lit", flush=True)
    sim.set_light((0.6, 0.0, 0.8, 0.25))
    _check(sim, scenes, cam, pal, light=(0.6, 0.0, 0.8, 0.25), stride=2)
    # rgb only, and after a step (new poses, same kernel)
    sim.set_light(None)
    a = g.batch_actions(0xCAFE, 0, scenes)
    sim.step(torch.from_numpy(a).cuda())
    state, _ = oracle.step(np.concatenate([s.agent_state for s in scenes]), np.concatenate([s.agent_dims for s in scenes]), a, 0.1)
    o = 0
    moved = []
    for s in scenes:
        m = g.Scene(agent_state=state[o:o + s.n_agents], agent_dims=s.agent_dims, agent_color=s.agent_color,
                    road_xy=s.road_xy, road_color=s.road_color, static_xyp=s.static_xyp, static_dims=s.static_dims,
                    static_color=s.static_color, signal_xyzr=s.signal_xyzr, signal_color=s.signal_color)
        moved.append(m)
        o += s.n_agents
    _check(sim, moved, cam, pal, stride=3, depth=False)


def test_full_uniform_workload_sampled_and_close_to_the_raster():
    from paper_2606_19641_amd import gp
    w = g.workload("uniform")
    pal = g.default_palette()
    sim = gp.Sim(w.scenes, w.camera, pal)
    rc, d, p = sim.render_raycast(depth=True, primid=True)
    rr, _, pr = sim.render(depth=True, primid=True)
    torch.cuda.synchronize()
    got, gp_ = rc.cpu().numpy(), p.cpu().numpy()
    rng = np.random.default_rng(0)
    for v in rng.choice(sim.n_views, 12, replace=False):
        s, a = divmod(int(v), w.scenes[0].n_agents)
        ref = oracle.render_scene_view(w.scenes[s], w.camera, pal, a, 0, backend="raycast")
        assert np.array_equal(got[v], ref.rgb) and np.array_equal(gp_[v], ref.primid), v
    agree = float((p == pr).float().mean().item())
    print(f"raycast vs raster primitive agreement {agree:.5f}", flush=True)
    assert agree > 0.995


@pytest.mark.parametrize("shape", [(70, 42), (33, 61)])
def test_non_square_rig_and_roadless_scene_both_backends(shape):
    """The four-camera rig at a non-square size whose rows are not whole dwords,
    and a scene without roads holding obstacles and lights: the ray caster and
    the raster (its lights variant) each match the oracle on every view."""
    from paper_2606_19641_amd import gp
    W, H = shape
    cam = g.camera_for(W, H, cams=g.STUDENT_RIG)
    pal = g.mixed_palette()
    pal[6:9] = g.default_palette()[6:9]
    a = g.make_scene(0x5EED0002, 9, 7, 300, n_static=12, n_signals=15)
    src = g.make_scene(0x5EED0003, 10, 6, 200, n_static=10, n_signals=12)
    roadless = g.Scene(agent_state=src.agent_state, agent_dims=src.agent_dims, agent_color=src.agent_color,
                       road_xy=np.zeros((0, 4, 2), np.float32), road_color=np.zeros(0, np.uint8),
                       static_xyp=src.static_xyp, static_dims=src.static_dims, static_color=src.static_color,
                       signal_xyzr=src.signal_xyzr, signal_color=src.signal_color)
    scenes = [a, roadless]
    sim = gp.Sim(scenes, cam, pal)
    _check(sim, scenes, cam, pal)
    rgb, d, p = sim.render(depth=True, primid=True)
    torch.cuda.synchronize()
    got, gpid = rgb.cpu().numpy(), p.cpu().numpy()
    o = 0
    for sc in scenes:
        for e in range(sc.n_agents):
            for c in range(4):
                v = (o + e) * 4 + c
                ref = oracle.render_scene_view(sc, cam, pal, e, c)
                assert np.array_equal(got[v], ref.rgb) and np.array_equal(gpid[v], ref.primid), (o, e, c)
        o += sc.n_agents
