"""Serving on the GPU: the batched step + render gives each sim exactly what
it gets alone, and a Poisson-driven serving run returns, for every request,
the images of a sequential replay of its rollout."""
import time

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g
from paper_2606_19641_amd import serve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp
    gp.lib()


def _scenes():
    scenes = [g.crowded_scene(61, n_agents=10, n_roads=60), g.crowded_scene(62, n_agents=5, n_roads=30),
              g.crowded_scene(63, n_agents=7, n_roads=40), g.make_scene(0x5EED0005, 3, 12, 600)]
    scenes[0].road_color[:] = 1          # one road colour: rgb kernel
    scenes[1].road_color[:] = 1
    return scenes                         # scene 2 has mixed road colours: general kernel


def _acts(step, scenes):
    return [g.actions(9, step, np.full(s.n_agents, i), np.arange(s.n_agents)) for i, s in enumerate(scenes)]


def test_batch_step_render_matches_each_sim_alone_and_oracle():
    from paper_2606_19641_amd import gp
    cam = g.camera_for(64)
    pal = g.mixed_palette()
    scenes = _scenes()
    batch = [gp.Sim([s], cam, pal) for s in scenes]
    alone = [gp.Sim([s], cam, pal) for s in scenes]
    rgb_b = [x.new_rgb() for x in batch]
    rgb_a = [x.new_rgb() for x in alone]
    nb = gp.batch_required_bytes(batch)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    staging = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
    host = [s.agent_state.copy() for s in scenes]
    for step in range(3):
        acts = _acts(step, scenes)
        gp.batch_step_render(batch, acts, rgb_b, ws, staging)
        torch.cuda.synchronize()             # staging may be rewritten after this
        for x, a, r in zip(alone, acts, rgb_a):
            x.step(torch.from_numpy(a).cuda())
            x.render(rgb=r)
        torch.cuda.synchronize()
        for k in range(len(scenes)):
            assert torch.equal(rgb_b[k], rgb_a[k]), (step, k)
            assert torch.equal(batch[k].get_state(), alone[k].get_state())
            host[k], _ = oracle.step(host[k], scenes[k].agent_dims, acts[k], 0.1)
        torch.cuda.synchronize()
    for k, s in enumerate(scenes):
        cur = g.Scene(agent_state=host[k], agent_dims=s.agent_dims, agent_color=s.agent_color,
                      road_xy=s.road_xy, road_color=s.road_color)
        got = rgb_b[k].cpu().numpy()
        for a in range(0, s.n_agents, 3):
            assert np.array_equal(got[a], oracle.render_scene_view(cur, cam, pal, a, 0).rgb), (k, a)


def test_batch_rejects_mixed_sizes_and_duplicates():
    from paper_2606_19641_amd import gp
    pal = g.mixed_palette()
    s = _scenes()[1]
    a = gp.Sim([s], g.camera_for(64), pal)
    b = gp.Sim([s], g.camera_for(32), pal)
    nb = gp.batch_required_bytes([a, a])
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    st = torch.empty(nb, dtype=torch.uint8, pin_memory=True)
    act = np.zeros((s.n_agents, 2), np.float32)
    with pytest.raises(gp.GpError):
        gp.batch_step_render([a, b], [act, act], [a.new_rgb(), b.new_rgb()], ws, st)
    with pytest.raises(gp.GpError):
        gp.batch_step_render([a, a], [act, act], [a.new_rgb(), a.new_rgb()], ws, st)
    with pytest.raises(gp.GpError):                      # workspace too small
        gp.batch_step_render([a], [act], [a.new_rgb()], ws[:256], st)


def test_serving_run_images_match_sequential_replay():
    from paper_2606_19641_amd import gp
    cam = g.camera_for(64)
    pal = g.mixed_palette()
    scenes = _scenes()
    ex = serve.GpuExecutor(cam, pal, budget_bytes=64 << 20, n_streams=2, max_batch_agents=1024,
                           max_batch_rollouts=8)
    frames = {}

    def on_complete(q, r):
        frames[q.rid] = r.handle["rgb"].cpu().numpy()

    srv = serve.Server(ex, budget_bytes=64 << 20, on_complete=on_complete)
    ids = [srv.open(s) for s in scenes]
    assert all(srv.admitted(i) for i in ids)
    arrivals = serve.poisson_arrivals(rate=3000.0, duration=0.03, seed=8)
    rng = np.random.default_rng(4)
    picks = rng.integers(0, len(ids), size=len(arrivals))
    sent = {}

    def actions_for(i, rid):
        s = scenes[rid]
        a = g.actions(31, i, np.full(s.n_agents, rid), np.arange(s.n_agents))
        sent.setdefault(rid, []).append(a)
        return a

    print(f"serving {len(arrivals)} requests over {len(ids)} rollouts", flush=True)
    serve.drive(srv, arrivals, lambda i: ids[picks[i]], actions_for, time.perf_counter)
    torch.cuda.synchronize()
    ok = sorted((q for q in srv.done if q.status == serve.OK), key=lambda q: q.rid)
    assert len(ok) == len(arrivals)
    by_roll = {}
    for q in ok:
        by_roll.setdefault(q.rollout, []).append(q)
    for rid, qs in by_roll.items():
        ref = gp.Sim([scenes[rid]], cam, pal)
        rgb = ref.new_rgb()
        for q, a in zip(sorted(qs, key=lambda q: q.t_arrival), sent[rid]):
            assert np.array_equal(q.actions, a)
            ref.step(torch.from_numpy(a).cuda())
            ref.render(rgb=rgb)
            assert np.array_equal(frames[q.rid], rgb.cpu().numpy()), (rid, q.rid)
    summ = srv.summary(0.0, 0.03)
    assert summ["p99_ms"] >= summ["p50_ms"] > 0



def test_burst_batches_overlap_on_device_and_match_alone():
    """A burst of requests (one per rollout, all at once) is launched as
    several batches on different streams whose work overlaps on the device
    (event spans), and every rollout's images equal its own sim stepped and
    rendered alone."""
    from paper_2606_19641_amd import gp
    cam = g.camera_for(128)
    pal = g.default_palette()
    scenes = [g.crowded_scene(900 + i, n_agents=96, n_roads=400, radius=40.0) for i in range(8)]
    ex = serve.GpuExecutor(cam, pal, budget_bytes=256 << 20, n_streams=4, max_batch_agents=1024,
                           max_batch_rollouts=2)
    ex.record_spans = True
    frames = {}

    def on_complete(q, r):
        frames[q.rollout] = r.handle["rgb"].cpu().numpy()

    srv = serve.Server(ex, budget_bytes=256 << 20, max_batch_rollouts=2, on_complete=on_complete)
    ids = [srv.open(s) for s in scenes]
    acts = {rid: g.actions(55, 0, np.full(scenes[k].n_agents, k), np.arange(scenes[k].n_agents))
            for k, rid in enumerate(ids)}
    for rid in ids:
        srv.submit(rid, acts[rid], now=0.0)
    launched = srv.pump(time.perf_counter())
    assert launched == 4                     # four slots, two rollouts each
    while not srv.idle():
        srv.pump(time.perf_counter())
    spans = sorted(ex.device_spans())
    print("device spans (ms):", [(round(a, 4), round(b, 4)) for a, b in spans], flush=True)
    overlaps = sum(1 for (a0, a1), (b0, b1) in zip(spans, spans[1:]) if b0 < a1)
    assert overlaps >= 1, spans
    for k, rid in enumerate(ids):
        ref = gp.Sim([scenes[k]], cam, pal)
        rgb = ref.new_rgb()
        ref.step(torch.from_numpy(acts[rid]).cuda())
        ref.render(rgb=rgb)
        assert np.array_equal(frames[rid], rgb.cpu().numpy()), rid
