"""Every-view parity at the benchmark sizes: the images of whole workloads
(not samples) after graph-replayed steps of an episode equal the oracle's,
rgb bit for bit.  The oracle renders the views on the host's cores."""
import os

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

THREADS = max(1, min(16, os.cpu_count() or 1))


def _moved(scenes, state):
    out, o = [], 0
    for s in scenes:
        out.append(g.Scene(agent_state=state[o:o + s.n_agents].copy(), agent_dims=s.agent_dims,
                           agent_color=s.agent_color, road_xy=s.road_xy, road_color=s.road_color))
        o += s.n_agents
    return out


def _every_view(scenes, cam, pal, rgb, views=None, label=""):
    """Compare the listed (scene, agent, camera) views (default: all) of rgb
    [V][H][W][3] with the oracle."""
    n_cams = len(cam.cam_dirs)
    base = np.cumsum([0] + [s.n_agents for s in scenes])
    if views is None:
        views = [(si, a, k) for si, s in enumerate(scenes) for a in range(s.n_agents) for k in range(n_cams)]
    refs = oracle.render_views([(scenes[si], a, k) for si, a, k in views], cam, pal, threads=THREADS)
    bad = []
    for (si, a, k), ref in zip(views, refs):
        v = (base[si] + a) * n_cams + k
        if not np.array_equal(rgb[v], ref.rgb):
            bad.append(((si, a, k), int((rgb[v] != ref.rgb).any(-1).sum())))
    assert not bad, f"{label}: {len(bad)} of {len(views)} views differ, first {bad[:5]}"
    return len(views)


def _graph_steps(w, steps, check_at, views_fn=None):
    from paper_2606_19641_amd import gp
    pal = g.default_palette()
    sim = gp.Sim(w.scenes, w.camera, pal)
    rgb = sim.new_rgb()
    st = np.concatenate([s.agent_state for s in w.scenes])
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    acts = [g.batch_actions(w.seed, k, w.scenes) for k in range(steps)]
    dev = [torch.from_numpy(a).cuda() for a in acts]
    checked = 0
    for k in range(steps):
        sim.step_render_graph(dev[k], rgb)
        st, _ = oracle.step(st, dims, acts[k], 0.1)
        if k in check_at:
            torch.cuda.synchronize()
            got = sim.get_state().cpu().numpy()
            assert np.array_equal(got.view(np.uint32), st.view(np.uint32)), f"state after step {k}"
            moved = _moved(w.scenes, st)
            views = views_fn(moved) if views_fn else None
            if views is None:
                img = rgb.cpu().numpy()
            else:
                # gather the listed views on the device first
                n_cams = len(w.camera.cam_dirs)
                base = np.cumsum([0] + [s.n_agents for s in w.scenes])
                idx = [(base[si] + a) * n_cams + kk for si, a, kk in views]
                sub = rgb.index_select(0, torch.tensor(idx, device="cuda")).cpu().numpy()
                img = _Lookup({v: sub[n] for n, v in enumerate(idx)})
            checked += _every_view(moved, w.camera, pal, img, views, label=f"step {k}")
            print(f"step {k}: {checked} views checked", flush=True)
    return checked


class _Lookup:
    """rgb[v] for the gathered views only."""

    def __init__(self, d):
        self.d = d

    def __getitem__(self, v):
        return self.d[int(v)]


def test_uniform_every_view_at_three_episode_steps():
    """64 scenes x 32 agents, 2,000 strips, 128x128 (the benchmark
    workload): all 2,048 views after steps 1, 2 and 3 of the episode, the
    step + render replayed as one graph."""
    n = _graph_steps(g.workload("uniform"), 3, {0, 1, 2})
    assert n == 3 * 2048


def test_uneven_every_view_of_sixteen_scenes():
    """The first 16 scenes of the uneven workload (agents U{4..128}, strips
    U{500..8000}, three cameras at 128x128): every view after two graph
    steps."""
    w = g.workload("uneven", n_scenes=16)
    n = _graph_steps(w, 2, {1})
    assert n == 3 * sum(s.n_agents for s in w.scenes)


@pytest.mark.parametrize("res", [64, 128, 256, 512])
def test_sweep_64_views_per_resolution(res):
    """The resolution sweep's full workload (64 scenes x 64 agents, 4,000
    strips): 64 views spread over the scenes after two graph steps."""
    w = g.workload("sweep", resolution=res)
    rng = np.random.default_rng(res)
    picks = sorted({(int(rng.integers(64)), int(rng.integers(64)), 0) for _ in range(80)})[:64]
    n = _graph_steps(w, 2, {1}, views_fn=lambda moved: picks)
    assert n == len(picks) >= 60
