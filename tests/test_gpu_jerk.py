"""Jerk-actuated step on the GPU vs the oracle (App. A, twelve discrete jerk
actions): state, heading and actuators bit-identical over rollouts that mix
jerk steps, direct steps and infraction checks; set_state clears the
actuators, fork copies them; the full workloads step bit-identically."""
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


def _jerk_actions(seed, n):
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 12, n)
    wild = rng.random(n) < 0.05                        # out-of-range indices coast
    k[wild] = rng.integers(12, 256, int(wild.sum()))
    return k.astype(np.uint8)


def _oracle_infractions(scenes, state, halted):
    out_s, out_h = [], []
    o = 0
    for sc in scenes:
        n = sc.n_agents
        st, hl, _ = oracle.infractions(state[o:o + n], sc.agent_dims, sc.road_xy, halted[o:o + n])
        out_s.append(st), out_h.append(hl)
        o += n
    return np.concatenate(out_s), np.concatenate(out_h)


def test_jerk_rollout_matches_oracle_with_halting_and_direct_steps():
    from paper_2606_19641_amd import gp
    scenes = [g.crowded_scene(91, n_agents=24, n_roads=40, radius=14.0),
              g.make_scene(0x5EED0003, 4, 33, 700), g.make_scene(0x5EED0002, 5, 70, 1200)]
    cam = g.camera_for(48)
    pal = g.mixed_palette()
    sim = gp.Sim(scenes, cam, pal)
    n = sim.n_agents
    dims = np.concatenate([s.agent_dims for s in scenes])
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    act = np.zeros((n, 4), np.float32)
    halted = np.zeros(n, np.uint8)
    assert np.array_equal(sim.get_actuators().cpu().numpy(), act)         # zero after create
    for k in range(40):
        if k % 10 == 7:                                  # a direct step leaves the actuators alone
            a = g.batch_actions(0xBEEF, k, scenes)
            sim.step(torch.from_numpy(a).cuda())
            state, _ = oracle.step(state, dims, a, 0.1, halted=halted)
        else:
            ks = _jerk_actions(k, n)
            print(f"jerk step {k}", flush=True)
            sim.step_jerk(torch.from_numpy(ks).cuda())
            state, _, act = oracle.step_jerk(state, dims, act, ks, 0.1, halted=halted)
        if k % 5 == 4:
            sim.check_infractions()
            state, halted = _oracle_infractions(scenes, state, halted)
        got_s = sim.get_state().cpu().numpy()
        got_a = sim.get_actuators().cpu().numpy()
        assert np.array_equal(got_s, state), k
        assert np.array_equal(got_a, act), k
    assert 0 < int(halted.sum()) < n
    assert np.any(act[:, 2] != 0) and np.any(act[:, 0] != 0)
    # the heading cosines the render uses come from the jerk step too
    rgb, _, _ = sim.render()
    torch.cuda.synchronize()
    got = rgb.cpu().numpy()
    o = 0
    for sc in scenes:
        cur = g.Scene(agent_state=state[o:o + sc.n_agents], agent_dims=sc.agent_dims,
                      agent_color=sc.agent_color, road_xy=sc.road_xy, road_color=sc.road_color)
        for a in range(0, sc.n_agents, 5):
            assert np.array_equal(got[o + a], oracle.render_scene_view(cur, cam, pal, a, 0).rgb), (o, a)
        o += sc.n_agents


def test_set_state_clears_and_fork_copies_the_actuators():
    from paper_2606_19641_amd import gp
    scenes = [g.make_scene(0x5EED0001, 2, 9, 120)]
    cam = g.camera_for(32)
    pal = g.mixed_palette()
    a = gp.Sim(scenes, cam, pal)
    b = gp.Sim(scenes, cam, pal)
    for k in range(6):
        a.step_jerk(torch.from_numpy(_jerk_actions(100 + k, a.n_agents)).cuda())
    b.fork_from(a)
    torch.cuda.synchronize()
    assert torch.equal(a.get_actuators(), b.get_actuators())
    assert bool((a.get_actuators() != 0).any())
    for k in range(4):
        ks = torch.from_numpy(_jerk_actions(200 + k, a.n_agents)).cuda()
        a.step_jerk(ks)
        b.step_jerk(ks)
    torch.cuda.synchronize()
    assert torch.equal(a.get_state(), b.get_state()) and torch.equal(a.get_actuators(), b.get_actuators())
    a.set_state(a.get_state().clone())
    torch.cuda.synchronize()
    assert not bool((a.get_actuators() != 0).any())
    with pytest.raises(ValueError):
        a.step_jerk(torch.zeros(a.n_agents, dtype=torch.int32, device="cuda"))


@pytest.mark.parametrize("name", ["uniform", "uneven"])
def test_full_workload_jerk_steps_bit_identical(name):
    from paper_2606_19641_amd import gp
    w = g.workload(name)
    sim = gp.Sim(w.scenes, w.camera, g.default_palette())
    n = sim.n_agents
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    state = np.concatenate([s.agent_state for s in w.scenes]).astype(np.float32)
    act = np.zeros((n, 4), np.float32)
    print(f"{name}: {n} agents", flush=True)
    for k in range(8):
        ks = _jerk_actions(300 + k, n)
        sim.step_jerk(torch.from_numpy(ks).cuda())
        state, _, act = oracle.step_jerk(state, dims, act, ks, 0.1)
    assert np.array_equal(sim.get_state().cpu().numpy(), state)
    assert np.array_equal(sim.get_actuators().cpu().numpy(), act)
