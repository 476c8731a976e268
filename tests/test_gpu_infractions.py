"""Infraction check and halting on the GPU vs the oracle (App. A: agents that
collide or leave the drivable area are halted in place), and fork."""
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


def _oracle_rollout_step(scenes, state, halted, act):
    """step every scene, then check it; returns (state, halted, flags)."""
    out_s, out_h, out_f = [], [], []
    o = 0
    for sc in scenes:
        n = sc.n_agents
        st, _ = oracle.step(state[o:o + n], sc.agent_dims, act[o:o + n], 0.1, halted=halted[o:o + n])
        st, hl, fl = oracle.infractions(st, sc.agent_dims, sc.road_xy, halted[o:o + n])
        out_s.append(st), out_h.append(hl), out_f.append(fl)
        o += n
    return np.concatenate(out_s), np.concatenate(out_h), np.concatenate(out_f)


def _scenes():
    crowded = g.crowded_scene(81, n_agents=30, n_roads=50, radius=12.0)   # many overlaps, strips
    gen = g.make_scene(0x5EED0003, 7, 40, 900)                            # lane-placed agents
    src = g.make_scene(0x5EED0001, 2, 3, 16)
    lone = g.Scene(agent_state=src.agent_state, agent_dims=src.agent_dims, agent_color=src.agent_color,
                   road_xy=np.zeros((0, 4, 2), np.float32), road_color=np.zeros(0, np.uint8))   # no road
    return [crowded, gen, lone]


def test_check_and_halting_match_oracle_over_a_rollout():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    cam = g.camera_for(48)
    pal = g.mixed_palette()
    sim = gp.Sim(scenes, cam, pal)
    state = np.concatenate([s.agent_state for s in scenes]).astype(np.float32)
    halted = np.zeros(sim.n_agents, np.uint8)
    st0, hl0, fl0 = [], [], []
    o = 0
    for sc in scenes:      # check the initial state first
        st, hl, fl = oracle.infractions(state[o:o + sc.n_agents], sc.agent_dims, sc.road_xy,
                                        halted[o:o + sc.n_agents])
        st0.append(st), hl0.append(hl), fl0.append(fl)
        o += sc.n_agents
    state, halted, flags = np.concatenate(st0), np.concatenate(hl0), np.concatenate(fl0)
    got = sim.check_infractions().cpu().numpy()
    assert np.array_equal(got, flags)
    assert np.array_equal(sim.get_state().cpu().numpy(), state)
    assert flags.any() and (flags & 1).any() and (flags & 2).any()
    n_halted = []
    for k in range(12):
        act = g.batch_actions(0xC0FFEE, k, scenes) * np.float32(3.0)      # aggressive, to make infractions
        sim.step(torch.from_numpy(act).cuda())
        gflags = sim.check_infractions().cpu().numpy()
        state, halted, flags = _oracle_rollout_step(scenes, state, halted, act)
        assert np.array_equal(gflags, flags), k
        assert np.array_equal(sim.get_state().cpu().numpy(), state), k
        n_halted.append(int(halted.sum()))
    assert n_halted[-1] > n_halted[0]                 # infractions happened along the way
    assert np.all(state[halted == 1, 3] == 0.0)
    # halted agents are still rendered (they stay observable)
    rgb, _, _ = sim.render()
    torch.cuda.synchronize()
    cur = []
    o = 0
    for sc in scenes:
        cur.append(g.Scene(agent_state=state[o:o + sc.n_agents], agent_dims=sc.agent_dims,
                           agent_color=sc.agent_color, road_xy=sc.road_xy, road_color=sc.road_color))
        o += sc.n_agents
    got_rgb = rgb.cpu().numpy()
    base = np.cumsum([0] + [s.n_agents for s in scenes])
    for si, sc in enumerate(cur):
        for a in range(0, sc.n_agents, 7):
            assert np.array_equal(got_rgb[base[si] + a], oracle.render_scene_view(sc, cam, pal, a, 0).rgb)


def test_set_state_clears_halted_and_fork_copies_it():
    from paper_2606_19641_amd import gp
    scenes = _scenes()
    cam = g.camera_for(32)
    pal = g.mixed_palette()
    a = gp.Sim(scenes, cam, pal)
    b = gp.Sim(scenes, cam, pal)
    flags = a.check_infractions()
    assert (flags.cpu().numpy() & 4).any()
    b.fork_from(a)
    for k in range(3):
        act = torch.from_numpy(g.batch_actions(5, k, scenes)).cuda()
        a.step(act)
        b.step(act)
    torch.cuda.synchronize()
    assert torch.equal(a.get_state(), b.get_state())
    ra, _, _ = a.render()
    rb, _, _ = b.render()
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    # a fresh episode: set_state clears halted, the agents move again
    init = torch.from_numpy(np.concatenate([s.agent_state for s in scenes]).astype(np.float32)).cuda()
    a.set_state(init)
    act = torch.from_numpy(np.tile(np.array([[3.0, 0.0]], np.float32), (a.n_agents, 1))).cuda()
    a.step(act)
    torch.cuda.synchronize()
    moved = (a.get_state()[:, 3] > 0).cpu().numpy()
    assert moved.all()
    with pytest.raises(gp.GpError):
        gp.Sim(scenes[:2], cam, pal).fork_from(a)
