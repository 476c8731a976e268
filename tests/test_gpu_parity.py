"""HIP path vs the CPU oracle, through the C ABI, on the same seeded inputs.

Bar: agent state bit-identical after every step; rgb and primitive ids
bit-identical; depth within 1e-5 relative (bit-identical expected)."""
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


def _sim(scenes, cam, pal, **launch):
    from paper_2606_19641_amd import gp
    s = gp.Sim(scenes, cam, pal)
    if launch:
        s.set_launch(**launch)
    return s


def _views_of(scenes, cam):
    out = []
    for si, s in enumerate(scenes):
        for a in range(s.n_agents):
            for k in range(len(cam.cam_dirs)):
                out.append((si, a, k))
    return out


def _compare_views(scenes, cam, pal, rgb, depth, primid, picks, label=""):
    """Compare GPU images of the picked (scene, agent, cam) views with the oracle."""
    n_cams = len(cam.cam_dirs)
    base = np.cumsum([0] + [s.n_agents for s in scenes])
    for (si, a, k) in picks:
        v = (base[si] + a) * n_cams + k
        ref = oracle.render_scene_view(scenes[si], cam, pal, a, k)
        got_rgb = rgb[v]
        assert np.array_equal(got_rgb, ref.rgb), f"{label} rgb view {(si, a, k)}: " \
            f"{int((got_rgb != ref.rgb).any(-1).sum())} px differ"
        if primid is not None:
            assert np.array_equal(primid[v], ref.primid), f"{label} primid view {(si, a, k)}"
        if depth is not None:
            d, r = depth[v], ref.depth
            assert np.array_equal(np.isinf(d), np.isinf(r))
            fin = np.isfinite(r)
            rel = np.abs(d[fin].astype(np.float64) - r[fin]) / np.abs(r[fin])
            assert rel.size == 0 or rel.max() <= 1e-5, f"{label} depth view {(si, a, k)} {rel.max()}"


def _host_scene_state(scenes, state):
    out, o = [], 0
    for s in scenes:
        out.append(g.Scene(agent_state=state[o:o + s.n_agents].copy(), agent_dims=s.agent_dims,
                           agent_color=s.agent_color, road_xy=s.road_xy, road_color=s.road_color))
        o += s.n_agents
    return out


# ------------------------------------------------------------------ step

def test_step_bit_identical_each_step_small():
    w = g.workload("small")
    pal = g.default_palette()
    sim = _sim(w.scenes, w.camera, pal)
    st = np.concatenate([s.agent_state for s in w.scenes])
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    for step in range(w.steps):
        act = g.batch_actions(w.seed, step, w.scenes)
        sim.step(torch.from_numpy(act).cuda())
        got = sim.get_state().cpu().numpy()
        ref, _ = oracle.step(st, dims, act, 0.1)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"step {step}"
        st = got        # next step from the same pre-state on both sides


def test_step_extreme_actions_bit_identical():
    scenes = [g.crowded_scene(1)]
    cam = g.camera_for(32)
    sim = _sim(scenes, cam, g.default_palette())
    n = scenes[0].n_agents
    rng = np.random.default_rng(3)
    act = (rng.standard_normal((n, 2)) * np.array([20.0, 2.0])).astype(np.float32)
    act[0] = (np.nan, np.nan)
    act[1] = (np.inf, -np.inf)
    st = scenes[0].agent_state.copy()
    for _ in range(5):
        sim.step(torch.from_numpy(act).cuda())
        got = sim.get_state().cpu().numpy()
        st, _ = oracle.step(st, scenes[0].agent_dims, act, 0.1)
        assert np.array_equal(got.view(np.uint32), st.view(np.uint32))


# ------------------------------------------------------------------ render

def test_small_workload_every_step_every_view():
    """The small workload (1 scene, 8 agents, 200 quads, 64x64), 10 steps;
    all views after every step, rgb + depth + primitive id."""
    w = g.workload("small")
    pal = g.default_palette()
    sim = _sim(w.scenes, w.camera, pal)
    st = np.concatenate([s.agent_state for s in w.scenes])
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    for step in range(w.steps + 1):
        rgb, depth, prim = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        hs = _host_scene_state(w.scenes, st)
        _compare_views(hs, w.camera, pal, rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(),
                       _views_of(hs, w.camera), f"step {step}")
        if step < w.steps:
            act = g.batch_actions(w.seed, step, w.scenes)
            sim.step(torch.from_numpy(act).cuda())
            st, _ = oracle.step(st, dims, act, 0.1)


@pytest.mark.parametrize("seed", range(6))
def test_crowded_three_cameras(seed):
    scenes = [g.crowded_scene(seed), g.crowded_scene(100 + seed, n_agents=9, n_roads=3)]
    cam = g.camera_for(48, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    sim = _sim(scenes, cam, pal)
    rgb, depth, prim = sim.render(depth=True, primid=True)
    torch.cuda.synchronize()
    _compare_views(scenes, cam, pal, rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(),
                   _views_of(scenes, cam))


@pytest.mark.parametrize("seed", range(4))
def test_rgb_kernel_matches_oracle_and_general_kernel(seed):
    """rgb-only renders of uniform-road-colour scenes take the rgb kernel
    (road coverage bitmask); it must equal the oracle and the general kernel."""
    scenes = [g.crowded_scene(200 + seed), g.crowded_scene(300 + seed, n_agents=40, n_roads=120)]
    for s in scenes:
        s.road_color[:] = 1
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    sim = _sim(scenes, cam, pal)
    fast, _, _ = sim.render()
    gen, _, _ = sim.render(depth=True)
    torch.cuda.synchronize()
    assert torch.equal(fast, gen)
    _compare_views(scenes, cam, pal, fast.cpu().numpy(), None, None, _views_of(scenes, cam))


def test_mixed_road_colours_rgb_only_takes_general_kernel():
    scenes = [g.crowded_scene(7)]
    cam = g.camera_for(48, cams=g.FRONT_AND_SIDES)
    pal = g.mixed_palette()
    sim = _sim(scenes, cam, pal)
    rgb, _, _ = sim.render()
    torch.cuda.synchronize()
    _compare_views(scenes, cam, pal, rgb.cpu().numpy(), None, None, _views_of(scenes, cam))


def test_rgb_kernel_box_list_overflow():
    """128 boxes crowded around the camera overflow a 256-entry LDS list; the
    rgb kernel then redoes the boxes band by band."""
    s = g.crowded_scene(41, n_agents=128, n_roads=60, radius=18.0)
    s.road_color[:] = 1
    cam = g.camera_for(128)
    pal = g.mixed_palette()
    for lv in (dict(batch_tris=256, band_rows=16), dict(batch_tris=512, band_rows=8)):
        sim = _sim([s], cam, pal, **lv)
        rgb, _, _ = sim.render()
        torch.cuda.synchronize()
        _compare_views([s], cam, pal, rgb.cpu().numpy(), None, None, [(0, a, 0) for a in range(0, 128, 9)])


def test_nonsquare_and_ragged_width():
    """Width not a multiple of 4 takes the byte-store path; 210x126 is the
    paper's student resolution (App. B)."""
    scenes = [g.crowded_scene(21), g.workload("small").scenes[0]]
    pal = g.mixed_palette()
    for cam in (g.Camera(width=210, height=126, focal_px=105.0, cam_dirs=g.FRONT_AND_SIDES),
                g.Camera(width=37, height=23, focal_px=18.5, cam_dirs=g.FRONT),
                g.Camera(width=12, height=9, focal_px=2.5, cam_dirs=g.FRONT),       # far line near a sample row
                g.Camera(width=16, height=16, focal_px=8.0, z_far=30.0, cam_dirs=g.FRONT_AND_SIDES)):
        sim = _sim(scenes, cam, pal)
        rgb, depth, prim = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        picks = [(0, a, k) for a in range(0, scenes[0].n_agents, 4) for k in range(len(cam.cam_dirs))]
        picks += [(1, a, k) for a in range(scenes[1].n_agents) for k in range(len(cam.cam_dirs))]
        fast, _, _ = sim.render()
        torch.cuda.synchronize()
        assert torch.equal(fast, rgb)
        _compare_views(scenes, cam, pal, rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(),
                       picks)


def test_image_pointer_alignment_and_pattern_widths():
    """Key-free rows of the rgb kernel are written 16 pixels at a time with
    16-byte stores when the width allows it and the image is 16-byte aligned;
    a 4-byte aligned image address takes the dword path.  Both give the same
    bits."""
    scenes = [g.crowded_scene(33), g.crowded_scene(34, n_agents=6, n_roads=80)]
    for s in scenes:
        s.road_color[:] = 1
    pal = g.mixed_palette()
    for cam in (g.camera_for(48, cams=g.FRONT_AND_SIDES),
                g.Camera(width=80, height=20, focal_px=40.0, cam_dirs=g.FRONT),
                g.Camera(width=16, height=40, focal_px=8.0, cam_dirs=g.FRONT)):
        sim = _sim(scenes, cam, pal)
        ref, _, _ = sim.render()
        n = ref.numel()
        buf = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
        for off in (4, 8, 16):
            out = buf[off:off + n].view(ref.shape)
            sim.render(rgb=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (cam.width, off)
        from paper_2606_19641_amd import gp
        with pytest.raises(gp.GpError):          # the ABI asks for a 4-byte aligned image
            sim.render(rgb=buf[1:1 + n].view(ref.shape))
        picks = [(si, a, k) for si, s in enumerate(scenes) for a in range(0, s.n_agents, 5)
                 for k in range(len(cam.cam_dirs))]
        _compare_views(scenes, cam, pal, ref.cpu().numpy(), None, None, picks)


def test_student_rig_four_cameras_both_resolutions():
    """The student's rig (App. B): front, front-left, front-right and rear
    cameras at 210x126 and 434x252 (rows not a whole number of dwords)."""
    scenes = [g.crowded_scene(71, n_agents=16, n_roads=60), g.workload("student", n_scenes=1).scenes[0]]
    scenes[0].road_color[:] = 1
    pal = g.mixed_palette()
    for w, h in g.STUDENT_RESOLUTIONS:
        cam = g.Camera(width=w, height=h, focal_px=w / 2.0, cam_dirs=g.STUDENT_RIG)
        sim = _sim(scenes, cam, pal)
        fast, _, _ = sim.render()
        gen, depth, prim = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        assert torch.equal(fast, gen)
        picks = [(0, a, k) for a in range(0, 16, 5) for k in range(4)]
        picks += [(1, a, k) for a in range(0, scenes[1].n_agents, 11) for k in range(4)]
        _compare_views(scenes, cam, pal, fast.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(), picks,
                       f"{w}x{h}")


def test_degenerate_scenes():
    """A lone agent (empty view), no roads, a huge road quad (guard band),
    zero-area and clockwise road strips, a flat box, boxes behind the camera."""
    lone = g.Scene(agent_state=np.array([[0, 0, 0.3, 5]], np.float32),
                   agent_dims=np.array([[4.5, 2, 1.5]], np.float32),
                   agent_color=np.array([2], np.uint8), road_xy=np.zeros((0, 4, 2), np.float32),
                   road_color=np.zeros(0, np.uint8))
    roads = np.array([[[-1e5, -1e5], [1e5, -1e5], [1e5, 1e5], [-1e5, 1e5]],
                      [[5, 1], [9, 1], [9, 1], [5, 1]],             # zero area
                      [[4, -3], [4, 3], [30, 3], [30, -3]],         # clockwise
                      [[6, -5], [14, 5], [14, -5], [6, 5]],         # self-intersecting (bow tie)
                      [[0.2, -40], [0.3, -40], [0.3, 40], [0.2, 40]]], np.float32)   # crosses the near plane
    odd = g.Scene(agent_state=np.array([[0, 0, 0, 0], [8, 0, 0.2, 0], [-10, 0, 0, 0], [3, 0.5, 1.0, 0]], np.float32),
                  agent_dims=np.array([[4, 2, 1.5], [8, 3, 0.0], [4, 2, 1.8], [4.5, 2, 1.4]], np.float32),
                  agent_color=np.array([2, 3, 4, 5], np.uint8), road_xy=roads,
                  road_color=np.array([1, 5, 1, 1, 1], np.uint8))
    uniform = g.Scene(agent_state=odd.agent_state, agent_dims=odd.agent_dims, agent_color=odd.agent_color,
                      road_xy=roads, road_color=np.ones(len(roads), np.uint8))
    pal = g.mixed_palette()
    for scenes in ([lone, odd], [lone, uniform]):
        for res in (32, 64):
            cam = g.camera_for(res, cams=g.FRONT_AND_SIDES)
            sim = _sim(scenes, cam, pal)
            rgb, depth, prim = sim.render(depth=True, primid=True)
            fast, _, _ = sim.render()
            torch.cuda.synchronize()
            _compare_views(scenes, cam, pal, rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(),
                           _views_of(scenes, cam))
            assert torch.equal(fast, rgb)
            assert np.all(prim.cpu().numpy()[:3] == -1)        # the lone agent sees nothing


def test_overflow_fallback_path():
    """A view with more triangles than one LDS batch holds goes band by band
    with flushes; the image must not change."""
    scene = g.make_scene(77, 0, 24, 8000)
    cam = g.camera_for(128)
    pal = g.default_palette()
    sim = _sim([scene], cam, pal, batch_tris=256, band_rows=16)
    rgb, depth, prim = sim.render(depth=True, primid=True)
    torch.cuda.synchronize()
    picks = [(0, a, 0) for a in range(0, 24, 3)]
    _compare_views([scene], cam, pal, rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(), picks)


def _launch_variants():
    out = []
    for sched in (0, 1):
        for band_rows in (8, 16, 32, 64):
            for batch in (256, 512, 1024):
                for threads in (256, 512):
                    out.append(dict(sched=sched, band_rows=band_rows, batch_tris=batch,
                                    block_threads=threads, blocks_per_cu=2))
    return out


def test_every_launch_variant_gives_identical_bits():
    w = g.workload("uneven", n_scenes=6)
    pal = g.default_palette()
    sim = _sim(w.scenes, w.camera, pal)
    ref = None
    for lv in _launch_variants():
        try:
            sim.set_launch(**lv)
        except Exception as e:      # a variant beyond the device's LDS limit is refused up front
            assert "LDS" in str(e)
            continue
        rgb, depth, prim = sim.render(depth=True, primid=True)
        fast, _, _ = sim.render()
        torch.cuda.synchronize()
        cur = (rgb.cpu().numpy(), depth.cpu().numpy(), prim.cpu().numpy(), fast.cpu().numpy())
        if ref is None:
            ref = cur
            picks = [(s, a, k) for s in range(0, 6, 2) for a in (0, w.scenes[s].n_agents - 1) for k in range(3)]
            _compare_views(w.scenes, w.camera, pal, *cur[:3], picks)
            assert np.array_equal(cur[0], cur[3])
        else:
            for a, b in zip(ref, cur):
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), lv


def test_direct_and_queued_persistent_launch_at_the_resident_boundary():
    """With the persistent schedule, a render of no more views than resident
    workgroups gives each view a workgroup of its own (no queue); one view
    more takes the queue.  Both equal the per-scene launches bit for bit, and
    sampled views of the direct form equal the oracle."""
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cam = g.camera_for(32)
    pal = g.default_palette()
    for n_views in (n_cu, n_cu + 1):
        print(f"resident boundary: {n_views} views on {n_cu} CUs", flush=True)
        sizes = [32] * (n_views // 32) + ([n_views % 32] if n_views % 32 else [])
        scenes = [g.make_scene(0x5EED0B0, i, n, 300) for i, n in enumerate(sizes)]
        sim = _sim(scenes, cam, pal)
        assert sim.n_views == n_views
        out = {}
        for sched in (0, 1):
            sim.set_launch(sched=sched, blocks_per_cu=1)
            rgb, d, p = sim.render(depth=True, primid=True)
            fast, _, _ = sim.render()
            torch.cuda.synchronize()
            out[sched] = [x.cpu().numpy() for x in (rgb, d, p, fast)]
        for a, b in zip(out[0], out[1]):
            assert np.array_equal(a.view(np.uint8), b.view(np.uint8)), n_views
        assert np.array_equal(out[1][0], out[1][3])
        picks = [(0, 0, 0), (len(scenes) - 1, sizes[-1] - 1, 0)]
        _compare_views(scenes, cam, pal, *out[1][:3], picks, label=f"{n_views} views")


def test_uniform_full_size_bench_launch_sampled():
    """64 scenes x 32 agents, 2,000 quads, 128x128, in the launch the bench
    times (persistent, rgb only) for 3 steps; sampled views vs the oracle."""
    w = g.workload("uniform")
    pal = g.default_palette()
    sim = _sim(w.scenes, w.camera, pal)
    rgb = sim.new_rgb()
    st = np.concatenate([s.agent_state for s in w.scenes])
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    rng = np.random.default_rng(5)
    for step in range(3):
        act = g.batch_actions(w.seed, step, w.scenes)
        sim.step(torch.from_numpy(act).cuda())
        sim.render(rgb=rgb)
        st, _ = oracle.step(st, dims, act, 0.1)
    torch.cuda.synchronize()
    assert np.array_equal(sim.get_state().cpu().numpy().view(np.uint32), st.view(np.uint32))
    hs = _host_scene_state(w.scenes, st)
    picks = [(int(rng.integers(64)), int(rng.integers(32)), 0) for _ in range(12)] + [(63, 31, 0), (0, 0, 0)]
    _compare_views(hs, w.camera, pal, rgb.cpu().numpy(), None, None, picks)


def test_uneven_full_size_graph_sampled():
    """256 uneven scenes, 3 cameras, 128x128: step + render replayed as a
    hipGraph (the bench's batched form); sampled views vs the oracle, and the
    graph result equals the eager per-scene result."""
    w = g.workload("uneven")
    pal = g.default_palette()
    sim = _sim(w.scenes, w.camera, pal)
    sim2 = _sim(w.scenes, w.camera, pal, sched=0)
    rgb = sim.new_rgb()
    rgb2 = sim2.new_rgb()
    act_d = torch.empty((sim.n_agents, 2), dtype=torch.float32, device="cuda")
    st = np.concatenate([s.agent_state for s in w.scenes])
    dims = np.concatenate([s.agent_dims for s in w.scenes])
    for step in range(2):
        act = g.batch_actions(w.seed, step, w.scenes)
        act_d.copy_(torch.from_numpy(act))
        sim.step_render_graph(act_d, rgb)
        sim2.step(act_d)
        sim2.render(rgb=rgb2)
        torch.cuda.synchronize()
        assert torch.equal(rgb, rgb2), f"graph vs plain at step {step}"
        st, _ = oracle.step(st, dims, act, 0.1)
    hs = _host_scene_state(w.scenes, st)
    rng = np.random.default_rng(9)
    picks = []
    for _ in range(10):
        si = int(rng.integers(256))
        picks.append((si, int(rng.integers(w.scenes[si].n_agents)), int(rng.integers(3))))
    _compare_views(hs, w.camera, pal, rgb.cpu().numpy(), None, None, picks)
    # the launch the bench's tuner picks for this workload: the same bits
    tuned = sim.new_rgb()
    sim.set_launch(band_rows=16, batch_tris=512, block_threads=256, blocks_per_cu=3)
    sim.render(rgb=tuned)
    torch.cuda.synchronize()
    assert torch.equal(tuned, rgb)


def test_sweep_full_size_every_resolution_sampled():
    """The resolution sweep at full size (64 scenes x 64 agents, 4,000 quads
    each) at 64x64, 128x128, 256x256 and 512x512: step + render replayed as a
    hipGraph for 2 steps; sampled views (rgb, depth, primitive ids) vs the
    oracle, and the launches the bench's tuner picked on these shapes give the
    same bits.  Sampled views are gathered on the device before the copy."""
    tuned = {64: [dict(band_rows=64, batch_tris=256, blocks_per_cu=3)],
             128: [dict(band_rows=32, batch_tris=256, blocks_per_cu=3)],
             256: [dict(band_rows=16, batch_tris=256, blocks_per_cu=2), dict(band_rows=16, batch_tris=512, blocks_per_cu=2)],
             512: [dict(band_rows=8, batch_tris=256, blocks_per_cu=3)]}
    pal = g.default_palette()
    rng = np.random.default_rng(64)
    for res in (64, 128, 256, 512):
        print(f"sweep {res}x{res}", flush=True)
        w = g.workload("sweep", resolution=res)
        sim = _sim(w.scenes, w.camera, pal)
        rgb = sim.new_rgb()
        act_d = torch.empty((sim.n_agents, 2), dtype=torch.float32, device="cuda")
        st = np.concatenate([s.agent_state for s in w.scenes])
        dims = np.concatenate([s.agent_dims for s in w.scenes])
        for step in range(2):
            act = g.batch_actions(w.seed, step, w.scenes)
            act_d.copy_(torch.from_numpy(act))
            sim.step_render_graph(act_d, rgb)
            st, _ = oracle.step(st, dims, act, 0.1)
        torch.cuda.synchronize()
        assert np.array_equal(sim.get_state().cpu().numpy().view(np.uint32), st.view(np.uint32))
        rgb2, d, p = sim.render(depth=True, primid=True)
        torch.cuda.synchronize()
        assert torch.equal(rgb, rgb2), res
        hs = _host_scene_state(w.scenes, st)
        n = 6 if res == 512 else 10
        picks = [(int(rng.integers(64)), int(rng.integers(64)), 0) for _ in range(n)] + [(63, 63, 0), (0, 0, 0)]
        idx = torch.tensor([si * 64 + a for si, a, _ in picks], device="cuda")
        got_rgb, got_d, got_p = rgb.index_select(0, idx).cpu().numpy(), d.index_select(0, idx).cpu().numpy(), \
            p.index_select(0, idx).cpu().numpy()
        for k, (si, a, c) in enumerate(picks):
            ref = oracle.render_scene_view(hs[si], w.camera, pal, a, c)
            assert np.array_equal(got_rgb[k], ref.rgb), (res, si, a)
            assert np.array_equal(got_p[k], ref.primid), (res, si, a)
            fin = np.isfinite(ref.depth)
            assert np.array_equal(np.isfinite(got_d[k]), fin), (res, si, a)
            rel = np.abs(got_d[k][fin].astype(np.float64) - ref.depth[fin]) / np.abs(ref.depth[fin])
            assert rel.size == 0 or rel.max() <= 1e-5, (res, si, a, rel.max())
        del rgb2, d, p
        for lv in tuned[res]:
            sim.set_launch(block_threads=256, **lv)
            other = sim.new_rgb()
            sim.render(rgb=other)
            torch.cuda.synchronize()
            assert torch.equal(other, rgb), (res, lv)
        del sim, rgb, other
        torch.cuda.empty_cache()


def test_state_save_restore_reproduces_images():
    w = g.workload("uniform", n_scenes=3)
    pal = g.default_palette()
    a = _sim(w.scenes, w.camera, pal)
    acts = [torch.from_numpy(g.batch_actions(w.seed, k, w.scenes)).cuda() for k in range(10)]
    for k in range(5):
        a.step(acts[k])
    saved = a.get_state().clone()
    for k in range(5, 10):
        a.step(acts[k])
    ra, _, _ = a.render()
    b = _sim(w.scenes, w.camera, pal)
    b.set_state(saved)
    for k in range(5, 10):
        b.step(acts[k])
    rb, _, _ = b.render()
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    assert torch.equal(a.get_state(), b.get_state())


def test_bad_arguments_rejected():
    from paper_2606_19641_amd import gp
    w = g.workload("small")
    sim = _sim(w.scenes, w.camera, g.default_palette())
    with pytest.raises(gp.GpError):
        sim.set_launch(band_rows=12)
    with pytest.raises(gp.GpError):
        sim.set_launch(batch_tris=100)
    with pytest.raises(ValueError):
        sim.step(torch.zeros((3, 2), device="cuda"))
    bad = g.Camera(width=0, height=64, focal_px=32.0)
    with pytest.raises(gp.GpError):
        gp.Sim(w.scenes, bad, g.default_palette())


def test_graph_takes_each_steps_own_action_buffer():
    """step_render_graph with a different action tensor at every step (the
    graph's step node is updated in place, no copy, no re-capture) equals the
    eager step + render on the same actions, and the state equals the
    oracle's; an image-pointer change in between rebuilds the graph."""
    w = g.workload("uniform")
    scenes = w.scenes[:4]
    pal = g.default_palette()
    sim = _sim(scenes, w.camera, pal)
    ref = _sim(scenes, w.camera, pal, sched=0)
    rgb_a, rgb_b, rgb_r = sim.new_rgb(), sim.new_rgb(), ref.new_rgb()
    acts = [torch.from_numpy(g.batch_actions(w.seed, k, scenes)).cuda() for k in range(6)]
    st = np.concatenate([s.agent_state for s in scenes])
    dims = np.concatenate([s.agent_dims for s in scenes])
    for k, a in enumerate(acts):
        out = rgb_a if k != 3 else rgb_b
        sim.step_render_graph(a, out)
        ref.step(a)
        ref.render(rgb=rgb_r)
        torch.cuda.synchronize()
        assert torch.equal(out, rgb_r), f"graph vs eager at step {k}"
        st, _ = oracle.step(st, dims, a.cpu().numpy(), 0.1)
        assert np.array_equal(sim.get_state().cpu().numpy().view(np.uint32), st.view(np.uint32)), k


_RASTERS = [
    dict(sched=1, raster=1, view_waves=1, blocks_per_cu=8),
    dict(sched=1, raster=1, view_waves=2, blocks_per_cu=8),
    dict(sched=1, raster=1, view_waves=4, blocks_per_cu=4),
    dict(sched=0, raster=1, view_waves=2, blocks_per_cu=8),
    dict(sched=1, raster=2, road_wgs_per_cu=1),
    dict(sched=1, raster=2, road_wgs_per_cu=8),
    dict(sched=1, raster=2, road_wgs_per_cu=16),
    dict(sched=0, raster=2, road_wgs_per_cu=8),
    dict(sched=1, raster=0, blocks_per_cu=3),
]


def _raster_case(case):
    pal = g.default_palette()
    if case == "crowded":
        # dense boxes all around: views whose box lists exceed the chip-wide
        # raster's capacity take its per-item set-up path
        scenes = [g.crowded_scene(700 + k, n_agents=64, n_roads=300, radius=18.0) for k in range(3)]
        return scenes, g.camera_for(128, cams=g.FRONT_AND_SIDES), pal
    if case == "uneven":
        w = g.workload("uneven", n_scenes=8)
        return w.scenes, w.camera, pal
    if case == "w208":
        # rows that are not whole 64-sample words, 13 groups of 16 per row
        w = g.workload("uneven", n_scenes=4)
        return w.scenes, g.camera_for(208, 120, cams=g.FRONT_AND_SIDES), pal
    if case == "roads":
        # dense strips all around: views with more road triangles than the
        # chip-wide raster's per-view list holds
        scenes = [g.crowded_scene(800 + k, n_agents=6, n_roads=1500, radius=30.0) for k in range(3)]
        return scenes, g.camera_for(128, cams=g.FRONT_AND_SIDES), pal
    res = int(case[5:])
    w = g.workload("sweep", resolution=res, n_scenes=3 if res == 512 else 6)
    return w.scenes, w.camera, pal


@pytest.mark.parametrize("case", ["crowded", "roads", "uneven", "w208", "sweep64", "sweep128", "sweep256", "sweep512"])
def test_every_rasteriser_gives_identical_bits(case):
    """The rgb-only render through every rasteriser (banded, wave-split with
    1, 2 and 4 wavefronts per view, chip-wide with several grids, per-scene
    and persistent) equals the general kernel's rgb bit for bit, after a step
    too; sampled views equal the oracle."""
    print(f"rasterisers: {case}", flush=True)
    scenes, cam, pal = _raster_case(case)
    sim = _sim(scenes, cam, pal)
    for step in range(2):
        if step:
            act = g.batch_actions(1234, 0, scenes)
            sim.step(torch.from_numpy(act).cuda())
        ref, _, _ = sim.render(depth=True, primid=True)
        for lv in _RASTERS:
            sim.set_launch(**lv)
            out = sim.new_rgb()
            sim.render(rgb=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (case, step, lv)
            # twice in a row: the passes leave their counters and coverage words clean
            sim.render(rgb=out)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (case, step, lv, "second render")
    st = sim.get_state().cpu().numpy()
    hs = _host_scene_state(scenes, st)
    picks = [(0, 0, 0), (len(scenes) - 1, scenes[-1].n_agents - 1, len(cam.cam_dirs) - 1), (1, 3, 0)]
    _compare_views(hs, cam, pal, ref.cpu().numpy(), None, None, picks)


def test_scene_order_does_not_change_any_view():
    """The same scenes given in another order make another work queue (other
    XCD segments, another view order, other workgroups and neighbours for
    every view): each view's image, depth and primitive ids stay the same
    bits, through every rasteriser."""
    print("scene-order determinism", flush=True)
    w = g.workload("uneven", n_scenes=12)
    pal = g.default_palette()
    perm = np.random.default_rng(5).permutation(len(w.scenes))
    a = _sim(w.scenes, w.camera, pal)
    b = _sim([w.scenes[i] for i in perm], w.camera, pal)
    n_cams = len(w.camera.cam_dirs)
    base_a = np.cumsum([0] + [s.n_agents for s in w.scenes])
    pb = [w.scenes[i] for i in perm]
    base_b = np.cumsum([0] + [s.n_agents for s in pb])
    # view index in b of every view of a
    idx = np.empty(a.n_views, np.int64)
    for jb, ia in enumerate(perm):
        n = w.scenes[ia].n_agents * n_cams
        idx[base_a[ia] * n_cams:base_a[ia] * n_cams + n] = np.arange(base_b[jb] * n_cams, base_b[jb] * n_cams + n)
    idx_t = torch.from_numpy(idx).cuda()
    ra, da, pa = a.render(depth=True, primid=True)
    rb, db, pb_ = b.render(depth=True, primid=True)
    assert torch.equal(ra, rb.index_select(0, idx_t))
    assert torch.equal(da.view(torch.int32), db.index_select(0, idx_t).view(torch.int32))
    assert torch.equal(pa, pb_.index_select(0, idx_t))
    for lv in _RASTERS:
        a.set_launch(**lv)
        b.set_launch(**lv)
        oa, ob = a.new_rgb(), b.new_rgb()
        a.render(rgb=oa)
        b.render(rgb=ob)
        torch.cuda.synchronize()
        assert torch.equal(oa, ra), lv
        assert torch.equal(ob.index_select(0, idx_t), ra), lv
