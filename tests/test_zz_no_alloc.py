"""The allocation-free render entry point (gp_sim_render_noalloc): its scratch
lives in a static device array instead of the sim's workspace.  Called
through the C ABI, its images equal gp_sim_render's (the chip-wide raster
through the workspace) bit for bit, on two calls in a row of which the second
renders a smaller input; the array keeps the first call's contents, so the
second call must clear what it needs.  A sim whose scratch exceeds the array
is refused."""
import ctypes as C

import numpy as np
import pytest

from paper_2606_19641_amd import scenegen as g

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _noalloc(sim, rgb):
    from paper_2606_19641_amd import gp
    L = gp.lib()
    fn = L.gp_sim_render_noalloc
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    fn.restype = C.c_int
    return fn(sim._h, rgb.data_ptr(), None)


def _reference(sim):
    # the existing entry point with the same (chip-wide) kernels on the workspace
    sim.set_launch(sched=1, raster=2)
    ref, _, _ = sim.render()
    return ref


def test_noalloc_render_equals_render_two_calls_second_smaller():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp
    pal = g.default_palette()
    big = g.workload("uneven", n_scenes=3)         # three cameras, up to 8,000 strips per scene
    small = g.workload("uniform", n_scenes=2)       # 64 views
    assert sum(s.n_agents for s in small.scenes) < 3 * sum(s.n_agents for s in big.scenes)
    sim_a = gp.Sim(big.scenes, big.camera, pal)
    sim_b = gp.Sim(small.scenes, small.camera, pal)
    for sim, w in ((sim_a, big), (sim_b, small)):
        print(f"noalloc render: {sim.n_views} views", flush=True)
        for step in range(2):
            if step:
                sim.step(torch.from_numpy(g.batch_actions(w.seed, 0, w.scenes)).cuda())
            ref = _reference(sim)
            out = sim.new_rgb()
            out.fill_(7)
            assert _noalloc(sim, out) == gp.GP_OK, gp.lib().gp_last_error()
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (sim.n_views, step)
    # the first sim again, after the smaller one
    ref = _reference(sim_a)
    out = sim_a.new_rgb()
    assert _noalloc(sim_a, out) == gp.GP_OK
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_refuses_what_it_cannot_serve():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp
    pal = g.default_palette()
    # 4,096 views at 512x512: coverage words alone need 134 MB, beyond the array
    w = g.workload("sweep", resolution=512)
    sim = gp.Sim(w.scenes, w.camera, pal)
    out = sim.new_rgb()
    assert _noalloc(sim, out) == gp.GP_EINVAL
    assert b"scratch" in gp.lib().gp_last_error()
    del sim, out
    torch.cuda.empty_cache()
    # an image width the chip-wide raster does not take
    w = g.workload("small")
    sim = gp.Sim(w.scenes, g.camera_for(48), pal)
    assert _noalloc(sim, sim.new_rgb()) == gp.GP_EINVAL
