"""The autotuner: its search space on the CPU; on the GPU, a search over real
launch settings keeps only result-identical variants, applies the fastest and
round-trips its cache."""
import json

import pytest

from paper_2606_19641_amd import tune


def test_candidates_cover_the_space_with_the_persistent_schedule():
    space = tune._grid(band_rows=(8, 16), batch_tris=(256,), block_threads=(256, 512), blocks_per_cu=(2, 3))
    c = tune.candidates(space)
    assert len(c) == 2 * 1 * 2 * 2
    assert all(x["sched"] == 1 for x in c)
    assert len({tuple(sorted(x.items())) for x in c}) == len(c)


def test_search_spaces_cover_every_rasteriser_and_bench_space_is_small():
    for space in (tune.DEFAULT_SPACE, tune.BENCH_SPACE):
        assert {c["raster"] for c in space} == {0, 1, 2}
    assert len(tune.BENCH_SPACE) <= 16


def test_cache_key_names_the_kernel_sources_and_scene_shape(monkeypatch):
    class Props:
        gcnArchName = "gfx950:sramecc+:xnack-"

    class Cam:
        width, height, cam_dirs = 128, 128, ((1.0, 0.0),)

    class FakeSim:
        device = "cuda:0"
        camera = Cam()
        light = None
        scene_shapes = ((32, 2000, 0, 0),)

    torch = pytest.importorskip("torch")
    monkeypatch.setattr(torch.cuda, "get_device_properties", lambda d: Props())
    a = FakeSim()
    k = tune.workload_key(a)
    assert k.startswith("gfx950|128x128|cams1|") and tune.kernel_source_sha()[:12] in k
    b = FakeSim()
    b.scene_shapes = ((32, 2000, 3, 0),)          # static obstacles change the key
    c = FakeSim()
    c.light = (0.0, 0.0, 1.0, 0.3)                # so does the light
    d = FakeSim()
    d.scene_shapes = ((32, 2000, 0, 2),)          # and traffic lights
    assert len({k, tune.workload_key(b), tune.workload_key(c), tune.workload_key(d)}) == 4


@pytest.mark.gpu
def test_tuner_applies_a_result_identical_setting_and_caches_it(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_19641_amd import gp, scenegen as g
    w = g.workload("uniform", n_scenes=4)
    sim = gp.Sim(w.scenes, w.camera, g.default_palette())
    ref = sim.new_rgb()
    sim.render(rgb=ref)
    torch.cuda.synchronize()
    space = tune._grid(raster=(2,), road_wgs_per_cu=(4, 8, 16)) + \
        [dict(raster=1, view_waves=2, blocks_per_cu=8), dict(raster=0, band_rows=32, blocks_per_cu=3)]
    cache = tmp_path / "tuned.json"
    best = tune.tune(sim, w.scenes, space=space, reps=2, cache=str(cache))
    assert sim.get_launch() == best
    out = sim.new_rgb()
    sim.render(rgb=out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    table = json.loads(cache.read_text())
    assert any(v["launch"] == best for v in table.values())
    sim.set_launch(raster=0, band_rows=8, blocks_per_cu=1)
    again = tune.tune(sim, w.scenes, space=space, reps=2, cache=str(cache))   # from the cache
    assert again == best and sim.get_launch() == best
