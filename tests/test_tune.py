"""The autotuner: its search space on the CPU; on the GPU, a search over real
launch settings keeps only result-identical variants, applies the fastest and
round-trips its cache."""
import json

import pytest

from paper_2606_19641_amd import tune


def test_candidates_cover_the_space_with_the_persistent_schedule():
    space = {"band_rows": (8, 16), "batch_tris": (256,), "block_threads": (256, 512), "blocks_per_cu": (2, 3)}
    c = tune.candidates(space)
    assert len(c) == 2 * 1 * 2 * 2
    assert all(x["sched"] == 1 for x in c)
    assert len({tuple(sorted(x.items())) for x in c}) == len(c)


def test_bench_space_is_small():
    n = 1
    for v in tune.BENCH_SPACE.values():
        n *= len(v)
    assert n <= 24


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
    space = {"band_rows": (16, 32), "batch_tris": (256,), "block_threads": (256, 512), "blocks_per_cu": (1, 3)}
    cache = tmp_path / "tuned.json"
    best = tune.tune(sim, w.scenes, space=space, reps=2, cache=str(cache))
    assert sim.get_launch() == best
    out = sim.new_rgb()
    sim.render(rgb=out)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    table = json.loads(cache.read_text())
    assert any(v["launch"] == best for v in table.values())
    sim.set_launch(band_rows=8, blocks_per_cu=1)
    again = tune.tune(sim, w.scenes, space=space, reps=2, cache=str(cache))   # from the cache
    assert again == best and sim.get_launch() == best
