"""Autotuner for the renderer's launch settings.

Every launch setting of gp_sim_render gives the same image bits (the per-pixel
winner is a maximum over a total order, so the rasteriser, its band or item
sizes, LDS batch sizes, block sizes and the number of resident workgroups only
change speed).  The tuner still checks that: a candidate whose rgb-only image,
or whose rgb / depth / primitive-id render, differs from the reference
setting's bits is rejected, and then the search raises without caching
anything.  The fastest setting wins; results are cached in a JSON file keyed by
(GPU architecture, resolution, cameras, per-scene shape of agents, strips,
static obstacles and traffic lights, light on or off, a hash of the kernel
sources).
"""
from __future__ import annotations

import glob
import hashlib
import itertools
import json
import os
from typing import Dict, Iterable, List, Optional

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned_launch.json")

# Search spaces: lists of partial launch settings, each applied on top of the
# sim's current one.  The rasteriser is a dimension of the search: the
# chip-wide passes with their workgroups per CU, the wave-split raster with
# its wavefronts per view, the banded raster with its band rows, LDS batch,
# block size and workgroups per CU.


def _grid(**dims) -> List[dict]:
    keys = list(dims)
    return [dict(zip(keys, vals)) for vals in itertools.product(*(dims[k] for k in keys))]


DEFAULT_SPACE = (
    _grid(raster=(2,), road_wgs_per_cu=(2, 4, 6, 8, 12, 16))
    + _grid(raster=(1,), view_waves=(1, 2, 4), blocks_per_cu=(4, 6, 8))
    + _grid(raster=(0,), band_rows=(8, 16, 32, 64), batch_tris=(256, 512, 1024), block_threads=(256, 512),
            blocks_per_cu=(1, 2, 3, 4))
)

# the short search the benchmark runs before timing (a few hundred renders)
BENCH_SPACE = (
    _grid(raster=(2,), road_wgs_per_cu=(4, 8, 16))
    + [dict(raster=1, view_waves=2, blocks_per_cu=8), dict(raster=1, view_waves=4, blocks_per_cu=4)]
    + _grid(raster=(0,), band_rows=(8, 16, 32), batch_tris=(256,), block_threads=(256,), blocks_per_cu=(2, 3))
    + _grid(raster=(0,), band_rows=(16,), batch_tris=(256, 512), block_threads=(512,), blocks_per_cu=(1, 2))
)


def kernel_source_sha() -> str:
    """sha256 over the HIP sources and headers the library is built from."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if f.endswith((".hip", ".h")):
            with open(f, "rb") as fh:
                h.update(os.path.basename(f).encode())
                h.update(fh.read())
    return h.hexdigest()


def workload_key(sim, scenes=None) -> str:
    import torch
    arch = torch.cuda.get_device_properties(sim.device).gcnArchName.split(":")[0]
    sig = hashlib.sha1()
    for shape in sim.scene_shapes:
        sig.update(("%d,%d,%d,%d;" % shape).encode())
    cam = sim.camera
    light = "lit" if sim.light is not None else "flat"
    return (f"{arch}|{cam.width}x{cam.height}|cams{len(cam.cam_dirs)}|{sig.hexdigest()[:12]}|{light}|"
            f"src{kernel_source_sha()[:12]}")


def candidates(space: Iterable[dict] = DEFAULT_SPACE) -> List[dict]:
    out = []
    for c in space:
        d = dict(c)
        d["sched"] = 1
        out.append(d)
    return out


def time_render(sim, rgb, reps: int = 5) -> float:
    """Mean milliseconds of one rgb render: `reps` renders back to back between
    two HIP events on the current stream, queued behind a short spin kernel so
    that host launch gaps stay out of the measurement."""
    import torch
    stream = torch.cuda.current_stream()
    sim.render(rgb=rgb)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda._sleep(1_000_000)
    a.record(stream)
    for _ in range(reps):
        sim.render(rgb=rgb)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def warm_up(sim, rgb, seconds: float = 0.1) -> None:
    """Render until about `seconds` of GPU work has run: the clocks rise only
    under sustained load, and a setting timed on a cold GPU looks slower."""
    import time
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(20):
            sim.render(rgb=rgb)
        torch.cuda.synchronize()


def tune(sim, scenes=None, space: Iterable[dict] = DEFAULT_SPACE, reps: int = 5,
         cache: Optional[str] = CACHE, verbose: bool = False) -> dict:
    """Pick the fastest result-identical launch setting for `sim`; applies it
    and returns it.  Raises (caching nothing) if any setting changed a bit."""
    import torch
    from .gp import GpError
    key = workload_key(sim)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table:
            sim.set_launch(**table[key]["launch"])
            return table[key]["launch"]
    base = sim.get_launch()
    base["sched"] = 1
    sim.set_launch(**base)
    rgb_ref = sim.new_rgb()
    sim.render(rgb=rgb_ref)
    full_ref = [t.clone() for t in sim.render(depth=True, primid=True)]
    rgb = sim.new_rgb()
    warm_up(sim, rgb_ref)
    # two interleaved passes over every setting, each keeping its faster time,
    # so that a drift of the clocks during the search favours none of them
    settings = [dict(base)]
    for c in candidates(space):
        full = dict(base)
        full.update(c)
        if full not in settings:
            settings.append(full)
    times = [float("inf")] * len(settings)
    ok = [True] * len(settings)
    rejected = []
    for _pass in range(2):
        for n, cand in enumerate(settings):
            if not ok[n]:
                continue
            try:
                sim.set_launch(**cand)
            except GpError:
                ok[n] = False
                continue
            ms = time_render(sim, rgb, reps)
            same = torch.equal(rgb, rgb_ref)
            if same and _pass == 0:
                full = sim.render(depth=True, primid=True)
                same = all(torch.equal(a.view(torch.uint8), b.view(torch.uint8)) for a, b in zip(full, full_ref))
            if not same:
                ok[n] = False
                rejected.append(cand)
                continue
            times[n] = min(times[n], ms)
            if verbose:
                print(f"tune {cand} {ms:.4f} ms", flush=True)
    if rejected:
        sim.set_launch(**base)
        raise RuntimeError(f"launch settings changed the image: {rejected[:3]}")
    n_best = min((n for n in range(len(settings)) if ok[n]), key=lambda n: times[n])
    best, best_ms = dict(settings[n_best]), times[n_best]
    sim.set_launch(**best)
    if cache:
        table = {}
        if os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
        table[key] = {"launch": best, "ms": best_ms}
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return best
