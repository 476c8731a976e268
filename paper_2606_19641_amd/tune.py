"""Autotuner for the renderer's launch settings.

Every launch setting of gp_sim_render gives the same image bits (the per-pixel
winner is a maximum over a total order, so band size, LDS batch size, block size
and the number of resident workgroups only change speed).  The tuner still
checks that: a candidate whose rgb differs from the reference setting's bits is
rejected, and the fastest surviving setting wins.  Results are cached in a JSON
file keyed by (GPU architecture, resolution, cameras, workload signature).
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Dict, Iterable, List, Optional

DEFAULT_SPACE = {
    "band_rows": (8, 16, 32, 64),
    "batch_tris": (256, 512, 1024),
    "block_threads": (256, 512),
    "blocks_per_cu": (1, 2, 3, 4),
}

# the short search the benchmark runs before timing (a few hundred renders)
BENCH_SPACE = {
    "band_rows": (16, 32),
    "batch_tris": (256, 512),
    "block_threads": (256,),
    "blocks_per_cu": (2, 3, 4),
}

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_launch.json")


def workload_key(sim, scenes) -> str:
    import torch
    arch = torch.cuda.get_device_properties(sim.device).gcnArchName.split(":")[0]
    sig = hashlib.sha1()
    for s in scenes:
        sig.update(f"{s.n_agents},{s.n_roads};".encode())
    cam = sim.camera
    return f"{arch}|{cam.width}x{cam.height}|cams{len(cam.cam_dirs)}|{sig.hexdigest()[:12]}"


def candidates(space: Dict[str, Iterable[int]] = DEFAULT_SPACE) -> List[dict]:
    keys = list(space)
    out = []
    for vals in itertools.product(*(space[k] for k in keys)):
        d = dict(zip(keys, vals))
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


def tune(sim, scenes, space: Dict[str, Iterable[int]] = DEFAULT_SPACE, reps: int = 5,
         cache: Optional[str] = CACHE, verbose: bool = False) -> dict:
    """Pick the fastest result-identical launch setting for `sim`; applies it and returns it."""
    import torch
    from .gp import GpError
    key = workload_key(sim, scenes)
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
    report = []
    for _pass in range(2):
        for n, cand in enumerate(settings):
            if not ok[n]:
                continue
            try:
                sim.set_launch(**cand)
            except GpError:
                ok[n] = False
                report.append((cand, None, "refused"))
                continue
            ms = time_render(sim, rgb, reps)
            if not torch.equal(rgb, rgb_ref):
                ok[n] = False
                report.append((cand, ms, "rejected: image bits differ"))
                continue
            times[n] = min(times[n], ms)
            if verbose:
                print(f"tune {cand} {ms:.4f} ms", flush=True)
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
    rejected = [r for r in report if r[2].startswith("rejected")]
    if rejected:
        raise RuntimeError(f"launch settings changed the image: {rejected[:3]}")
    return best
