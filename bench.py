"""Benchmark of the Gigapixel hot path on one MI355X.

One step = the kinematic step of every agent + the render of every view
(rgb, uint8) of one batch of synthetic scenes already resident in HBM.
Default workload: 64 scenes x 32 agents, 2,000 road quads each, one forward
camera at 128x128.  The batched form (one persistent-kernel render plus the
step, replayed as one hipGraph) is timed, and the plain form (per-scene
launches of the same kernels) is timed beside it on the same GPU.

Prints ONE JSON line.  With --gpus N > 1 it exits with a message: the path
needs no communication and this benchmark runs on one GPU only.
"""
from __future__ import annotations

import argparse
import glob
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 64 * 2.4e9          # vector lane-ops/s: 256 CUs, 4 SIMDs x 16 lanes, 2.4 GHz
METRIC = "agent-views/sec at 128×128 RGB (batched vs plain, same GPU); p99 step latency"
HBM_PEAK_GBS = 8000.0
COPY_BYTES = 256 << 20
# the workloads' episodes: 100 steps of random actions from the initial placement
EPISODE_STEPS = 100
RASTER_KERNELS = {0: "k_render (banded)", 1: "k_render_rgb (wave-split)",
                  2: "k_chip_setup + k_chip_roads + k_chip_resolve (chip-wide)"}
# the kernel field of a counter summary (profsum hbm --kernel) for each rasteriser
COUNTER_KERNELS = {0: "k_render<", 1: "k_render_rgb", 2: "k_chip"}


def kernel_source_sha() -> str:
    """sha256 over the HIP sources and headers (the tuner's cache key uses it too)."""
    from paper_2606_19641_amd import tune
    return tune.kernel_source_sha()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_counters(workload_name: str, launch: dict):
    """HBM traffic and VALU busy of the render kernel from a committed rocprofv3
    counter summary (profiles/*_counters.txt) of that kernel taken on the same
    kernel source, workload and launch setting, or None when there is none."""
    kernel = COUNTER_KERNELS.get(launch.get("raster"))
    sha = kernel_source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_counters.txt"))):
        kv = {}
        with open(path) as f:
            for line in f:
                if ":" in line and not line.startswith((" ", "#", "\t")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        try:
            if not (kv["kernel_source_sha256"] == sha and kv["workload"] == workload_name
                    and kv["kernel"] == kernel and json.loads(kv["launch"]) == launch):
                continue
            return {"traffic": float(kv["traffic_bytes_per_launch"]),
                    "valu_busy_pct": float(kv["valu_busy_pct"]),
                    "lds_bank_conflict_pct": float(kv["lds_bank_conflict_pct"]),
                    "valu_insts": float(kv["valu_insts_per_launch"]),
                    "source": os.path.relpath(path, ROOT)}
        except (KeyError, ValueError):
            continue
    return None


def _workload(args):
    from paper_2606_19641_amd import scenegen as g
    if args.workload == "sweep":
        return g.workload("sweep", resolution=args.res)
    if args.workload == "student":
        return g.workload("student", resolution=args.res if args.res in (210, 434) else 210)
    return g.workload(args.workload)


def _describe(w):
    na = [s.n_agents for s in w.scenes]
    nr = [s.n_roads for s in w.scenes]
    cams = len(w.camera.cam_dirs)
    if len(set(na)) == 1 and len(set(nr)) == 1:
        body = f"{len(w.scenes)} scenes x {na[0]} agents, {nr[0]} road quads each"
    else:
        body = (f"{len(w.scenes)} scenes, agents {min(na)}..{max(na)} (total {sum(na)}), "
                f"road quads {min(nr)}..{max(nr)}")
    return (f"{w.name}: {body}, {cams} camera(s) per agent at {w.camera.width}x{w.camera.height} "
            f"uint8 RGB")


def render_bytes(w) -> int:
    """Algorithmic HBM bytes of one render launch: every image written once,
    every scene's geometry read once (road strip 32 B corners + 1 B colour;
    agent 16 B state + 8 B heading cosines + 16 B dims + 1 B colour), one
    8 B view record per view."""
    img = w.camera.width * w.camera.height * 3
    geo = sum(33 * s.n_roads + 41 * s.n_agents for s in w.scenes)
    return w.n_views * (img + 8) + geo


def step_bytes(w) -> int:
    """Agent step: read state 16 B + dims 16 B + action 8 B, write state 16 B + cosines 8 B."""
    return 64 * w.n_agents


def _oracle_rate(w, budget_s: float, threads: int):
    """Views/s of the oracle over whole steps of the workload (step, then every
    view), stopped when the budget is spent (a step may be cut short)."""
    import oracle
    from paper_2606_19641_amd import scenegen as g
    cams = len(w.camera.cam_dirs)
    pal = g.default_palette()
    st = np.concatenate([s.agent_state for s in w.scenes])
    chunk = max(threads * 4, 16)
    done, steps = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        st, _ = oracle.step(st, np.concatenate([s.agent_dims for s in w.scenes]),
                            g.batch_actions(w.seed, steps, w.scenes), 0.1)
        scenes, o = [], 0
        for s in w.scenes:
            scenes.append(g.Scene(agent_state=st[o:o + s.n_agents], agent_dims=s.agent_dims,
                                  agent_color=s.agent_color, road_xy=s.road_xy, road_color=s.road_color))
            o += s.n_agents
        items = [(s, a, k) for s in scenes for a in range(s.n_agents) for k in range(cams)]
        for b in range(0, len(items), chunk):
            oracle.render_views(items[b:b + chunk], w.camera, pal, threads=threads)
            done += len(items[b:b + chunk])
            if time.perf_counter() - t0 >= budget_s:
                break
        steps += 1
    return done, steps, time.perf_counter() - t0


def cpu_baseline(w, budget_s: float):
    """The oracle on the host cores (all of them, then one) on a bounded sample."""
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    threads = max(1, threads)
    done, steps, dt = _oracle_rate(w, budget_s, threads)
    d1, _, t1 = _oracle_rate(w, max(1.0, budget_s / 4), 1)
    return {"value": done / dt, "unit": "agent-views/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "single_thread_value": d1 / t1,
            "sample": f"{done} views over {steps} step(s) of the same workload ({w.n_views} views per "
                      f"step; agent step + every view; {threads} threads, {dt:.1f} s); single thread: "
                      f"{d1} views in {t1:.1f} s"}


def serve_bench(args):
    """Serving at Poisson load: resident rollouts (agents U{8..128}, road quads
    U{500..8000}, one 128x128 forward view per agent), requests = one step +
    render of a rollout; one JSON line with the per-rate results."""
    import torch
    from paper_2606_19641_amd import scenegen as g
    from paper_2606_19641_amd import serve
    pool = g.workload("serve", n_scenes=args.serve_pool)
    pal = g.default_palette()
    budget = args.serve_budget_gib << 30
    ex = serve.GpuExecutor(pool.camera, pal, budget_bytes=budget, n_streams=args.serve_streams,
                           max_batch_agents=args.serve_resident * 128, max_batch_rollouts=args.serve_resident)
    rates = [float(r) for r in args.serve_rates.split(",")]
    rows = []
    # request payloads are generated before the timed runs (the client's cost,
    # not the server's): 8 action sets per scene of the pool, used in turn
    bank = [[g.actions(pool.seed, k, np.full(sc.n_agents, si), np.arange(sc.n_agents)) for k in range(8)]
            for si, sc in enumerate(pool.scenes)]
    scene_of = {}
    for ri, rate in enumerate(rates):
        srv = serve.Server(ex, budget_bytes=budget, max_batch_rollouts=args.serve_resident)
        nxt = [0]
        open_ids = []

        def open_one():
            si = nxt[0] % len(pool.scenes)
            nxt[0] += 1
            rid = srv.open(pool.scenes[si])
            scene_of[rid] = si
            open_ids.append(rid)

        for _ in range(args.serve_resident):
            open_one()
        torch.cuda.synchronize()
        life = args.serve_life
        count = {}
        rng = np.random.default_rng(1000 + ri)
        arrivals = serve.poisson_arrivals(rate, args.serve_seconds, seed=2000 + ri)

        retiring = []

        def pick(i):
            while retiring:                        # their last request is queued: close, replace
                srv.close(retiring.pop())
                open_one()
            k = int(rng.integers(len(open_ids)))
            rid = open_ids[k]
            count[rid] = count.get(rid, 0) + 1
            if count[rid] == life:
                open_ids.pop(k)
                retiring.append(rid)
            return rid

        def actions_for(i, rid):
            return bank[scene_of[rid]][i % len(bank[0])]

        gc.collect()
        gc.disable()                               # no collector pauses inside the timed run
        try:
            t0 = serve.drive(srv, arrivals, pick, actions_for, time.perf_counter)
            t1 = time.perf_counter() - t0
        finally:
            gc.enable()
        torch.cuda.synchronize()
        summ = srv.summary(0.0, max(args.serve_seconds, t1))
        summ.update({"offered_per_s": rate, "wall_s": t1, "admitted_rollouts": nxt[0]})
        rows.append(summ)
        print(f"serve rate {rate:.0f}/s: {summ['completed_per_s']:.0f} done/s, p50 {summ['p50_ms']:.3f} ms, "
              f"p99 {summ['p99_ms']:.3f} ms, mean batch {summ['mean_batch_rollouts']:.1f}", file=sys.stderr,
              flush=True)
        for rid in list(srv.rollouts):
            srv.cancel(rid)
        srv.pump(time.perf_counter())
        torch.cuda.synchronize()
        srv.pump(time.perf_counter())
    top = rows[-1]
    out = {
        "metric": "serving: completed requests/s at Poisson load (one step + 128x128 render of a rollout "
                  "per request); p50/p99 latency arrival-to-completion",
        "value": top["completed_per_s"], "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
        "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded scenes standing in for nuPlan)",
        "config": {"workload": f"serve: {args.serve_resident} resident rollouts from a pool of "
                               f"{len(pool.scenes)} scenes (agents U{{8..128}}, road quads U{{500..8000}}), "
                               f"128x128 forward view, rollout life {args.serve_life} requests, "
                               f"{args.serve_streams} streams, {args.serve_seconds} s per rate",
                   "seed": pool.seed},
        "rates": rows,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the GPU needs about 0.1 s of steady work to reach its full clocks: 1,000
    # warm-up steps (~0.1 s) before the timed ones
    ap.add_argument("--warmup", type=int, default=1000)
    ap.add_argument("--workload", default="uniform",
                    choices=["small", "uniform", "uneven", "sweep", "serve", "student"])
    ap.add_argument("--res", type=int, default=128)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--lat-steps", type=int, default=1000, help="graph replays sampled for the latency percentiles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--tuned", default="", help="launch settings JSON (skips the autotuner)")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch settings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--serve-rates", default="1000,2000,5000,10000,20000")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-resident", type=int, default=64)
    ap.add_argument("--serve-pool", type=int, default=256)
    ap.add_argument("--serve-life", type=int, default=EPISODE_STEPS, help="requests per rollout (one episode)")
    ap.add_argument("--serve-streams", type=int, default=4)
    ap.add_argument("--serve-budget-gib", type=int, default=16)
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the rendering path needs no "
              "inter-GPU communication and each GPU owns whole scenes, so N GPUs give N times the "
              "one-GPU figure by construction, which this benchmark does not claim.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serve":
        serve_bench(args)
        return

    import torch
    from paper_2606_19641_amd import gp
    from paper_2606_19641_amd import scenegen as g

    w = _workload(args)
    pal = g.default_palette()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    K, W = args.steps, args.warmup
    sim = gp.Sim(w.scenes, w.camera, pal, device="cuda:0")
    V = sim.n_views
    # Every step this benchmark runs belongs to an episode of E steps of random
    # actions from the workload's initial placement: with random actions the
    # agents leave the road network within a few hundred steps and the views
    # empty out, so a longer run would time a different (cheaper) workload.
    # Episode step e takes action set e; the state returns to the initial one
    # at every episode start.  The inputs are built first (host work, GPU idle).
    E = EPISODE_STEPS
    state0 = sim.get_state()
    acts = torch.from_numpy(np.stack([g.batch_actions(w.seed, k, w.scenes) for k in range(E)])).to(dev)
    rgb = sim.new_rgb()
    stream = torch.cuda.current_stream()

    def replay(k):
        """Step k of the run (episode step k mod E) as one graph replay."""
        if k % E == 0:
            sim.set_state(state0)
        sim.step_render_graph(acts[k % E], rgb)

    if args.tuned:
        sim.set_launch(**json.loads(args.tuned))
    elif not args.no_tune:
        # the autotuner: fastest of the result-identical launch settings (a7)
        from paper_2606_19641_amd import tune
        tune.tune(sim, w.scenes, space=tune.BENCH_SPACE, reps=5, cache=None)
    launch = sim.get_launch()
    launch["sched"] = gp.SCHED_PERSISTENT
    sim.set_launch(**launch)

    # ---- batched: step + persistent render as one graph replay per step.  W
    # warm-up steps, continued (untimed) until at least 0.1 s of steady work
    # has run, since the clocks rise only under sustained load
    t_w = time.perf_counter()
    for k in range(W):
        replay(k)
    torch.cuda.synchronize()
    k = W
    while time.perf_counter() - t_w < 0.1:
        for _ in range(16):
            replay(k)
            k += 1
        torch.cuda.synchronize()
    settle_steps = k - W
    # the timed steps: one episode from its start (more than E steps run
    # further episodes, each from the initial state again)
    sim.set_state(state0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        if k and k % E == 0:
            sim.set_state(state0)
        sim.step_render_graph(acts[k % E], rgb)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    batched = V * K / wall

    # ---- step latency: its own run of lat_steps graph replays (actions reused in
    # turn), one event pair each, for the p50 / p99
    n_lat = max(args.lat_steps, 1)
    lev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n_lat)]
    for k in range(n_lat):
        if k % E == 0:
            sim.set_state(state0)
        lev[k][0].record(stream)
        sim.step_render_graph(acts[k % E], rgb)
        lev[k][1].record(stream)
    torch.cuda.synchronize()
    lat_ms = np.array([a.elapsed_time(b) for a, b in lev])

    # ---- the render kernel alone (eager, persistent), events on its stream,
    # over the states of one episode: after each untimed step, RR renders
    # back to back between one event pair (which spreads the dispatch latency
    # an event pair adds over RR launches); a short spin kernel first lets the
    # launches queue up, so host launch gaps do not enter the event times
    rk, RR = max(10, min(K, E)), 3
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(rk)]
    sim.set_state(state0)
    torch.cuda._sleep(1_000_000)
    for k in range(rk):
        sim.step(acts[k % E])
        rev[k][0].record(stream)
        for _ in range(RR):
            sim.render(rgb=rgb)
        rev[k][1].record(stream)
    torch.cuda.synchronize()
    render_ms = float(np.mean([a.elapsed_time(b) for a, b in rev])) / RR

    # ---- the infraction check (collision / off-road, halting) on the same state,
    # timed apart: it is not part of the step + render graph
    flags = torch.empty(sim.n_agents, dtype=torch.uint8, device=dev)
    state_c = sim.get_state()
    iev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(10)]
    torch.cuda._sleep(1_000_000)
    for a, b in iev:
        a.record(stream)
        sim.check_infractions(flags)
        b.record(stream)
    torch.cuda.synchronize()
    infr_ms = float(np.mean([a.elapsed_time(b) for a, b in iev]))
    sim.set_state(state_c)              # the check halted offenders: restore the state

    # ---- the ray-cast backend over the states of one episode (every fifth
    # step; same images up to edge pixels), timed apart: the raster is the
    # measured path
    rc_rgb = sim.new_rgb()
    sim.render_raycast(rgb=rc_rgb)
    rev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(E // 5)]
    sim.set_state(state0)
    torch.cuda.synchronize()
    torch.cuda._sleep(1_000_000)
    for k in range(E):
        sim.step(acts[k])
        if k % 5 == 4:
            a, b = rev[k // 5]
            a.record(stream)
            sim.render_raycast(rgb=rc_rgb)
            b.record(stream)
    torch.cuda.synchronize()
    raycast_ms = float(np.mean([a.elapsed_time(b) for a, b in rev]))
    del rc_rgb

    # ---- plain: per-scene launches of the same kernels, no graph
    plain = None
    if not args.no_plain:
        sim.set_launch(sched=gp.SCHED_PLAIN)
        sim.set_state(state0)
        for k in range(min(W, 20)):         # the clocks are up by now
            sim.step(acts[k % E])
            sim.render(rgb=rgb)
        sim.set_state(state0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(K):
            if k and k % E == 0:
                sim.set_state(state0)
            sim.step(acts[k % E])
            sim.render(rgb=rgb)
        torch.cuda.synchronize()
        plain = V * K / (time.perf_counter() - t1)
        sim.set_launch(sched=gp.SCHED_PERSISTENT)

    if args.copy_calibration:
        # a plain streaming kernel of known size: 256 MiB read, 256 MiB written
        src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    rb = render_bytes(w)
    achieved = rb / (render_ms * 1e-3) / 1e9
    # the render kernel's work rates: pixel samples resolved, and primitives
    # considered before culling (every view: the other boxes' 6 faces, the
    # obstacles' faces, every road strip and light of its scene)
    cams = len(w.camera.cam_dirs)
    prims = sum(s.n_agents * cams * (6 * (s.n_agents - 1 + getattr(s, "n_static", 0)) + s.n_roads
                                     + getattr(s, "n_signals", 0)) for s in w.scenes)
    rates = {"pixels_per_s": V * w.camera.width * w.camera.height / (render_ms * 1e-3),
             "primitives_per_s": prims / (render_ms * 1e-3), "primitives_per_step": prims}
    meas = measured_counters(args.workload if args.workload != "sweep" else f"sweep{args.res}", launch)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": batched,
        "unit": "agent-views/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "settle_steps": settle_steps,
        "ms_per_step": wall / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded scenes standing in for nuPlan)",
        "config": {"workload": _describe(w), "views_per_step": V, "seed": w.seed,
                   "schedule": ("one workgroup per view, the dispatcher balancing uneven views"
                                if launch.get("raster") == 1 else
                                "three chip-wide passes" if launch.get("raster") == 2 else
                                "persistent work queue (one workgroup per view when the views fit the resident grid)")
                               + " + hipGraph (step + render)",
                   "launch": launch},
        "plain_value": plain,
        "batched_over_plain": (batched / plain) if plain else None,
        "p50_step_ms": float(np.percentile(lat_ms, 50)),
        "p99_step_ms": float(np.percentile(lat_ms, 99)),
        "latency_samples": int(n_lat),
        "render_kernel_ms": render_ms,
        "infraction_check_ms": infr_ms,
        "raycast_render_ms": raycast_ms,
        "render_rates": rates,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": meas["traffic"] if meas else None,
                     "kernel": RASTER_KERNELS.get(launch.get("raster"), "k_render"), "bytes_per_launch": rb,
                     "valu_busy_pct": meas["valu_busy_pct"] if meas else None,
                     "lds_bank_conflict_pct": meas["lds_bank_conflict_pct"] if meas else None,
                     "counters_from": meas["source"] if meas else None},
        # the plain VALU roof beside the HBM one: wave instructions x 64 lanes
        # over the kernel time, against 256 CUs x 64 lanes x 2.4 GHz
        "valu_roof": ({"achieved": meas["valu_insts"] * 64 / (render_ms * 1e-3), "peak": VALU_PEAK,
                       "unit": "lane-ops/s", "frac": meas["valu_insts"] * 64 / (render_ms * 1e-3) / VALU_PEAK}
                      if meas else None),
        "cpu_baseline": cpu,
        "paper_context": "~50k agent steps/s from pixels on 1 NVIDIA A100L (workload not stated)",
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
