"""Seeded synthetic driving scenes, actions and workload configurations.

This module only draws inputs. It holds none of the renderer's or the
dynamics' arithmetic, and both the HIP path and the CPU oracle receive the
same arrays from it.

The paper's scenes come from nuPlan (Sec. 4; App. A "Other Details"), which
is not available here.  A synthetic stand-in with the same ingredients is
generated instead: a road map made of lane strips (App. A: lane polylines
become thin planar strips) and vehicle cuboids placed on the lanes.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: every draw is a hash of (seed, stream, i, j, k), so a value does
not depend on how scenes are batched or in which order they are built.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream tags, one per kind of draw
S_ROADNET, S_SCENE, S_AGENT, S_ACTION = 1, 2, 3, 4

# palette indices used by the generated scenes
COLOR_BACKGROUND, COLOR_ROAD, COLOR_VEHICLE = 0, 1, 2
COLOR_SIGNAL_RED, COLOR_SIGNAL_YELLOW, COLOR_SIGNAL_GREEN = 6, 7, 8


def splitmix64(x):
    """SplitMix64 finaliser on uint64 (scalar or array); arithmetic wraps mod 2**64."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def keyed_u64(seed, stream, i=0, j=0, k=0):
    """One 64-bit draw for the counter (seed, stream, i, j, k); arrays broadcast."""
    h = splitmix64(np.uint64(seed) ^ splitmix64(np.uint64(stream)))
    for v in (i, j, k):
        h = splitmix64(h ^ splitmix64(np.asarray(v, dtype=np.uint64)))
    return h


def keyed_uniform(seed, stream, i=0, j=0, k=0):
    """Uniform float64 in [0, 1) with 24 random bits (so it is exact in float32)."""
    return (keyed_u64(seed, stream, i, j, k) >> np.uint64(40)).astype(np.float64) * (2.0 ** -24)


@dataclasses.dataclass
class Scene:
    """Host arrays of one scene, float32 SoA as the boundary takes them."""
    agent_state: np.ndarray  # [n_agents, 4] x, y, psi, v   (m, m, rad, m/s)
    agent_dims: np.ndarray   # [n_agents, 3] L, W, H        (m)
    agent_color: np.ndarray  # [n_agents] uint8 palette index
    road_xy: np.ndarray      # [n_roads, 4, 2] corners at z = 0, counter-clockwise seen from +z
    road_color: np.ndarray   # [n_roads] uint8 palette index
    # static obstacles (cuboids that never move): [k, 3] x, y, psi; [k, 3] L, W, H; [k] colour
    static_xyp: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3), np.float32))
    static_dims: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3), np.float32))
    static_color: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.uint8))
    # traffic lights (spheres): [g, 4] x, y, z (centre), radius; [g] colour of the light's state
    signal_xyzr: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 4), np.float32))
    signal_color: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(0, np.uint8))

    @property
    def n_agents(self) -> int:
        return int(self.agent_state.shape[0])

    @property
    def n_roads(self) -> int:
        return int(self.road_xy.shape[0])

    @property
    def n_static(self) -> int:
        return int(self.static_xyp.shape[0])

    @property
    def n_signals(self) -> int:
        return int(self.signal_xyzr.shape[0])


@dataclasses.dataclass
class Camera:
    width: int = 128
    height: int = 128
    focal_px: float = 64.0          # W/2 gives a 90 degree horizontal field of view
    cam_height: float = 1.6
    z_near: float = 0.5
    z_far: float = 100.0
    cam_dirs: Sequence[Sequence[float]] = ((1.0, 0.0),)   # (cos, sin) of each camera's yaw offset


FRONT = ((1.0, 0.0),)
FRONT_AND_SIDES = ((1.0, 0.0), (0.5, 0.8660254), (0.5, -0.8660254))   # 0, +60, -60 degrees
# the student's rig (App. B): front, front-left, front-right, rear; the paper
# gives no yaw offsets, so the side cameras take +-60 degrees as above
STUDENT_RIG = ((1.0, 0.0), (0.5, 0.8660254), (0.5, -0.8660254), (-1.0, 0.0))
STUDENT_RESOLUTIONS = ((210, 126), (434, 252))


def default_palette() -> np.ndarray:
    pal = np.zeros((256, 3), dtype=np.uint8)
    pal[COLOR_BACKGROUND] = (0, 0, 0)
    pal[COLOR_ROAD] = (128, 128, 128)
    pal[COLOR_VEHICLE] = (0, 0, 255)      # the paper colours every agent blue
    pal[COLOR_SIGNAL_RED] = (255, 32, 32)
    pal[COLOR_SIGNAL_YELLOW] = (255, 200, 0)
    pal[COLOR_SIGNAL_GREEN] = (32, 224, 64)
    return pal


def camera_for(width: int, height: int | None = None, cams=FRONT) -> Camera:
    height = width if height is None else height
    return Camera(width=width, height=height, focal_px=width / 2.0, cam_dirs=cams)


# ---------------------------------------------------------------- road network

MAP_HALF = 100.0       # every map is [-100, 100]^2 m
LANE_WIDTH = 3.5
ROADS_PER_AXIS = 4


def road_network(seed: int, scene: int, n_quads: int) -> np.ndarray:
    """Manhattan grid: 4 east-west and 4 north-south roads of two opposing lanes.

    The 16 lanes (each 200 m long, 3.5 m wide) are cut into n_quads segments in
    total; lane l gets n_quads // 16 segments plus one of the remainder if
    l < n_quads % 16.  Returns float32 [n_quads, 4, 2], counter-clockwise seen
    from above.
    """
    if n_quads < 16:
        raise ValueError("need at least one quad per lane (16)")
    base = np.array([-75.0, -25.0, 25.0, 75.0])
    jit = keyed_uniform(seed, S_ROADNET, scene, np.arange(2 * ROADS_PER_AXIS)) * 20.0 - 10.0
    lanes = []  # (start point, unit direction)
    for r in range(ROADS_PER_AXIS):
        y0 = base[r] + jit[r]
        lanes.append(((-MAP_HALF, y0 - LANE_WIDTH / 2), (1.0, 0.0)))    # eastbound, south lane
        lanes.append(((MAP_HALF, y0 + LANE_WIDTH / 2), (-1.0, 0.0)))    # westbound, north lane
    for r in range(ROADS_PER_AXIS):
        x0 = base[r] + jit[ROADS_PER_AXIS + r]
        lanes.append(((x0 + LANE_WIDTH / 2, -MAP_HALF), (0.0, 1.0)))    # northbound, east lane
        lanes.append(((x0 - LANE_WIDTH / 2, MAP_HALF), (0.0, -1.0)))    # southbound, west lane
    nl = len(lanes)
    counts = np.full(nl, n_quads // nl)
    counts[: n_quads % nl] += 1
    out = np.empty((n_quads, 4, 2), dtype=np.float64)
    hw = LANE_WIDTH / 2
    q = 0
    for li, ((sx, sy), (dx, dy)) in enumerate(lanes):
        n = int(counts[li])
        seg = 2 * MAP_HALF / n
        s0 = np.arange(n) * seg
        s1 = s0 + seg
        nx, ny = -dy, dx                   # left normal
        ax0, ay0 = sx + dx * s0, sy + dy * s0
        ax1, ay1 = sx + dx * s1, sy + dy * s1
        blk = out[q:q + n]
        blk[:, 0, 0], blk[:, 0, 1] = ax0 - hw * nx, ay0 - hw * ny
        blk[:, 1, 0], blk[:, 1, 1] = ax1 - hw * nx, ay1 - hw * ny
        blk[:, 2, 0], blk[:, 2, 1] = ax1 + hw * nx, ay1 + hw * ny
        blk[:, 3, 0], blk[:, 3, 1] = ax0 + hw * nx, ay0 + hw * ny
        q += n
    return out.astype(np.float32)


def place_agents(seed: int, scene: int, road_xy: np.ndarray, n_agents: int) -> tuple:
    """Vehicles on lane centrelines, heading along the lane +-U(0, 5 deg).

    L ~ U(4, 5.5), W ~ U(1.8, 2.2), H ~ U(1.4, 2.0) m, v0 ~ U(0, 15) m/s.
    """
    a = np.arange(n_agents)
    u = lambda c: keyed_uniform(seed, S_AGENT, scene, a, c)
    nq = road_xy.shape[0]
    qi = np.minimum((u(0) * nq).astype(np.int64), nq - 1)
    quad = road_xy[qi].astype(np.float64)
    back = 0.5 * (quad[:, 0] + quad[:, 3])
    front = 0.5 * (quad[:, 1] + quad[:, 2])
    t = u(1)
    pos = back + t[:, None] * (front - back)
    d = front - back
    lane_heading = np.arctan2(d[:, 1], d[:, 0])
    dev = np.deg2rad(5.0) * u(2) * np.where(u(3) < 0.5, -1.0, 1.0)
    psi = lane_heading + dev
    psi = np.where(psi > math.pi, psi - 2 * math.pi, psi)
    psi = np.where(psi <= -math.pi, psi + 2 * math.pi, psi)
    L = 4.0 + 1.5 * u(4)
    W = 1.8 + 0.4 * u(5)
    H = 1.4 + 0.6 * u(6)
    v = 15.0 * u(7)
    state = np.stack([pos[:, 0], pos[:, 1], psi, v], axis=1).astype(np.float32)
    dims = np.stack([L, W, H], axis=1).astype(np.float32)
    return state, dims


S_STATIC = 7


def place_statics(seed: int, scene: int, road_xy: np.ndarray, n_static: int) -> tuple:
    """Static obstacles on lane edges (a road's edge or the line between its two
    lanes): parked vehicles and barriers 1.75..2.25 m to either side of a lane
    segment's centreline, along the lane +-U(0, 10 deg); L ~ U(1, 6),
    W ~ U(0.5, 2.2), H ~ U(0.8, 2.0) m."""
    a = np.arange(n_static)
    u = lambda c: keyed_uniform(seed, S_STATIC, scene, a, c)
    nq = road_xy.shape[0]
    qi = np.minimum((u(0) * nq).astype(np.int64), nq - 1)
    quad = road_xy[qi].astype(np.float64)
    back = 0.5 * (quad[:, 0] + quad[:, 3])
    front = 0.5 * (quad[:, 1] + quad[:, 2])
    pos = back + u(1)[:, None] * (front - back)
    d = front - back
    heading = np.arctan2(d[:, 1], d[:, 0])
    side = np.where(u(2) < 0.5, -1.0, 1.0)
    nrm = np.stack([-np.sin(heading), np.cos(heading)], axis=1)
    pos = pos + (side * (1.75 + 0.5 * u(3)))[:, None] * nrm       # at the lane's edge
    psi = heading + np.deg2rad(10.0) * (2.0 * u(4) - 1.0)
    psi = np.where(psi > math.pi, psi - 2 * math.pi, psi)
    psi = np.where(psi <= -math.pi, psi + 2 * math.pi, psi)
    dims = np.stack([1.0 + 5.0 * u(5), 0.5 + 1.7 * u(6), 0.8 + 1.2 * u(7)], axis=1)
    xyp = np.stack([pos[:, 0], pos[:, 1], psi], axis=1).astype(np.float32)
    return xyp, dims.astype(np.float32)


S_SIGNAL = 8
SIGNAL_STATES = (COLOR_SIGNAL_RED, COLOR_SIGNAL_YELLOW, COLOR_SIGNAL_GREEN)


def place_signals(seed: int, scene: int, road_xy: np.ndarray, n_signals: int) -> tuple:
    """Traffic lights at lane-segment ends: 2.5..3.5 m to the side of the
    centreline, centre 3.5..5.5 m up, radius 0.25..0.4 m, state red / yellow /
    green with probabilities 0.45 / 0.1 / 0.45.  Returns (xyzr [g, 4], colour [g])."""
    a = np.arange(n_signals)
    u = lambda c: keyed_uniform(seed, S_SIGNAL, scene, a, c)
    nq = road_xy.shape[0]
    qi = np.minimum((u(0) * nq).astype(np.int64), nq - 1)
    quad = road_xy[qi].astype(np.float64)
    back = 0.5 * (quad[:, 0] + quad[:, 3])
    front = 0.5 * (quad[:, 1] + quad[:, 2])
    d = front - back
    heading = np.arctan2(d[:, 1], d[:, 0])
    nrm = np.stack([-np.sin(heading), np.cos(heading)], axis=1)
    side = np.where(u(1) < 0.5, -1.0, 1.0)
    pos = front + (side * (2.5 + u(2)))[:, None] * nrm
    xyzr = np.stack([pos[:, 0], pos[:, 1], 3.5 + 2.0 * u(3), 0.25 + 0.15 * u(4)], axis=1).astype(np.float32)
    st = u(5)
    color = np.where(st < 0.45, COLOR_SIGNAL_RED, np.where(st < 0.55, COLOR_SIGNAL_YELLOW, COLOR_SIGNAL_GREEN))
    return xyzr, color.astype(np.uint8)


def make_scene(seed: int, scene: int, n_agents: int, n_quads: int, n_static: int = 0,
               n_signals: int = 0) -> Scene:
    roads = road_network(seed, scene, n_quads)
    state, dims = place_agents(seed, scene, roads, n_agents)
    sc = Scene(agent_state=state, agent_dims=dims,
               agent_color=np.full(n_agents, COLOR_VEHICLE, dtype=np.uint8),
               road_xy=roads, road_color=np.full(n_quads, COLOR_ROAD, dtype=np.uint8))
    if n_static:
        sc.static_xyp, sc.static_dims = place_statics(seed, scene, roads, n_static)
        sc.static_color = np.full(n_static, COLOR_VEHICLE, dtype=np.uint8)   # agents and obstacles blue
    if n_signals:
        sc.signal_xyzr, sc.signal_color = place_signals(seed, scene, roads, n_signals)
    return sc


S_CROWD = 5


def crowded_scene(seed: int, n_agents: int = 24, n_roads: int = 40, radius: float = 25.0) -> Scene:
    """A dense test scene around agent 0 (at the origin): boxes in every
    orientation within `radius` m, some close enough to cross the near plane,
    some lower than the camera (top faces visible), and randomly oriented road
    strips that overlap each other."""
    a = np.arange(n_agents)
    u = lambda c: keyed_uniform(seed, S_CROWD, 0, a, c)
    r = radius * np.sqrt(u(0))
    th = 2 * math.pi * u(1)
    x = np.where(a == 0, 0.0, r * np.cos(th))
    y = np.where(a == 0, 0.0, r * np.sin(th))
    psi = 2 * math.pi * u(2) - math.pi
    L = 3.0 + 3.0 * u(3)
    W = 1.5 + 1.0 * u(4)
    H = 1.0 + 1.4 * u(5)
    v = 10.0 * u(6)
    state = np.stack([x, y, psi, v], axis=1).astype(np.float32)
    dims = np.stack([L, W, H], axis=1).astype(np.float32)
    q = np.arange(n_roads)
    ur = lambda c: keyed_uniform(seed, S_CROWD, 1, q, c)
    cx = 60.0 * ur(0) - 30.0
    cy = 60.0 * ur(1) - 30.0
    ang = 2 * math.pi * ur(2)
    half_len = 2.0 + 15.0 * ur(3)
    hw = LANE_WIDTH / 2
    dx, dy = np.cos(ang), np.sin(ang)
    nx, ny = -dy, dx
    roads = np.empty((n_roads, 4, 2))
    roads[:, 0] = np.stack([cx - half_len * dx - hw * nx, cy - half_len * dy - hw * ny], 1)
    roads[:, 1] = np.stack([cx + half_len * dx - hw * nx, cy + half_len * dy - hw * ny], 1)
    roads[:, 2] = np.stack([cx + half_len * dx + hw * nx, cy + half_len * dy + hw * ny], 1)
    roads[:, 3] = np.stack([cx - half_len * dx + hw * nx, cy - half_len * dy + hw * ny], 1)
    # a few strips wound clockwise (roads are two-sided)
    cw = ur(4) < 0.3
    roads[cw] = roads[cw][:, ::-1]
    acol = (COLOR_VEHICLE + (a % 3)).astype(np.uint8)        # distinct colours expose ties
    rcol = (COLOR_ROAD + 4 * (q % 2)).astype(np.uint8)
    return Scene(agent_state=state, agent_dims=dims, agent_color=acol,
                 road_xy=roads.astype(np.float32), road_color=rcol)


def mixed_palette() -> np.ndarray:
    """default_palette plus distinct colours for the crowded-scene indices."""
    pal = default_palette()
    pal[3] = (255, 0, 0)
    pal[4] = (0, 255, 0)
    pal[5] = (200, 200, 40)
    return pal


def uneven_counts(seed: int, n_scenes: int, agents=(4, 128), quads=(500, 8000)):
    """Per-scene (agents, quads) drawn uniformly from the inclusive integer ranges."""
    s = np.arange(n_scenes)
    ua = keyed_uniform(seed, S_SCENE, s, 0)
    uq = keyed_uniform(seed, S_SCENE, s, 1)
    na = agents[0] + np.minimum((ua * (agents[1] - agents[0] + 1)).astype(np.int64), agents[1] - agents[0])
    nq = quads[0] + np.minimum((uq * (quads[1] - quads[0] + 1)).astype(np.int64), quads[1] - quads[0])
    return na, nq


def actions(seed: int, step: int, scene_ids: np.ndarray, agent_ids: np.ndarray) -> np.ndarray:
    """Per-agent (accel, steer): accel ~ U(-3, 3) m/s^2, steer ~ U(-0.3, 0.3) rad.

    Keyed by (seed, step, scene, agent), so independent of batching.
    Returns float32 [n, 2].
    """
    u0 = keyed_uniform(seed, S_ACTION, step, scene_ids, agent_ids * 2)
    u1 = keyed_uniform(seed, S_ACTION, step, scene_ids, agent_ids * 2 + 1)
    return np.stack([6.0 * u0 - 3.0, 0.6 * u1 - 0.3], axis=1).astype(np.float32)


def batch_actions(seed: int, step: int, scenes: List[Scene]) -> np.ndarray:
    """Actions for every agent of a batch, in (scene, agent) order."""
    sid = np.concatenate([np.full(s.n_agents, i) for i, s in enumerate(scenes)])
    aid = np.concatenate([np.arange(s.n_agents) for s in scenes])
    return actions(seed, step, sid, aid)


# ---------------------------------------------------------------- workloads

SEEDS = {"small": 0x5EED0001, "uniform": 0x5EED0002, "uneven": 0x5EED0003,
         "sweep": 0x5EED0004, "serve": 0x5EED0005, "student": 0x5EED0006}


@dataclasses.dataclass
class Workload:
    name: str
    seed: int
    scenes: List[Scene]
    camera: Camera
    steps: int

    @property
    def n_agents(self) -> int:
        return sum(s.n_agents for s in self.scenes)

    @property
    def n_views(self) -> int:
        return self.n_agents * len(self.camera.cam_dirs)


def workload(name: str, resolution: int | None = None, n_scenes: int | None = None) -> Workload:
    """The five synthetic workloads (small / uniform / uneven / sweep / serve).

    small:   1 scene, 8 agents, 200 quads, 64x64, 10 steps
    uniform: 64 scenes x 32 agents, 2,000 quads, 128x128, 100 steps
    uneven:  256 scenes, agents U{4..128}, quads U{500..8000}, 3 cameras, 128x128
    sweep:   64 scenes x 64 agents, 4,000 quads, one camera at `resolution`
    serve:   pool of scenes with agents U{8..128}, quads U{500..8000}, 128x128
    student: 64 scenes x 32 agents, 2,000 quads, the 4-camera student rig at
             210x126 (resolution=210) or 434x252 (resolution=434)
    `n_scenes` truncates a workload (used for small samples of a large one).
    """
    seed = SEEDS[name]
    if name == "small":
        scenes = [make_scene(seed, 0, 8, 200)]
        cam, steps = camera_for(64), 10
    elif name == "uniform":
        n = 64 if n_scenes is None else n_scenes
        scenes = [make_scene(seed, s, 32, 2000) for s in range(n)]
        cam, steps = camera_for(128), 100
    elif name == "uneven":
        n = 256 if n_scenes is None else n_scenes
        na, nq = uneven_counts(seed, 256)
        scenes = [make_scene(seed, s, int(na[s]), int(nq[s])) for s in range(n)]
        cam, steps = camera_for(128, cams=FRONT_AND_SIDES), 100
    elif name == "sweep":
        n = 64 if n_scenes is None else n_scenes
        scenes = [make_scene(seed, s, 64, 4000) for s in range(n)]
        cam, steps = camera_for(128 if resolution is None else resolution), 100
    elif name == "serve":
        n = 64 if n_scenes is None else n_scenes
        na, nq = uneven_counts(seed, n, agents=(8, 128))
        scenes = [make_scene(seed, s, int(na[s]), int(nq[s])) for s in range(n)]
        cam, steps = camera_for(128), 100
    elif name == "student":
        n = 64 if n_scenes is None else n_scenes
        scenes = [make_scene(seed, s, 32, 2000) for s in range(n)]
        h = dict(STUDENT_RESOLUTIONS)[210 if resolution is None else resolution]
        w = 210 if resolution is None else resolution
        cam, steps = Camera(width=w, height=h, focal_px=w / 2.0, cam_dirs=STUDENT_RIG), 100
    else:
        raise KeyError(name)
    if n_scenes is not None and name == "small":
        scenes = scenes[:n_scenes]
    return Workload(name=name, seed=seed, scenes=scenes, camera=cam, steps=steps)
