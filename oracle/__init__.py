"""CPU oracle of the Gigapixel hot path (agent step + egocentric raster).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may use this package; the product path never does.  It
shares no code with the HIP library.  The arithmetic lives in gp_oracle.c
(plain C, binary32 with explicit fmaf, int64 coverage); this module only
compiles it with gcc and marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import concurrent.futures as _cf
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gp_oracle.c")
_LIB = os.path.join(_HERE, "libgp_oracle.so")
CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fPIC", "-shared", "-Wall"]

_lib = None


def build(force: bool = True) -> str:
    """Compile gp_oracle.c into libgp_oracle.so next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [("n_agents", C.c_int), ("n_roads", C.c_int),
                ("agent_state", C.c_void_p), ("agent_dims", C.c_void_p),
                ("agent_color", C.c_void_p), ("road_xy", C.c_void_p),
                ("road_color", C.c_void_p), ("n_static", C.c_int),
                ("static_xyp", C.c_void_p), ("static_dims", C.c_void_p),
                ("static_color", C.c_void_p), ("n_signals", C.c_int),
                ("signal_xyzr", C.c_void_p), ("signal_color", C.c_void_p)]


class _Camera(C.Structure):
    _fields_ = [("width", C.c_int), ("height", C.c_int),
                ("focal_px", C.c_float), ("cam_height", C.c_float),
                ("z_near", C.c_float), ("z_far", C.c_float),
                ("palette", C.c_void_p), ("shade", C.c_int), ("light", C.c_float * 3),
                ("ambient", C.c_float)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        L.gpo_sincos.argtypes = [C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.gpo_step.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float, C.c_void_p,
                               C.c_void_p]
        L.gpo_step_jerk.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_float,
                                    C.c_void_p, C.c_void_p]
        L.gpo_atan_small.argtypes = [C.c_float]
        L.gpo_atan_small.restype = C.c_float
        L.gpo_overlap.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gpo_in_strip.argtypes = [C.c_void_p, C.c_float, C.c_float]
        L.gpo_infractions.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_int, C.c_void_p, C.c_void_p]
        L.gpo_render_view.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_int, C.c_float,
                                      C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_longlong)]
        L.gpo_render_view.restype = C.c_longlong
        L.gpo_raycast_view.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_int, C.c_float,
                                       C.c_float, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        L.gpo_cover_tri.argtypes = [C.c_void_p, C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def sincos(t: float):
    s, c = C.c_float(), C.c_float()
    lib().gpo_sincos(C.c_float(t), C.byref(s), C.byref(c))
    return np.float32(s.value), np.float32(c.value)


def step(state: np.ndarray, dims: np.ndarray, act: np.ndarray, dt: float = 0.1, halted=None):
    """One kinematic step; returns (new_state [n,4], cos/sin psi [n,2]); inputs untouched.
    Agents flagged in `halted` (uint8 [n]) keep their state."""
    st = np.ascontiguousarray(state, dtype=np.float32).copy()
    dm = np.ascontiguousarray(dims, dtype=np.float32)
    ac = np.ascontiguousarray(act, dtype=np.float32)
    hl = None if halted is None else np.ascontiguousarray(halted, dtype=np.uint8)
    cs = np.empty((st.shape[0], 2), dtype=np.float32)
    lib().gpo_step(st.shape[0], _ptr(st), _ptr(dm), _ptr(ac), C.c_float(dt), _ptr(cs), _ptr(hl))
    return st, cs


def atan_small(x: float):
    """atan for |x| <= tan(0.5), the series the jerk step uses (binary32)."""
    return np.float32(lib().gpo_atan_small(C.c_float(x)))


def step_jerk(state: np.ndarray, dims: np.ndarray, actuators: np.ndarray, actions: np.ndarray,
              dt: float = 0.1, halted=None):
    """One jerk-actuated step (App. A, twelve discrete actions); returns
    (new_state [n,4], cos/sin psi [n,2], new_actuators [n,4] = a_lon, a_lat,
    steering, 0); inputs untouched.  Agents flagged in `halted` keep both."""
    st = np.ascontiguousarray(state, dtype=np.float32).copy()
    ac = np.ascontiguousarray(actuators, dtype=np.float32).copy()
    dm = np.ascontiguousarray(dims, dtype=np.float32)
    ix = np.ascontiguousarray(actions, dtype=np.uint8)
    hl = None if halted is None else np.ascontiguousarray(halted, dtype=np.uint8)
    assert st.shape[0] == ac.shape[0] == dm.shape[0] == ix.shape[0]
    cs = np.empty((st.shape[0], 2), dtype=np.float32)
    lib().gpo_step_jerk(st.shape[0], _ptr(st), _ptr(dm), _ptr(ac), _ptr(ix), C.c_float(dt), _ptr(cs), _ptr(hl))
    return st, cs, ac


def overlap(state_i, dims_i, state_j, dims_j) -> bool:
    """Footprints of two agents overlap with positive area (separating axes)."""
    a = [np.ascontiguousarray(x, dtype=np.float32) for x in (state_i, dims_i, state_j, dims_j)]
    return bool(lib().gpo_overlap(*[_ptr(x) for x in a]))


def in_strip(quad, px: float, py: float) -> bool:
    """The point lies in the road strip (on or inside each edge, either winding)."""
    q = np.ascontiguousarray(quad, dtype=np.float32).reshape(8)
    return bool(lib().gpo_in_strip(_ptr(q), C.c_float(px), C.c_float(py)))


def infractions(scene_state, dims, road_xy, halted, static_xyp=None, static_dims=None):
    """Collision / off-road check of one scene: returns (state with newly halted
    agents' speed zeroed, halted, flags) with flags bit 0 collision, bit 1
    off-road, bit 2 halted; inputs untouched.  static_xyp [k, 3] (x, y, psi)
    and static_dims [k, 3] are the scene's static obstacles."""
    st = np.ascontiguousarray(scene_state, dtype=np.float32).copy()
    dm = np.ascontiguousarray(dims, dtype=np.float32)
    rx = np.ascontiguousarray(road_xy, dtype=np.float32).reshape(-1, 8)
    hl = np.ascontiguousarray(halted, dtype=np.uint8).copy()
    fl = np.zeros(st.shape[0], dtype=np.uint8)
    sx = np.zeros((0, 3), np.float32) if static_xyp is None else np.ascontiguousarray(static_xyp, np.float32)
    sd = np.zeros((0, 3), np.float32) if static_dims is None else np.ascontiguousarray(static_dims, np.float32)
    assert sx.shape == sd.shape
    lib().gpo_infractions(st.shape[0], _ptr(st), _ptr(dm), rx.shape[0], _ptr(rx) if rx.size else None,
                          _ptr(hl), _ptr(fl), sx.shape[0], _ptr(sx) if sx.size else None,
                          _ptr(sd) if sd.size else None)
    return st, hl, fl


def scene_infractions(scene, state, halted):
    """infractions() of a scenegen.Scene-like object with the given agent state."""
    return infractions(state, scene.agent_dims, scene.road_xy, halted, *_statics(scene)[:2])


def _signals(scene):
    gx = getattr(scene, "signal_xyzr", None)
    if gx is None or len(gx) == 0:
        return None
    return scene.signal_xyzr, scene.signal_color


def _statics(scene):
    sx = getattr(scene, "static_xyp", None)
    if sx is None or len(sx) == 0:
        return None, None, None
    return scene.static_xyp, scene.static_dims, scene.static_color


def cover_tri(X, Y, W: int, H: int, count=None) -> np.ndarray:
    """Add the coverage of one snapped triangle (1/256 px units) to count [H, W] (uint8)."""
    x = np.ascontiguousarray(X, dtype=np.int32)
    y = np.ascontiguousarray(Y, dtype=np.int32)
    if count is None:
        count = np.zeros((H, W), dtype=np.uint8)
    lib().gpo_cover_tri(_ptr(x), _ptr(y), W, H, _ptr(count))
    return count


class View:
    """Output of one rendered view."""

    def __init__(self, rgb, depth, primid, n_tri, n_frag, key=None):
        self.rgb, self.depth, self.primid = rgb, depth, primid
        self.n_tri, self.n_frag = n_tri, n_frag
        self.key = key      # [H, W] uint64: each pixel's winning key (0 for background)


def render_view(state, dims, agent_color, road_xy, road_color, camera, palette,
                ego: int, cam_dir=(1.0, 0.0), light=None, statics=None, signals=None,
                backend: str = "raster") -> View:
    """Render one ego view.  `camera` has width, height, focal_px, cam_height, z_near, z_far.
    `light` = (lx, ly, lz, ambient) turns on directional shading (unit direction
    towards the light, world frame).  `statics` = (xyp [k, 3], dims [k, 3],
    colour [k]) are static obstacles, `signals` = (xyzr [g, 4], colour [g]) traffic lights.
    backend "raycast" casts one primary ray per pixel instead of rasterising."""
    st = np.ascontiguousarray(state, dtype=np.float32)
    dm = np.ascontiguousarray(dims, dtype=np.float32)
    ac = np.ascontiguousarray(agent_color, dtype=np.uint8)
    rx = np.ascontiguousarray(road_xy, dtype=np.float32).reshape(-1, 4, 2)
    rc = np.ascontiguousarray(road_color, dtype=np.uint8)
    pal = np.ascontiguousarray(palette, dtype=np.uint8).reshape(256, 3)
    sc = _Scene(st.shape[0], rx.shape[0], _ptr(st), _ptr(dm), _ptr(ac), _ptr(rx), _ptr(rc))
    if statics is not None and statics[0] is not None and len(statics[0]):
        sx = np.ascontiguousarray(statics[0], np.float32)
        sd = np.ascontiguousarray(statics[1], np.float32)
        scol = np.ascontiguousarray(statics[2], np.uint8)
        assert sx.shape == sd.shape == (scol.shape[0], 3)
        sc.n_static, sc.static_xyp, sc.static_dims, sc.static_color = sx.shape[0], _ptr(sx), _ptr(sd), _ptr(scol)
    if signals is not None and len(signals[0]):
        gx = np.ascontiguousarray(signals[0], np.float32)
        gc = np.ascontiguousarray(signals[1], np.uint8)
        assert gx.shape == (gc.shape[0], 4)
        sc.n_signals, sc.signal_xyzr, sc.signal_color = gx.shape[0], _ptr(gx), _ptr(gc)
    W, H = int(camera.width), int(camera.height)
    cm = _Camera(W, H, camera.focal_px, camera.cam_height, camera.z_near, camera.z_far, _ptr(pal))
    if light is not None:
        cm.shade = 1
        cm.light[0], cm.light[1], cm.light[2] = (float(np.float32(x)) for x in light[:3])
        cm.ambient = float(np.float32(light[3]))
    key = np.empty(H * W, dtype=np.uint64)
    rgb = np.empty((H, W, 3), dtype=np.uint8)
    depth = np.empty((H, W), dtype=np.float32)
    prim = np.empty((H, W), dtype=np.int32)
    nf = C.c_longlong(0)
    if backend == "raycast":
        lib().gpo_raycast_view(C.byref(sc), C.byref(cm), int(ego), C.c_float(cam_dir[0]), C.c_float(cam_dir[1]),
                               _ptr(key), _ptr(rgb), _ptr(depth), _ptr(prim))
        return View(rgb, depth, prim, -1, -1)
    if backend != "raster":
        raise ValueError(backend)
    nt = lib().gpo_render_view(C.byref(sc), C.byref(cm), int(ego), C.c_float(cam_dir[0]),
                               C.c_float(cam_dir[1]), _ptr(key), _ptr(rgb), _ptr(depth),
                               _ptr(prim), C.byref(nf))
    return View(rgb, depth, prim, int(nt), int(nf.value), key.reshape(H, W))


def render_scene_view(scene, camera, palette, ego: int, cam: int = 0, light=None, backend: str = "raster") -> View:
    """Render view (ego, cam) of a scenegen.Scene-like object."""
    return render_view(scene.agent_state, scene.agent_dims, scene.agent_color, scene.road_xy,
                       scene.road_color, camera, palette, ego, camera.cam_dirs[cam], light, _statics(scene),
                       _signals(scene), backend)


def render_views(items, camera, palette, threads: int = 1):
    """Render a list of (scene, ego, cam) items; threads > 1 runs views concurrently
    (ctypes releases the GIL during each call)."""
    fn = lambda it: render_scene_view(it[0], camera, palette, it[1], it[2])
    if threads <= 1:
        return [fn(it) for it in items]
    with _cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, items))
