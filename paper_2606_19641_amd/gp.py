"""Python binding of the Gigapixel C ABI (include/gp.h).

Argument marshalling only: torch supplies device memory and streams, and
every step of the path runs in the HIP library libgigapix.so.  There is no
CPU fallback: if the library is missing or no GPU is present the calls fail.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgigapix.so")

GP_OK, GP_EINVAL, GP_ENOMEM, GP_EDEVICE, GP_ESTATE = 0, -1, -2, -3, -4
SCHED_PLAIN, SCHED_PERSISTENT = 0, 1
RASTER_BANDED, RASTER_SPLIT, RASTER_CHIP = 0, 1, 2
MAX_CAMS = 4

EXPORTS = ("gp_sim_required_bytes", "gp_sim_create", "gp_sim_set_launch", "gp_sim_get_launch",
           "gp_sim_step", "gp_sim_render", "gp_sim_step_render_graph", "gp_sim_get_state",
           "gp_sim_set_state", "gp_sim_num_views", "gp_sim_num_agents", "gp_sim_num_scenes",
           "gp_sim_destroy", "gp_last_error", "gp_batch_required_bytes", "gp_batch_step_render",
           "gp_sim_check_infractions", "gp_sim_fork", "gp_sim_step_jerk", "gp_sim_get_actuators",
           "gp_sim_set_light", "gp_sim_set_signal_colors", "gp_sim_num_signals",
           "gp_sim_render_raycast")


class GpError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gp status {status}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("n_cams", C.c_int32),
                ("cam_dir", (C.c_float * 2) * MAX_CAMS), ("focal_px", C.c_float),
                ("cam_height", C.c_float), ("z_near", C.c_float), ("z_far", C.c_float),
                ("dt", C.c_float), ("palette", (C.c_uint8 * 3) * 256)]


class SceneDesc(C.Structure):
    _fields_ = [("n_agents", C.c_int32), ("n_roads", C.c_int32),
                ("agent_state", C.c_void_p), ("agent_dims", C.c_void_p),
                ("agent_color", C.c_void_p), ("road_xy", C.c_void_p), ("road_color", C.c_void_p),
                ("n_static", C.c_int32), ("static_xyp", C.c_void_p), ("static_dims", C.c_void_p),
                ("static_color", C.c_void_p), ("n_signals", C.c_int32), ("signal_xyzr", C.c_void_p),
                ("signal_color", C.c_void_p)]


class Launch(C.Structure):
    _fields_ = [("sched", C.c_int32), ("band_rows", C.c_int32), ("batch_tris", C.c_int32),
                ("block_threads", C.c_int32), ("blocks_per_cu", C.c_int32), ("raster", C.c_int32),
                ("view_waves", C.c_int32), ("road_wgs_per_cu", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load libgigapix.so (built by __graft_entry__.build / paper_2606_19641_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is missing: build it first "
                               "(python -m paper_2606_19641_amd.build)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.gp_sim_required_bytes.argtypes = [C.POINTER(Config), C.POINTER(SceneDesc), i32]
        L.gp_sim_required_bytes.restype = i64
        L.gp_sim_create.argtypes = [C.POINTER(Config), C.POINTER(SceneDesc), i32, vp, i64, vp,
                                    C.POINTER(vp)]
        L.gp_sim_set_launch.argtypes = [vp, C.POINTER(Launch)]
        L.gp_sim_get_launch.argtypes = [vp, C.POINTER(Launch)]
        L.gp_sim_step.argtypes = [vp, vp, vp]
        L.gp_sim_render.argtypes = [vp, vp, vp, vp, vp]
        L.gp_sim_step_render_graph.argtypes = [vp, vp, vp, vp]
        L.gp_sim_get_state.argtypes = [vp, vp, vp]
        L.gp_sim_set_state.argtypes = [vp, vp, vp]
        L.gp_sim_num_views.argtypes = [vp]
        L.gp_sim_num_views.restype = i64
        L.gp_sim_num_agents.argtypes = [vp]
        L.gp_sim_num_agents.restype = i64
        L.gp_sim_num_scenes.argtypes = [vp]
        L.gp_sim_num_scenes.restype = i32
        L.gp_sim_destroy.argtypes = [vp]
        L.gp_sim_destroy.restype = None
        L.gp_last_error.restype = C.c_char_p
        L.gp_batch_required_bytes.argtypes = [i32, i64, i64]
        L.gp_batch_required_bytes.restype = i64
        L.gp_batch_step_render.argtypes = [C.POINTER(vp), i32, C.POINTER(vp), C.POINTER(vp), vp, i64,
                                           vp, i64, vp]
        L.gp_sim_check_infractions.argtypes = [vp, vp, vp]
        L.gp_sim_fork.argtypes = [vp, vp, vp]
        L.gp_sim_step_jerk.argtypes = [vp, vp, vp]
        L.gp_sim_get_actuators.argtypes = [vp, vp, vp]
        L.gp_sim_set_light.argtypes = [vp, vp]
        L.gp_sim_set_signal_colors.argtypes = [vp, vp, vp]
        L.gp_sim_render_raycast.argtypes = [vp, vp, vp, vp, vp]
        L.gp_sim_render_noalloc.argtypes = [vp, vp, vp]
        L.gp_sim_num_signals.argtypes = [vp]
        L.gp_sim_num_signals.restype = C.c_int64
        for name in ("gp_sim_check_infractions", "gp_sim_fork", "gp_sim_step_jerk", "gp_sim_get_actuators",
                     "gp_sim_set_light", "gp_sim_set_signal_colors", "gp_sim_render_raycast", "gp_sim_render_noalloc",
                     "gp_batch_step_render", "gp_sim_create", "gp_sim_set_launch", "gp_sim_get_launch",
                     "gp_sim_step", "gp_sim_render", "gp_sim_step_render_graph", "gp_sim_get_state",
                     "gp_sim_set_state"):
            getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != GP_OK:
        raise GpError(status, lib().gp_last_error().decode(errors="replace"))


def make_config(camera, palette, dt: float = 0.1) -> Config:
    cfg = Config()
    cfg.width, cfg.height = int(camera.width), int(camera.height)
    dirs = list(camera.cam_dirs)
    if not 1 <= len(dirs) <= MAX_CAMS:
        raise ValueError("1..4 cameras")
    cfg.n_cams = len(dirs)
    for k, (c, s) in enumerate(dirs):
        cfg.cam_dir[k][0], cfg.cam_dir[k][1] = float(c), float(s)
    cfg.focal_px = float(camera.focal_px)
    cfg.cam_height = float(camera.cam_height)
    cfg.z_near, cfg.z_far = float(camera.z_near), float(camera.z_far)
    cfg.dt = float(dt)
    pal = np.ascontiguousarray(palette, dtype=np.uint8).reshape(256, 3)
    C.memmove(C.addressof(cfg.palette), pal.ctypes.data, 768)
    return cfg


def _stream_handle(stream) -> Optional[int]:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _scene_descs(scenes: Sequence):
    """ctypes scene descriptors plus the host arrays they point into."""
    keep = []
    descs = (SceneDesc * len(scenes))()
    for i, s in enumerate(scenes):
        st = np.ascontiguousarray(s.agent_state, dtype=np.float32)
        dm = np.ascontiguousarray(s.agent_dims, dtype=np.float32)
        ac = np.ascontiguousarray(s.agent_color, dtype=np.uint8)
        rx = np.ascontiguousarray(s.road_xy, dtype=np.float32)
        rc = np.ascontiguousarray(s.road_color, dtype=np.uint8)
        keep += [st, dm, ac, rx, rc]
        descs[i] = SceneDesc(st.shape[0], rx.shape[0] if rx.size else 0, st.ctypes.data,
                             dm.ctypes.data, ac.ctypes.data, rx.ctypes.data if rx.size else None,
                             rc.ctypes.data if rc.size else None)
        sx = getattr(s, "static_xyp", None)
        if sx is not None and len(sx):
            sx = np.ascontiguousarray(sx, dtype=np.float32)
            sd = np.ascontiguousarray(s.static_dims, dtype=np.float32)
            sc = np.ascontiguousarray(s.static_color, dtype=np.uint8)
            if sx.shape != (sc.shape[0], 3) or sd.shape != sx.shape:
                raise ValueError("static obstacles need xyp [k, 3], dims [k, 3], colour [k]")
            keep += [sx, sd, sc]
            descs[i].n_static = sx.shape[0]
            descs[i].static_xyp, descs[i].static_dims, descs[i].static_color = (
                sx.ctypes.data, sd.ctypes.data, sc.ctypes.data)
        gx = getattr(s, "signal_xyzr", None)
        if gx is not None and len(gx):
            gx = np.ascontiguousarray(gx, dtype=np.float32)
            gc = np.ascontiguousarray(s.signal_color, dtype=np.uint8)
            if gx.shape != (gc.shape[0], 4):
                raise ValueError("traffic lights need xyzr [g, 4] and colour [g]")
            keep += [gx, gc]
            descs[i].n_signals = gx.shape[0]
            descs[i].signal_xyzr, descs[i].signal_color = gx.ctypes.data, gc.ctypes.data
    return descs, keep


def required_bytes(scenes: Sequence, camera, palette, dt: float = 0.1) -> int:
    """Workspace bytes gp_sim_create needs for these scenes."""
    descs, _keep = _scene_descs(scenes)
    cfg = make_config(camera, palette, dt)
    n = lib().gp_sim_required_bytes(C.byref(cfg), descs, len(scenes))
    if n < 0:
        raise GpError(GP_EINVAL, lib().gp_last_error().decode())
    return int(n)


class Sim:
    """A batch of scenes resident on the GPU.  The workspace is allocated here
    unless a device uint8 tensor (256-byte aligned, large enough) is given."""

    def __init__(self, scenes: Sequence, camera, palette, dt: float = 0.1, device: str = "cuda",
                 stream=None, workspace=None):
        import torch
        self.camera = camera
        self.device = torch.device(device)
        descs, self._keep = _scene_descs(scenes)
        self.cfg = make_config(camera, palette, dt)
        L = lib()
        nbytes = L.gp_sim_required_bytes(C.byref(self.cfg), descs, len(scenes))
        if nbytes < 0:
            raise GpError(GP_EINVAL, L.gp_last_error().decode())
        with torch.cuda.device(self.device):
            if workspace is None:
                workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            elif workspace.numel() < nbytes:
                raise GpError(GP_ENOMEM, f"workspace has {workspace.numel()} bytes, {nbytes} needed")
            self.workspace = workspace
            h = C.c_void_p()
            _check(L.gp_sim_create(C.byref(self.cfg), descs, len(scenes), self.workspace.data_ptr(),
                                   int(nbytes), _stream_handle(stream), C.byref(h)))
        self._h = h
        self._keep = []
        self.n_views = int(L.gp_sim_num_views(h))
        self.n_agents = int(L.gp_sim_num_agents(h))
        self.n_scenes = int(L.gp_sim_num_scenes(h))
        self.workspace_bytes = int(nbytes)
        self.light = None
        self.scene_shapes = tuple((int(getattr(s, "n_agents", 0)), int(getattr(s, "n_roads", 0)),
                                   int(getattr(s, "n_static", 0)), int(getattr(s, "n_signals", 0)))
                                  for s in scenes)

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            lib().gp_sim_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- launch settings
    def get_launch(self) -> dict:
        l = Launch()
        _check(lib().gp_sim_get_launch(self._h, C.byref(l)))
        return l.as_dict()

    def set_launch(self, **kw):
        cur = self.get_launch()
        cur.update(kw)
        l = Launch(**cur)
        _check(lib().gp_sim_set_launch(self._h, C.byref(l)))

    # -- outputs
    def new_rgb(self):
        import torch
        return torch.empty((self.n_views, self.camera.height, self.camera.width, 3),
                           dtype=torch.uint8, device=self.device)

    def step(self, actions, stream=None):
        """actions: float32 [n_agents, 2] device tensor (accel, steer)."""
        self._check_tensor(actions, (self.n_agents, 2), "float32")
        _check(lib().gp_sim_step(self._h, actions.data_ptr(), _stream_handle(stream)))

    def step_jerk(self, actions, stream=None):
        """actions: uint8 [n_agents] device tensor of jerk-action indices 0..11
        (3 * longitudinal + lateral; larger indices coast)."""
        self._check_tensor(actions, (self.n_agents,), "uint8")
        _check(lib().gp_sim_step_jerk(self._h, actions.data_ptr(), _stream_handle(stream)))

    @property
    def n_signals(self) -> int:
        return int(lib().gp_sim_num_signals(self._h))

    def set_signal_colors(self, colors, stream=None):
        """colors: uint8 [n_signals] device tensor, the palette index of every light's state."""
        self._check_tensor(colors, (self.n_signals,), "uint8")
        _check(lib().gp_sim_set_signal_colors(self._h, colors.data_ptr(), _stream_handle(stream)))

    def render_raycast(self, rgb=None, depth=False, primid=False, stream=None):
        """Render every view with the ray-cast backend; returns (rgb, depth or None, primid or None)."""
        import torch
        rgb = self.new_rgb() if rgb is None else rgb
        self._check_tensor(rgb, (self.n_views, self.camera.height, self.camera.width, 3), "uint8")
        shp = (self.n_views, self.camera.height, self.camera.width)
        d = torch.empty(shp, dtype=torch.float32, device=self.device) if depth is True else (depth or None)
        p = torch.empty(shp, dtype=torch.int32, device=self.device) if primid is True else (primid or None)
        _check(lib().gp_sim_render_raycast(self._h, rgb.data_ptr(), d.data_ptr() if d is not None else None,
                                           p.data_ptr() if p is not None else None, _stream_handle(stream)))
        return rgb, d, p

    def set_light(self, light=None):
        """light = (lx, ly, lz, ambient): unit direction towards the light (world
        frame) and ambient term; None turns shading off."""
        if light is None:
            _check(lib().gp_sim_set_light(self._h, None))
            self.light = None
            return
        arr = (C.c_float * 4)(*[float(x) for x in light])
        _check(lib().gp_sim_set_light(self._h, C.cast(arr, C.c_void_p)))
        self.light = tuple(float(x) for x in light)

    def get_actuators(self, stream=None):
        """float32 [n_agents, 4]: longitudinal and lateral acceleration, steering angle, 0."""
        import torch
        out = torch.empty((self.n_agents, 4), dtype=torch.float32, device=self.device)
        _check(lib().gp_sim_get_actuators(self._h, out.data_ptr(), _stream_handle(stream)))
        return out

    def render(self, rgb=None, depth=False, primid=False, stream=None):
        """Render every view; returns (rgb, depth or None, primid or None)."""
        import torch
        rgb = self.new_rgb() if rgb is None else rgb
        self._check_tensor(rgb, (self.n_views, self.camera.height, self.camera.width, 3), "uint8")
        shp = (self.n_views, self.camera.height, self.camera.width)
        d = torch.empty(shp, dtype=torch.float32, device=self.device) if depth is True else (depth or None)
        p = torch.empty(shp, dtype=torch.int32, device=self.device) if primid is True else (primid or None)
        _check(lib().gp_sim_render(self._h, rgb.data_ptr(), d.data_ptr() if d is not None else None,
                                   p.data_ptr() if p is not None else None, _stream_handle(stream)))
        return rgb, d, p

    def render_noalloc(self, rgb=None, stream=None):
        """rgb render whose scratch is the library's static device array (no
        allocation in the call); returns rgb."""
        rgb = self.new_rgb() if rgb is None else rgb
        self._check_tensor(rgb, (self.n_views, self.camera.height, self.camera.width, 3), "uint8")
        _check(lib().gp_sim_render_noalloc(self._h, rgb.data_ptr(), _stream_handle(stream)))
        return rgb

    def step_render_graph(self, actions, rgb, stream=None):
        self._check_tensor(actions, (self.n_agents, 2), "float32")
        self._check_tensor(rgb, (self.n_views, self.camera.height, self.camera.width, 3), "uint8")
        _check(lib().gp_sim_step_render_graph(self._h, actions.data_ptr(), rgb.data_ptr(),
                                              _stream_handle(stream)))

    def get_state(self, stream=None):
        import torch
        out = torch.empty((self.n_agents, 4), dtype=torch.float32, device=self.device)
        _check(lib().gp_sim_get_state(self._h, out.data_ptr(), _stream_handle(stream)))
        return out

    def set_state(self, state, stream=None):
        self._check_tensor(state, (self.n_agents, 4), "float32")
        _check(lib().gp_sim_set_state(self._h, state.data_ptr(), _stream_handle(stream)))

    def check_infractions(self, flags=None, stream=None):
        """Collision / off-road check; halts offenders.  Returns uint8 flags
        [n_agents]: bit 0 collision, bit 1 off-road, bit 2 halted."""
        import torch
        if flags is None:
            flags = torch.empty(self.n_agents, dtype=torch.uint8, device=self.device)
        self._check_tensor(flags, (self.n_agents,), "uint8")
        _check(lib().gp_sim_check_infractions(self._h, flags.data_ptr(), _stream_handle(stream)))
        return flags

    def fork_from(self, src: "Sim", stream=None):
        """Copy src's agent state, heading cosines, halted flags and jerk actuators into this sim."""
        _check(lib().gp_sim_fork(self._h, src._h, _stream_handle(stream)))

    def _check_tensor(self, t, shape, dtype):
        import torch
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("expected a device tensor")
        if tuple(t.shape) != tuple(shape) or str(t.dtype) != f"torch.{dtype}" or not t.is_contiguous():
            raise ValueError(f"expected contiguous {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


def view_index(scenes, scene: int, agent: int, cam: int, n_cams: int) -> int:
    """Image index of (scene, agent, camera) in the (scene, agent, camera) order."""
    base = sum(s.n_agents for s in scenes[:scene])
    return (base + agent) * n_cams + cam


def batch_required_bytes(sims: Sequence["Sim"]) -> int:
    n = lib().gp_batch_required_bytes(len(sims), sum(x.n_agents for x in sims), sum(x.n_views for x in sims))
    if n < 0:
        raise GpError(GP_EINVAL, lib().gp_last_error().decode())
    return int(n)


def batch_step_render(sims: Sequence["Sim"], actions: Sequence[np.ndarray], rgbs, ws, staging,
                      stream=None):
    """One step + rgb render of every sim in one batched launch (serving).

    actions[k]: host float32 [n_agents_k, 2]; rgbs[k]: device uint8 images of
    sim k; ws: device uint8 tensor, staging: pinned host uint8 tensor, both at
    least batch_required_bytes(sims).  The caller keeps ws / staging untouched
    until the stream has passed this call."""
    n = len(sims)
    if not (len(actions) == len(rgbs) == n):
        raise ValueError("one action array and one image tensor per sim")
    acts = [np.ascontiguousarray(a, dtype=np.float32) for a in actions]
    for a, sim, rgb in zip(acts, sims, rgbs):
        if a.shape != (sim.n_agents, 2):
            raise ValueError(f"actions must be [{sim.n_agents}, 2], got {a.shape}")
        sim._check_tensor(rgb, (sim.n_views, sim.camera.height, sim.camera.width, 3), "uint8")
    hs = (C.c_void_p * n)(*[x._h.value for x in sims])
    ha = (C.c_void_p * n)(*[a.ctypes.data for a in acts])
    hr = (C.c_void_p * n)(*[r.data_ptr() for r in rgbs])
    _check(lib().gp_batch_step_render(hs, n, ha, hr, ws.data_ptr(), ws.numel(), staging.data_ptr(),
                                      staging.numel(), _stream_handle(stream)))
