"""Independent float64 ray caster used to pin the oracle's raster.

Written from the geometry, not from the oracle: one ray per pixel centre,
slab intersection with each cuboid in its own frame (only rays that enter a
box from outside count, which is what culling back faces means), and the
z = 0 plane with a point-in-quad test for the road strips.  The ray
parameter equals the planar camera depth, so the near/far interval applies to
it directly.

For each pixel it also reports whether the pixel is ambiguous for a raster
with snapped vertices: an edge passes close to the sample (detected by four
jittered rays at (+-delta, +-delta) px), a hit lies near the near or far
plane, the two nearest hits have nearly equal depth, or the ray grazes the
hit face.
"""
from __future__ import annotations

import math

import numpy as np


def _camera(state, ego, cam_dir):
    x, y, psi = (float(v) for v in state[ego, :3])
    ck, sk = float(cam_dir[0]), float(cam_dir[1])
    yaw = math.atan2(math.sin(psi) * ck + math.cos(psi) * sk, math.cos(psi) * ck - math.sin(psi) * sk)
    fwd = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    right = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    up = np.array([0.0, 0.0, 1.0])
    return np.array([x, y]), fwd, right, up


def _rays(cam, ox, oy):
    """World directions of pixel rays with camera-space direction (u, -v, 1)."""
    W, H, f = cam.width, cam.height, float(cam.focal_px)
    i, j = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    u = (i + 0.5 + ox - W / 2.0) / f
    v = (j + 0.5 + oy - H / 2.0) / f
    return u, -v


def _cast(scene, cam, palette, ego, cam_dir, ox=0.0, oy=0.0, with_flags=False):
    st = np.asarray(scene.agent_state, dtype=np.float64)
    dm = np.asarray(scene.agent_dims, dtype=np.float64)
    roads = np.asarray(scene.road_xy, dtype=np.float64).reshape(-1, 4, 2)
    na = st.shape[0]
    pos, fwd, right, up = _camera(st, ego, cam_dir)
    hcam = float(cam.cam_height)
    ru, rv = _rays(cam, ox, oy)
    # world ray: origin (pos, hcam), direction d = ru*right + rv*up + fwd; parameter = depth
    dx = ru * right[0] + fwd[0]
    dy = ru * right[1] + fwd[1]
    dz = rv
    shape = ru.shape
    zn, zf = float(cam.z_near), float(cam.z_far)
    best_t = np.full(shape, np.inf)
    best_cls = np.full(shape, -1)
    best_prim = np.full(shape, -1, dtype=np.int64)
    second_t = np.full(shape, np.inf)
    graze = np.zeros(shape, dtype=bool)
    near_plane = np.zeros(shape, dtype=bool)
    dnorm = np.sqrt(dx * dx + dy * dy + dz * dz)

    def offer(t, hit, cls, prim, cosang):
        nonlocal best_t, best_cls, best_prim, second_t, graze
        hit = hit & (t >= zn) & (t <= zf)
        near_plane[...] |= hit & ((np.abs(t - zn) <= 1e-4 * zn) | (np.abs(t - zf) <= 1e-4 * zf))
        # ordering: smaller depth, then higher class, then lower primitive index
        better = hit & ((t < best_t) | ((t == best_t) & ((cls > best_cls) | ((cls == best_cls) & (prim < best_prim)))))
        # the runner-up depth among distinct primitives for tie detection
        second_t = np.where(better, np.minimum(second_t, best_t), np.where(hit, np.minimum(second_t, t), second_t))
        graze = np.where(better, np.abs(cosang) < 1e-3, graze)
        best_t = np.where(better, t, best_t)
        best_cls = np.where(better, cls, best_cls)
        best_prim = np.where(better, prim, best_prim)

    for j in range(na):
        if j == ego:
            continue
        bx, by, psi = st[j, 0], st[j, 1], st[j, 2]
        L, Wd, Hb = dm[j]
        c, s = math.cos(psi), math.sin(psi)
        # ray in the box frame (a along heading, b to the left, z up; origin at box centre)
        px, py, pz = pos[0] - bx, pos[1] - by, hcam - Hb / 2.0
        oa, ob, oz = px * c + py * s, -px * s + py * c, pz
        da, db = dx * c + dy * s, -dx * s + dy * c
        half = (L / 2.0, Wd / 2.0, Hb / 2.0)
        o = (oa, ob, oz)
        dd = (da, db, dz)
        t_in = np.full(shape, -np.inf)
        t_out = np.full(shape, np.inf)
        face = np.full(shape, -1)
        # axis a: +a face 0 (front), -a face 2 (back); axis b: +b face 1, -b face 3; z: top 4, bottom 5
        faces = ((0, 2), (1, 3), (4, 5))
        for ax in range(3):
            with np.errstate(divide="ignore", invalid="ignore"):
                t1 = (-half[ax] - o[ax]) / dd[ax]
                t2 = (half[ax] - o[ax]) / dd[ax]
            # entering through the -side if d > 0, through the +side if d < 0
            enter = np.where(dd[ax] > 0, t1, t2)
            leave = np.where(dd[ax] > 0, t2, t1)
            par = dd[ax] == 0
            inside_slab = np.abs(o[ax]) < half[ax]
            enter = np.where(par, np.where(inside_slab, -np.inf, np.inf), enter)
            leave = np.where(par, np.where(inside_slab, np.inf, -np.inf), leave)
            fid = np.where(dd[ax] > 0, faces[ax][1], faces[ax][0])
            upd = enter > t_in
            face = np.where(upd, fid, face)
            t_in = np.maximum(t_in, enter)
            t_out = np.minimum(t_out, leave)
        hit = (t_in <= t_out) & (t_in > 0) & np.isfinite(t_in)
        # cosine between the ray and the entered face normal
        nrm = {0: (c, s, 0.0), 2: (-c, -s, 0.0), 1: (-s, c, 0.0), 3: (s, -c, 0.0), 4: (0.0, 0.0, 1.0), 5: (0.0, 0.0, -1.0)}
        cosang = np.zeros(shape)
        for fi, n in nrm.items():
            m = face == fi
            cosang = np.where(m, (dx * n[0] + dy * n[1] + dz * n[2]) / dnorm, cosang)
        offer(np.where(hit, t_in, np.inf), hit, 1, 6 * j + face, cosang)

    # road plane z = 0 (two-sided)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = -hcam / dz
    down = dz < 0
    hx = pos[0] + t * dx
    hy = pos[1] + t * dy
    cosang = dz / dnorm
    # all strips share the plane, so the lowest covering index is the road candidate
    first_road = np.full(shape, -1, dtype=np.int64)
    for r in range(roads.shape[0]):
        q = roads[r]
        # point in convex quad of either orientation: all edge cross products share a sign
        cr = []
        for k in range(4):
            ax_, ay_ = q[k]
            bx_, by_ = q[(k + 1) % 4]
            cr.append((bx_ - ax_) * (hy - ay_) - (by_ - ay_) * (hx - ax_))
        cr = np.stack(cr)
        inside = np.all(cr > 0, axis=0) | np.all(cr < 0, axis=0)
        first_road = np.where(down & inside & (first_road < 0), r, first_road)
    hit = first_road >= 0
    offer(np.where(hit, t, np.inf), hit, 0, 6 * na + first_road, cosang)

    colour_idx = np.zeros(shape, dtype=np.int64)
    isbox = best_prim >= 0
    isbox_cls = isbox & (best_cls == 1)
    isroad = isbox & (best_cls == 0)
    ac = np.asarray(scene.agent_color).astype(np.int64)
    rc = np.asarray(scene.road_color).astype(np.int64)
    colour_idx[isbox_cls] = ac[best_prim[isbox_cls] // 6]
    colour_idx[isroad] = rc[best_prim[isroad] - 6 * na]
    rgb = np.asarray(palette)[colour_idx]
    depth = np.where(isbox, best_t, np.inf)
    prim = np.where(isbox, best_prim, -1)
    if not with_flags:
        return rgb, depth, prim
    with np.errstate(invalid="ignore"):
        tie = np.isfinite(second_t) & (np.abs(second_t - best_t) <= 1e-5 * best_t)
    return rgb, depth, prim, graze | near_plane | tie


def raycast(scene, cam, palette, ego, cam_index=0, delta=0.05):
    """Return (rgb, depth, primid, ambiguous) for one view; delta in pixels."""
    cam_dir = cam.cam_dirs[cam_index]
    rgb, depth, prim, amb = _cast(scene, cam, palette, ego, cam_dir, with_flags=True)
    for sx in (-delta, delta):
        for sy in (-delta, delta):
            _, d2, p2, a2 = _cast(scene, cam, palette, ego, cam_dir, sx, sy, with_flags=True)
            amb |= (p2 != prim) | a2
    return rgb, depth, prim, amb
