"""Oracle pins for traffic lights (Sec. 3.1: traffic lights are small spheres).

Against float64 geometry written here from the ray-sphere definition: for
every pixel sample, the ray through it meets the sphere iff the centre's
distance to the ray is below r, and the visible point is the near
intersection; pixels within 1e-4 r of tangency (or 1e-4 m of the near / far
plane) are ambiguous in binary32 and skipped.  Plus the on-axis closed form
(a disc of half-angle asin(r / Z)), occlusion against a box, near-plane
clipping, numbering after the roads, and unlit (emissive) colours."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g


def _lone_ego(x=0.0, y=0.0, psi=0.0):
    return g.Scene(agent_state=np.array([[x, y, psi, 0.0]], np.float32),
                   agent_dims=np.array([[4.5, 2.0, 1.6]], np.float32), agent_color=np.array([2], np.uint8),
                   road_xy=np.zeros((0, 4, 2), np.float32), road_color=np.zeros(0, np.uint8))


def _float64_spheres(cam, ego_xy, psi, spheres):
    """(prim index into spheres or -1, depth) per pixel by float64 ray casting."""
    W, H, f = cam.width, cam.height, cam.focal_px
    cx, cy = 0.5 * W, 0.5 * H
    fx, fy = math.cos(psi), math.sin(psi)
    best = np.full((H, W), np.inf)
    idx = np.full((H, W), -1)
    amb = np.zeros((H, W), bool)
    for k, (x, y, z, r) in enumerate(spheres):
        dx, dy = x - ego_xy[0], y - ego_xy[1]
        c = np.array([dx * fy - dy * fx, z - cam.cam_height, dx * fx + dy * fy])   # right, up, forward
        for j in range(H):
            for i in range(W):
                D = np.array([i + 0.5 - cx, cy - (j + 0.5), f])
                s0 = D @ c / (D @ D)
                w = c - s0 * D
                dist = math.sqrt(w @ w)
                if abs(dist - r) < 1e-4 * r:
                    amb[j, i] = True
                    continue
                if dist >= r:
                    continue
                z_hit = (s0 - math.sqrt((r * r - w @ w) / (D @ D))) * f
                if abs(z_hit - cam.z_near) < 1e-4 or abs(z_hit - cam.z_far) < 1e-4:
                    amb[j, i] = True
                    continue
                if cam.z_near <= z_hit <= cam.z_far and z_hit < best[j, i]:
                    best[j, i], idx[j, i] = z_hit, k
    return idx, best, amb


@pytest.mark.parametrize("seed", range(3))
def test_spheres_match_float64_ray_casting(seed):
    rng = np.random.default_rng(seed)
    cam = g.camera_for(40)
    sc = _lone_ego(psi=float(rng.uniform(-3, 3)))
    n = 6
    fwd = np.array([math.cos(sc.agent_state[0, 2]), math.sin(sc.agent_state[0, 2])])
    side = np.array([-fwd[1], fwd[0]])
    spheres = []
    for _ in range(n):
        dist = rng.uniform(1.0, 30.0)
        p = dist * fwd + rng.uniform(-0.6, 0.6) * dist * side
        spheres.append((p[0], p[1], rng.uniform(0.5, 4.0), rng.uniform(0.3, 2.5)))
    sc.signal_xyzr = np.array(spheres, np.float32)
    sc.signal_color = np.array([6, 7, 8, 6, 7, 8], np.uint8)
    v = oracle.render_scene_view(sc, cam, g.default_palette(), 0, 0)
    sp = [tuple(float(x) for x in s) for s in sc.signal_xyzr]
    idx, depth, amb = _float64_spheres(cam, (0.0, 0.0), float(sc.agent_state[0, 2]), sp)
    sig0 = 6 * 1 + 0
    got = np.where(v.primid >= 0, v.primid - sig0, -1)
    ok = ~amb
    assert np.array_equal(got[ok], idx[ok])
    hit = ok & (idx >= 0)
    assert hit.sum() > 50
    assert np.allclose(v.depth[hit], depth[hit], rtol=1e-5)
    pal = g.default_palette()
    assert np.array_equal(v.rgb[hit], pal[sc.signal_color[idx[hit]]])


def test_sphere_on_the_axis_is_a_disc_of_half_angle_asin_r_over_z():
    cam = g.camera_for(64)
    for Z, r in ((10.0, 1.0), (6.0, 2.5), (40.0, 3.0)):
        sc = _lone_ego()
        sc.signal_xyzr = np.array([[Z, 0.0, cam.cam_height, r]], np.float32)
        sc.signal_color = np.array([6], np.uint8)
        v = oracle.render_scene_view(sc, cam, g.default_palette(), 0, 0)
        tan2 = r * r / (Z * Z - r * r)
        W = cam.width
        a = np.arange(W) + 0.5 - W / 2
        rho2 = (a[None, :] ** 2 + a[:, None] ** 2) / cam.focal_px ** 2
        inside = rho2 < tan2 * (1 - 1e-5)
        outside = rho2 > tan2 * (1 + 1e-5)
        cov = v.primid >= 0
        assert np.all(cov[inside]) and not np.any(cov[outside]), (Z, r)
        # depth at a centre pixel, whose ray makes the angle t with the axis,
        # tan t = sqrt(0.5) / f: near hit Z cos t - sqrt(r^2 - Z^2 sin^2 t) along
        # the ray, planar depth that times cos t
        c = W // 2
        t = math.atan(math.sqrt(0.5) / cam.focal_px)
        z = (Z * math.cos(t) - math.sqrt(r * r - (Z * math.sin(t)) ** 2)) * math.cos(t)
        assert v.depth[c, c] == pytest.approx(z, rel=1e-5)


def test_occlusion_with_boxes_and_the_near_plane():
    cam = g.camera_for(48)
    pal = g.default_palette()
    # a box 8 m ahead, a light in front of it and one behind it, both at box height
    sc = g.Scene(agent_state=np.array([[0, 0, 0, 0], [8, 0, 0, 0]], np.float32),
                 agent_dims=np.array([[4.5, 2, 1.6], [4.5, 2.0, 2.0]], np.float32),
                 agent_color=np.array([2, 2], np.uint8), road_xy=np.zeros((0, 4, 2), np.float32),
                 road_color=np.zeros(0, np.uint8))
    sc.signal_xyzr = np.array([[4.0, 0.0, 1.0, 0.4], [14.0, 0.0, 1.0, 0.6]], np.float32)
    sc.signal_color = np.array([6, 8], np.uint8)
    v = oracle.render_scene_view(sc, cam, pal, 0, 0)
    sig0 = 12
    assert np.any(v.primid == sig0)                   # the near light shows
    assert not np.any(v.primid == sig0 + 1)           # the far one is behind the box
    # a light cut by the near plane (centre 0.3 m ahead, r 0.4): its near part
    # is clipped, nothing behind shows through; a light behind the camera: nothing
    sc2 = _lone_ego()
    sc2.signal_xyzr = np.array([[0.3, 0.0, 1.6, 0.4], [-5.0, 0.0, 1.6, 1.0]], np.float32)
    sc2.signal_color = np.array([6, 6], np.uint8)
    v2 = oracle.render_scene_view(sc2, cam, pal, 0, 0)
    assert not np.any(v2.primid >= 0)


def test_numbering_after_roads_and_lights_are_unlit():
    sc = g.make_scene(0x5EED0002, 2, 10, 600, n_static=10, n_signals=40)
    cam = g.camera_for(64, cams=g.FRONT_AND_SIDES)
    pal = g.default_palette()
    sig0 = 6 * (sc.n_agents + sc.n_static) + sc.n_roads
    seen = 0
    for ego in range(sc.n_agents):
        for c in range(3):
            flat = oracle.render_scene_view(sc, cam, pal, ego, c)
            lit = oracle.render_scene_view(sc, cam, pal, ego, c, light=(0.0, 0.0, 1.0, 0.0))
            m = flat.primid >= sig0
            seen += int(m.sum())
            assert np.all(flat.primid[m] < sig0 + sc.n_signals)
            assert np.array_equal(lit.rgb[m], flat.rgb[m])
            assert np.array_equal(flat.rgb[m], pal[sc.signal_color[flat.primid[m] - sig0]])
    assert seen > 20
