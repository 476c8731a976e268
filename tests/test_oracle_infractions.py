"""Oracle pins for the infraction check (collision, off-road, halting; App. A).

Collision is checked against an independent float64 construction (the
intersection polygon of the two footprints by convex clipping, and the
distance between them), off-road against point-in-rectangle closed forms and
the scene generator's placement (agents start on lane centrelines)."""
import math

import numpy as np
import pytest

import oracle
from paper_2606_19641_amd import scenegen as g


def _box(x, y, psi, L=4.0, W=2.0):
    return np.array([x, y, psi, 0.0], np.float32), np.array([L, W, 1.5], np.float32)


def _corners64(x, y, psi, L, W):
    c, s = math.cos(psi), math.sin(psi)
    out = []
    for a, b in ((1, 1), (-1, 1), (-1, -1), (1, -1)):
        out.append((x + a * L / 2 * c - b * W / 2 * s, y + a * L / 2 * s + b * W / 2 * c))
    return out


def _clip_area(p, q):
    """Area of convex polygon p clipped by convex polygon q (both CCW), float64."""
    def inside(pt, a, b):
        return (b[0] - a[0]) * (pt[1] - a[1]) - (b[1] - a[1]) * (pt[0] - a[0]) >= 0

    def cut(a, b, c, d):
        x1, y1, x2, y2, x3, y3, x4, y4 = *a, *b, *c, *d
        den = (x1 - x2) * (y3 - y4) - (y1 - y2) * (x3 - x4)
        t = ((x1 - x3) * (y3 - y4) - (y1 - y3) * (x3 - x4)) / den
        return (x1 + t * (x2 - x1), y1 + t * (y2 - y1))

    out = list(p)
    for i in range(len(q)):
        a, b = q[i], q[(i + 1) % len(q)]
        inp, out = out, []
        for k in range(len(inp)):
            cur, prev = inp[k], inp[k - 1]
            if inside(cur, a, b):
                if not inside(prev, a, b):
                    out.append(cut(prev, cur, a, b))
                out.append(cur)
            elif inside(prev, a, b):
                out.append(cut(prev, cur, a, b))
        if not out:
            return 0.0
    return 0.5 * abs(sum(out[k][0] * out[k - 1][1] - out[k - 1][0] * out[k][1] for k in range(len(out))))


def _seg_dist(p, a, b):
    ax, ay = b[0] - a[0], b[1] - a[1]
    t = max(0.0, min(1.0, ((p[0] - a[0]) * ax + (p[1] - a[1]) * ay) / (ax * ax + ay * ay)))
    return math.hypot(p[0] - a[0] - t * ax, p[1] - a[1] - t * ay)


def _poly_dist(p, q):
    d = min(_seg_dist(v, q[k], q[(k + 1) % 4]) for v in p for k in range(4))
    return min(d, min(_seg_dist(v, p[k], p[(k + 1) % 4]) for v in q for k in range(4)))


def test_axis_aligned_overlap_gap_and_touch():
    a = _box(0.0, 0.0, 0.0)
    assert oracle.overlap(*a, *_box(3.9, 0.0, 0.0))
    assert not oracle.overlap(*a, *_box(4.1, 0.0, 0.0))
    assert not oracle.overlap(*a, *_box(4.0, 0.0, 0.0))          # touching is not a collision
    assert oracle.overlap(*a, *_box(0.0, 1.9, 0.0))
    assert not oracle.overlap(*a, *_box(0.0, 2.0, 0.0))
    assert oracle.overlap(*a, *_box(0.0, 0.0, 1.0))              # concentric, any heading


def test_rotated_corner_cases():
    # a 45-degree box whose corner reaches 0.1 m into / stops 0.1 m short of a box's side
    d = math.sqrt(2.0)          # half diagonal of a 2 x 2 square
    sq = dict(L=2.0, W=2.0)
    a = _box(0.0, 0.0, 0.0, **sq)
    assert oracle.overlap(*a, *_box(1.0 + d - 0.1, 0.0, math.pi / 4, **sq))
    assert not oracle.overlap(*a, *_box(1.0 + d + 0.1, 0.0, math.pi / 4, **sq))


@pytest.mark.parametrize("seed", range(4))
def test_random_pairs_match_float64_polygon_geometry(seed):
    rng = np.random.default_rng(seed)
    checked = 0
    for _ in range(1500):
        xi, yi, xj, yj = rng.uniform(-4, 4, 4)
        pi_, pj = rng.uniform(-math.pi, math.pi, 2)
        Li, Lj = rng.uniform(3.5, 6.0, 2)
        Wi, Wj = rng.uniform(1.6, 2.6, 2)
        si, di = _box(xi, yi, pi_, Li, Wi)
        sj, dj = _box(xj, yj, pj, Lj, Wj)
        got = oracle.overlap(si, di, sj, dj)
        assert got == oracle.overlap(sj, dj, si, di)                    # symmetric
        P = _corners64(*map(float, (si[0], si[1], si[2], di[0], di[1])))
        Q = _corners64(*map(float, (sj[0], sj[1], sj[2], dj[0], dj[1])))
        area = _clip_area(P, Q)
        if area > 1e-3:
            assert got, (xi, yi, pi_, xj, yj, pj)
            checked += 1
        elif area == 0.0 and _poly_dist(P, Q) > 1e-3:
            assert not got, (xi, yi, pi_, xj, yj, pj)
            checked += 1
    assert checked > 1400


def test_in_strip_closed_forms_and_windings():
    ccw = np.array([[0, 0], [2, 0], [2, 1], [0, 1]], np.float32)
    for q in (ccw, ccw[::-1].copy()):
        assert oracle.in_strip(q, 1.0, 0.5)
        assert oracle.in_strip(q, 0.0, 0.5) and oracle.in_strip(q, 2.0, 1.0)   # edge, vertex: inside
        assert not oracle.in_strip(q, 2.01, 0.5) and not oracle.in_strip(q, 1.0, -0.01)
    # a rotated strip
    c, s = math.cos(0.7), math.sin(0.7)
    rot = np.array([[x * c - y * s, x * s + y * c] for x, y in ccw], np.float32)
    px, py = 1.0 * c - 0.5 * s, 1.0 * s + 0.5 * c
    assert oracle.in_strip(rot, px, py)
    assert not oracle.in_strip(rot, px + 2.0 * c, py + 2.0 * s)


def test_generated_agents_start_on_road_and_off_road_away_from_it():
    for seed, n_q in ((0x5EED0002, 2000), (0x5EED0003, 700)):
        sc = g.make_scene(seed, 1, 24, n_q)
        st, hl, fl = oracle.infractions(sc.agent_state, sc.agent_dims, sc.road_xy, np.zeros(24, np.uint8))
        assert not np.any(fl & 2)                       # on lane centrelines
        far = sc.agent_state.copy()
        far[:, 0] += 1000.0                             # far outside the 200 m map
        st2, hl2, fl2 = oracle.infractions(far, sc.agent_dims, sc.road_xy, np.zeros(24, np.uint8))
        assert np.all(fl2 & 2) and np.all(hl2 == 1) and np.all(st2[:, 3] == 0.0)


def test_halting_latches_zeroes_speed_and_freezes_the_step():
    a, da = _box(0.0, 0.0, 0.0)
    b, db = _box(3.0, 0.0, 0.0)
    c, dc = _box(20.0, 0.0, 0.0)
    state = np.stack([a, b, c])
    state[:, 3] = [5.0, 6.0, 7.0]
    dims = np.stack([da, db, dc])
    road = np.array([[[-100, -10], [100, -10], [100, 10], [-100, 10]]], np.float32)
    st, hl, fl = oracle.infractions(state, dims, road, np.zeros(3, np.uint8))
    assert list(fl) == [1 | 4, 1 | 4, 0] and list(hl) == [1, 1, 0]
    assert list(st[:, 3]) == [0.0, 0.0, 7.0]
    act = np.full((3, 2), 2.0, np.float32)
    nxt, cs = oracle.step(st, dims, act, 0.1, halted=hl)
    assert np.array_equal(nxt[:2], st[:2]) and not np.array_equal(nxt[2], st[2])
    s0, c0 = oracle.sincos(float(st[0, 2]))
    assert cs[0, 0] == c0 and cs[0, 1] == s0
    # halted stays halted once the cause is gone
    st[1, 0] = 50.0
    st3, hl3, fl3 = oracle.infractions(st, dims, road, hl)
    assert list(hl3) == [1, 1, 0] and list(fl3) == [4, 4, 0]
