"""Oracle pins for the jerk-actuated step (App. A, "Action Space and Dynamics":
twelve discrete actions, longitudinal jerks {-15, -4, 0, 4} x lateral jerks
{-4, 0, 4} m/s^3, integrated into accelerations, then speed and steering, with
g-force, speed, steering and steering-rate limits; wheelbase 0.6 L).

The pins come from outside the oracle's own formulas: float64 integration of
constant jerk, the libm arctangent, the geometry of a steady turn (a chord
polygon inscribed in a circle of radius v^2 / a_lat), and the direct step,
which its own tests pin."""
import math

import numpy as np
import pytest

import oracle

DT = 0.1
LON = (-15.0, -4.0, 0.0, 4.0)
LAT = (-4.0, 0.0, 4.0)
T = np.float32(0.546302497)


def _agent(v=10.0, psi=0.0, L=4.5):
    st = np.array([[0.0, 0.0, psi, v]], np.float32)
    dm = np.array([[L, 2.0, 1.5]], np.float32)
    return st, dm, np.zeros((1, 4), np.float32)


def _roll(st, dm, ac, ks, halted=None):
    out = []
    for k in ks:
        st, cs, ac = oracle.step_jerk(st, dm, ac, np.array([k], np.uint8), DT, halted=halted)
        out.append((st, cs, ac))
    return out


def test_atan_series_against_libm():
    xs = np.linspace(-float(T), float(T), 40001).astype(np.float32)
    for x in xs:
        got, ref = float(oracle.atan_small(float(x))), math.atan(float(x))
        assert abs(got - ref) <= float(np.spacing(np.float32(abs(ref)))), x
        assert oracle.atan_small(-float(x)) == -oracle.atan_small(float(x))     # odd
    assert oracle.atan_small(0.0) == 0.0
    assert oracle.atan_small(float(T)) == np.float32(0.5)


@pytest.mark.parametrize("k", range(12))
def test_each_action_from_rest_of_the_actuators(k):
    st, dm, ac = _agent(v=10.0)
    l = 0.6 * 4.5
    st1, cs1, ac1 = oracle.step_jerk(st, dm, ac, np.array([k], np.uint8), DT)
    jl, jt = LON[k // 3], LAT[k % 3]
    a_lon = jl * DT
    v1 = 10.0 + a_lon * DT
    assert ac1[0, 0] == pytest.approx(a_lon, rel=1e-6)
    assert st1[0, 3] == pytest.approx(v1, rel=1e-6)
    a_lat = jt * DT                                   # far below the rate limit at 10 m/s
    delta = math.atan(a_lat * l / (v1 * v1))
    assert ac1[0, 2] == pytest.approx(delta, rel=1e-5, abs=1e-9)
    assert ac1[0, 1] == pytest.approx(a_lat, rel=1e-5, abs=1e-9)   # realised = commanded
    assert ac1[0, 3] == 0.0
    # the pose is the direct step's with the realised acceleration and steering
    ref, cs = oracle.step(st, dm, np.array([[ac1[0, 0], ac1[0, 2]]], np.float32), DT)
    assert np.array_equal(ref, st1) and np.array_equal(cs, cs1)


def test_out_of_range_index_coasts():
    st, dm, _ = _agent(v=7.0, psi=0.3)
    ac = np.array([[1.0, -0.5, 0.05, 0.0]], np.float32)
    ref = oracle.step_jerk(st, dm, ac, np.array([7], np.uint8), DT)      # (0, 0) jerks
    for k in (12, 13, 100, 255):
        got = oracle.step_jerk(st, dm, ac, np.array([k], np.uint8), DT)
        assert all(np.array_equal(a, b) for a, b in zip(got, ref)), k


def test_constant_jerk_matches_float64_integration_and_limits():
    st, dm, ac = _agent(v=0.0)
    a, v = 0.0, 0.0
    for n, (s1, _, a1) in enumerate(_roll(st, dm, ac, [10] * 40)):       # (+4, 0)
        a = min(a + 4.0 * DT, 3.0)
        v = min(v + a * DT, 30.0)
        assert a1[0, 0] == pytest.approx(a, abs=2e-6), n
        assert s1[0, 3] == pytest.approx(v, rel=2e-5, abs=2e-6), n
    assert a1[0, 0] == 3.0                                               # g-limit
    # hard braking: the acceleration falls 1.5 per step to -6, then the stop
    st, dm, ac = _agent(v=3.0)
    seq = _roll(st, dm, ac, [1] * 12)                                    # (-15, 0)
    accs = [float(x[2][0, 0]) for x in seq]
    assert accs[:2] == pytest.approx([-1.5, -3.0], abs=1e-6)
    assert min(accs) >= -6.0
    stopped = [i for i, x in enumerate(seq) if x[0][0, 3] == 0.0]
    assert stopped and all(seq[i][2][0, 0] == 0.0 for i in stopped)     # the clip cancels it
    assert all(float(x[0][0, 3]) >= 0.0 for x in seq)
    assert all(x[2][0, 2] == 0.0 and x[2][0, 1] == 0.0 for x in seq)    # no lateral command, no steering


def test_steering_rate_and_angle_bounds():
    st, dm, ac = _agent(v=2.0)          # low speed: the lateral command asks for a large angle
    prev = 0.0
    deltas = []
    for s1, _, a1 in _roll(st, dm, ac, [8] * 20):                        # (0, +4)
        d = float(a1[0, 2])
        assert d - prev <= 0.6 * DT + 1e-7
        assert abs(d) <= 0.5
        deltas.append(d)
        prev = d
    assert deltas[0] == pytest.approx(0.06, abs=1e-7)                   # rate-limited from the start
    assert deltas[-1] == np.float32(0.5)                                 # saturates at the angle bound
    # lateral g-limit: the commanded lateral acceleration never passes 4 m/s^2
    st, dm, ac = _agent(v=20.0)
    for s1, _, a1 in _roll(st, dm, ac, [8] * 30):
        assert abs(float(a1[0, 1])) <= 4.0 * (1 + 1e-5)


def test_steady_turn_lies_on_a_circle_of_radius_v2_over_alat():
    st, dm, ac = _agent(v=10.0)
    seq = _roll(st, dm, ac, [8] * 10)                          # lateral acceleration to 4
    st, ac = seq[-1][0], seq[-1][2]
    a_lat = float(ac[0, 1])
    assert a_lat == pytest.approx(4.0, rel=1e-4)
    pts = []
    for s1, _, a1 in _roll(st, dm, ac, [7] * 60):                        # hold (zero jerks)
        pts.append((float(s1[0, 0]), float(s1[0, 1])))
        assert float(a1[0, 1]) == pytest.approx(a_lat, rel=1e-5)
        assert float(s1[0, 3]) == pytest.approx(10.0, rel=1e-6)
    P = np.array(pts, np.float64)
    # centre from three points, then every point at the same distance
    (x1, y1), (x2, y2), (x3, y3) = P[0], P[20], P[40]
    d = 2 * (x1 * (y2 - y3) + x2 * (y3 - y1) + x3 * (y1 - y2))
    ux = ((x1**2 + y1**2) * (y2 - y3) + (x2**2 + y2**2) * (y3 - y1) + (x3**2 + y3**2) * (y1 - y2)) / d
    uy = ((x1**2 + y1**2) * (x3 - x2) + (x2**2 + y2**2) * (x1 - x3) + (x3**2 + y3**2) * (x2 - x1)) / d
    r = np.hypot(P[:, 0] - ux, P[:, 1] - uy)
    assert np.ptp(r) < 2e-3
    # chord polygon of a circle of radius v^2 / a_lat: chord v dt, turn v dt kappa per step
    kappa = a_lat / 100.0
    R_poly = 10.0 * DT / (2 * math.sin(10.0 * DT * kappa / 2))
    assert r.mean() == pytest.approx(R_poly, rel=1e-3)
    assert r.mean() == pytest.approx(100.0 / a_lat, rel=2e-3)


def test_halted_agents_keep_state_and_actuators():
    rng = np.random.default_rng(3)
    n = 8
    st = np.column_stack([rng.uniform(-50, 50, (n, 2)), rng.uniform(-3, 3, n), rng.uniform(0, 20, n)]).astype(np.float32)
    dm = np.column_stack([rng.uniform(3.5, 6, n), rng.uniform(1.6, 2.5, n), np.full(n, 1.5)]).astype(np.float32)
    ac = np.column_stack([rng.uniform(-6, 3, n), rng.uniform(-4, 4, n), rng.uniform(-0.5, 0.5, n), np.zeros(n)]).astype(np.float32)
    hl = (np.arange(n) % 2).astype(np.uint8)
    ks = rng.integers(0, 12, n).astype(np.uint8)
    st1, cs1, ac1 = oracle.step_jerk(st, dm, ac, ks, DT, halted=hl)
    h = hl == 1
    assert np.array_equal(st1[h], st[h]) and np.array_equal(ac1[h], ac[h])
    assert not np.array_equal(st1[~h], st[~h])
    for i in np.nonzero(h)[0]:
        s, c = oracle.sincos(float(st[i, 2]))
        assert cs1[i, 0] == c and cs1[i, 1] == s
