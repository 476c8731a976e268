"""Pins of the oracle's sincos and kinematic step against mathematics that
does not come from the oracle: libm in float64, closed-form straight-line
motion, the float64 semi-implicit recurrence, clamp bounds."""
import math

import numpy as np
import pytest

import oracle


def _ulp32(x):
    x = np.float32(abs(x))
    return float(np.spacing(x)) if x != 0 else float(np.finfo(np.float32).smallest_subnormal)


def test_sincos_vs_libm_dense():
    # dense sweep of [-4, 4]; error measured in units of the larger of the
    # result's ulp and 2^-26 (absolute floor near the zeros of sin and cos)
    ts = np.linspace(-4.0, 4.0, 20001).astype(np.float32)
    worst = 0.0
    for t in ts:
        s, c = oracle.sincos(float(t))
        es, ec = math.sin(float(t)), math.cos(float(t))
        worst = max(worst,
                    abs(float(s) - es) / max(_ulp32(es), 2.0 ** -26),
                    abs(float(c) - ec) / max(_ulp32(ec), 2.0 ** -26))
    assert worst <= 2.0, worst


def test_sincos_special_values():
    assert oracle.sincos(0.0) == (np.float32(0.0), np.float32(1.0))
    for t in (0.1, 0.7, 1.3, 2.9, 3.5):
        s1, c1 = oracle.sincos(t)
        s2, c2 = oracle.sincos(-t)
        assert s1 == -s2 and c1 == c2          # odd / even symmetry
        assert abs(float(s1) ** 2 + float(c1) ** 2 - 1.0) < 4e-7


def _one(x=0.0, y=0.0, psi=0.0, v=10.0, L=4.5):
    st = np.array([[x, y, psi, v]], dtype=np.float32)
    dm = np.array([[L, 2.0, 1.5]], dtype=np.float32)
    return st, dm


def test_step_zero_steer_keeps_heading_bits_and_goes_straight():
    psi0 = np.float32(0.3)
    st, dm = _one(psi=psi0, v=5.0)
    act = np.array([[1.0, 0.0]], dtype=np.float32)
    x64, y64, v64 = 0.0, 0.0, 5.0
    for k in range(10):
        st, cs = oracle.step(st, dm, act, 0.1)
        assert st[0, 2] == psi0                 # heading bit-unchanged
        v64 = min(max(v64 + 1.0 * 0.1, 0.0), 30.0)
        x64 += v64 * 0.1 * math.cos(float(psi0))
        y64 += v64 * 0.1 * math.sin(float(psi0))
    assert abs(st[0, 3] - v64) <= 1e-5 * v64
    assert abs(st[0, 0] - x64) <= 1e-5 * abs(x64)
    assert abs(st[0, 1] - y64) <= 1e-5 * abs(y64)


def test_step_constant_steer_follows_float64_recurrence():
    # constant speed and steer: psi grows by v dt tan(delta)/(0.6 L) per step
    L, v, delta, dt = 4.8, 8.0, 0.2, 0.1
    st, dm = _one(v=v, L=L)
    act = np.array([[0.0, delta]], dtype=np.float32)
    x, y, psi = 0.0, 0.0, 0.0
    d32 = float(np.float32(delta))
    for _ in range(40):
        st, _ = oracle.step(st, dm, act, dt)
        psi += v * dt * math.tan(d32) / (0.6 * float(np.float32(L)))
        psi = psi - 2 * math.pi if psi > math.pi else psi
        x += v * dt * math.cos(psi)
        y += v * dt * math.sin(psi)
    # 40 steps around most of a circle of radius 0.6 L / tan(delta)
    R = 0.6 * L / math.tan(d32)
    assert abs(st[0, 2] - psi) <= 1e-5 * max(1.0, abs(psi))
    assert math.hypot(st[0, 0] - x, st[0, 1] - y) <= 1e-5 * R * 10


def test_step_clamps():
    st = np.array([[0, 0, 0, 29.9], [0, 0, 0, 0.1], [0, 0, 0, 5.0]], dtype=np.float32)
    dm = np.full((3, 3), 4.5, dtype=np.float32)
    act = np.array([[100.0, 3.0], [-100.0, -3.0], [np.nan, np.nan]], dtype=np.float32)
    out, cs = oracle.step(st, dm, act, 0.1)
    assert out[0, 3] == np.float32(30.0)                   # speed capped
    assert out[1, 3] == np.float32(0.0)                    # no reversing
    # steer clamped to +-0.5: heading change equals that of steer = 0.5 exactly
    ref, _ = oracle.step(st[:1], dm[:1], np.array([[100.0, 0.5]], np.float32), 0.1)
    assert out[0, 2] == ref[0, 2]
    # NaN actions take the lower bound of each clamp (fmin/fmax semantics)
    ref2, _ = oracle.step(st[2:], dm[2:], np.array([[-6.0, -0.5]], np.float32), 0.1)
    assert np.array_equal(out[2], ref2[0])
    # the stored (cos, sin) is sincos of the new heading
    for k in range(3):
        s, c = oracle.sincos(float(out[k, 2]))
        assert cs[k, 0] == c and cs[k, 1] == s


def _f32_exact(x):
    """binary32 nearest to the exact rational x, ties to even (one rounding)."""
    from fractions import Fraction
    x = Fraction(x)
    c = np.float32(float(x))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - x)
        even = (int(np.array(cand).view(np.uint32)) & 1) == 0
        if best is None or d < best[0] or (d == best[0] and even):
            best = (d, cand)
    return best[1]


def _fmaf(a, b, c):
    # fused a * b + c of binary32 operands, rounded once
    from fractions import Fraction
    return _f32_exact(Fraction(float(np.float32(a))) * Fraction(float(np.float32(b))) + Fraction(float(np.float32(c))))


def test_step_acceleration_and_steer_clamp_values():
    # App. A ("Action Space and Dynamics") clips the acceleration; the bounds
    # read here are [-6, 3] m/s^2 and |steer| <= 0.5 rad.  From v = 10 (far
    # from the speed bounds) the new speed is the fused v + a dt with a at the
    # bound, so a wrong bound changes the value.
    dt = np.float32(0.1)
    st = np.array([[0, 0, 0, 10.0]] * 4, dtype=np.float32)
    dm = np.full((4, 3), 4.5, dtype=np.float32)
    act = np.array([[100.0, 0.0], [-100.0, 0.0], [np.nan, 0.0], [2.5, 0.0]], dtype=np.float32)
    out, _ = oracle.step(st, dm, act, 0.1)
    assert out[0, 3] == _fmaf(3.0, dt, 10.0)
    assert out[1, 3] == _fmaf(-6.0, dt, 10.0)
    assert out[2, 3] == _fmaf(-6.0, dt, 10.0)      # NaN takes the lower bound
    assert out[3, 3] == _fmaf(2.5, dt, 10.0)       # inside the bounds: unchanged
    # steering: a command past the bound turns like 0.5 rad, whose heading
    # change v1 dt tan(0.5) / (0.6 L) is fixed in float64 (a bound of 0.45 or
    # 0.55 would move it by more than 10%)
    st2 = np.array([[0, 0, 0, 10.0]] * 3, dtype=np.float32)
    act2 = np.array([[0.0, 3.0], [0.0, -3.0], [0.0, np.nan]], dtype=np.float32)
    out2, _ = oracle.step(st2, dm[:3], act2, 0.1)
    v1 = float(_fmaf(0.0, dt, 10.0))
    dpsi = v1 * float(dt) * math.tan(0.5) / (0.6 * 4.5)
    assert abs(float(out2[0, 2]) - dpsi) <= 1e-6 * dpsi
    assert abs(float(out2[1, 2]) + dpsi) <= 1e-6 * dpsi
    assert abs(float(out2[2, 2]) + dpsi) <= 1e-6 * dpsi   # NaN steer: -0.5
    # speed bounds by value: 0 and 30 exactly
    st3 = np.array([[0, 0, 0, 0.2], [0, 0, 0, 29.95]], dtype=np.float32)
    out3, _ = oracle.step(st3, dm[:2], np.array([[-6.0, 0.0], [3.0, 0.0]], np.float32), 0.1)
    assert out3[0, 3] == np.float32(0.0) and out3[1, 3] == np.float32(30.0)


def test_step_heading_wraps_into_half_open_interval():
    st = np.array([[0, 0, np.float32(3.1), 20.0], [0, 0, np.float32(-3.1), 20.0]], dtype=np.float32)
    dm = np.full((2, 3), 4.0, dtype=np.float32)
    act = np.array([[0.0, 0.5], [0.0, -0.5]], dtype=np.float32)
    out, _ = oracle.step(st, dm, act, 0.1)
    assert -math.pi < out[0, 2] <= math.pi and out[0, 2] < 0
    assert -math.pi < out[1, 2] <= math.pi and out[1, 2] > 0
