"""Pins of the oracle's dynamics (App. A.1) against closed forms and
identities that the equations fix, independent of the oracle's code."""
import math

import numpy as np
import pytest

import oracle

DT = 0.1


def _state(x, y, yaw, vx, vy, length=4.5, width=2.0, valid=1):
    n = len(x)
    return {"x": np.asarray(x, float), "y": np.asarray(y, float), "yaw": np.asarray(yaw, float),
            "vx": np.asarray(vx, float), "vy": np.asarray(vy, float),
            "length": np.full(n, length), "width": np.full(n, width),
            "valid": np.full(n, valid, np.uint8)}


def _roll(s, accel, curv, steps):
    ctrl = np.ones(len(s["x"]), np.uint8)
    out = [s]
    for t in range(steps):
        s = oracle.bicycle_forward(s, accel[t], curv[t], ctrl, s, DT)
        out.append(s)
    return out


def test_straight_line_constant_accel_closed_form():
    # kappa = 0, constant a, velocity along the yaw: yaw stays, the speed grows
    # linearly, x_n = x0 + cos(yaw) (v0 n dt + a n^2 dt^2 / 2).
    rng = np.random.default_rng(0)
    n, steps = 64, 40
    yaw = rng.uniform(-math.pi, math.pi, n)
    v0 = rng.uniform(5, 15, n)
    a = rng.uniform(-0.1, 3, n)
    s = _state(rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), yaw, v0 * np.cos(yaw), v0 * np.sin(yaw))
    traj = _roll(s, np.tile(a, (steps, 1)), np.zeros((steps, n)), steps)
    for k in (1, 7, steps):
        disp = v0 * k * DT + 0.5 * a * (k * DT) ** 2
        np.testing.assert_allclose(traj[k]["x"], s["x"] + np.cos(yaw) * disp, rtol=0, atol=1e-11)
        np.testing.assert_allclose(traj[k]["y"], s["y"] + np.sin(yaw) * disp, rtol=0, atol=1e-11)
        np.testing.assert_allclose(traj[k]["yaw"], yaw, rtol=0, atol=0)
        np.testing.assert_allclose(np.hypot(traj[k]["vx"], traj[k]["vy"]), v0 + a * k * DT, atol=1e-11)


def test_constant_curvature_polygon_closed_form():
    # a = 0, constant kappa, aligned velocity: each step turns by phi = kappa v dt
    # after a straight chord v dt, so x_n = x0 + v dt sin(n phi/2)/sin(phi/2) cos(yaw0 + (n-1) phi/2).
    rng = np.random.default_rng(1)
    n, steps = 32, 50
    yaw0 = rng.uniform(-math.pi, math.pi, n)
    v = rng.uniform(2, 15, n)
    k = rng.uniform(-0.1, 0.1, n)
    s = _state(rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), yaw0, v * np.cos(yaw0), v * np.sin(yaw0))
    traj = _roll(s, np.zeros((steps, n)), np.tile(k, (steps, 1)), steps)
    phi = k * v * DT
    for m in (1, 13, steps):
        ratio = np.sin(m * phi / 2) / np.sin(phi / 2)
        np.testing.assert_allclose(traj[m]["x"], s["x"] + v * DT * ratio * np.cos(yaw0 + (m - 1) * phi / 2), atol=1e-10)
        np.testing.assert_allclose(traj[m]["y"], s["y"] + v * DT * ratio * np.sin(yaw0 + (m - 1) * phi / 2), atol=1e-10)
        np.testing.assert_allclose(traj[m]["yaw"], yaw0 + m * phi, atol=1e-12)


def test_inverse_recovers_action_and_state():
    # inverse(s, forward(s, a, kappa)) = (a, kappa) whenever v' >= 0 and
    # |kappa D| < pi; then forward(s, inverse(...)) reproduces s' exactly.
    rng = np.random.default_rng(2)
    n = 500
    yaw = rng.uniform(-math.pi, math.pi, n)
    v = rng.uniform(0.5, 20, n)
    slip = rng.uniform(-0.3, 0.3, n)  # velocity not aligned with yaw is allowed
    s = _state(rng.uniform(-100, 100, n), rng.uniform(-100, 100, n), yaw,
               v * np.cos(yaw + slip), v * np.sin(yaw + slip))
    a = rng.uniform(-3, 3, n)
    k = rng.uniform(-0.3, 0.3, n)
    ctrl = np.ones(n, np.uint8)
    s1 = oracle.bicycle_forward(s, a, k, ctrl, s, DT)
    ra, rk, rv = oracle.bicycle_inverse(s, s1, DT)
    assert rv.all()
    np.testing.assert_allclose(ra, a, atol=1e-9)
    np.testing.assert_allclose(rk, k, atol=1e-9)
    s2 = oracle.bicycle_forward(s, ra, rk, ctrl, s, DT)
    for f in ("x", "y", "yaw", "vx", "vy"):
        np.testing.assert_allclose(s2[f], s1[f], atol=1e-9)


def test_inverse_heading_wraps_across_pi():
    # yaw just below pi turning left crosses to -pi in atan2 terms; the wrapped
    # difference keeps kappa small and positive.
    s = _state([0.0], [0.0], [math.pi - 0.01], [10 * math.cos(math.pi - 0.01)], [10 * math.sin(math.pi - 0.01)])
    s1 = oracle.bicycle_forward(s, [0.0], [0.05], np.ones(1, np.uint8), s, DT)
    a, k, v = oracle.bicycle_inverse(s, s1, DT)
    assert abs(k[0] - 0.05) < 1e-12 and abs(a[0]) < 1e-12


def test_inverse_zero_distance_gives_zero_curvature_and_invalid_pairs():
    s = _state([0.0, 1.0], [0.0, 1.0], [0.3, 0.3], [0.0, 1.0], [0.0, 0.0])
    s1 = dict(s)
    s1["valid"] = np.array([1, 0], np.uint8)
    a, k, v = oracle.bicycle_inverse(s, s1, DT)
    assert k[0] == 0.0 and a[0] == 0.0 and v[0] == 1
    assert v[1] == 0 and a[1] == 0.0 and k[1] == 0.0


def test_forward_is_rigid_motion_equivariant():
    # Rotating and translating the initial state rotates/translates the result.
    rng = np.random.default_rng(3)
    n = 200
    s = _state(rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), rng.uniform(-3, 3, n),
               rng.uniform(-10, 10, n), rng.uniform(-10, 10, n))
    a, k = rng.uniform(-3, 3, n), rng.uniform(-0.1, 0.1, n)
    ctrl = np.ones(n, np.uint8)
    phi, tx, ty = 0.7, 12.0, -5.0
    c, sn = math.cos(phi), math.sin(phi)
    r = dict(s)
    r["x"], r["y"] = c * s["x"] - sn * s["y"] + tx, sn * s["x"] + c * s["y"] + ty
    r["vx"], r["vy"] = c * s["vx"] - sn * s["vy"], sn * s["vx"] + c * s["vy"]
    r["yaw"] = s["yaw"] + phi
    s1 = oracle.bicycle_forward(s, a, k, ctrl, s, DT)
    r1 = oracle.bicycle_forward(r, a, k, ctrl, r, DT)
    np.testing.assert_allclose(r1["x"], c * s1["x"] - sn * s1["y"] + tx, atol=1e-10)
    np.testing.assert_allclose(r1["y"], sn * s1["x"] + c * s1["y"] + ty, atol=1e-10)
    np.testing.assert_allclose(r1["yaw"], s1["yaw"] + phi, atol=1e-12)
    np.testing.assert_allclose(r1["vx"], c * s1["vx"] - sn * s1["vy"], atol=1e-10)


def test_playback_and_frozen_objects():
    rng = np.random.default_rng(4)
    n = 6
    s = _state(rng.normal(size=n), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n))
    s["valid"] = np.array([1, 1, 0, 0, 1, 1], np.uint8)
    log = _state(rng.normal(size=n), rng.normal(size=n), rng.normal(size=n), rng.normal(size=n),
                 rng.normal(size=n), length=5.0, width=2.1)
    log["valid"] = np.array([0, 1, 1, 0, 1, 1], np.uint8)
    ctrl = np.array([0, 0, 1, 1, 1, 0], np.uint8)
    out = oracle.bicycle_forward(s, np.ones(n), np.ones(n) * 0.1, ctrl, log, DT)
    for i in (0, 1, 5):      # uncontrolled: replay the log, including valid
        for f in out:
            assert out[f][i] == log[f][i]
    for i in (2, 3):         # controlled but invalid: frozen
        for f in out:
            assert out[f][i] == s[f][i]
    assert out["valid"][4] == 1 and out["length"][4] == s["length"][4]


def test_delta_dynamics_inverse_identity():
    rng = np.random.default_rng(5)
    n = 100
    s = _state(rng.uniform(-50, 50, n), rng.uniform(-50, 50, n), rng.uniform(-3, 3, n),
               rng.normal(size=n), rng.normal(size=n))
    d = rng.uniform(-2, 2, (3, n))
    ctrl = np.ones(n, np.uint8)
    s1 = oracle.delta_forward(s, d[0], d[1], d[2], ctrl, s, DT)
    np.testing.assert_allclose(s1["vx"], d[0] / DT, atol=1e-9)
    dx, dy, dyaw, v = oracle.delta_inverse(s, s1)
    np.testing.assert_allclose(np.stack([dx, dy, dyaw]), d, atol=1e-12)
    assert v.all()


def test_infeasibility_thresholds():
    # Sec. 3.4: |a| > 6 m/s^2 or |kappa| > 0.3 1/m from inverse kinematics.
    # Transitions made by the bicycle model itself within the limits are
    # feasible; just beyond either limit they are not.
    rng = np.random.default_rng(6)
    n = 400
    yaw = rng.uniform(-math.pi, math.pi, n)
    v = rng.uniform(2, 20, n)
    s = _state(rng.uniform(-80, 80, n), rng.uniform(-80, 80, n), yaw, v * np.cos(yaw), v * np.sin(yaw))
    ctrl = np.ones(n, np.uint8)
    a = rng.uniform(-5.9, 5.9, n)
    k = rng.uniform(-0.29, 0.29, n)
    s1 = oracle.bicycle_forward(s, a, k, ctrl, s, DT)
    assert not oracle.infeasibility(s, s1, DT).any()
    for aa, kk, expect in ((6.1, 0.0, 1), (-6.1, 0.0, 1), (0.0, 0.31, 1), (0.0, -0.31, 1), (5.9, 0.29, 0)):
        s2 = oracle.bicycle_forward(s, np.full(n, aa), np.full(n, kk), ctrl, s, DT)
        assert (oracle.infeasibility(s, s2, DT) == expect).all(), (aa, kk)
    s3 = dict(s1)
    s3["valid"] = np.zeros(n, np.uint8)
    s4 = oracle.bicycle_forward(s, np.full(n, 9.0), np.zeros(n), ctrl, s, DT)
    assert not oracle.infeasibility(s, dict(s4, valid=s3["valid"]), DT).any()
    # a delta-action jump of 0.5 rad in one 0.1 s step at 10 m/s is infeasible
    d = oracle.delta_forward(_state([0.0], [0.0], [0.0], [10.0], [0.0]), [1.0], [0.0], [0.5], np.ones(1, np.uint8),
                             _state([0.0], [0.0], [0.0], [0.0], [0.0]), DT)
    d["vx"], d["vy"] = np.array([10 * math.cos(0.5)]), np.array([10 * math.sin(0.5)])
    assert oracle.infeasibility(_state([0.0], [0.0], [0.0], [10.0], [0.0]), d, DT)[0] == 1
    np.testing.assert_array_equal(oracle.reward([0, 1, 1, 0], [0, 0, 1, 1]), [0.0, -1.0, -2.0, -1.0])
