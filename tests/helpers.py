"""Shared helpers of the GPU parity tests: tolerances, near-tie accounting and
device setup.  The tolerance is the one the workload states for float32
states and metrics: |gpu - oracle| <= 1e-5 (absolute, quantity units) or
<= 1e-4 * |oracle| (relative); angles are compared modulo 2 pi."""
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

ATOL = 1e-5
RTOL = 1e-4
BAND = 1e-4   # near-tie band for masks [m]
FIELDS = ("x", "y", "yaw", "vx", "vy", "length", "width")


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    from paper_2310_08710_amd import wm
    wm.lib()   # raises if the HIP library is missing: no fallback
    return torch.device("cuda:0")


def f64(d):
    return {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in d.items()}


def within(g, o, atol=ATOL, rtol=RTOL):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    return (np.abs(g - o) <= atol) | (np.abs(g - o) <= rtol * np.abs(o))


def angle_within(g, o, atol=ATOL, rtol=RTOL):
    d = np.asarray(g, np.float64) - np.asarray(o, np.float64)
    d = d - 2 * math.pi * np.round(d / (2 * math.pi))
    return (np.abs(d) <= atol) | (np.abs(d) <= rtol * np.abs(np.asarray(o, np.float64)))


def assert_state_close(g, o, where="", mask=None, atol=ATOL, rtol=RTOL):
    for f in FIELDS:
        ok = angle_within(g[f], o[f], atol, rtol) if f == "yaw" else within(g[f], o[f], atol, rtol)
        if mask is not None:
            ok = ok | ~mask
        if not ok.all():
            bad = np.flatnonzero(~ok.reshape(-1))[:5]
            raise AssertionError("%s field %s: %d mismatches, first %s gpu=%s oracle=%s" % (
                where, f, (~ok).sum(), bad, np.asarray(g[f]).reshape(-1)[bad], np.asarray(o[f]).reshape(-1)[bad]))
    np.testing.assert_array_equal(g["valid"], o["valid"], err_msg=where + " valid")


def offroad_decisive(ref, band=BAND):
    """Per object: +1 decisively off road, -1 decisively on road, 0 near tie
    (some corner within the band or with an ambiguous nearest point).  `ref`
    must come from oracle.offroad(..., band=band); band may be per object."""
    band = np.broadcast_to(np.asarray(band, np.float64), ref["margin"].shape)[:, None]
    cm, amb = ref["corner_margin"], ref["ambiguous"].astype(bool)
    off = ((cm > band) & ~amb).any(axis=1)
    on = ((cm < -band) & ~amb).all(axis=1) | (cm == -float(np.finfo(np.float32).max)).all(axis=1)
    return np.where(off, 1, np.where(on, -1, 0))


def compare_offroad(g_mask, g_margin, ref, where="", band=BAND):
    """Masks bit-exact on decisive objects; margins within tolerance (plus the
    band when the states differ) on objects whose corners have a unique
    nearest point (no other point within the band of its distance: float32
    cannot order distances closer than its rounding at the scene's scale, and
    the margin depends on which point is taken).  Returns the near-tie count."""
    dec = offroad_decisive(ref, band)
    exp = (dec > 0).astype(np.uint8)
    sel = dec != 0
    bad = np.flatnonzero(sel & (g_mask != exp))
    assert bad.size == 0, "%s offroad mask mismatches at %s" % (where, bad[:10])
    clean = ~(ref["ambiguous"].astype(bool) | ref["tied"].astype(bool)).any(axis=1)
    extra = np.broadcast_to(np.asarray(band, np.float64) - BAND, ref["margin"].shape)
    ok = within(g_margin, ref["margin"]) | (np.abs(g_margin - ref["margin"]) <= extra + ATOL) | ~clean
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, "%s offroad margin mismatches at %s gpu=%s oracle=%s" % (
        where, bad[:5], g_margin[bad[:5]], ref["margin"][bad[:5]])
    return int((dec == 0).sum())


def compare_collision(g_col, g_mm, o_col, o_mm, where="", band=BAND):
    """Collision masks bit-exact where the oracle's max margin is outside the
    band; max margins within tolerance (plus the band beyond BAND)."""
    band = np.broadcast_to(np.asarray(band, np.float64), o_mm.shape)
    tie = np.abs(o_mm) < band
    bad = np.flatnonzero(~tie & (g_col != o_col))
    assert bad.size == 0, "%s collision mismatches at %s" % (where, bad[:10])
    ok = within(g_mm, o_mm) | (np.abs(g_mm - o_mm) <= band - BAND + ATOL)
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, "%s overlap margin mismatches at %s gpu=%s oracle=%s" % (
        where, bad[:5], g_mm[bad[:5]], o_mm[bad[:5]])
    return int(tie.sum())


# Largest distance from a box's centre to its corner, for the boxes of the
# synthetic scenes (length <= 5.5 m, width <= 2.2 m): 2.97 m < 3 m.
HALF_DIAGONAL = 3.0


def state_delta(g, o):
    """Per object: how far any point of the box can have moved between two
    states, |dp| + HALF_DIAGONAL * |dyaw|.  A separating-axis margin moves by
    at most the sum of this for its two boxes, a corner's signed side offset by
    at most this (margins are 1-Lipschitz in the positions involved)."""
    dp = np.hypot(np.asarray(g["x"], np.float64) - o["x"], np.asarray(g["y"], np.float64) - o["y"])
    dyaw = np.asarray(g["yaw"], np.float64) - o["yaw"]
    dyaw = np.abs(dyaw - 2 * math.pi * np.round(dyaw / (2 * math.pi)))
    both = (np.asarray(g["valid"]) == 1) & (np.asarray(o["valid"]) == 1)
    return np.where(both, dp + HALF_DIAGONAL * dyaw, 0.0)


def scenario_band(delta, obj_off):
    """Per object: BAND + twice the largest state_delta of its scenario (a pair
    margin involves two boxes; a per-object maximum may switch partners)."""
    out = np.zeros_like(delta)
    for s in range(len(obj_off) - 1):
        sl = slice(obj_off[s], obj_off[s + 1])
        if obj_off[s + 1] > obj_off[s]:
            out[sl] = BAND + 2.0 * delta[sl].max()
    return out


# Trajectory tolerance: float32 rounding of positions at the scene's scale
# (100 m), of velocities at 15 m/s and of yaw at pi accumulates over the
# steps; the workload's relative tolerance 1e-4 is applied at that scale.
SCALE = {"x": 100.0, "y": 100.0, "vx": 15.0, "vy": 15.0, "yaw": math.pi, "length": 5.5, "width": 2.2}


def assert_traj_close(g, o, where=""):
    for f in FIELDS:
        d = np.asarray(g[f], np.float64) - o[f]
        if f == "yaw":
            d = d - 2 * math.pi * np.round(d / (2 * math.pi))
        ok = np.abs(d) <= RTOL * np.maximum(np.abs(o[f]), SCALE[f])
        if not ok.all():
            bad = np.flatnonzero(~ok.reshape(-1))[:5]
            raise AssertionError("%s field %s: %d beyond 1e-4 of the scene scale, first %s gpu=%s oracle=%s" % (
                where, f, (~ok).sum(), bad, np.asarray(g[f]).reshape(-1)[bad], np.asarray(o[f]).reshape(-1)[bad]))
    np.testing.assert_array_equal(g["valid"], o["valid"], err_msg=where + " valid")


# Gradient tolerance: per scenario the norm error ||g - o|| / ||o|| <= 1e-3;
# the element-wise maximum |g - o| / max |o| is reported beside it and held to
# the same 1e-3.
GRAD_TOL = 1e-3


def grad_errors(g, o):
    """(norm error, element-wise maximum error) of one scenario's gradient:
    ||g - o||_2 / ||o||_2 and max |g - o| / max |o|."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = np.abs(o).max()
    return float(np.linalg.norm(g - o) / np.linalg.norm(o)), float(np.abs(g - o).max() / scale)


def assert_grad_close(g, o, where=""):
    """Bound both gradient errors of one scenario and print them (the
    element-wise maximum is reported next to the norm error)."""
    norm, elem = grad_errors(g, o)
    print("gradient %s: norm error %.3e, element-wise max %.3e" % (where, norm, elem))
    assert norm <= GRAD_TOL, (where, "norm", norm)
    assert elem <= GRAD_TOL, (where, "element-wise", elem)
    return norm, elem
