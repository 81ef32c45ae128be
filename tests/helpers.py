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


def offroad_decisive(ref):
    """Per object: +1 decisively off road, -1 decisively on road, 0 near tie
    (some corner within the band or with an ambiguous nearest point)."""
    cm, amb = ref["corner_margin"], ref["ambiguous"].astype(bool)
    off = ((cm > BAND) & ~amb).any(axis=1)
    on = ((cm < -BAND) & ~amb).all(axis=1) | (cm == -float(np.finfo(np.float32).max)).all(axis=1)
    return np.where(off, 1, np.where(on, -1, 0))


def compare_offroad(g_mask, g_margin, ref, where=""):
    """Masks bit-exact on decisive objects, margins within tolerance on objects
    whose winning corner is unambiguous.  Returns the near-tie count."""
    dec = offroad_decisive(ref)
    exp = (dec > 0).astype(np.uint8)
    sel = dec != 0
    bad = np.flatnonzero(sel & (g_mask != exp))
    assert bad.size == 0, "%s offroad mask mismatches at %s" % (where, bad[:10])
    clean = ~ref["ambiguous"].astype(bool).any(axis=1)
    ok = within(g_margin, ref["margin"]) | ~clean
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, "%s offroad margin mismatches at %s gpu=%s oracle=%s" % (
        where, bad[:5], g_margin[bad[:5]], ref["margin"][bad[:5]])
    return int((dec == 0).sum())


def compare_collision(g_col, g_mm, o_col, o_mm, where=""):
    tie = np.abs(o_mm) < BAND
    bad = np.flatnonzero(~tie & (g_col != o_col))
    assert bad.size == 0, "%s collision mismatches at %s" % (where, bad[:10])
    ok = within(g_mm, o_mm)
    bad = np.flatnonzero(~ok)
    assert bad.size == 0, "%s overlap margin mismatches at %s gpu=%s oracle=%s" % (
        where, bad[:5], g_mm[bad[:5]], o_mm[bad[:5]])
    return int(tie.sum())
