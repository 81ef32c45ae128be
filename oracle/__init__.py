"""FP64 CPU oracle of the simulator hot path (ctypes wrapper of wm_oracle.c).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library.  Every function takes host numpy arrays (float32 inputs are widened
to float64 exactly) and returns numpy arrays.

Each wrapper names the paper passage its C function follows; the C source
states the readings taken where the paper is silent or ambiguous.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wm_oracle.c")
_LIB = os.path.join(_HERE, "libwm_oracle.so")
NO_VALUE = -float(np.finfo(np.float32).max)
FIELDS = ("x", "y", "yaw", "vx", "vy", "length", "width")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, IEEE semantics, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _State(C.Structure):
    _fields_ = [(f, C.POINTER(C.c_double)) for f in FIELDS] + [("valid", C.POINTER(C.c_uint8))]


class _Roadgraph(C.Structure):
    _fields_ = [("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("dir_x", C.POINTER(C.c_double)), ("dir_y", C.POINTER(C.c_double)),
                ("type", C.POINTER(C.c_int8)), ("valid", C.POINTER(C.c_uint8))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        d, i32, u8 = C.c_double, C.c_int32, C.c_uint8
        P = C.POINTER
        _lib.or_sat_margin.restype = d
        _lib.or_sat_margin.argtypes = [d] * 10
    return _lib


def _p(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


class OState:
    """Owned float64 state arrays (shape [n] or [T, n]) plus a C view."""

    def __init__(self, fields: Dict[str, np.ndarray]):
        self.a = {f: np.ascontiguousarray(fields[f], dtype=np.float64) for f in FIELDS}
        self.a["valid"] = np.ascontiguousarray(fields["valid"], dtype=np.uint8)
        self.c = _State(*[_p(self.a[f], C.c_double) for f in FIELDS], _p(self.a["valid"], C.c_uint8))

    @classmethod
    def empty(cls, shape):
        d = {f: np.zeros(shape) for f in FIELDS}
        d["valid"] = np.zeros(shape, np.uint8)
        return cls(d)

    def __getitem__(self, k):
        return self.a[k]


class ORoadgraph:
    def __init__(self, rg: Dict[str, np.ndarray]):
        self.a = {k: np.ascontiguousarray(rg[k], dtype=np.float64) for k in ("x", "y", "dir_x", "dir_y")}
        self.a["type"] = np.ascontiguousarray(rg["type"], dtype=np.int8)
        self.a["valid"] = np.ascontiguousarray(rg["valid"], dtype=np.uint8)
        self.c = _Roadgraph(*[_p(self.a[k], C.c_double) for k in ("x", "y", "dir_x", "dir_y")],
                            _p(self.a["type"], C.c_int8), _p(self.a["valid"], C.c_uint8))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def bicycle_forward(cur, accel, curvature, controlled, log_next, dt) -> Dict[str, np.ndarray]:
    """Bicycle forward step, App. A.1 (forward dynamics equation) + log
    playback of uncontrolled objects (Sec. 4.3)."""
    cs, ls = OState(cur), OState(log_next)
    n = cs.a["x"].shape[0]
    out = OState.empty(n)
    a, k, c = _f64(accel), _f64(curvature), _u8(controlled)
    lib().or_bicycle_forward(C.c_int(n), C.byref(cs.c), _p(a, C.c_double), _p(k, C.c_double),
                             _p(c, C.c_uint8), C.byref(ls.c), C.c_double(dt), C.byref(out.c))
    return out.a


def bicycle_inverse(cur, nxt, dt):
    """Bicycle inverse kinematics, App. A.1 (inverse kinematics equation).
    Returns (accel, curvature, valid)."""
    cs, ns = OState(cur), OState(nxt)
    n = cs.a["x"].shape[0]
    a, k, v = np.zeros(n), np.zeros(n), np.zeros(n, np.uint8)
    lib().or_bicycle_inverse(C.c_int(n), C.byref(cs.c), C.byref(ns.c), C.c_double(dt),
                             _p(a, C.c_double), _p(k, C.c_double), _p(v, C.c_uint8))
    return a, k, v


def infeasibility(cur, nxt, dt):
    """Kinematic infeasibility of each transition, Sec. 3.4: inverse
    kinematics gives |a| > 6 m/s^2 or |kappa| > 0.3 1/m.  uint8 [n]."""
    cs, ns = OState(cur), OState(nxt)
    n = cs.a["x"].shape[0]
    out = np.zeros(n, np.uint8)
    lib().or_infeasibility(C.c_int(n), C.byref(cs.c), C.byref(ns.c), C.c_double(dt), _p(out, C.c_uint8))
    return out


def reward(collision, offroad):
    """Sparse per-object reward of Sec. 5.2: -1[collision] - 1[off-road]."""
    return -(np.asarray(collision, np.float64) + np.asarray(offroad, np.float64))


def discretize(values, lo: float, hi: float, bins: int):
    """Discretized actions (Sec. 5.2): nearest of `bins` evenly spaced values
    over [lo, hi], decided in binary32.  Returns (index int32, snapped float32)."""
    v = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
    idx = np.zeros(v.shape[0], np.int32)
    snp = np.zeros(v.shape[0], np.float32)
    lib().or_discretize(C.c_int(v.shape[0]), _p(v, C.c_float), C.c_float(lo), C.c_float(hi), C.c_int(bins),
                        _p(idx, C.c_int32), _p(snp, C.c_float))
    return idx, snp


def delta_forward(cur, dx, dy, dyaw, controlled, log_next, dt):
    """Delta action space forward step, App. A.1 (delta equations)."""
    cs, ls = OState(cur), OState(log_next)
    n = cs.a["x"].shape[0]
    out = OState.empty(n)
    ax, ay, at, c = _f64(dx), _f64(dy), _f64(dyaw), _u8(controlled)
    lib().or_delta_forward(C.c_int(n), C.byref(cs.c), _p(ax, C.c_double), _p(ay, C.c_double),
                           _p(at, C.c_double), _p(c, C.c_uint8), C.byref(ls.c), C.c_double(dt),
                           C.byref(out.c))
    return out.a


def delta_inverse(cur, nxt):
    """Delta action space inverse, App. A.1.  Returns (dx, dy, dyaw, valid)."""
    cs, ns = OState(cur), OState(nxt)
    n = cs.a["x"].shape[0]
    dx, dy, dt_, v = np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n, np.uint8)
    lib().or_delta_inverse(C.c_int(n), C.byref(cs.c), C.byref(ns.c), _p(dx, C.c_double),
                           _p(dy, C.c_double), _p(dt_, C.c_double), _p(v, C.c_uint8))
    return dx, dy, dt_, v


def sat_margin(a, b) -> float:
    """Separating-axis overlap margin of two boxes (x, y, yaw, length, width),
    Sec. 3.4 Collision."""
    return lib().or_sat_margin(*[float(v) for v in a], *[float(v) for v in b])


def overlap(obj_off, state, matrix: bool = False):
    """Collision metric, Sec. 3.4.  Returns (collision u8 [n], max_margin [n],
    pair_margin list of [N_s, N_s] blocks or None)."""
    off = _i32(obj_off)
    S = off.shape[0] - 1
    st = OState(state)
    n = int(off[-1])
    col, mm = np.zeros(n, np.uint8), np.zeros(n)
    counts = np.diff(off).astype(np.int64)
    pm = np.zeros(int((counts ** 2).sum())) if matrix else None
    lib().or_overlap(C.c_int(S), _p(off, C.c_int32), C.byref(st.c),
                     _p(pm, C.c_double) if matrix else None, _p(col, C.c_uint8), _p(mm, C.c_double))
    blocks = None
    if matrix:
        blocks, pos = [], 0
        for N in counts:
            blocks.append(pm[pos:pos + N * N].reshape(N, N))
            pos += N * N
    return col, mm, blocks


def offroad(obj_off, rg_off, state, rg, band: float = 1e-4):
    """Off-road metric, Sec. 3.4.  Returns dict with per-object 'offroad',
    'margin' and per-corner 'nearest' (scenario-local index), 'corner_margin',
    'ambiguous' (another point within `band` of the nearest distance lies on
    the other side, or |margin| < band) and 'tied' (another point within
    `band` of the nearest distance at all), each [n, 4]."""
    off, roff = _i32(obj_off), _i32(rg_off)
    S = off.shape[0] - 1
    st, g = OState(state), ORoadgraph(rg)
    n = int(off[-1])
    out = {"offroad": np.zeros(n, np.uint8), "margin": np.zeros(n),
           "nearest": np.zeros((n, 4), np.int32), "corner_margin": np.zeros((n, 4)),
           "ambiguous": np.zeros((n, 4), np.uint8), "tied": np.zeros((n, 4), np.uint8)}
    lib().or_offroad(C.c_int(S), _p(off, C.c_int32), _p(roff, C.c_int32), C.byref(st.c), C.byref(g.c),
                     C.c_double(band), _p(out["margin"], C.c_double), _p(out["offroad"], C.c_uint8),
                     _p(out["nearest"], C.c_int32), _p(out["corner_margin"], C.c_double),
                     _p(out["ambiguous"], C.c_uint8), _p(out["tied"], C.c_uint8))
    return out


def log_divergence(sim, log):
    """Displacement error per object, Sec. 3.4."""
    a, b = OState(sim), OState(log)
    n = a.a["x"].shape[0]
    out = np.zeros(n)
    lib().or_log_divergence(C.c_int(n), C.byref(a.c), C.byref(b.c), _p(out, C.c_double))
    return out


def observe(obj_off, rg_off, state, rg, ego, k: int, max_objects: int):
    """Default observation, Sec. 3.2.  ego [S, E] global ids.  Returns
    (rg_idx int32 [S, E, k], rg_feat [S, E, k, 4], obj_feat [S, E, max_objects, 8])."""
    off, roff = _i32(obj_off), _i32(rg_off)
    S = off.shape[0] - 1
    eg = _i32(ego).reshape(S, -1)
    E = eg.shape[1]
    st, g = OState(state), ORoadgraph(rg)
    idx = np.zeros((S, E, k), np.int32)
    rf = np.zeros((S, E, k, 4))
    of = np.zeros((S, E, max_objects, 8))
    lib().or_observe(C.c_int(S), _p(off, C.c_int32), _p(roff, C.c_int32), C.byref(st.c), C.byref(g.c),
                     _p(eg, C.c_int32), C.c_int(E), C.c_int(k), C.c_int(max_objects),
                     _p(idx, C.c_int32), _p(rf, C.c_double), _p(of, C.c_double))
    return idx, rf, of


def rollout(obj_off, rg_off, init, accel, curvature, controlled, log_seq, rg, T: int, dt: float,
            metrics: bool = True, want_loss: bool = True):
    """Rollout of T steps, Sec. 5.1 (Rollout) and Sec. 4.1 (step): metrics on
    each successor state.  log_seq fields are [T+1, n] (row 0 = initial
    time); accel/curvature [T, n].  Returns dict of [T, n] arrays (+ 'loss' [S])."""
    off = _i32(obj_off)
    roff = _i32(rg_off) if rg_off is not None else None
    S = off.shape[0] - 1
    n = int(off[-1])
    st, ls = OState(init), OState(log_seq)
    g = ORoadgraph(rg) if (rg is not None and metrics) else None
    traj = OState.empty((T, n))
    a, k, c = _f64(accel), _f64(curvature), _u8(controlled)
    out = {"collision": np.zeros((T, n), np.uint8), "overlap_margin": np.zeros((T, n)),
           "offroad": np.zeros((T, n), np.uint8), "offroad_margin": np.zeros((T, n)),
           "log_div": np.zeros((T, n)), "loss": np.zeros(S)}
    P = lambda key, ct: _p(out[key], ct) if metrics else None  # noqa: E731
    lib().or_rollout(C.c_int(S), _p(off, C.c_int32), _p(roff, C.c_int32) if roff is not None else None,
                     C.byref(st.c), _p(a, C.c_double), _p(k, C.c_double), _p(c, C.c_uint8), C.byref(ls.c),
                     C.byref(g.c) if g is not None else None, C.c_int(T), C.c_double(dt), C.byref(traj.c),
                     P("collision", C.c_uint8), P("overlap_margin", C.c_double),
                     P("offroad", C.c_uint8) if g is not None else None,
                     P("offroad_margin", C.c_double) if g is not None else None,
                     P("log_div", C.c_double), _p(out["loss"], C.c_double) if want_loss else None)
    out["traj"] = traj.a
    return out


# IDM sim-agent parameters (Sec. 3.5; values are readings, the paper gives
# none): desired speed v0 [m/s], minimum gap s0 [m], time headway [s],
# maximum acceleration and comfortable deceleration [m/s^2], exponent,
# hardest braking [m/s^2], lookahead pose spacing [m] and pose count.
IDM_DEFAULT = {"v0": 30.0, "s0": 2.0, "headway": 1.5, "a_max": 2.0, "b_comf": 3.0, "delta": 4.0,
               "brake": 8.0, "step": 2.0, "poses": 25}


class _OIdm(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("v0", "s0", "headway", "a_max", "b_comf", "delta", "brake", "step")] + \
        [("poses", C.c_int)]


def rollout_idm(obj_off, rg_off, init, accel, curvature, controlled, log_seq, rg, T: int, dt: float,
                idm=None):
    """Rollout of T steps in which the uncontrolled objects with a fully
    valid log window are IDM sim agents (Sec. 3.5).  Returns the dict of
    rollout() without 'loss', plus 'idm_margin' [T, n] (each agent's
    decision margin per step, +inf for other objects)."""
    par = dict(IDM_DEFAULT)
    par.update(idm or {})
    off = _i32(obj_off)
    roff = _i32(rg_off) if rg_off is not None else None
    S = off.shape[0] - 1
    n = int(off[-1])
    st, ls = OState(init), OState(log_seq)
    g = ORoadgraph(rg) if rg is not None else None
    traj = OState.empty((T, n))
    a, k, c = _f64(accel), _f64(curvature), _u8(controlled)
    out = {"collision": np.zeros((T, n), np.uint8), "overlap_margin": np.zeros((T, n)),
           "offroad": np.zeros((T, n), np.uint8), "offroad_margin": np.zeros((T, n)),
           "log_div": np.zeros((T, n)), "idm_margin": np.zeros((T, n))}
    prm = _OIdm(*[float(par[q]) for q in ("v0", "s0", "headway", "a_max", "b_comf", "delta", "brake", "step")],
                int(par["poses"]))
    lib().or_rollout_idm(C.c_int(S), _p(off, C.c_int32), _p(roff, C.c_int32) if roff is not None else None,
                         C.byref(st.c), _p(a, C.c_double), _p(k, C.c_double), _p(c, C.c_uint8), C.byref(ls.c),
                         C.byref(g.c) if g is not None else None, C.c_int(T), C.c_double(dt), C.byref(prm),
                         C.byref(traj.c), _p(out["collision"], C.c_uint8), _p(out["overlap_margin"], C.c_double),
                         _p(out["offroad"], C.c_uint8) if g is not None else None,
                         _p(out["offroad_margin"], C.c_double) if g is not None else None,
                         _p(out["log_div"], C.c_double), _p(out["idm_margin"], C.c_double))
    out["traj"] = traj.a
    return out


def state_loss(obj_off, state, log, controlled):
    """Loss terms of one state against the log at the same step, per scenario."""
    off = _i32(obj_off)
    S = off.shape[0] - 1
    st, lg = OState(state), OState(log)
    c = _u8(controlled)
    out = np.zeros(S)
    lib().or_state_loss(C.c_int(S), _p(off, C.c_int32), C.byref(st.c), C.byref(lg.c), _p(c, C.c_uint8),
                        _p(out, C.c_double))
    return out


def rollout_loss(obj_off, init, accel, curvature, controlled, log_seq, T: int, dt: float):
    """Per-scenario training loss of a rollout (the loss read for the
    paper's differentiable-simulation use, Sec. 1 / Sec. 6)."""
    off = _i32(obj_off)
    S = off.shape[0] - 1
    st, ls = OState(init), OState(log_seq)
    a, k, c = _f64(accel), _f64(curvature), _u8(controlled)
    loss = np.zeros(S)
    lib().or_rollout_loss(C.c_int(S), _p(off, C.c_int32), C.byref(st.c), _p(a, C.c_double),
                          _p(k, C.c_double), _p(c, C.c_uint8), C.byref(ls.c), C.c_int(T),
                          C.c_double(dt), _p(loss, C.c_double))
    return loss


def rollout_grad(obj_off, init, accel, curvature, controlled, log_seq, T: int, dt: float, dloss=None):
    """Hand-written reverse-mode gradient of the rollout loss with respect to
    the actions (full tape).  Returns (grad_accel [T, n], grad_curvature [T, n], loss [S])."""
    off = _i32(obj_off)
    S = off.shape[0] - 1
    n = int(off[-1])
    st, ls = OState(init), OState(log_seq)
    a, k, c = _f64(accel), _f64(curvature), _u8(controlled)
    dl = _f64(np.ones(S) if dloss is None else dloss)
    ga, gk, loss = np.zeros((T, n)), np.zeros((T, n)), np.zeros(S)
    lib().or_rollout_grad(C.c_int(S), _p(off, C.c_int32), C.byref(st.c), _p(a, C.c_double),
                          _p(k, C.c_double), _p(c, C.c_uint8), C.byref(ls.c), C.c_int(T), C.c_double(dt),
                          _p(dl, C.c_double), _p(ga, C.c_double), _p(gk, C.c_double), _p(loss, C.c_double))
    return ga, gk, loss
