"""Python binding of the C ABI in include/wm.h (argument marshalling only).

Every function takes torch tensors on a ROCm device, passes their device
pointers and the current HIP stream to libwm.so, and returns after the launch
(no synchronization).  All computation happens in the HIP kernels; if the
library is missing this module raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Dict, Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwm.so")

WM_OK, WM_ERR_NULL, WM_ERR_RANGE, WM_ERR_SHAPE, WM_ERR_WORKSPACE, WM_ERR_UNSUPPORTED, WM_ERR_DEVICE = range(7)
MAX_OBJECTS = 1024
MAX_TOPK = 1024
MAX_OBSERVE_POINTS = 32768
NO_VALUE = -float(np.finfo(np.float32).max)
STATE_FIELDS = ("x", "y", "yaw", "vx", "vy", "length", "width")

_P = C.c_void_p


class CBatch(C.Structure):
    _fields_ = [("num_scenarios", C.c_int32), ("total_objects", C.c_int32), ("total_rg_points", C.c_int32),
                ("max_objects", C.c_int32), ("max_rg_points", C.c_int32), ("obj_off", _P), ("rg_off", _P)]


class CState(C.Structure):
    _fields_ = [(f, _P) for f in STATE_FIELDS] + [("valid", _P)]


class CRoadgraph(C.Structure):
    _fields_ = [("x", _P), ("y", _P), ("dir_x", _P), ("dir_y", _P), ("type", _P), ("valid", _P)]


class CAction(C.Structure):
    _fields_ = [("accel", _P), ("curvature", _P), ("controlled", _P)]


class CMetrics(C.Structure):
    _fields_ = [("collision", _P), ("offroad", _P), ("overlap_margin", _P), ("offroad_margin", _P),
                ("log_div", _P), ("infeasible", _P), ("reward", _P)]


class CDeltaAction(C.Structure):
    _fields_ = [("dx", _P), ("dy", _P), ("dyaw", _P), ("controlled", _P)]


class CTuning(C.Structure):
    _fields_ = [("unit_objects", C.c_int32), ("edge_splits", C.c_int32)]


class CIdm(C.Structure):
    _fields_ = [(k, C.c_float) for k in ("desired_speed", "min_gap", "time_headway", "max_accel", "comfort_decel",
                                         "exponent", "max_brake", "lookahead_step")] + [("lookahead_poses", C.c_int32)]


# IDM sim-agent parameters used when none are given (Sec. 3.5 gives none;
# a urban-speed reading): v0 30 m/s, s0 2 m, headway 1.5 s, a_max 2 m/s^2,
# b 3 m/s^2, delta 4, hardest braking 8 m/s^2, 25 lookahead poses 2 m apart.
IDM_DEFAULT = {"desired_speed": 30.0, "min_gap": 2.0, "time_headway": 1.5, "max_accel": 2.0, "comfort_decel": 3.0,
               "exponent": 4.0, "max_brake": 8.0, "lookahead_step": 2.0, "lookahead_poses": 25}


class WMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("wm error %d (%s): %s" % (code, error_string(code), msg))
        self.code = code


_lib = None


def lib() -> C.CDLL:
    """Load libwm.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwm.so is not built (%s); run `python -m paper_2310_08710_amd.build`" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        L.wm_workspace_bytes.restype = C.c_size_t
        L.wm_workspace_bytes.argtypes = [C.POINTER(CBatch), C.c_int32, C.c_int32]
        L.wm_rollout_workspace_bytes.restype = C.c_size_t
        L.wm_rollout_workspace_bytes.argtypes = [C.POINTER(CBatch), C.c_int32, C.c_int32]
        L.wm_error_string.restype = C.c_char_p
        L.wm_error_string.argtypes = [C.c_int]
        L.wm_last_error_message.restype = C.c_char_p
        L.wm_step.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                              C.POINTER(CRoadgraph), C.c_float, C.POINTER(CState), C.POINTER(CMetrics), _P,
                              C.c_size_t, _P]
        L.wm_step_prepared.argtypes = L.wm_step.argtypes
        L.wm_step_observe.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                                      C.POINTER(CRoadgraph), C.c_float, C.POINTER(CState), C.POINTER(CMetrics), _P,
                                      C.c_int32, C.c_int32, _P, _P, _P, _P, C.c_size_t, _P]
        L.wm_step_noalloc.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                                      C.POINTER(CRoadgraph), C.c_float, C.POINTER(CState), C.POINTER(CMetrics), _P]
        L.wm_roadgraph_prepare.argtypes = [C.POINTER(CBatch), C.POINTER(CRoadgraph), _P, C.c_size_t, _P]
        L.wm_inverse_action.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CState), C.c_float, _P, _P,
                                        _P, _P]
        L.wm_overlap.argtypes = [C.POINTER(CBatch), C.POINTER(CState), _P, _P, _P, _P, _P, _P]
        L.wm_offroad.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CRoadgraph), _P, _P, _P,
                                 C.POINTER(CTuning), _P, C.c_size_t, _P]
        L.wm_observe.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CRoadgraph), _P, C.c_int32,
                                 C.c_int32, _P, _P, _P, _P]
        L.wm_observe_seq.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.c_int32, C.POINTER(CRoadgraph), _P,
                                     C.c_int32, C.c_int32, _P, _P, _P, _P]
        L.wm_rollout.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                                 C.POINTER(CRoadgraph), C.c_int32, C.c_float, C.c_int32, C.POINTER(CState),
                                 C.POINTER(CState), C.POINTER(CMetrics), _P, C.POINTER(CTuning), _P, C.c_size_t, _P]
        L.wm_rollout_idm.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                                     C.POINTER(CRoadgraph), C.c_int32, C.c_float, C.POINTER(CIdm),
                                     C.POINTER(CState), C.POINTER(CMetrics), C.POINTER(CTuning), _P, C.c_size_t, _P]
        L.wm_rollout_scan_counts.argtypes = [C.POINTER(CBatch), _P, C.c_size_t, C.POINTER(C.c_uint64), _P]
        L.wm_rollout_backward.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction),
                                          C.POINTER(CState), C.c_int32, C.c_float, C.c_int32, C.POINTER(CState),
                                          _P, _P, _P, _P, C.c_size_t, _P]
        L.wm_step_delta.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CDeltaAction),
                                    C.POINTER(CState), C.c_float, C.POINTER(CState), _P]
        L.wm_inverse_delta.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CState), _P, _P, _P, _P, _P]
        L.wm_discretize.argtypes = [_P, C.c_int32, C.c_float, C.c_float, C.c_int32, _P, _P, _P]
        L.wm_profile_enable.argtypes = [C.c_int]
        L.wm_profile_collect.argtypes = [C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_int32)]
        L.wm_autotune.argtypes = [C.POINTER(CBatch), C.POINTER(CState), C.POINTER(CAction), C.POINTER(CState),
                                  C.POINTER(CRoadgraph), C.c_int32, C.c_float, _P, C.c_size_t, C.POINTER(CTuning),
                                  _P]
        _lib = L
    return _lib


def error_string(code: int) -> str:
    return lib().wm_error_string(code).decode()


def _check(rc: int):
    if rc != WM_OK:
        raise WMError(rc, lib().wm_last_error_message().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else t.data_ptr()


def _need(t: Optional[torch.Tensor], numel: int, dtype: torch.dtype, name: str, optional: bool = True):
    """Raise ValueError unless t is a contiguous tensor of `dtype` with at least
    `numel` elements (the library trusts device pointers, so a short tensor
    would become an out-of-bounds device access).  None passes when optional."""
    if t is None:
        if optional:
            return
        raise ValueError("%s is required" % name)
    if t.dtype != dtype:
        raise ValueError("%s has dtype %s, expected %s" % (name, t.dtype, dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < numel:
        raise ValueError("%s has %d elements, %d needed" % (name, t.numel(), numel))


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


# ---------------------------------------------------------------------------
# Containers
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Batch:
    """Packed batch: device offsets plus the host sizes the ABI needs."""
    obj_off: torch.Tensor            # int32 [S+1] (device)
    rg_off: torch.Tensor             # int32 [S+1] (device)
    num_scenarios: int
    total_objects: int
    total_rg_points: int
    max_objects: int
    max_rg_points: int

    @classmethod
    def from_offsets(cls, obj_off: np.ndarray, rg_off: np.ndarray, device) -> "Batch":
        obj_off = np.asarray(obj_off, np.int32)
        rg_off = np.asarray(rg_off, np.int32)
        S = obj_off.shape[0] - 1
        return cls(torch.from_numpy(obj_off).to(device), torch.from_numpy(rg_off).to(device), S,
                   int(obj_off[-1]), int(rg_off[-1]), int(np.diff(obj_off).max()) if S else 0,
                   int(np.diff(rg_off).max()) if S else 0)

    def c(self) -> CBatch:
        _need(self.obj_off, self.num_scenarios + 1, torch.int32, "batch.obj_off", False)
        _need(self.rg_off, self.num_scenarios + 1, torch.int32, "batch.rg_off", False)
        return CBatch(self.num_scenarios, self.total_objects, self.total_rg_points, self.max_objects,
                      self.max_rg_points, self.obj_off.data_ptr(), self.rg_off.data_ptr())

    def workspace_bytes(self, T: int = 0, ckpt_every: int = 0) -> int:
        b = self.c()
        return int(lib().wm_workspace_bytes(C.byref(b), T, ckpt_every))

    def workspace(self, T: int = 0, ckpt_every: int = 0) -> torch.Tensor:
        return torch.empty(max(self.workspace_bytes(T, ckpt_every), 1), dtype=torch.uint8,
                           device=self.obj_off.device)


@dataclasses.dataclass
class State:
    """SoA state tensors ([n] or time-major [T, n]); float32 + uint8 valid."""
    x: torch.Tensor
    y: torch.Tensor
    yaw: torch.Tensor
    vx: torch.Tensor
    vy: torch.Tensor
    length: torch.Tensor
    width: torch.Tensor
    valid: torch.Tensor

    def c(self, numel: int = 0, name: str = "state") -> CState:
        """C view; every field must hold at least `numel` entries."""
        for f in STATE_FIELDS:
            _need(getattr(self, f), numel, torch.float32, "%s.%s" % (name, f), False)
        _need(self.valid, numel, torch.uint8, name + ".valid", False)
        return CState(*[getattr(self, f).data_ptr() for f in STATE_FIELDS], self.valid.data_ptr())

    @classmethod
    def empty(cls, shape, device) -> "State":
        return cls(*[torch.empty(shape, dtype=torch.float32, device=device) for _ in STATE_FIELDS],
                   torch.empty(shape, dtype=torch.uint8, device=device))

    @classmethod
    def from_numpy(cls, d: Dict[str, np.ndarray], device) -> "State":
        return cls(*[torch.from_numpy(np.ascontiguousarray(d[f], np.float32)).to(device) for f in STATE_FIELDS],
                   torch.from_numpy(np.ascontiguousarray(d["valid"], np.uint8)).to(device))

    def numpy(self) -> Dict[str, np.ndarray]:
        return {f: getattr(self, f).cpu().numpy() for f in STATE_FIELDS + ("valid",)}

    def row(self, t: int) -> "State":
        return State(*[getattr(self, f)[t] for f in STATE_FIELDS + ("valid",)])


@dataclasses.dataclass
class Roadgraph:
    x: torch.Tensor
    y: torch.Tensor
    dir_x: torch.Tensor
    dir_y: torch.Tensor
    type: torch.Tensor
    valid: torch.Tensor

    def c(self, numel: int = 0) -> CRoadgraph:
        """C view; every field must hold at least `numel` points."""
        for f in ("x", "y", "dir_x", "dir_y"):
            _need(getattr(self, f), numel, torch.float32, "rg." + f, False)
        _need(self.type, numel, torch.int8, "rg.type", False)
        _need(self.valid, numel, torch.uint8, "rg.valid", False)
        return CRoadgraph(self.x.data_ptr(), self.y.data_ptr(), self.dir_x.data_ptr(), self.dir_y.data_ptr(),
                          self.type.data_ptr(), self.valid.data_ptr())

    @classmethod
    def from_numpy(cls, d: Dict[str, np.ndarray], device) -> "Roadgraph":
        f = lambda k, dt: torch.from_numpy(np.ascontiguousarray(d[k], dt)).to(device)  # noqa: E731
        return cls(f("x", np.float32), f("y", np.float32), f("dir_x", np.float32), f("dir_y", np.float32),
                   f("type", np.int8), f("valid", np.uint8))


@dataclasses.dataclass
class Action:
    accel: torch.Tensor
    curvature: torch.Tensor
    controlled: torch.Tensor

    def c(self, numel: int = 0, n: int = 0) -> CAction:
        """C view; accel / curvature hold at least `numel` entries, controlled `n`."""
        _need(self.accel, numel, torch.float32, "accel", False)
        _need(self.curvature, numel, torch.float32, "curvature", False)
        _need(self.controlled, n, torch.uint8, "controlled", False)
        return CAction(self.accel.data_ptr(), self.curvature.data_ptr(), self.controlled.data_ptr())


@dataclasses.dataclass
class Metrics:
    collision: Optional[torch.Tensor] = None
    offroad: Optional[torch.Tensor] = None
    overlap_margin: Optional[torch.Tensor] = None
    offroad_margin: Optional[torch.Tensor] = None
    log_div: Optional[torch.Tensor] = None
    infeasible: Optional[torch.Tensor] = None
    reward: Optional[torch.Tensor] = None

    FIELDS = ("collision", "offroad", "overlap_margin", "offroad_margin", "log_div", "infeasible", "reward")

    @classmethod
    def empty(cls, shape, device) -> "Metrics":
        u8 = lambda: torch.empty(shape, dtype=torch.uint8, device=device)  # noqa: E731
        f32 = lambda: torch.empty(shape, dtype=torch.float32, device=device)  # noqa: E731
        return cls(u8(), u8(), f32(), f32(), f32(), u8(), f32())

    def row(self, t: int) -> "Metrics":
        return Metrics(*[None if getattr(self, f) is None else getattr(self, f)[t] for f in self.FIELDS])

    def c(self, numel: int = 0) -> CMetrics:
        """C view; every given member must hold at least `numel` entries."""
        for f in self.FIELDS:
            _need(getattr(self, f), numel, torch.uint8 if f in ("collision", "offroad", "infeasible") else
                  torch.float32, "metrics." + f)
        return CMetrics(_ptr(self.collision), _ptr(self.offroad), _ptr(self.overlap_margin),
                        _ptr(self.offroad_margin), _ptr(self.log_div), _ptr(self.infeasible), _ptr(self.reward))


def _tune(t):
    if t is None:
        return None
    return C.byref(CTuning(int(t[0]), int(t[1])))


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def _step(fn, batch, cur, act, log_next, rg, dt, nxt, metrics, ws, stream):
    N = batch.total_objects
    b, c, a, l, n = batch.c(), cur.c(N, "cur"), act.c(N, N), log_next.c(N, "log_next"), nxt.c(N, "next")
    r = rg.c(batch.total_rg_points) if rg is not None else None
    m = metrics.c(N) if metrics is not None else None
    _check(fn(C.byref(b), C.byref(c), C.byref(a), C.byref(l), C.byref(r) if r is not None else None, dt, C.byref(n),
              C.byref(m) if m is not None else None, _ptr(ws), ws.numel() if ws is not None else 0, _stream(stream)))


def step(batch: Batch, cur: State, act: Action, log_next: State, rg: Optional[Roadgraph], dt: float, nxt: State,
         metrics: Optional[Metrics] = None, ws: Optional[torch.Tensor] = None, stream=None):
    _step(lib().wm_step, batch, cur, act, log_next, rg, dt, nxt, metrics, ws, stream)


def step_noalloc(batch: Batch, cur: State, act: Action, log_next: State, rg: Optional[Roadgraph], dt: float,
                 nxt: State, metrics: Optional[Metrics] = None, stream=None):
    """step() with the library's device-resident workspace (no ws argument)."""
    N = batch.total_objects
    b, c, a, l, n = batch.c(), cur.c(N, "cur"), act.c(N, N), log_next.c(N, "log_next"), nxt.c(N, "next")
    r = rg.c(batch.total_rg_points) if rg is not None else None
    m = metrics.c(N) if metrics is not None else None
    _check(lib().wm_step_noalloc(C.byref(b), C.byref(c), C.byref(a), C.byref(l), C.byref(r) if r is not None else None,
                                 dt, C.byref(n), C.byref(m) if m is not None else None, _stream(stream)))


def roadgraph_prepare(batch: Batch, rg: Roadgraph, ws: torch.Tensor, stream=None):
    """Compact the road edges into `ws` once for step_prepared()."""
    b, r = batch.c(), rg.c(batch.total_rg_points)
    _check(lib().wm_roadgraph_prepare(C.byref(b), C.byref(r), ws.data_ptr(), ws.numel(), _stream(stream)))


def step_prepared(batch: Batch, cur: State, act: Action, log_next: State, rg: Optional[Roadgraph], dt: float,
                  nxt: State, metrics: Optional[Metrics], ws: torch.Tensor, stream=None):
    """step() reusing the edges that roadgraph_prepare() compacted into `ws`."""
    _step(lib().wm_step_prepared, batch, cur, act, log_next, rg, dt, nxt, metrics, ws, stream)


def step_observe(batch: Batch, cur: State, act: Action, log_next: State, rg: Roadgraph, dt: float, nxt: State,
                 metrics: Optional[Metrics], ws: Optional[torch.Tensor], ego: torch.Tensor, E: int, k: int,
                 rg_idx: torch.Tensor, rg_feat: Optional[torch.Tensor] = None, obj_feat: Optional[torch.Tensor] = None,
                 stream=None):
    """One closed-loop step: step_prepared() then observe() of the successor
    `nxt`, in one library call (off-road metrics read the edges that
    roadgraph_prepare() compacted into `ws`)."""
    N = batch.total_objects
    b, c, a, l, n = batch.c(), cur.c(N, "cur"), act.c(N, N), log_next.c(N, "log_next"), nxt.c(N, "next")
    r = rg.c(batch.total_rg_points)
    m = metrics.c(N) if metrics is not None else None
    _observe_sizes(batch, 1, ego, E, k, rg_idx, rg_feat, obj_feat)
    _need(ws, 0, torch.uint8, "ws")
    _check(lib().wm_step_observe(C.byref(b), C.byref(c), C.byref(a), C.byref(l), C.byref(r), dt, C.byref(n),
                                 C.byref(m) if m is not None else None, ego.data_ptr(), E, k, rg_idx.data_ptr(),
                                 _ptr(rg_feat), _ptr(obj_feat), _ptr(ws), ws.numel() if ws is not None else 0,
                                 _stream(stream)))


def inverse_action(batch: Batch, cur: State, nxt: State, dt: float, accel: torch.Tensor, curvature: torch.Tensor,
                   valid_out: Optional[torch.Tensor] = None, stream=None):
    N = batch.total_objects
    b, c, n = batch.c(), cur.c(N, "cur"), nxt.c(N, "next")
    _need(accel, N, torch.float32, "accel", False)
    _need(curvature, N, torch.float32, "curvature", False)
    _need(valid_out, N, torch.uint8, "valid_out")
    _check(lib().wm_inverse_action(C.byref(b), C.byref(c), C.byref(n), dt, accel.data_ptr(), curvature.data_ptr(),
                                   _ptr(valid_out), _stream(stream)))


def step_delta(batch: Batch, cur: State, dx: torch.Tensor, dy: torch.Tensor, dyaw: torch.Tensor,
               controlled: torch.Tensor, log_next: State, dt: float, nxt: State, stream=None):
    N = batch.total_objects
    b, c, l, n = batch.c(), cur.c(N, "cur"), log_next.c(N, "log_next"), nxt.c(N, "next")
    for t, nm in ((dx, "dx"), (dy, "dy"), (dyaw, "dyaw")):
        _need(t, N, torch.float32, nm, False)
    _need(controlled, N, torch.uint8, "controlled", False)
    a = CDeltaAction(dx.data_ptr(), dy.data_ptr(), dyaw.data_ptr(), controlled.data_ptr())
    _check(lib().wm_step_delta(C.byref(b), C.byref(c), C.byref(a), C.byref(l), dt, C.byref(n), _stream(stream)))


def inverse_delta(batch: Batch, cur: State, nxt: State, dx: torch.Tensor, dy: torch.Tensor, dyaw: torch.Tensor,
                  valid_out: Optional[torch.Tensor] = None, stream=None):
    N = batch.total_objects
    b, c, n = batch.c(), cur.c(N, "cur"), nxt.c(N, "next")
    for t, nm in ((dx, "dx"), (dy, "dy"), (dyaw, "dyaw")):
        _need(t, N, torch.float32, nm, False)
    _need(valid_out, N, torch.uint8, "valid_out")
    _check(lib().wm_inverse_delta(C.byref(b), C.byref(c), C.byref(n), dx.data_ptr(), dy.data_ptr(), dyaw.data_ptr(),
                                  _ptr(valid_out), _stream(stream)))


def discretize(values: torch.Tensor, lo: float, hi: float, bins: int, index: torch.Tensor,
               snapped: Optional[torch.Tensor] = None, stream=None):
    _need(values, 0, torch.float32, "values", False)
    _need(index, values.numel(), torch.int32, "index", False)
    _need(snapped, values.numel(), torch.float32, "snapped")
    _check(lib().wm_discretize(values.data_ptr(), values.numel(), lo, hi, bins, index.data_ptr(), _ptr(snapped),
                               _stream(stream)))


def overlap(batch: Batch, st: State, collision=None, max_margin=None, pair_off=None, margin=None, mask=None,
            stream=None):
    """Collision metric; with `margin` / `mask` also the per-scenario pair
    matrices, whose total size is read back from pair_off[S] (a synchronizing
    copy, so the matrix form is not for graph capture)."""
    N = batch.total_objects
    b, s = batch.c(), st.c(N)
    _need(collision, N, torch.uint8, "collision")
    _need(max_margin, N, torch.float32, "max_margin")
    if margin is not None or mask is not None:
        _need(pair_off, batch.num_scenarios + 1, torch.int64, "pair_off", False)
        # the last block ends at pair_off[S] (host copy: a synchronizing read)
        pairs = int(pair_off[batch.num_scenarios].item())
        _need(margin, pairs, torch.float32, "margin")
        _need(mask, pairs, torch.uint8, "mask")
    _check(lib().wm_overlap(C.byref(b), C.byref(s), _ptr(pair_off), _ptr(margin), _ptr(mask), _ptr(collision),
                            _ptr(max_margin), _stream(stream)))


def offroad(batch: Batch, st: State, rg: Roadgraph, ws: torch.Tensor, offroad=None, margin=None, nearest=None,
            tune=None, stream=None):
    N = batch.total_objects
    b, s, r = batch.c(), st.c(N), rg.c(batch.total_rg_points)
    _need(offroad, N, torch.uint8, "offroad")
    _need(margin, N, torch.float32, "margin")
    _need(nearest, 4 * N, torch.int32, "nearest")
    _need(ws, 0, torch.uint8, "ws", False)
    _check(lib().wm_offroad(C.byref(b), C.byref(s), C.byref(r), _ptr(offroad), _ptr(margin), _ptr(nearest),
                            _tune(tune), ws.data_ptr(), ws.numel(), _stream(stream)))


def _observe_sizes(batch, T, ego, E, k, rg_idx, rg_feat, obj_feat):
    slots = batch.num_scenarios * max(E, 0)
    _need(ego, slots, torch.int32, "ego", False)
    _need(rg_idx, T * slots * max(k, 0), torch.int32, "rg_idx", False)
    _need(rg_feat, T * slots * max(k, 0) * 4, torch.float32, "rg_feat")
    _need(obj_feat, T * slots * batch.max_objects * 8, torch.float32, "obj_feat")


def observe(batch: Batch, st: State, rg: Roadgraph, ego: torch.Tensor, E: int, k: int, rg_idx: torch.Tensor,
            rg_feat=None, obj_feat=None, stream=None):
    b, s, r = batch.c(), st.c(batch.total_objects), rg.c(batch.total_rg_points)
    _observe_sizes(batch, 1, ego, E, k, rg_idx, rg_feat, obj_feat)
    _check(lib().wm_observe(C.byref(b), C.byref(s), C.byref(r), ego.data_ptr(), E, k, rg_idx.data_ptr(),
                            _ptr(rg_feat), _ptr(obj_feat), _stream(stream)))


def observe_seq(batch: Batch, traj: State, T: int, rg: Roadgraph, ego: torch.Tensor, E: int, k: int,
                rg_idx: torch.Tensor, rg_feat: Optional[torch.Tensor] = None, obj_feat: Optional[torch.Tensor] = None,
                stream=None):
    """Observation of every row of a [T, n] state sequence in one launch;
    outputs are [T, ...] with each row as in observe()."""
    b, st, r = batch.c(), traj.c(T * batch.total_objects, "traj"), rg.c(batch.total_rg_points)
    _observe_sizes(batch, T, ego, E, k, rg_idx, rg_feat, obj_feat)
    _check(lib().wm_observe_seq(C.byref(b), C.byref(st), T, C.byref(r), ego.data_ptr(), E, k, rg_idx.data_ptr(),
                                _ptr(rg_feat), _ptr(obj_feat), _stream(stream)))


def rollout(batch: Batch, init: State, act_seq: Action, log_seq: State, rg: Optional[Roadgraph], T: int, dt: float,
            ws: torch.Tensor, ckpt_every: int = 0, ckpt: Optional[State] = None, traj: Optional[State] = None,
            metrics: Optional[Metrics] = None, loss: Optional[torch.Tensor] = None, tune=None, stream=None):
    N = batch.total_objects
    b, i, a, l = batch.c(), init.c(N, "init"), act_seq.c(T * N, N), log_seq.c((T + 1) * N, "log_seq")
    r = rg.c(batch.total_rg_points) if rg is not None else None
    ck = ckpt.c(-(-T // max(ckpt_every, 1)) * N, "ckpt") if ckpt is not None else None
    tr = traj.c(T * N, "traj") if traj is not None else None
    m = metrics.c(T * N) if metrics is not None else None
    _need(loss, batch.num_scenarios, torch.float32, "loss")
    _need(ws, 0, torch.uint8, "ws", False)
    _check(lib().wm_rollout(C.byref(b), C.byref(i), C.byref(a), C.byref(l), C.byref(r) if r is not None else None,
                            T, dt, ckpt_every, C.byref(ck) if ck is not None else None,
                            C.byref(tr) if tr is not None else None, C.byref(m) if m is not None else None,
                            _ptr(loss), _tune(tune), ws.data_ptr(), ws.numel(), _stream(stream)))


def rollout_idm(batch: Batch, init: State, act_seq: Action, log_seq: State, rg: Optional[Roadgraph], T: int,
                dt: float, ws: torch.Tensor, idm: Optional[dict] = None, traj: Optional[State] = None,
                metrics: Optional[Metrics] = None, tune=None, stream=None):
    """Fused rollout with IDM sim agents (every uncontrolled object with a
    fully valid log window); idm overrides entries of IDM_DEFAULT."""
    par = dict(IDM_DEFAULT)
    par.update(idm or {})
    p = CIdm(*[float(par[k]) for k in ("desired_speed", "min_gap", "time_headway", "max_accel", "comfort_decel",
                                       "exponent", "max_brake", "lookahead_step")], int(par["lookahead_poses"]))
    N = batch.total_objects
    b, i, a, l = batch.c(), init.c(N, "init"), act_seq.c(T * N, N), log_seq.c((T + 1) * N, "log_seq")
    r = rg.c(batch.total_rg_points) if rg is not None else None
    tr = traj.c(T * N, "traj") if traj is not None else None
    m = metrics.c(T * N) if metrics is not None else None
    _need(ws, 0, torch.uint8, "ws", False)
    _check(lib().wm_rollout_idm(C.byref(b), C.byref(i), C.byref(a), C.byref(l), C.byref(r) if r is not None else None,
                                T, dt, C.byref(p), C.byref(tr) if tr is not None else None,
                                C.byref(m) if m is not None else None, _tune(tune), ws.data_ptr(), ws.numel(),
                                _stream(stream)))


def rollout_scan_counts(batch: Batch, ws: torch.Tensor, stream=None):
    """Work counts of the last fused rollout run with workspace ws: (blocks
    folded, chunk-box object tests, block-box corner tests); waits for the
    stream."""
    _need(ws, 0, torch.uint8, "ws", False)
    out = (C.c_uint64 * 3)()
    _check(lib().wm_rollout_scan_counts(C.byref(batch.c()), ws.data_ptr(), ws.numel(), out, _stream(stream)))
    return int(out[0]), int(out[1]), int(out[2])


def rollout_backward(batch: Batch, init: State, act_seq: Action, log_seq: State, T: int, dt: float, ckpt_every: int,
                     ckpt: State, dloss: torch.Tensor, grad_accel: torch.Tensor, grad_curvature: torch.Tensor,
                     ws: torch.Tensor, stream=None):
    N = batch.total_objects
    b, i, a, l = batch.c(), init.c(N, "init"), act_seq.c(T * N, N), log_seq.c((T + 1) * N, "log_seq")
    ck = ckpt.c(-(-T // max(ckpt_every, 1)) * N, "ckpt")
    _need(dloss, batch.num_scenarios, torch.float32, "dloss", False)
    _need(grad_accel, T * N, torch.float32, "grad_accel", False)
    _need(grad_curvature, T * N, torch.float32, "grad_curvature", False)
    _need(ws, 0, torch.uint8, "ws", False)
    _check(lib().wm_rollout_backward(C.byref(b), C.byref(i), C.byref(a), C.byref(l), T, dt, ckpt_every,
                                     C.byref(ck), dloss.data_ptr(), grad_accel.data_ptr(), grad_curvature.data_ptr(),
                                     ws.data_ptr(), ws.numel(), _stream(stream)))


def autotune(batch: Batch, init: State, act_seq: Action, log_seq: State, rg: Optional[Roadgraph], T: int, dt: float,
             ws: torch.Tensor, stream=None):
    N = batch.total_objects
    b, i, a, l = batch.c(), init.c(N, "init"), act_seq.c(T * N, N), log_seq.c((T + 1) * N, "log_seq")
    r = rg.c(batch.total_rg_points) if rg is not None else None
    _need(ws, 0, torch.uint8, "ws", False)
    best = CTuning(0, 0)
    _check(lib().wm_autotune(C.byref(b), C.byref(i), C.byref(a), C.byref(l), C.byref(r) if r is not None else None,
                             T, dt, ws.data_ptr(), ws.numel(), C.byref(best), _stream(stream)))
    return best.unit_objects, best.edge_splits


PROF_ROLLOUT, PROF_BACKWARD, PROF_OBSERVE, PROF_OFFROAD = range(4)


def profile_enable(on: bool = True):
    _check(lib().wm_profile_enable(1 if on else 0))


def profile_collect(which: int):
    """(total kernel ms, launches) of one entry point's main kernel since the
    last collect (waits for the recorded events)."""
    ms = C.c_float(0.0)
    cnt = C.c_int32(0)
    _check(lib().wm_profile_collect(which, C.byref(ms), C.byref(cnt)))
    return float(ms.value), int(cnt.value)


class RolloutLoss(torch.autograd.Function):
    """Differentiable rollout: forward = wm_rollout (loss + checkpoints, and
    the step metrics into `metrics` unless it is None), backward =
    wm_rollout_backward (hand-written adjoint).  Inputs accel / curvature
    [T, n] float32; returns the per-scenario loss [S].  Call as
    apply(accel, curvature, batch, init, controlled, log_seq, rg, T, dt,
    ckpt_every, metrics)."""

    @staticmethod
    def forward(ctx, accel, curvature, batch, init, controlled, log_seq, rg, T, dt, ckpt_every, metrics):
        dev = accel.device
        accel = accel.detach().contiguous()
        curvature = curvature.detach().contiguous()
        act = Action(accel, curvature, controlled)
        n_ck = (T + ckpt_every - 1) // ckpt_every
        ckpt = State.empty((n_ck, batch.total_objects), dev)
        ws = batch.workspace(T, ckpt_every)
        loss = torch.empty(batch.num_scenarios, dtype=torch.float32, device=dev)
        rollout(batch, init, act, log_seq, rg, T, dt, ws, ckpt_every=ckpt_every, ckpt=ckpt, metrics=metrics, loss=loss)
        ctx.saved = (batch, init, act, log_seq, T, dt, ckpt_every, ckpt, ws)
        return loss

    @staticmethod
    def backward(ctx, dloss):
        batch, init, act, log_seq, T, dt, ckpt_every, ckpt, ws = ctx.saved
        ga = torch.empty_like(act.accel)
        gk = torch.empty_like(act.curvature)
        rollout_backward(batch, init, act, log_seq, T, dt, ckpt_every, ckpt, dloss.contiguous().float(), ga, gk, ws)
        return ga, gk, None, None, None, None, None, None, None, None, None


# ---------------------------------------------------------------------------
# Upload helpers for host scenes
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DeviceScene:
    batch: Batch
    log_seq: State          # [T+1, n] rollout window, row 0 = initial time
    init: State             # [n] (views of log_seq row 0 copied)
    rg: Roadgraph
    act_seq: Action         # [T, n]
    ego: torch.Tensor       # int32 [S * E]
    T: int
    dt: float


def upload(scene, device) -> DeviceScene:
    """Copy a host scene (synth.Scene) to the device in the ABI's layouts."""
    batch = Batch.from_offsets(scene.obj_off, scene.rg_off, device)
    lw = scene.log_window()
    log_seq = State.from_numpy(lw, device)
    init = State.from_numpy({k: v[0] for k, v in lw.items()}, device)
    rg = Roadgraph.from_numpy(scene.rg, device)
    act = Action(torch.from_numpy(np.ascontiguousarray(scene.accel)).to(device),
                 torch.from_numpy(np.ascontiguousarray(scene.curvature)).to(device),
                 torch.from_numpy(np.ascontiguousarray(scene.controlled)).to(device))
    ego = torch.from_numpy(np.ascontiguousarray(scene.ego.reshape(-1))).to(device)
    return DeviceScene(batch, log_seq, init, rg, act, ego, scene.steps, scene.dt)
