"""Seeded synthetic scenes shaped like the paper's driving workloads.

This module builds INPUTS only: object boxes, logged trajectories, oriented
road-graph polylines and actions.  It contains none of the simulator's own
arithmetic (no bicycle step, no overlap, offroad, divergence or observation
math), so that both the HIP path and the FP64 oracle can consume the same
arrays without sharing any computation.

Workload shape (Sec. 3.1, Sec. 5.1, App. A.3): scenes of up to 128 objects,
logs sampled every 0.1 s, one second of history (states 0..10) followed by an
80-step future, and a static road graph of oriented points (Sec. 3.4,
Off-Road).  The real dataset is not available, so the generator stands in for
it with uniform boxes in a 200 m x 200 m square and random lanes.

Logged trajectories are produced by integrating a continuous-time unicycle
path exactly along circular arcs (constant curvature and constant
longitudinal acceleration inside each 0.1 s interval).  This is a different
model from the paper's discrete bicycle update, the same way real logs are not
produced by the simulator's dynamics, so expert actions recovered by inverse
dynamics reproduce the logs only approximately.

Every array is generated in float64 and stored as float32 (uint8 / int8 /
int32 for flags and offsets).  Random streams are per scenario:
``PCG64(SeedSequence([seed_base + config, scenario]))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

DT = 0.1
T0 = 10              # index of the current state: 11 history states 0..10
BOX = 100.0          # objects and lanes live in [-BOX, BOX]^2
LANE_HALF_WIDTH = 1.8
POINT_SPACING = 0.5
VERTEX_SPACING = 10.0
MAX_TURN = 0.35
TYPE_LANE_CENTER = 0
TYPE_ROAD_EDGE = 1

STATE_FIELDS = ("x", "y", "yaw", "vx", "vy", "length", "width")


@dataclasses.dataclass
class ConfigSpec:
    """Sizes of one workload (see the module docstring for the shapes)."""
    name: str
    scenarios: int
    objects: tuple          # (lo, hi) inclusive; lo == hi for a fixed size
    rg_points: tuple        # (lo, hi) inclusive
    steps: int
    controlled_per_scenario: Optional[int]   # None: every object is controlled
    log_noise: bool         # logs use perturbed actions (configs 1-4)


CONFIGS: Dict[int, ConfigSpec] = {
    0: ConfigSpec("plain step, 1 scenario x 16 objects, 1000 road points, 10 steps",
                  1, (16, 16), (1000, 1000), 10, None, False),
    1: ConfigSpec("batched step + metrics, 256 scenarios x 128 objects, 30000 road points, 80 steps",
                  256, (128, 128), (30000, 30000), 80, None, True),
    2: ConfigSpec("ragged, 1024 scenarios, objects U{8..128}, road points U{2000..30000}, 80 steps",
                  1024, (8, 128), (2000, 30000), 80, None, True),
    3: ConfigSpec("differentiable rollout, 512 scenarios x 128 objects (8 controlled), 30000 road points, 80 steps",
                  512, (128, 128), (30000, 30000), 80, 8, True),
    4: ConfigSpec("observation + rollout, 4096 scenarios, objects U{32..128}, road points U{10000..30000}, 80 steps",
                  4096, (32, 128), (10000, 30000), 80, 8, True),
}


@dataclasses.dataclass
class Scene:
    """A packed (CSR) batch of scenarios, all arrays host numpy.

    Object arrays are indexed by the global object id ``obj_off[s] + i``;
    road-graph arrays by ``rg_off[s] + j``.  Logs are time-major:
    ``log[f][t, g]`` for t in 0..T0+T.
    """
    config: int
    seed_base: int
    obj_off: np.ndarray          # int32 [S+1]
    rg_off: np.ndarray           # int32 [S+1]
    log: Dict[str, np.ndarray]   # float32 [T0+T+1, n] per STATE_FIELDS, 'valid' uint8
    rg: Dict[str, np.ndarray]    # 'x','y','dir_x','dir_y' float32, 'type' int8, 'valid' uint8
    accel: np.ndarray            # float32 [T, n]
    curvature: np.ndarray        # float32 [T, n]
    controlled: np.ndarray       # uint8 [n]
    ego: np.ndarray              # int32 [S, E] global object ids (E = 8 or N_s if fewer)
    steps: int
    dt: float = DT

    @property
    def num_scenarios(self) -> int:
        return int(self.obj_off.shape[0] - 1)

    @property
    def total_objects(self) -> int:
        return int(self.obj_off[-1])

    @property
    def total_rg_points(self) -> int:
        return int(self.rg_off[-1])

    @property
    def max_objects(self) -> int:
        return int(np.max(np.diff(self.obj_off))) if self.num_scenarios else 0

    @property
    def max_rg_points(self) -> int:
        return int(np.max(np.diff(self.rg_off))) if self.num_scenarios else 0

    def state_at(self, t: int) -> Dict[str, np.ndarray]:
        """Logged state at absolute log index t (the rollout starts at T0)."""
        return {k: v[t] for k, v in self.log.items()}

    def log_window(self) -> Dict[str, np.ndarray]:
        """Logs for the rollout window: [T+1, n], index 0 = the initial state."""
        return {k: np.ascontiguousarray(v[T0:T0 + self.steps + 1]) for k, v in self.log.items()}


def _rng(seed_base: int, config: int, scenario: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed_base + config, scenario])))


def _fold(u: np.ndarray) -> np.ndarray:
    """Mirror-fold coordinates into [-BOX, BOX]: a straight path folded this
    way is the same as a path whose heading reflects at the box walls."""
    w = (u + BOX) % (4.0 * BOX)
    return np.where(w <= 2.0 * BOX, w, 4.0 * BOX - w) - BOX


def _polylines(rng: np.random.Generator, lanes: int, n_pts: int) -> np.ndarray:
    """Lane center lines: n_pts points at 0.5 m spacing, a vertex every 10 m
    with a heading change U(-0.35, 0.35) rad, reflected at the box walls.
    Returns float64 [lanes, n_pts, 2]."""
    per_vertex = int(round(VERTEX_SPACING / POINT_SPACING))
    n_vert = max(1, -(-(n_pts - 1) // per_vertex))
    start = rng.uniform(-BOX, BOX, size=(lanes, 2))
    heading = rng.uniform(-math.pi, math.pi, size=lanes)
    turns = rng.uniform(-MAX_TURN, MAX_TURN, size=(lanes, n_vert))
    seg_heading = heading[:, None] + np.cumsum(turns, axis=1)            # [lanes, n_vert]
    h = np.repeat(seg_heading, per_vertex, axis=1)[:, :max(n_pts - 1, 0)]
    steps = POINT_SPACING * np.stack([np.cos(h), np.sin(h)], axis=-1)
    raw = np.concatenate([start[:, None, :], start[:, None, :] + np.cumsum(steps, axis=1)], axis=1)
    return _fold(raw)


def _unit_dirs(pts: np.ndarray) -> np.ndarray:
    """Unit vector from each point to the next one of the same polyline
    (axis -2); the last point repeats its predecessor's direction."""
    d = np.empty_like(pts)
    if pts.shape[-2] == 1:
        d[..., 0, 0], d[..., 0, 1] = 1.0, 0.0
        return d
    seg = pts[..., 1:, :] - pts[..., :-1, :]
    nrm = np.linalg.norm(seg, axis=-1, keepdims=True)
    nrm[nrm == 0] = 1.0
    d[..., :-1, :] = seg / nrm
    d[..., -1, :] = d[..., -2, :]
    return d


def make_roadgraph(rng: np.random.Generator, n_points: int, lanes: int = 8):
    """8 lanes x 3 polylines (center type 0; right edge type 1 in the lane
    direction; left edge type 1 stored reversed so the road lies on the left
    of every edge direction).  floor(P/24) points per polyline, remaining
    points are padded invalid.  Returns dict of float64/int arrays [P]."""
    per = n_points // (3 * lanes)
    used = per * 3 * lanes
    xy = np.zeros((n_points, 2))
    dd = np.zeros((n_points, 2))
    ty = np.zeros(n_points, np.int8)
    if per > 0:
        c = _polylines(rng, lanes, per)                                  # [L, per, 2]
        dc = _unit_dirs(c)
        normal = np.stack([-dc[..., 1], dc[..., 0]], axis=-1)            # left normal
        right = c - LANE_HALF_WIDTH * normal
        left = (c + LANE_HALF_WIDTH * normal)[:, ::-1, :]
        polys = np.stack([c, right, left], axis=1)                       # [L, 3, per, 2]
        xy[:used] = polys.reshape(-1, 2)
        dd[:used] = _unit_dirs(polys).reshape(-1, 2)
        ty[:used] = np.broadcast_to(np.array([TYPE_LANE_CENTER, TYPE_ROAD_EDGE, TYPE_ROAD_EDGE],
                                             np.int8)[None, :, None], (lanes, 3, per)).reshape(-1)
    valid = np.concatenate([np.ones(used, np.uint8), np.zeros(n_points - used, np.uint8)])
    return {"x": xy[:, 0], "y": xy[:, 1], "dir_x": dd[:, 0], "dir_y": dd[:, 1],
            "type": ty, "valid": valid}


def _arc_advance(x, y, yaw, v, a, kappa, dt):
    """Exact motion along a circular arc of curvature kappa while the speed
    changes linearly from v to v + a*dt (continuous-time unicycle; distinct
    from the simulator's discrete update)."""
    s = v * dt + 0.5 * a * dt * dt
    half = 0.5 * kappa * s
    safe = np.where(half == 0, 1.0, half)
    sinc = np.where(np.abs(half) < 1e-8, 1.0 - half * half / 6.0, np.sin(half) / safe)
    mid = yaw + half
    return (x + s * np.cos(mid) * sinc, y + s * np.sin(mid) * sinc,
            yaw + kappa * s, v + a * dt)


def _draw_objects(rng: np.random.Generator, n: int, n_states: int, noise: bool, box: float = BOX):
    """Per-scenario random draws for the object tracks (see make_logs)."""
    d = {
        "x": rng.uniform(-box, box, size=n), "y": rng.uniform(-box, box, size=n),
        "yaw": rng.uniform(-math.pi, math.pi, size=n),
        "length": rng.uniform(4.0, 5.5, size=n), "width": rng.uniform(1.8, 2.2, size=n),
        "speed": rng.uniform(0.0, 15.0, size=n),
        "a_base": rng.uniform(-3.0, 3.0, size=n), "k_base": rng.uniform(-0.1, 0.1, size=n),
    }
    if noise:
        d["a_noise"] = rng.normal(0.0, 0.5, size=(n_states - 1, n))
        d["k_noise"] = rng.normal(0.0, 0.5 * 0.1 / 3.0, size=(n_states - 1, n))
    return d


def make_logs(draws: Dict[str, np.ndarray], n_states: int, noise: bool, dt: float = DT):
    """Logged object tracks [n_states, n] from the initial boxes and actions.

    Initial boxes: x, y ~ U(-100, 100), yaw ~ U[-pi, pi), length ~ U(4, 5.5),
    width ~ U(1.8, 2.2), speed ~ U(0, 15).  Each interval uses the base action
    (accel ~ U(-3, 3), curvature ~ U(-0.1, 0.1)), plus N(0, 0.5^2) accel noise
    and N(0, (0.5 * 0.1/3)^2) curvature noise when `noise`, clipped to the
    action ranges, with accel raised so the speed never drops below 0.5 m/s.
    """
    n = draws["x"].shape[0]
    out = {f: np.empty((n_states, n)) for f in STATE_FIELDS}
    x, y, yaw, v = draws["x"], draws["y"], draws["yaw"], draws["speed"]
    for t in range(n_states):
        out["x"][t], out["y"][t], out["yaw"][t] = x, y, yaw
        out["vx"][t], out["vy"][t] = v * np.cos(yaw), v * np.sin(yaw)
        out["length"][t], out["width"][t] = draws["length"], draws["width"]
        if t == n_states - 1:
            break
        a, k = draws["a_base"], draws["k_base"]
        if noise:
            a = np.clip(a + draws["a_noise"][t], -3.0, 3.0)
            k = np.clip(k + draws["k_noise"][t], -0.1, 0.1)
        a = np.maximum(a, (0.5 - v) / dt)
        x, y, yaw, v = _arc_advance(x, y, yaw, v, a, k, dt)
    return out


def make_scene(config: int, seed_base: int = 1000, scenarios: Optional[int] = None,
               invalid_frac: float = 0.0, rg_invalid_frac: float = 0.0,
               objects: Optional[tuple] = None, rg_points: Optional[tuple] = None,
               steps: Optional[int] = None, controlled_per_scenario: Optional[int] = -1,
               object_box: float = BOX, on_road_frac: float = 0.0) -> Scene:
    """Build the packed scene for one of the workload configs (0..4).

    Optional overrides shrink a config for tests (``scenarios``, ``objects``,
    ``rg_points``, ``steps``).  ``invalid_frac`` marks that fraction of
    objects invalid in every logged state; ``rg_invalid_frac`` marks that
    fraction of road points invalid.  ``object_box`` shrinks the square the
    objects start in (denser scenes, more overlaps); ``on_road_frac`` moves
    that fraction of objects onto a random lane-center point, heading along
    the lane.  The first ``scenarios`` scenarios of a config are identical to
    the full config's first scenarios (for the same options).
    """
    spec = CONFIGS[config]
    S = spec.scenarios if scenarios is None else scenarios
    T = spec.steps if steps is None else steps
    o_lo, o_hi = spec.objects if objects is None else objects
    p_lo, p_hi = spec.rg_points if rg_points is None else rg_points
    ctrl_k = spec.controlled_per_scenario if controlled_per_scenario == -1 else controlled_per_scenario
    n_states = T0 + T + 1

    counts, pcounts, per_draw, per_valid, per_rg, per_act = [], [], [], [], [], []
    for s in range(S):
        rng = _rng(seed_base, config, s)
        n = int(rng.integers(o_lo, o_hi + 1))
        p = int(rng.integers(p_lo, p_hi + 1))
        draws = _draw_objects(rng, n, n_states, spec.log_noise, object_box)
        valid = np.ones(n, np.uint8)
        if invalid_frac > 0:
            valid = (rng.random(n) >= invalid_frac).astype(np.uint8)
        rg = make_roadgraph(rng, p)
        if on_road_frac > 0:
            centers = np.flatnonzero((rg["type"] == TYPE_LANE_CENTER) & (rg["valid"] == 1))
            pick = rng.random(n) < on_road_frac
            if centers.size:
                at = centers[rng.integers(0, centers.size, size=n)]
                draws["x"] = np.where(pick, rg["x"][at], draws["x"])
                draws["y"] = np.where(pick, rg["y"][at], draws["y"])
                draws["yaw"] = np.where(pick, np.arctan2(rg["dir_y"][at], rg["dir_x"][at]), draws["yaw"])
                draws["k_base"] = np.where(pick, 0.0, draws["k_base"])
        if rg_invalid_frac > 0:
            rg["valid"] = rg["valid"] * (rng.random(p) >= rg_invalid_frac).astype(np.uint8)
        if config == 0:
            acc = rng.uniform(-3.0, 3.0, size=(T, n))
            cur = rng.uniform(-0.1, 0.1, size=(T, n))
        else:
            acc = np.broadcast_to(draws["a_base"], (T, n))
            cur = np.broadcast_to(draws["k_base"], (T, n))
        ctrl = np.ones(n, np.uint8) if ctrl_k is None else (np.arange(n) < ctrl_k).astype(np.uint8)
        counts.append(n)
        pcounts.append(p)
        per_draw.append(draws)
        per_valid.append(valid)
        per_rg.append(rg)
        per_act.append((acc, cur, ctrl))

    # integrate every scenario's tracks together (the draws above fix the values)
    all_draws = {k: np.concatenate([d[k] for d in per_draw], axis=-1) for k in per_draw[0]}
    logs64 = make_logs(all_draws, n_states, spec.log_noise)
    obj_off = np.zeros(S + 1, np.int32)
    obj_off[1:] = np.cumsum(counts)
    rg_off = np.zeros(S + 1, np.int32)
    rg_off[1:] = np.cumsum(pcounts)
    log = {f: np.ascontiguousarray(logs64[f].astype(np.float32)) for f in STATE_FIELDS}
    vcat = np.concatenate(per_valid)
    log["valid"] = np.ascontiguousarray(np.broadcast_to(vcat, (n_states, vcat.shape[0])).astype(np.uint8))
    rg = {k: np.ascontiguousarray(np.concatenate([r[k] for r in per_rg]).astype(
        np.float32 if k in ("x", "y", "dir_x", "dir_y") else per_rg[0][k].dtype)) for k in per_rg[0]}
    accel = np.ascontiguousarray(np.concatenate([a for a, _, _ in per_act], axis=1).astype(np.float32))
    curvature = np.ascontiguousarray(np.concatenate([c for _, c, _ in per_act], axis=1).astype(np.float32))
    controlled = np.concatenate([c for _, _, c in per_act]).astype(np.uint8)
    E = 8
    ego = np.stack([obj_off[s] + np.minimum(np.arange(E), counts[s] - 1) for s in range(S)]).astype(np.int32)
    return Scene(config=config, seed_base=seed_base, obj_off=obj_off, rg_off=rg_off, log=log, rg=rg,
                 accel=accel, curvature=curvature, controlled=controlled, ego=ego, steps=T)
