"""Benchmark of the simulator hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Workload: 256 scenarios x 128 objects, 30,000 road points per scenario
(about 20,000 road-edge points), an 80-step rollout at dt = 0.1 s (synthetic
scenes shaped like the paper's runtime benchmark, Sec. 5.1 / App. A.3).  One
timed step is one expert rollout (RolloutExpert in the paper's runtime
table): expert actions from inverse kinematics on the logs, then the fused
persistent rollout kernel with every metric (collision, off-road,
displacement) at every step.  The step is captured once as a HIP graph and
the K timed steps are K replays: value = agent-steps/s = valid objects x 80 x
K / wall time; the per-replay median and minimum come from HIP events
between the replays.

Also reported on the same line: the dominant kernel against the FP32 roofline
(HIP events around the persistent kernel over K more steps), the FP64 CPU
oracle on bounded samples of the workloads, the plain per-step form
(separate launches per operation, captured in a HIP graph), the
differentiable rollout (forward + adjoint) of the configurations with
8 and with all objects controlled, the observation (8 egos per scenario,
k = 1000), the ragged batches of 1,024 and 4,096 scenarios, the closed loop
of step + observation, IDM agents and the per-step latency at batch 1 and 16.
Progress goes to stderr; stdout carries exactly one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12        # MI355X FP32 vector peak [FLOP/s] (published)
PEAK_HBM = 8.0e12           # MI355X HBM3E [B/s] (published)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def edge_counts(scene):
    is_edge = (scene.rg["type"] == 1) & (scene.rg["valid"] == 1)
    c = np.concatenate([[0], np.cumsum(is_edge.astype(np.int64))])
    return c[scene.rg_off[1:]] - c[scene.rg_off[:-1]]


def rollout_ops(scene, T):
    """Algorithmic FP32 operations of one fused rollout launch: per agent-step,
    off-road 4 corners x E_s edge points x 6 ops, overlap 20 ops x (N_s - 1)
    (40 ops per pair, each pair shared by two agents), dynamics and
    displacement 35 ops."""
    N = np.diff(scene.obj_off).astype(np.float64)
    E = edge_counts(scene).astype(np.float64)
    per_step = (N * (4.0 * E * 6.0 + 20.0 * np.maximum(N - 1, 0) + 35.0)).sum()
    return per_step * T, float((4.0 * N * E).sum() * T)


def rollout_executed_ops(scene, T, counts):
    """FP32 operations one fused rollout launch executes, from the kernel's
    own work counts (wm_rollout_scan_counts): a folded road-edge block is 32
    points x the 16 corners of a group at the 6 ops of a corner-point pair; a
    box test (chunk box against an object circle, block box against a corner)
    10 ops (4 subtractions, 2 max3, a product, an FMA, a comparison); overlap,
    dynamics and displacement as in rollout_ops.  Returns (ops, corner-point
    pairs)."""
    folded, ctests, btests = counts
    N = np.diff(scene.obj_off).astype(np.float64)
    rest = (N * (20.0 * np.maximum(N - 1, 0) + 35.0)).sum() * T
    pairs = 512.0 * folded
    return 6.0 * pairs + 10.0 * (ctests + btests) + rest, pairs


def rollout_roofline(scene, T, kernel_ms, counts, traffic):
    """The k_rollout roofline entry: achieved by the method's algorithmic
    count (rollout_ops), the executed work beside it."""
    ops, pairs = rollout_ops(scene, T)
    achieved = ops / (kernel_ms * 1e-3)
    xops, xpairs = rollout_executed_ops(scene, T, counts)
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": traffic, "kernel": "k_rollout", "kernel_ms": kernel_ms,
            "ops_per_launch": ops, "corner_edge_pairs_per_launch": pairs,
            "count": "algorithmic: every corner of every valid object against every road-edge point each step "
                     "(Sec. 3.4 Off-Road); the kernel evaluates only the road-edge blocks that a corner can "
                     "reach (exact result), so this rate can exceed the FP32 peak",
            "executed": {"ops_per_launch": xops, "corner_point_pairs": xpairs, "tflops": xops / (kernel_ms * 1e-3) / 1e12,
                         "frac": xops / (kernel_ms * 1e-3) / PEAK_FP32, "blocks_folded": counts[0],
                         "box_tests": counts[1] + counts[2], "pairs_vs_algorithmic": xpairs / pairs}}


# Algorithmic FP32 ops of the adjoint (FMA = 2): per ordered pair (controlled
# object, valid partner) and step, the separating-axis margin (49: offsets 2,
# relative rotation 6, absolute values 2, four projections 12, four gaps 24,
# minimum 3), the gradient through the arg-min axis (9), the sigmoid and its
# derivative (7) and the accumulation (6): 71; per controlled object and step,
# the recomputed bicycle step (20) and its adjoint with the log term (50): 70.
# The adjoint first tests every (controlled object, partner) pair against a
# distance bound (offsets 2, squared distance 2, radius sum 3, its square
# doubled 2, comparison 1: 10) and evaluates the 71-op term only where the
# term can be non-zero in FP32.
ADJ_OPS_PER_PAIR = 71
ADJ_OPS_PER_OBJECT = 70
ADJ_OPS_PER_TEST = 10
ADJ_CULL_GAP = 9.0   # metres; the same bound as the kernel's


def adjoint_executed_ops(obj_off, controlled, init, log_seq, traj, T):
    """Ops one adjoint launch executes, and the pair terms it evaluates: every
    (controlled object, partner) pair is tested at every step, and the terms
    within the bound sqrt(2) (r_i + r_j + ADJ_CULL_GAP) (r = half length + half
    width; an object is never its own partner) are evaluated.  States:
    controlled objects from the trajectory, the others from the log.  Scenes
    of uniform object count."""
    import torch
    off = obj_off.cpu().numpy()
    S, N = len(off) - 1, int(off[1] - off[0])
    assert (np.diff(off) == N).all(), "uniform object counts only"
    ctrl = (controlled != 0) & (init.valid != 0)
    nc = int(ctrl.sum())
    near = 0
    for t in range(1, T + 1):
        x = torch.where(ctrl, traj.x[t - 1], log_seq.x[t]).view(S, N)
        y = torch.where(ctrl, traj.y[t - 1], log_seq.y[t]).view(S, N)
        ln = torch.where(ctrl, init.length, log_seq.length[t])
        wd = torch.where(ctrl, init.width, log_seq.width[t])
        r = (0.5 * (ln + wd)).view(S, N)
        d2 = (x[:, :, None] - x[:, None, :]) ** 2 + (y[:, :, None] - y[:, None, :]) ** 2
        rs = r[:, :, None] + r[:, None, :] + ADJ_CULL_GAP
        m = (d2 <= 2.0 * rs * rs) & ctrl.view(S, N)[:, :, None]
        m &= ~torch.eye(N, dtype=torch.bool, device=m.device)[None]
        near += int(m.sum())
    ops = T * (ADJ_OPS_PER_TEST * nc * N + ADJ_OPS_PER_OBJECT * nc) + ADJ_OPS_PER_PAIR * near
    return float(ops), float(near), float(T * nc * (N - 1))


# The method's work of the adjoint, as counted for its roofline: per scenario
# and step, every unordered pair of valid objects with a controlled member
# (nc (N - 1) - nc (nc - 1) / 2 pairs; 988 at N = 128 with 8 controlled) costs
# about 40 FP32 ops for the separating-axis margin and its soft-overlap term,
# three times over (the recomputed forward, the term, its reverse).  The
# executed count above sits beside it: the kernel skips pairs whose term is
# exactly zero in FP32.
ADJ_ALG_OPS_PER_PAIR = 120


def adjoint_algorithmic_ops(obj_off, controlled, valid, T):
    """(ops, pairs) of one adjoint launch over T steps by the count above;
    host arrays, `valid` of the initial state."""
    off = np.asarray(obj_off).astype(np.int64)
    ctrl = (np.asarray(controlled) != 0) & (np.asarray(valid) != 0)
    vld = np.asarray(valid) != 0
    cc = np.concatenate([[0], np.cumsum(ctrl)])
    cv = np.concatenate([[0], np.cumsum(vld)])
    nc = cc[off[1:]] - cc[off[:-1]]
    nv = cv[off[1:]] - cv[off[:-1]]
    pairs = float(np.sum(nc * np.maximum(nv - 1, 0) - nc * (nc - 1) // 2))
    return ADJ_ALG_OPS_PER_PAIR * pairs * T, pairs * T


# Algorithmic work of the default observation per ego and state row: each of
# the scenario's P_s road points costs 5 FP32 ops for its key dx^2 + dy^2 from
# the ego centre (two differences, a product and an FMA) and 4 for one
# selection pass (compare with the bound, count, place).  Bytes written: k
# road entries of 20 B (index and four features) and max_objects object
# entries of 32 B; the bound is HBM (the writes), with the VALU fraction
# beside it.
OBS_OPS_PER_POINT = 9


def observe_roofline(out_bytes, ops, kernel_ms):
    sec = kernel_ms * 1e-3
    return {"bound": "hbm", "achieved": out_bytes / sec / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": out_bytes / sec / PEAK_HBM, "traffic": None, "kernel": "k_observe", "kernel_ms": kernel_ms,
            "bytes_per_launch": out_bytes,
            "valu": {"achieved": ops / sec / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": ops / sec / PEAK_FP32, "ops_per_launch": ops}}


def adjoint_roofline(alg_ops, alg_pairs, xops, xnear, kernel_ms):
    """The adjoint kernel against the FP32 peak by the method's count, with
    the executed count beside it."""
    sec = kernel_ms * 1e-3
    r = {"bound": "alu", "achieved": alg_ops / sec / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
         "frac": alg_ops / sec / PEAK_FP32, "kernel": "k_rollout_backward", "kernel_ms": kernel_ms,
         "ops_per_launch": alg_ops, "pair_steps_with_a_controlled_member": alg_pairs}
    if xops is not None:
        r["executed"] = {"ops_per_launch": xops, "pair_terms_evaluated": xnear, "achieved": xops / sec / 1e12,
                         "frac": xops / sec / PEAK_FP32}
    return r


# The sources k_rollout is compiled from: its counters stay valid while these
# and the tuning are unchanged.
ROLLOUT_SOURCES = ("paper_2310_08710_amd/csrc/wm_kernels.hip", "paper_2310_08710_amd/csrc/wm_device.h",
                   "paper_2310_08710_amd/csrc/wm_internal.h", "include/wm.h")


def rollout_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in ROLLOUT_SOURCES:
        h.update(open(os.path.join(ROOT, rel), "rb").read())
    return h.hexdigest()


def recorded_traffic(tune):
    """HBM-side bytes per k_rollout launch from the committed rocprofv3
    counter runs, or None when k_rollout's sources or the tuning changed
    since."""
    path = os.path.join(ROOT, "profiles", "k_rollout_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != rollout_sources_sha256() or list(rec.get("tuning", [])) != list(tune or []):
        return None
    return float(rec["traffic_bytes_per_launch"])


def cpu_info():
    """nproc, the cores this process may run on and the CPU model string."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"nproc": os.cpu_count(), "usable_cores": usable, "model": model}


def _f64(d):
    return {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in d.items()}


def _scenario(scene, lw, s):
    """Host inputs of scenario s alone (local offsets)."""
    o0, o1 = int(scene.obj_off[s]), int(scene.obj_off[s + 1])
    p0, p1 = int(scene.rg_off[s]), int(scene.rg_off[s + 1])
    sub = {k: v[:, o0:o1] for k, v in lw.items()}
    return (np.array([0, o1 - o0], np.int32), np.array([0, p1 - p0], np.int32), sub,
            _f64({k: v[p0:p1] for k, v in scene.rg.items()}), scene.accel[:, o0:o1], scene.curvature[:, o0:o1],
            scene.controlled[o0:o1])


def _pool_time(fn, items, threads):
    """Wall time of fn over items on `threads` threads (the oracle's C calls
    release the interpreter lock, so the threads run in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.perf_counter()
    if threads == 1:
        res = [fn(i) for i in items]
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            res = list(ex.map(fn, items))
    return res, time.perf_counter() - t0


def cpu_forward(scene, scen_ids, threads):
    """The FP64 oracle's rollout with every metric on the given scenarios, one
    scenario per task: (agent-steps/s, wall seconds)."""
    import oracle
    lw = scene.log_window()
    T = scene.steps

    def one(s):
        oo, ro, sub, rg, a, k, c = _scenario(scene, lw, s)
        oracle.rollout(oo, ro, _f64({q: v[0] for q, v in sub.items()}), a, k, c, _f64(sub), rg, T, scene.dt,
                       metrics=True, want_loss=False)
        return int(sub["valid"][0].sum())

    oracle.lib()
    objs, wall = _pool_time(one, scen_ids, threads)
    return sum(objs) * T / wall, wall


def cpu_fwd_bwd(scene, scen_ids, threads):
    """The FP64 oracle's loss and hand-written reverse-mode gradient (its
    forward runs inside, with a full tape) on the given scenarios:
    (rollout scenario-steps/s, wall seconds)."""
    import oracle
    lw = scene.log_window()
    T = scene.steps

    def one(s):
        oo, _, sub, _, a, k, c = _scenario(scene, lw, s)
        oracle.rollout_grad(oo, _f64({q: v[0] for q, v in sub.items()}), a, k, c, _f64(sub), T, scene.dt)
        return 1

    oracle.lib()
    n, wall = _pool_time(one, scen_ids, threads)
    return sum(n) * T / wall, wall


def cpu_baselines(scene1, threads):
    """The oracle as it stands on the host cores: the config-1 forward on all
    `threads` and on one thread, and fwd+bwd samples of the differentiable
    and the 4,096-scenario workloads."""
    from paper_2310_08710_amd import synth
    info = cpu_info()
    sample = 2 * threads
    rate, wall = cpu_forward(scene1, range(sample), threads)
    rate1, wall1 = cpu_forward(scene1, range(1), 1)
    out = {"value": rate, "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
           "sample": "%d of the 256 scenarios of the bench workload, all 80 steps with every metric, FP64 C oracle, "
                     "one scenario per thread (%.1f s wall)" % (sample, wall),
           "nproc": info["nproc"], "usable_cores": info["usable_cores"], "cpu_model": info["model"],
           "single_thread": {"value": rate1, "unit": "agent-steps/s", "sample": "scenario 0 (%.1f s)" % wall1}}
    log("cpu oracle: %.3e agent-steps/s on %d threads (%.1f s); one thread %.3e" % (rate, threads, wall, rate1))
    for cfg, key, n_s in ((3, "fwd_bwd_config3", 512), (4, "fwd_bwd_config4", 1024)):
        sc = synth.make_scene(cfg, scenarios=n_s)
        r, w = cpu_fwd_bwd(sc, range(n_s), threads)
        out[key] = {"value": r, "unit": "rollout scenario-steps/s", "cores": threads,
                    "sample": "%d scenarios of the %s workload, loss-only forward + reverse-mode gradient "
                              "(full tape), FP64, one scenario per task (%.1f s wall)" % (
                                  n_s, "512 x 128" if cfg == 3 else "4096-scenario", w)}
        log("cpu oracle fwd+bwd config %d: %.3e scenario-steps/s (%.1f s)" % (cfg, r, w))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip plain / fwd+bwd / observation")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune", type=str, default=None, help="unit_objects,edge_splits (skips the autotuner)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the adjoint of config 1 (every object controlled), for profiling it")
    ap.add_argument("--observe-only", action="store_true",
                    help="only time the observation of config 1 (one row, then the 80 logged rows) and exit")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device once (calibrates HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_probe:
        import torch
        src = torch.ones(args.copy_probe * 262144, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB" % args.copy_probe)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (scenarios are independent, "
              "so N GPUs would each run their own share of the batch); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_08710_amd import synth, wm

    dev = torch.device("cuda:0")
    wm.lib()
    if args.adjoint_only:
        print(json.dumps(adjoint_only(dev)), flush=True)
        return
    t = time.perf_counter()
    scene = synth.make_scene(1)
    ds = wm.upload(scene, dev)
    torch.cuda.synchronize()
    S, n, T = scene.num_scenarios, scene.total_objects, scene.steps
    log("scene: %d scenarios, %d objects, %d road points, T=%d (%.1fs)" % (S, n, scene.total_rg_points, T,
                                                                          time.perf_counter() - t))

    # expert actions for the whole window in one launch: rows 0..T-1 -> 1..T
    inv_batch = wm.Batch(ds.batch.obj_off, ds.batch.rg_off, 1, T * n, ds.batch.total_rg_points, 0, 0)
    lg = ds.log_seq
    cur = wm.State(*[getattr(lg, f)[:T] for f in wm.STATE_FIELDS + ("valid",)])
    nxt = wm.State(*[getattr(lg, f)[1:] for f in wm.STATE_FIELDS + ("valid",)])
    ea = torch.empty((T, n), device=dev)
    ek = torch.empty((T, n), device=dev)
    expert = wm.Action(ea, ek, ds.act_seq.controlled)
    if args.observe_only:
        obs = {"workload": "default observation of config 1: 8 egos per scenario, k = 1000, logged rows 1..80"}
        observation(obs, scene, ds, dev, nxt)
        print(json.dumps(obs), flush=True)
        return
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    ws = ds.batch.workspace(T, 10)

    tune = None
    if args.tune:
        tune = tuple(int(v) for v in args.tune.split(","))
    elif not args.no_autotune:
        wm.inverse_action(inv_batch, cur, nxt, scene.dt, ea, ek)
        tune = wm.autotune(ds.batch, ds.init, expert, ds.log_seq, ds.rg, T, scene.dt, ws)
        log("autotuned (unit_objects, edge_splits) =", tune)

    def step():
        wm.inverse_action(inv_batch, cur, nxt, scene.dt, ea, ek)
        wm.rollout(ds.batch, ds.init, expert, ds.log_seq, ds.rg, T, scene.dt, ws, traj=traj, metrics=met,
                   tune=tune)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # the step as one HIP graph (captured on a side stream, replayed on the
    # current one)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    graph.replay()
    torch.cuda.synchronize()
    # timed region: K replays; HIP events between them give the per-step
    # median and minimum, the wall clock over all K gives `value`
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        graph.replay()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    del graph
    # kernel timing: K more steps launched directly, with HIP events around
    # k_rollout on the stream it runs on (events inside a graph are not timed)
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_ROLLOUT)
    t1 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    eager_wall = time.perf_counter() - t1
    kms, launches = wm.profile_collect(wm.PROF_ROLLOUT)
    wm.profile_enable(False)
    valid_objs = int(scene.log["valid"][synth.T0].sum())
    value = valid_objs * T * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    kernel_ms = kms / max(launches, 1)
    roof = rollout_roofline(scene, T, kernel_ms, wm.rollout_scan_counts(ds.batch, ws), recorded_traffic(tune))
    log("fused rollout (graph replays): %.3f ms/step (median %.3f, min %.3f), kernel %.3f ms, %.3e agent-steps/s, "
        "%.1f TFLOP/s algorithmic, %.1f TFLOP/s executed (%.2f%% of the corner-point pairs)"
        % (ms_per_step, step_ms[len(step_ms) // 2], step_ms[0], kernel_ms, value, roof["achieved"],
           roof["executed"]["tflops"], 100 * roof["executed"]["pairs_vs_algorithmic"]))
    assert torch.isfinite(met.offroad_margin).all() and torch.isfinite(traj.x).all()

    out = {
        "metric": "agent-steps/s (step+metrics)",
        "value": value,
        "unit": "agent-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "step_ms_median": step_ms[len(step_ms) // 2],
        "step_ms_min": step_ms[0],
        "timing": "K replays of the step captured as one HIP graph; the kernel time comes from K more steps "
                  "launched directly (%.3f ms per step)" % (1e3 * eager_wall / args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "expert rollout of 256 scenarios x 128 objects, 30000 road points "
                               "(~20000 road edges) per scenario, 80 steps, every metric every step",
                   "scenarios": S, "objects_per_scenario": 128, "rg_points": 30000, "T": T,
                   "tuning": list(tune) if tune else None},
        "roofline": roof,
    }

    if not args.no_extras:
        extras(out, scene, ds, dev, inv_batch, cur, nxt, ea, ek, expert, tune, traj, met)

    if not args.no_cpu:
        threads = max(1, min(cpu_info()["usable_cores"], 16))
        out["cpu_baseline"] = cpu_baselines(scene, threads)
    print(json.dumps(out), flush=True)


def observe_once(scene, ds, dev, st, reps=3, E=8, K=1000):
    """Time the default observation of one state row for every scenario's E
    egos (k = K): wall ms per call and the k_observe roofline entry."""
    import torch
    from paper_2310_08710_amd import wm
    S = scene.num_scenarios
    P = float(np.sum(np.diff(scene.rg_off)))
    idx = torch.empty(S * E * K, dtype=torch.int32, device=dev)
    rf = torch.empty(S * E * K * 4, device=dev)
    of = torch.empty(S * E * ds.batch.max_objects * 8, device=dev)
    wm.observe(ds.batch, st, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_OBSERVE)
    t0 = time.perf_counter()
    for _ in range(reps):
        wm.observe(ds.batch, st, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    oms = 1e3 * (time.perf_counter() - t0) / reps
    kms, kl = wm.profile_collect(wm.PROF_OBSERVE)
    wm.profile_enable(False)
    out_bytes = S * E * (K * 20.0 + ds.batch.max_objects * 32.0)
    ops = OBS_OPS_PER_POINT * P * E
    okm = kms / max(kl, 1)
    return oms, observe_roofline(out_bytes, ops, okm), (idx, rf, of)


def observation(out, scene, ds, dev, rows_state, reps=3):
    """Time the default observation of config 1 (8 egos per scenario, k =
    1000): one state row, then every row of `rows_state` (T rows) in one
    launch.  Besides the output rate, `point_reads_TBps` is the rate at which
    the kernel reads road points (x, y, valid: 9 B) from cache, once per ego
    and row."""
    import torch
    from paper_2310_08710_amd import wm
    S, T = scene.num_scenarios, scene.steps
    E, K = 8, 1000
    point_bytes = 9.0 * float(np.sum(np.diff(scene.rg_off))) * E
    oms, roof, bufs = observe_once(scene, ds, dev, ds.init, reps, E, K)
    del bufs
    okm = roof["kernel_ms"]
    out["observe"] = {"egos_per_s": S * E / (oms * 1e-3), "ms": oms, "kernel_ms": okm, "k": K, "egos": S * E,
                      "roofline": roof, "point_reads_TBps": point_bytes / (okm * 1e-3) / 1e12}
    log("observe: %.3f ms for %d egos (kernel %.3f ms, %.1f%% of HBM)" % (oms, S * E, okm, 100 * roof["frac"]))

    # every row of a trajectory in one launch
    idx = torch.empty((T, S * E * K), dtype=torch.int32, device=dev)
    rf = torch.empty((T, S * E * K * 4), device=dev)
    of = torch.empty((T, S * E * ds.batch.max_objects * 8), device=dev)
    wm.observe_seq(ds.batch, rows_state, T, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_OBSERVE)
    t0 = time.perf_counter()
    wm.observe_seq(ds.batch, rows_state, T, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    sms = 1e3 * (time.perf_counter() - t0)
    kms, kl = wm.profile_collect(wm.PROF_OBSERVE)
    wm.profile_enable(False)
    skm = kms / max(kl, 1)
    out_bytes = T * S * E * (K * 20.0 + ds.batch.max_objects * 32.0)
    ops = T * OBS_OPS_PER_POINT * float(np.sum(np.diff(scene.rg_off))) * E
    sroof = observe_roofline(out_bytes, ops, skm)
    out["observe_seq"] = {"ms": sms, "kernel_ms": skm, "rows": T, "egos_per_row": S * E, "k": K,
                          "ego_steps_per_s": T * S * E / (sms * 1e-3), "roofline": sroof,
                          "point_reads_TBps": T * point_bytes / (skm * 1e-3) / 1e12}
    log("observe_seq: %.3f ms for %d steps x %d egos (%.1f%% of HBM)" % (sms, T, S * E, 100 * sroof["frac"]))


def extras(out, scene, ds, dev, inv_batch, cur, nxt, ea, ek, expert, tune, fused_traj, fused_met):
    import torch
    from paper_2310_08710_amd import synth, wm
    S, n, T = scene.num_scenarios, scene.total_objects, scene.steps
    reps = 3

    # plain form: one launch per operation and step, replayed as a HIP graph
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    ws0 = ds.batch.workspace()
    fields = ("collision", "offroad", "overlap_margin", "offroad_margin", "log_div")

    def plain():
        # the road edges are compacted once per rollout, as in the fused form
        wm.inverse_action(inv_batch, cur, nxt, scene.dt, ea, ek)
        wm.roadgraph_prepare(ds.batch, ds.rg, ws0)
        c = ds.init
        for t in range(1, T + 1):
            act = wm.Action(ea[t - 1], ek[t - 1], ds.act_seq.controlled)
            m = wm.Metrics(*[getattr(met, f)[t - 1] for f in fields])
            wm.step_prepared(ds.batch, c, act, ds.log_seq.row(t), ds.rg, scene.dt, traj.row(t - 1), m, ws0)
            c = traj.row(t - 1)

    pms = _time_graph(plain, reps)
    fused_ms = out["ms_per_step"]
    same = all(torch.equal(getattr(fused_met, f), getattr(met, f)) for f in fields) and \
        torch.equal(fused_traj.x, traj.x)
    out["plain"] = {"value": n * T / (pms * 1e-3), "unit": "agent-steps/s", "ms_per_rollout": pms,
                    "form": "road-edge compaction once, then per-step launches (dynamics, overlap, off-road) "
                            "in one HIP graph",
                    "fused_speedup": pms / fused_ms, "identical_outputs": bool(same)}
    log("plain graph: %.3f ms/rollout (fused speedup %.2fx, identical %s)" % (pms, pms / fused_ms, same))
    del traj, met

    # differentiable rollout: forward (every metric + loss + checkpoints) + adjoint
    a = ea.clone().requires_grad_(True)
    k = ek.clone().requires_grad_(True)
    fmet = wm.Metrics.empty((T, n), dev)

    def fwd_bwd():
        a.grad = None
        k.grad = None
        L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, ds.rg, T, scene.dt, 10,
                                 fmet)
        L.sum().backward()

    fwd_bwd()
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_BACKWARD)
    t0 = time.perf_counter()
    for _ in range(reps):
        fwd_bwd()
    torch.cuda.synchronize()
    fbms = 1e3 * (time.perf_counter() - t0) / reps
    bms, bl = wm.profile_collect(wm.PROF_BACKWARD)
    wm.profile_enable(False)
    bkm = bms / max(bl, 1)
    # the trajectory of these actions: the expert rollout, every object controlled
    xops, xnear, _ = adjoint_executed_ops(ds.batch.obj_off, ds.act_seq.controlled, ds.init, ds.log_seq, fused_traj,
                                          T)
    alg, alg_pairs = adjoint_algorithmic_ops(scene.obj_off, scene.controlled, scene.log["valid"][synth.T0], T)
    out["fwd_bwd"] = {"value": S * T / (fbms * 1e-3), "unit": "rollout scenario-steps/s",
                      "agent_steps_per_s": n * T / (fbms * 1e-3), "ms_per_rollout": fbms,
                      "backward_kernel_ms": bkm, "controlled": "all objects", "checkpoint_every": 10,
                      "backward_roofline": adjoint_roofline(alg, alg_pairs, xops, xnear, bkm)}
    log("fwd+bwd: %.3f ms/rollout (adjoint kernel %.3f ms, %.1f%% of FP32 by the method's count)" % (
        fbms, bkm, 100 * out["fwd_bwd"]["backward_roofline"]["frac"]))
    del a, k, fmet

    observation(out, scene, ds, dev, fused_traj, reps)
    closed_loop(out, scene, ds, dev, fused_ms)
    step_latency(out, dev)
    ragged(out, dev)
    idm(out, scene, ds, dev, tune)
    fwd_bwd_config3(out, dev)
    config4(out, dev)


def closed_loop(out, scene, ds, dev, fused_ms, E=8, K=1000):
    """Closed-loop simulation of the bench workload: 80 calls of
    wm_step_observe (dynamics, every metric, then the successor's default
    observation for 8 egos per scenario, k = 1000, with road and object
    features), captured as one HIP graph; per-step latency and the cost
    against the fused rollout of the same 80 steps (which has no
    observation)."""
    import torch
    from paper_2310_08710_amd import wm
    S, n, T = scene.num_scenarios, scene.total_objects, scene.steps
    maxN = ds.batch.max_objects
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    idx = torch.empty((S * E * K,), dtype=torch.int32, device=dev)
    rf = torch.empty((S * E * K * 4,), device=dev)
    of = torch.empty((S * E * maxN * 8,), device=dev)
    ws = ds.batch.workspace()
    wm.roadgraph_prepare(ds.batch, ds.rg, ws)
    acts = [wm.Action(ds.act_seq.accel[t], ds.act_seq.curvature[t], ds.act_seq.controlled) for t in range(T)]

    def loop():
        c = ds.init
        for t in range(1, T + 1):
            wm.step_observe(ds.batch, c, acts[t - 1], ds.log_seq.row(t), ds.rg, scene.dt, traj.row(t - 1),
                            met.row(t - 1), ws, ds.ego, E, K, idx, rf, of)
            c = traj.row(t - 1)

    ms = _time_graph(loop, 3)
    out["closed_loop"] = {"ms_per_rollout": ms, "ms_per_step": ms / T, "unit": "agent-steps/s",
                          "value": n * T / (ms * 1e-3), "ego_observations_per_s": S * E * T / (ms * 1e-3),
                          "vs_fused_rollout": ms / fused_ms,
                          "workload": "80 x wm_step_observe on the bench workload (every metric, then 8 egos per "
                                      "scenario, k = 1000, road and object features), one HIP graph"}
    log("closed loop: %.3f ms per 80 steps (%.3f ms/step, %.2fx the fused rollout)" % (ms, ms / T, ms / fused_ms))


def step_latency(out, dev, reps=50):
    """Per-step latency of the plain step on a prepared road graph (one HIP
    graph replay per step): transition only and transition + every metric,
    for the 1 x 16-object scene and for 1 and 16 scenarios of 128 objects with
    30,000 road points (the paper's Step / Transition / Metrics rows at batch
    1 and 16); plus the 80-step expert rollout at those batches."""
    import torch
    from paper_2310_08710_amd import synth, wm
    res = {}
    for key, cfg, S in (("config0_1x16", 0, None), ("bs1_128", 1, 1), ("bs16_128", 1, 16)):
        sc = synth.make_scene(cfg, scenarios=S)
        ds = wm.upload(sc, dev)
        n, T = sc.total_objects, sc.steps
        ws = ds.batch.workspace()
        wm.roadgraph_prepare(ds.batch, ds.rg, ws)
        act = wm.Action(ds.act_seq.accel[0], ds.act_seq.curvature[0], ds.act_seq.controlled)
        nxt = wm.State.empty(n, dev)
        met = wm.Metrics.empty(n, dev)
        tr = _time_graph(lambda: wm.step_prepared(ds.batch, ds.init, act, ds.log_seq.row(1), None, sc.dt, nxt, None,
                                                  ws), reps, median=True)
        st = _time_graph(lambda: wm.step_prepared(ds.batch, ds.init, act, ds.log_seq.row(1), ds.rg, sc.dt, nxt, met,
                                                  ws), reps, median=True)
        wsr = ds.batch.workspace(T, 0)
        traj = wm.State.empty((T, n), dev)
        mets = wm.Metrics.empty((T, n), dev)
        ro = _time_graph(lambda: wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, wsr, traj=traj,
                                            metrics=mets), 5, median=True)
        res[key] = {"scenarios": sc.num_scenarios, "objects": n, "rg_points_per_scenario": int(sc.rg_off[1]),
                    "transition_ms": tr, "step_ms": st, "metrics_ms": st - tr,
                    "step_agent_steps_per_s": n / (st * 1e-3), "rollout_steps": T, "rollout_ms": ro}
        log("step latency %s: transition %.4f ms, step + metrics %.4f ms, %d-step rollout %.3f ms" % (
            key, tr, st, T, ro))
    out["step_latency"] = res


def config4(out, dev, reps=3, E=8, K=1000):
    """4,096 ragged scenarios (objects U{32..128}, road points U{10000..30000}):
    the default observation of 8 egos per scenario (32,768 egos, k = 1000),
    then the 80-step fused rollout with every metric, loss and checkpoints
    every 10 steps plus the adjoint (RolloutLoss forward + backward), 8
    controlled objects per scenario."""
    import torch
    from paper_2310_08710_amd import synth, wm
    t = time.perf_counter()
    sc = synth.make_scene(4)
    ds = wm.upload(sc, dev)
    log("config 4 scene: %d scenarios, %d objects, %d road points (%.1f s)" % (
        sc.num_scenarios, sc.total_objects, sc.total_rg_points, time.perf_counter() - t))
    S, n, T = sc.num_scenarios, sc.total_objects, sc.steps
    oms, oroof, bufs = observe_once(sc, ds, dev, ds.init, reps, E, K)
    del bufs
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)
    fmet = wm.Metrics.empty((T, n), dev)

    def fb():
        a.grad = None
        k.grad = None
        L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, ds.rg, T, sc.dt, 10, fmet)
        L.sum().backward()

    fb()
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_BACKWARD)
    wm.profile_collect(wm.PROF_ROLLOUT)
    t0 = time.perf_counter()
    for _ in range(reps):
        fb()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    bms, bl = wm.profile_collect(wm.PROF_BACKWARD)
    fms, fl = wm.profile_collect(wm.PROF_ROLLOUT)
    wm.profile_enable(False)
    bkm, fkm = bms / max(bl, 1), fms / max(fl, 1)
    valid = int(sc.log["valid"][synth.T0].sum())
    fops, _ = rollout_ops(sc, T)
    alg, alg_pairs = adjoint_algorithmic_ops(sc.obj_off, sc.controlled, sc.log["valid"][synth.T0], T)
    out["config4"] = {
        "workload": "4096 ragged scenarios, objects U{32..128}, road points U{10000..30000}, 8 egos and 8 controlled "
                    "objects per scenario, k = 1000, 80 steps, checkpoint every 10",
        "observe": {"ms": oms, "egos": S * E, "egos_per_s": S * E / (oms * 1e-3), "roofline": oroof},
        "fwd_bwd": {"value": S * T / (ms * 1e-3), "unit": "rollout scenario-steps/s",
                    "agent_steps_per_s": valid * T / (ms * 1e-3), "ms_per_rollout": ms,
                    "forward_kernel_ms": fkm, "forward_roofline_frac": fops / (fkm * 1e-3) / PEAK_FP32,
                    "backward_kernel_ms": bkm,
                    "backward_roofline": adjoint_roofline(alg, alg_pairs, None, None, bkm)},
        "observe_plus_fwd_bwd_ms": oms + ms}
    log("config 4: observe %.3f ms (%.1f%% of HBM), fwd+bwd %.3f ms/rollout (forward kernel %.3f ms, adjoint %.3f ms)"
        % (oms, 100 * oroof["frac"], ms, fkm, bkm))


def fwd_bwd_config3(out, dev, reps=3):
    """Differentiable rollout on 512 scenarios x 128 objects (8 controlled per
    scenario), 30,000 road points, 80 steps, checkpoint every 10: the forward
    with loss and checkpoints, then the hand-written adjoint (RolloutLoss
    forward + backward), in rollout scenario-steps/s."""
    import torch
    from paper_2310_08710_amd import synth, wm
    sc = synth.make_scene(3)
    ds = wm.upload(sc, dev)
    S, T = sc.num_scenarios, sc.steps
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)

    fmet = wm.Metrics.empty((T, sc.total_objects), dev)

    def fb(met):
        a.grad = None
        k.grad = None
        L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, ds.rg, T, sc.dt, 10, met)
        L.sum().backward()

    res = {"unit": "rollout scenario-steps/s",
           "workload": "512 scenarios x 128 objects (8 controlled), 30000 road points, 80 steps, checkpoint every 10"}
    tr = wm.State.empty((T, sc.total_objects), dev)
    wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, None, T, sc.dt, ds.batch.workspace(T, 0), traj=tr)
    xops, xnear, _ = adjoint_executed_ops(ds.batch.obj_off, ds.act_seq.controlled, ds.init, ds.log_seq, tr, T)
    del tr
    for key, met in (("full_metrics", fmet), ("loss_only", None)):
        fb(met)
        torch.cuda.synchronize()
        wm.profile_enable(True)
        wm.profile_collect(wm.PROF_BACKWARD)
        wm.profile_collect(wm.PROF_ROLLOUT)
        t0 = time.perf_counter()
        for _ in range(reps):
            fb(met)
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
        bms, bl = wm.profile_collect(wm.PROF_BACKWARD)
        fms, fl = wm.profile_collect(wm.PROF_ROLLOUT)
        wm.profile_enable(False)
        bkm = bms / max(bl, 1)
        alg, alg_pairs = adjoint_algorithmic_ops(sc.obj_off, sc.controlled, sc.log["valid"][synth.T0], T)
        res[key] = {"value": S * T / (ms * 1e-3), "agent_steps_per_s": sc.total_objects * T / (ms * 1e-3),
                    "ms_per_rollout": ms, "forward_kernel_ms": fms / max(fl, 1), "backward_kernel_ms": bkm,
                    "backward_roofline": adjoint_roofline(alg, alg_pairs, xops, xnear, bkm)}
        log("fwd+bwd (512 x 128, 8 controlled, %s): %.3f ms/rollout (forward kernel %.3f ms, adjoint %.3f ms)" % (
            key, ms, fms / max(fl, 1), bms / max(bl, 1)))
    res["value"] = res["full_metrics"]["value"]
    out["fwd_bwd_config3"] = res


def adjoint_only(dev, reps=3):
    """The adjoint alone, for profiling it: config 1 with every object
    controlled, the forward with the loss and checkpoints only (no road
    graph), then the adjoint; its kernel time and executed work."""
    import torch
    from paper_2310_08710_amd import synth, wm
    sc = synth.make_scene(1)
    ds = wm.upload(sc, dev)
    T, n = sc.steps, sc.total_objects
    ctrl = torch.ones_like(ds.act_seq.controlled)
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)

    def fb():
        a.grad = None
        k.grad = None
        L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ctrl, ds.log_seq, None, T, sc.dt, 10, None)
        L.sum().backward()

    fb()
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_BACKWARD)
    for _ in range(reps):
        fb()
    torch.cuda.synchronize()
    bms, bl = wm.profile_collect(wm.PROF_BACKWARD)
    wm.profile_enable(False)
    bkm = bms / max(bl, 1)
    tr = wm.State.empty((T, n), dev)
    wm.rollout(ds.batch, ds.init, wm.Action(ds.act_seq.accel, ds.act_seq.curvature, ctrl), ds.log_seq, None, T,
               sc.dt, ds.batch.workspace(T, 0), traj=tr)
    xops, xnear, tested = adjoint_executed_ops(ds.batch.obj_off, ctrl, ds.init, ds.log_seq, tr, T)
    return {"workload": "adjoint of config 1, every object controlled, loss only, checkpoint every 10",
            "backward_kernel_ms": bkm, "launches": bl, "ops_per_launch": xops, "pair_terms_evaluated": xnear,
            "pair_terms": tested, "tflops": xops / (bkm * 1e-3) / 1e12}


def idm(out, scene, ds, dev, tune):
    """The same 256 x 128 batch with 8 controlled objects per scenario and the
    other 120 as IDM sim agents (Sec. 3.5) against log playback of the same
    objects, both fused rollouts of 80 steps with every metric."""
    import torch
    from paper_2310_08710_amd import wm
    n, T = scene.total_objects, scene.steps
    ctrl = torch.zeros(n, dtype=torch.uint8, device=dev)
    off = np.asarray(scene.obj_off)
    for s in range(scene.num_scenarios):
        ctrl[int(off[s]):int(off[s]) + 8] = 1
    act = wm.Action(ds.act_seq.accel, ds.act_seq.curvature, ctrl)
    ws = ds.batch.workspace(T, 0)
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    ims = _time_graph(lambda: wm.rollout_idm(ds.batch, ds.init, act, ds.log_seq, ds.rg, T, scene.dt, ws, traj=traj,
                                             metrics=met, tune=tune), 3)
    pms = _time_graph(lambda: wm.rollout(ds.batch, ds.init, act, ds.log_seq, ds.rg, T, scene.dt, ws, traj=traj,
                                         metrics=met, tune=tune), 3)
    out["idm"] = {"ms_per_rollout": ims, "value": n * T / (ims * 1e-3), "unit": "agent-steps/s",
                  "playback_ms_per_rollout": pms, "agents_per_scenario": 120,
                  "parameters": dict(wm.IDM_DEFAULT)}
    log("IDM rollout: %.3f ms (playback of the same objects %.3f ms)" % (ims, pms))


def _time_graph(fn, reps, median=False):
    """Capture fn() as one HIP graph and return the mean wall time of a replay
    [ms], or with `median` the median of HIP-event times of single replays."""
    import torch
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    g.replay()
    torch.cuda.synchronize()
    if median:
        stream = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(stream)
        for i in range(reps):
            g.replay()
            ev[i + 1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]))
    else:
        t0 = time.perf_counter()
        for _ in range(reps):
            g.replay()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / reps
    del g
    return ms


def ragged(out, dev, T_cmp=10):
    """Ragged batch (1,024 scenarios, objects U{8..128}, road points
    U{2,000..30,000}): the fused persistent rollout (autotuned, HIP graph) over
    80 steps, and fused against the plain one-scenario-per-launch form over the
    first T_cmp steps (both as HIP graphs, identical outputs)."""
    import torch
    from paper_2310_08710_amd import synth, wm
    sc = synth.make_scene(2)
    ds = wm.upload(sc, dev)
    n, T = sc.total_objects, sc.steps
    valid = int(sc.log["valid"][synth.T0].sum())
    ws = ds.batch.workspace(T, 0)
    tune = wm.autotune(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws)
    met = wm.Metrics.empty((T, n), dev)
    traj = wm.State.empty((T, n), dev)

    def fused(steps):
        wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, steps, sc.dt, ws, traj=traj, metrics=met,
                   tune=tune)

    fms = _time_graph(lambda: fused(T), 3)
    # kernel time from HIP events around eager launches (events recorded
    # inside a captured graph are not timed)
    fused(T)
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_ROLLOUT)
    for _ in range(3):
        fused(T)
    torch.cuda.synchronize()
    kms, kl = wm.profile_collect(wm.PROF_ROLLOUT)
    wm.profile_enable(False)
    ops, _ = rollout_ops(sc, T)
    kernel_ms = kms / max(kl, 1)
    res = {"workload": "1024 ragged scenarios, objects U{8..128}, road points U{2000..30000}, 80 steps",
           "tuning": list(tune), "fused_ms_per_rollout": fms, "value": valid * T / (fms * 1e-3),
           "unit": "agent-steps/s", "kernel_ms": kernel_ms,
           "roofline_frac": ops / (kernel_ms * 1e-3) / PEAK_FP32}
    log("ragged fused: %.3f ms/rollout, %.3e agent-steps/s, kernel %.1f%% of FP32 peak" % (
        fms, res["value"], 100 * res["roofline_frac"]))

    # fused vs one launch sequence per scenario and step, first T_cmp steps
    off = np.asarray(sc.obj_off)
    counts = np.diff(off)
    rgc = np.diff(np.asarray(sc.rg_off))
    views = [wm.Batch(ds.batch.obj_off[s:s + 2], ds.batch.rg_off[s:s + 2], 1, n, ds.batch.total_rg_points,
                      int(counts[s]), int(rgc[s])) for s in range(sc.num_scenarios)]
    wsv = views[int(np.argmax(rgc))].workspace()
    ptraj = wm.State.empty((T_cmp, n), dev)
    pmet = wm.Metrics.empty((T_cmp, n), dev)
    acts = [wm.Action(ds.act_seq.accel[t], ds.act_seq.curvature[t], ds.act_seq.controlled) for t in range(T_cmp)]
    logs = [ds.log_seq.row(t + 1) for t in range(T_cmp)]
    rows = [ptraj.row(t) for t in range(T_cmp)]
    mets = [pmet.row(t) for t in range(T_cmp)]

    def plain():
        for v in views:
            c = ds.init
            for t in range(T_cmp):
                wm.step(v, c, acts[t], logs[t], ds.rg, sc.dt, rows[t], mets[t], wsv)
                c = rows[t]

    pms = _time_graph(plain, 2)
    f10 = _time_graph(lambda: fused(T_cmp), 5)
    same = all(torch.equal(getattr(met, f)[:T_cmp], getattr(pmet, f)) for f in wm.Metrics.FIELDS) and \
        torch.equal(traj.x[:T_cmp], ptraj.x)
    res.update({"steps_compared": T_cmp, "fused_ms": f10, "per_scenario_plain_ms": pms,
                "per_scenario_launches": int(sc.num_scenarios * T_cmp), "fused_speedup": pms / f10,
                "identical_outputs": bool(same)})
    log("ragged %d steps: fused %.3f ms vs per-scenario plain %.3f ms (%.1fx), identical=%s" % (
        T_cmp, f10, pms, pms / f10, same))
    out["ragged"] = res


if __name__ == "__main__":
    main()
