"""Benchmark of the simulator hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Workload: 256 scenarios x 128 objects, 30,000 road points per scenario
(about 20,000 road-edge points), an 80-step rollout at dt = 0.1 s (synthetic
scenes shaped like the paper's runtime benchmark, Sec. 5.1 / App. A.3).  One
timed step is one expert rollout (RolloutExpert in the paper's runtime
table): expert actions from inverse kinematics on the logs, then the fused
persistent rollout kernel with every metric (collision, off-road,
displacement) at every step.  value = agent-steps/s = objects x 80 x K / time.

Also reported on the same line: the dominant kernel against the FP32 roofline
(HIP events around the persistent kernel), the FP64 CPU oracle on a bounded
sample of the same workload, the plain per-step form (separate launches per
operation, captured in a HIP graph), the differentiable rollout (forward +
adjoint) and the observation (8 egos per scenario, k = 1000).
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


def adjoint_ops(scene, controlled):
    """Algorithmic ops of one adjoint launch over the scene's T steps; every
    object is valid in the synthetic scenes."""
    ctrl = np.asarray(controlled).astype(bool)
    off = np.asarray(scene.obj_off)
    nc = np.add.reduceat(ctrl.astype(np.int64), off[:-1]) if len(off) > 1 else np.zeros(0)
    N = np.diff(off).astype(np.int64)
    pairs = float((nc * np.maximum(N - 1, 0)).sum())
    return scene.steps * (ADJ_OPS_PER_PAIR * pairs + ADJ_OPS_PER_OBJECT * float(nc.sum())), scene.steps * pairs


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


def cpu_baseline(scene, sample, threads):
    """The FP64 oracle (as it stands) on the first `sample` scenarios of the
    workload, one scenario per thread; agent-steps/s."""
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    lw = scene.log_window()
    T = scene.steps

    def one(s):
        o0, o1 = int(scene.obj_off[s]), int(scene.obj_off[s + 1])
        p0, p1 = int(scene.rg_off[s]), int(scene.rg_off[s + 1])
        sub = {k: v[:, o0:o1] for k, v in lw.items()}
        f64 = lambda d: {k: (v.astype(np.float64) if v.dtype == np.float32 else v) for k, v in d.items()}  # noqa
        rg = f64({k: v[p0:p1] for k, v in scene.rg.items()})
        oracle.rollout(np.array([0, o1 - o0], np.int32), np.array([0, p1 - p0], np.int32),
                       f64({k: v[0] for k, v in sub.items()}), scene.accel[:, o0:o1], scene.curvature[:, o0:o1],
                       scene.controlled[o0:o1], f64(sub), rg, T, scene.dt, metrics=True, want_loss=False)
        return o1 - o0

    oracle.lib()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        objs = sum(ex.map(one, range(sample)))
    dt = time.perf_counter() - t0
    return objs * T / dt, dt


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-extras", action="store_true", help="skip plain / fwd+bwd / observation")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--tune", type=str, default=None, help="unit_objects,edge_splits (skips the autotuner)")
    ap.add_argument("--cpu-sample", type=int, default=8, help="scenarios of the oracle sample")
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
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_ROLLOUT)
    # HIP events between the steps on the stream the steps run on give the
    # per-step distribution; the wall clock over all K steps gives `value`
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(args.steps):
        step()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps))
    kms, launches = wm.profile_collect(wm.PROF_ROLLOUT)
    wm.profile_enable(False)
    valid_objs = int(scene.log["valid"][synth.T0].sum())
    value = valid_objs * T * args.steps / wall
    ms_per_step = 1e3 * wall / args.steps
    kernel_ms = kms / max(launches, 1)
    ops, pairs = rollout_ops(scene, T)
    achieved = ops / (kernel_ms * 1e-3)
    log("fused rollout: %.3f ms/step, kernel %.3f ms, %.3e agent-steps/s, %.1f TFLOP/s algorithmic" % (
        ms_per_step, kernel_ms, value, achieved / 1e12))
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "expert rollout of 256 scenarios x 128 objects, 30000 road points "
                               "(~20000 road edges) per scenario, 80 steps, every metric every step",
                   "scenarios": S, "objects_per_scenario": 128, "rg_points": 30000, "T": T,
                   "tuning": list(tune) if tune else None},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": recorded_traffic(tune), "kernel": "k_rollout",
                     "kernel_ms": kernel_ms, "ops_per_launch": ops, "corner_edge_pairs_per_launch": pairs},
    }

    if not args.no_extras:
        extras(out, scene, ds, dev, inv_batch, cur, nxt, ea, ek, expert, tune)

    if not args.no_cpu:
        try:
            threads = len(os.sched_getaffinity(0))
        except AttributeError:
            threads = os.cpu_count() or 1
        threads = max(1, min(threads, 16, args.cpu_sample))
        rate, secs = cpu_baseline(scene, args.cpu_sample, threads)
        out["cpu_baseline"] = {"value": rate, "unit": "agent-steps/s", "cores": threads, "kind": "oracle",
                               "sample": "%d of the 256 scenarios, all 80 steps with every metric, FP64 C oracle, "
                                         "one scenario per thread (%.1f s wall)" % (args.cpu_sample, secs)}
        log("cpu oracle: %.3e agent-steps/s on %d threads (%.1f s)" % (rate, threads, secs))
    print(json.dumps(out), flush=True)


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
    idx = torch.empty(S * E * K, dtype=torch.int32, device=dev)
    rf = torch.empty(S * E * K * 4, device=dev)
    of = torch.empty(S * E * ds.batch.max_objects * 8, device=dev)
    wm.observe(ds.batch, ds.init, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    wm.profile_enable(True)
    wm.profile_collect(wm.PROF_OBSERVE)
    t0 = time.perf_counter()
    for _ in range(reps):
        wm.observe(ds.batch, ds.init, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    oms = 1e3 * (time.perf_counter() - t0) / reps
    kms, kl = wm.profile_collect(wm.PROF_OBSERVE)
    wm.profile_enable(False)
    out_bytes = S * E * (K * 20 + ds.batch.max_objects * 32)
    okm = kms / max(kl, 1)
    out["observe"] = {"egos_per_s": S * E / (oms * 1e-3), "ms": oms, "kernel_ms": okm, "k": K, "egos": S * E,
                      "output_GBps": out_bytes / (okm * 1e-3) / 1e9,
                      "point_reads_TBps": point_bytes / (okm * 1e-3) / 1e12}
    log("observe: %.3f ms for %d egos (kernel %.3f ms)" % (oms, S * E, okm))

    # every row of a trajectory in one launch
    del idx, rf, of
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
    out["observe_seq"] = {"ms": sms, "kernel_ms": skm, "rows": T, "egos_per_row": S * E, "k": K,
                          "ego_steps_per_s": T * S * E / (sms * 1e-3),
                          "output_GBps": T * out_bytes / (skm * 1e-3) / 1e9,
                          "point_reads_TBps": T * point_bytes / (skm * 1e-3) / 1e12}
    log("observe_seq: %.3f ms for %d steps x %d egos" % (sms, T, S * E))


def extras(out, scene, ds, dev, inv_batch, cur, nxt, ea, ek, expert, tune):
    import torch
    from paper_2310_08710_amd import wm
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

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plain()
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plain()
    g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    pms = 1e3 * (time.perf_counter() - t0) / reps
    fused_ms = out["ms_per_step"]
    out["plain"] = {"value": n * T / (pms * 1e-3), "unit": "agent-steps/s", "ms_per_rollout": pms,
                    "form": "road-edge compaction once, then per-step launches (dynamics, overlap, off-road) "
                            "in one HIP graph",
                    "fused_speedup": pms / fused_ms}
    log("plain graph: %.3f ms/rollout (fused speedup %.2fx)" % (pms, pms / fused_ms))
    del g

    # fused rollout captured as a graph as well (whole rollout = 1 replay)
    traj2 = wm.State.empty((T, n), dev)
    met2 = wm.Metrics.empty((T, n), dev)
    ws1 = ds.batch.workspace(T, 10)

    def fused():
        wm.inverse_action(inv_batch, cur, nxt, scene.dt, ea, ek)
        wm.rollout(ds.batch, ds.init, expert, ds.log_seq, ds.rg, T, scene.dt, ws1, traj=traj2, metrics=met2,
                   tune=tune)

    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fused()
    torch.cuda.current_stream().wait_stream(side)
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        fused()
    g2.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        g2.replay()
    torch.cuda.synchronize()
    gms = 1e3 * (time.perf_counter() - t0) / reps
    out["fused_graph"] = {"ms_per_rollout": gms, "value": n * T / (gms * 1e-3), "unit": "agent-steps/s"}
    ok = all(torch.equal(getattr(met2, f), getattr(met, f)) for f in fields)
    out["fused_graph"]["equals_plain"] = bool(ok)
    del g2

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
    aops, apairs = adjoint_ops(scene, ds.act_seq.controlled.cpu().numpy())
    # the trajectory of these actions (traj2: the expert rollout, every object controlled)
    xops, xnear, _ = adjoint_executed_ops(ds.batch.obj_off, ds.act_seq.controlled, ds.init, ds.log_seq, traj2, T)
    out["fwd_bwd"] = {"value": S * T / (fbms * 1e-3), "unit": "rollout scenario-steps/s",
                      "agent_steps_per_s": n * T / (fbms * 1e-3), "ms_per_rollout": fbms,
                      "backward_kernel_ms": bkm, "controlled": "all objects",
                      "checkpoint_every": 10,
                      "backward_roofline": {"bound": "alu", "achieved": xops / (bkm * 1e-3) / 1e12,
                                            "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                                            "frac": xops / (bkm * 1e-3) / PEAK_FP32, "ops_per_launch": xops,
                                            "pair_terms_per_launch": apairs, "pair_terms_evaluated": xnear,
                                            "all_pairs_equivalent_tflops": aops / (bkm * 1e-3) / 1e12}}
    log("fwd+bwd: %.3f ms/rollout (adjoint kernel %.3f ms)" % (fbms, bms / max(bl, 1)))

    observation(out, scene, ds, dev, traj2, reps)

    ragged(out, dev)
    idm(out, scene, ds, dev, tune)
    fwd_bwd_config3(out, dev)


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
        aops, _ = adjoint_ops(sc, sc.controlled)
        res[key] = {"value": S * T / (ms * 1e-3), "agent_steps_per_s": sc.total_objects * T / (ms * 1e-3),
                    "ms_per_rollout": ms, "forward_kernel_ms": fms / max(fl, 1), "backward_kernel_ms": bkm,
                    "backward_tflops": xops / (bkm * 1e-3) / 1e12, "backward_frac": xops / (bkm * 1e-3) / PEAK_FP32,
                    "pair_terms_evaluated": xnear,
                    "all_pairs_equivalent_tflops": aops / (bkm * 1e-3) / 1e12}
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


def _time_graph(fn, reps):
    """Capture fn() as one HIP graph and return the mean wall time of a replay [ms]."""
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
