"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (autotuned rollout), on outputs the FP64 oracle recomputes
scenario by scenario (scenarios never interact, so a sampled scenario is an
independent sub-batch for the oracle)."""
import numpy as np
import pytest

import oracle
from helpers import assert_grad_close, device, f64, within
from paper_2310_08710_amd import synth
from test_gpu_rollout import METRICS, compare_rollout

pytestmark = pytest.mark.gpu


def _sub(scene, scen):
    """Host sub-batch of the given scenarios: (obj_off, rg_off, logs [T+1, n'],
    rg, accel, curvature, controlled, columns)."""
    off, roff = np.asarray(scene.obj_off), np.asarray(scene.rg_off)
    cols = np.concatenate([np.arange(off[s], off[s + 1]) for s in scen])
    pts = np.concatenate([np.arange(roff[s], roff[s + 1]) for s in scen])
    obj_off = np.concatenate([[0], np.cumsum([off[s + 1] - off[s] for s in scen])]).astype(np.int32)
    rg_off = np.concatenate([[0], np.cumsum([roff[s + 1] - roff[s] for s in scen])]).astype(np.int32)
    lw = {k: v[:, cols] for k, v in scene.log_window().items()}
    rg = f64({k: v[pts] for k, v in scene.rg.items()})
    return obj_off, rg_off, f64(lw), rg, scene.accel[:, cols], scene.curvature[:, cols], scene.controlled[cols], cols


def _oracle_expert(lw, dt):
    """Expert actions by the oracle's own inverse kinematics on the logs."""
    T = lw["x"].shape[0] - 1
    n = lw["x"].shape[1]
    a, k = np.zeros((T, n)), np.zeros((T, n))
    for t in range(T):
        a[t], k[t], _ = oracle.bicycle_inverse({q: v[t] for q, v in lw.items()},
                                               {q: v[t + 1] for q, v in lw.items()}, dt)
    return a, k


def test_config1_expert_rollout_full_size():
    """256 scenarios x 128 objects, 30000 road points, 80 steps: the benchmark's
    expert rollout (GPU inverse kinematics over the whole log window, then the
    fused rollout with every metric), checked on sampled scenarios against the
    oracle's own expert rollout."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(1)
    ds = wm.upload(sc, dev)
    n, T = sc.total_objects, sc.steps
    inv_batch = wm.Batch(ds.batch.obj_off, ds.batch.rg_off, 1, T * n, ds.batch.total_rg_points, 0, 0)
    F = wm.STATE_FIELDS + ("valid",)
    cur = wm.State(*[getattr(ds.log_seq, f)[:T] for f in F])
    nxt = wm.State(*[getattr(ds.log_seq, f)[1:] for f in F])
    ea, ek = torch.empty((T, n), device=dev), torch.empty((T, n), device=dev)
    wm.inverse_action(inv_batch, cur, nxt, sc.dt, ea, ek)
    expert = wm.Action(ea, ek, ds.act_seq.controlled)
    ws = ds.batch.workspace(T, 0)
    tune = wm.autotune(ds.batch, ds.init, expert, ds.log_seq, ds.rg, T, sc.dt, ws)
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    wm.rollout(ds.batch, ds.init, expert, ds.log_seq, ds.rg, T, sc.dt, ws, traj=traj, metrics=met, tune=tune)
    torch.cuda.synchronize()
    g_all = traj.numpy()
    gm_all = {f: getattr(met, f).cpu().numpy() for f in METRICS}
    print("tuning", tune, flush=True)
    for scen in ([0], [173]):
        obj_off, rg_off, lw, rg, _, _, ctrl, cols = _sub(sc, scen)
        a, k = _oracle_expert(lw, sc.dt)
        ref = oracle.rollout(obj_off, rg_off, {q: v[0] for q, v in lw.items()}, a, k, ctrl, lw, rg, T, sc.dt)
        ties = compare_rollout({q: v[:, cols] for q, v in g_all.items()}, {q: v[:, cols] for q, v in gm_all.items()},
                               None, ref, obj_off, rg_off, rg)
        print("scenario", scen, "near ties", ties, flush=True)


def test_config2_ragged_fused_vs_per_scenario_and_oracle():
    """1024 ragged scenarios (objects U{8..128}, road points U{2000..30000}),
    80 steps: the fused persistent rollout equals the plain per-scenario launch
    bit for bit on sampled scenarios and matches the oracle."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(2)
    ds = wm.upload(sc, dev)
    n, T = sc.total_objects, sc.steps
    ws = ds.batch.workspace(T, 0)
    tune = wm.autotune(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws)
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    loss = torch.empty(sc.num_scenarios, device=dev)
    wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, traj=traj, metrics=met, loss=loss,
               tune=tune)
    torch.cuda.synchronize()
    off = np.asarray(sc.obj_off)
    counts = np.diff(off)
    pick = [int(np.argmin(counts)), int(np.argmax(counts)), 511]
    # plain per-scenario launches (one-scenario views of the batch)
    ptraj = wm.State.empty((T, n), dev)
    pmet = wm.Metrics.empty((T, n), dev)
    for s in pick:
        view = wm.Batch(ds.batch.obj_off[s:s + 2], ds.batch.rg_off[s:s + 2], 1, n, ds.batch.total_rg_points,
                        int(counts[s]), int(sc.rg_off[s + 1] - sc.rg_off[s]))
        wsv = view.workspace()
        c = ds.init
        for t in range(1, T + 1):
            act = wm.Action(ds.act_seq.accel[t - 1], ds.act_seq.curvature[t - 1], ds.act_seq.controlled)
            m = wm.Metrics(*[getattr(pmet, f)[t - 1] for f in ("collision", "offroad", "overlap_margin",
                                                                 "offroad_margin", "log_div")])
            wm.step(view, c, act, ds.log_seq.row(t), ds.rg, sc.dt, ptraj.row(t - 1), m, wsv)
            c = ptraj.row(t - 1)
    torch.cuda.synchronize()
    for s in pick:
        sl = slice(off[s], off[s + 1])
        for f in wm.STATE_FIELDS + ("valid",):
            assert torch.equal(getattr(traj, f)[:, sl], getattr(ptraj, f)[:, sl]), (s, f)
        for f in METRICS:
            assert torch.equal(getattr(met, f)[:, sl], getattr(pmet, f)[:, sl]), (s, f)
    g_all = traj.numpy()
    gm_all = {f: getattr(met, f).cpu().numpy() for f in METRICS}
    for s in pick[:2]:
        obj_off, rg_off, lw, rg, a, k, ctrl, cols = _sub(sc, [s])
        ref = oracle.rollout(obj_off, rg_off, {q: v[0] for q, v in lw.items()}, a, k, ctrl, lw, rg, T, sc.dt)
        compare_rollout({q: v[:, cols] for q, v in g_all.items()}, {q: v[:, cols] for q, v in gm_all.items()},
                        loss.cpu().numpy()[[s]], ref, obj_off, rg_off, rg)


def test_config3_adjoint_full_size():
    """512 scenarios x 128 objects (8 controlled), 30000 road points, 80 steps,
    checkpoint every 10: GPU adjoint vs the oracle's reverse-mode gradient on
    the first 4 scenarios (relative error <= 1e-3 per scenario)."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(3)
    ds = wm.upload(sc, dev)
    T = sc.steps
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)
    L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, ds.rg, T, sc.dt, 10, None)
    L.sum().backward()
    torch.cuda.synchronize()
    obj_off, _, lw, _, oa, ok_, ctrl, cols = _sub(sc, [0, 1, 2, 3])
    ga_o, gk_o, loss_o = oracle.rollout_grad(obj_off, {q: v[0] for q, v in lw.items()}, oa, ok_, ctrl, lw, T, sc.dt)
    assert within(L.detach().cpu().numpy()[:4], loss_o, atol=1e-3, rtol=1e-3).all()
    ga, gk = a.grad.cpu().numpy()[:, cols], k.grad.cpu().numpy()[:, cols]
    for s in range(4):
        c = slice(obj_off[s], obj_off[s + 1])
        for name, g, o in (("accel", ga, ga_o), ("curvature", gk, gk_o)):
            assert_grad_close(g[:, c], o[:, c], "%s s=%d" % (name, s))
    assert np.isfinite(a.grad.cpu().numpy()).all()


@pytest.fixture(scope="module")
def config4():
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4)
    return sc, wm.upload(sc, dev), dev


def test_config4_observation_full_size(config4):
    """4096 ragged scenarios (objects U{32..128}, road points
    U{10000..30000}), 8 egos each, k = 1000: indices bit-exact and features
    within tolerance on sampled scenarios."""
    import torch
    from paper_2310_08710_amd import wm
    sc, ds, dev = config4
    S, E, K = sc.num_scenarios, 8, 1000
    maxN = ds.batch.max_objects
    idx = torch.empty(S * E * K, dtype=torch.int32, device=dev)
    rf = torch.empty(S * E * K * 4, device=dev)
    of = torch.empty(S * E * maxN * 8, device=dev)
    wm.observe(ds.batch, ds.init, ds.rg, ds.ego, E, K, idx, rf, of)
    torch.cuda.synchronize()
    gi = idx.cpu().numpy().reshape(S, E, K)
    gr = rf.cpu().numpy().reshape(S, E, K, 4)
    go = of.cpu().numpy().reshape(S, E, maxN, 8)
    st = sc.state_at(synth.T0)
    for s in (0, 2047, 4095):
        o0, o1 = sc.obj_off[s], sc.obj_off[s + 1]
        p0, p1 = sc.rg_off[s], sc.rg_off[s + 1]
        sub_st = f64({q: v[o0:o1] for q, v in st.items()})
        sub_rg = f64({q: v[p0:p1] for q, v in sc.rg.items()})
        ego = (sc.ego[s] - o0).reshape(1, E)
        oi, orf, oof = oracle.observe(np.array([0, o1 - o0], np.int32), np.array([0, p1 - p0], np.int32), sub_st,
                                      sub_rg, ego, K, maxN)
        np.testing.assert_array_equal(gi[s], oi[0])
        assert within(gr[s], orf[0]).all()
        ok = within(go[s], oof[0])
        d = go[s][..., 2] - oof[0][..., 2]
        ok[..., 2] = np.abs(d - 2 * np.pi * np.round(d / (2 * np.pi))) <= 1e-5
        assert ok.all()
    # the block-pruned form: logged rows 0..3 in one call (each row's bound
    # from the previous one), sampled scenarios against the oracle
    del idx, rf, of
    R = 4
    idx = torch.empty((R, S * E * K), dtype=torch.int32, device=dev)
    rf = torch.empty((R, S * E * K * 4), device=dev)
    wm.observe_seq(ds.batch, ds.log_seq, R, ds.rg, ds.ego, E, K, idx, rf, None)
    torch.cuda.synchronize()
    lw = sc.log_window()
    for r in range(R):
        gi = idx[r].cpu().numpy().reshape(S, E, K)
        gr = rf[r].cpu().numpy().reshape(S, E, K, 4)
        for s in (7, 2047, 4094):
            o0, o1 = sc.obj_off[s], sc.obj_off[s + 1]
            p0, p1 = sc.rg_off[s], sc.rg_off[s + 1]
            sub_st = f64({q: v[r, o0:o1] for q, v in lw.items()})
            sub_rg = f64({q: v[p0:p1] for q, v in sc.rg.items()})
            ego = (sc.ego[s] - o0).reshape(1, E)
            oi, orf, _ = oracle.observe(np.array([0, o1 - o0], np.int32), np.array([0, p1 - p0], np.int32), sub_st,
                                        sub_rg, ego, K, maxN)
            np.testing.assert_array_equal(gi[s], oi[0], err_msg="row %d scenario %d" % (r, s))
            assert within(gr[s], orf[0]).all()


def test_config4_adjoint_full_size(config4):
    """The same 4096 ragged scenarios: 80-step fused rollout with every metric
    plus adjoint; gradients of two sampled scenarios against the oracle."""
    import torch
    from paper_2310_08710_amd import wm
    sc, ds, dev = config4
    T = sc.steps
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)
    L = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, ds.rg, T, sc.dt, 10, None)
    L.sum().backward()
    torch.cuda.synchronize()
    for s in (1, 3000):
        obj_off, _, lw, _, oa, ok_, ctrl, cols = _sub(sc, [s])
        ga_o, gk_o, loss_o = oracle.rollout_grad(obj_off, {q: v[0] for q, v in lw.items()}, oa, ok_, ctrl, lw, T,
                                                 sc.dt)
        assert within(L.detach().cpu().numpy()[[s]], loss_o, atol=1e-3, rtol=1e-3).all()
        for name, g, o in (("accel", a.grad.cpu().numpy()[:, cols], ga_o),
                           ("curvature", k.grad.cpu().numpy()[:, cols], gk_o)):
            assert_grad_close(g, o, "%s s=%d" % (name, s))
