"""GPU parity of the fused rollout (Sec. 5.1 Rollout), of its adjoint
(differentiable simulation) and of the observation (Sec. 3.2), through the C
ABI, against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from helpers import (assert_grad_close, assert_traj_close, compare_collision, compare_offroad, device, f64,
                     scenario_band, state_delta, within)
from paper_2310_08710_amd import synth

pytestmark = pytest.mark.gpu


def _ragged(T=20, **kw):
    opts = dict(scenarios=6, objects=(5, 140), rg_points=(240, 5000), steps=T, invalid_frac=0.08,
                rg_invalid_frac=0.03, object_box=35, on_road_frac=0.5)
    opts.update(kw)
    return synth.make_scene(2, **opts)


def _run_fused(ds, sc, dev, tune=None, ckpt_every=0):
    import torch
    from paper_2310_08710_amd import wm
    n, T = sc.total_objects, sc.steps
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    loss = torch.empty(sc.num_scenarios, device=dev)
    ck = None
    if ckpt_every:
        ck = wm.State.empty(((T + ckpt_every - 1) // ckpt_every, n), dev)
    ws = ds.batch.workspace(T, ckpt_every)
    wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, ckpt_every=ckpt_every, ckpt=ck,
               traj=traj, metrics=met, loss=loss, tune=tune)
    torch.cuda.synchronize()
    return traj, met, loss, ck


def _run_plain(ds, sc, dev):
    import torch
    from paper_2310_08710_amd import wm
    n, T = sc.total_objects, sc.steps
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    ws = ds.batch.workspace()
    cur = ds.init
    for t in range(1, T + 1):
        act = wm.Action(ds.act_seq.accel[t - 1], ds.act_seq.curvature[t - 1], ds.act_seq.controlled)
        nxt = traj.row(t - 1)
        m = wm.Metrics(*[getattr(met, f.name)[t - 1] for f in __import__("dataclasses").fields(met)])
        wm.step(ds.batch, cur, act, ds.log_seq.row(t), ds.rg, sc.dt, nxt, m, ws)
        cur = nxt
    torch.cuda.synchronize()
    return traj, met


@pytest.mark.parametrize("seed", [1000, 2000])
def test_fused_rollout_matches_oracle(seed):
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _ragged(seed_base=seed)
    ctrl = sc.controlled.copy()
    ctrl[::5] = 0
    sc.controlled = ctrl
    ds = wm.upload(sc, dev)
    traj, met, loss, _ = _run_fused(ds, sc, dev)
    T, n = sc.steps, sc.total_objects
    g = traj.numpy()
    lw = sc.log_window()
    init = f64({k: v[0] for k, v in lw.items()})
    ref = oracle.rollout(sc.obj_off, sc.rg_off, init, sc.accel, sc.curvature, ctrl, f64(lw), f64(sc.rg), T, sc.dt)
    gm = {f: getattr(met, f).cpu().numpy() for f in METRICS}
    compare_rollout(g, gm, loss.cpu().numpy(), ref, sc.obj_off, sc.rg_off, f64(sc.rg))


METRICS = ("collision", "offroad", "overlap_margin", "offroad_margin", "log_div")


def compare_rollout(g, gm, loss, ref, obj_off, rg_off, rg):
    """GPU rollout outputs against the oracle's own rollout from the same
    inputs (g: trajectory fields [T, n]; gm: metrics [T, n]; loss [S] or
    None).  Trajectories: within 1e-4 of the scene scale at every step.
    Metrics: margins within tolerance plus the Lipschitz band of the measured
    state difference; masks bit-exact outside that band.  Returns the number
    of near ties."""
    T = g["x"].shape[0]
    n = g["x"].shape[1]
    ties = 0
    for t in range(T):
        gt = {k: v[t] for k, v in g.items()}
        ot = {k: v[t] for k, v in ref["traj"].items()}
        assert_traj_close(gt, ot, "t=%d" % t)
        delta = state_delta(gt, ot)
        band = scenario_band(delta, obj_off)
        ties += compare_collision(gm["collision"][t], gm["overlap_margin"][t], ref["collision"][t],
                                  ref["overlap_margin"][t], "t=%d" % t, band=band)
        r = oracle.offroad(obj_off, rg_off, ot, rg, band=float(band.max()))
        ties += compare_offroad(gm["offroad"][t], gm["offroad_margin"][t], r, "t=%d" % t, band=band)
        ld = gm["log_div"][t]
        assert (within(ld, ref["log_div"][t]) | (np.abs(ld - ref["log_div"][t]) <= delta + 1e-5)).all()
    assert ties <= 2 * T * n // 50, (ties, T * n)
    if loss is not None:
        assert within(loss, ref["loss"], atol=1e-3, rtol=1e-3).all()
    return ties


def test_fused_equals_plain_and_all_tunings():
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _ragged(T=12)
    ds = wm.upload(sc, dev)
    traj, met, loss, _ = _run_fused(ds, sc, dev)
    ptraj, pmet = _run_plain(ds, sc, dev)
    for f in synth.STATE_FIELDS + ("valid",):
        assert torch.equal(getattr(traj, f), getattr(ptraj, f)), f
    for f in wm.Metrics.FIELDS:
        assert torch.equal(getattr(met, f), getattr(pmet, f)), f
    for tune in ((64, 1), (64, 2), (64, 8), (128, 2), (128, 4), (256, 2)):
        t2, m2, l2, _ = _run_fused(ds, sc, dev, tune=tune)
        for f in ("collision", "offroad", "overlap_margin", "offroad_margin", "infeasible", "reward"):
            assert torch.equal(getattr(m2, f), getattr(met, f)), (tune, f)
        assert torch.equal(t2.x, traj.x)
        # the loss partials depend on the slice size only through summation order
        assert torch.allclose(l2, loss, rtol=1e-5, atol=1e-4)
    # a work-group larger than the fused kernel allows is refused before launch
    with pytest.raises(wm.WMError):
        _run_fused(ds, sc, dev, tune=(256, 4))
    # two identical runs are bitwise identical
    t3, m3, l3, _ = _run_fused(ds, sc, dev)
    assert torch.equal(l3, loss) and torch.equal(m3.offroad_margin, met.offroad_margin)


def test_checkpoints_are_the_trajectory():
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _ragged(T=23)
    ds = wm.upload(sc, dev)
    traj, met, loss, ck = _run_fused(ds, sc, dev, ckpt_every=5)
    assert ck.x.shape[0] == 5
    assert torch.equal(ck.x[0], ds.init.x) and torch.equal(ck.valid[0], ds.init.valid)
    for c in range(1, 5):
        assert torch.equal(ck.x[c], traj.x[5 * c - 1]) and torch.equal(ck.yaw[c], traj.yaw[5 * c - 1])


def _grad_scene(T=20, S=4, N=(24, 40)):
    sc = synth.make_scene(3, scenarios=S, objects=N, rg_points=(240, 480), steps=T, object_box=14)
    return sc


def test_adjoint_matches_oracle_gradient():
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _grad_scene()
    ds = wm.upload(sc, dev)
    T = sc.steps
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)
    dl = torch.tensor([1.0, 0.5, 2.0, 1.5], device=dev)
    loss = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, None, T, sc.dt, 5, None)
    (loss * dl).sum().backward()
    torch.cuda.synchronize()
    lw = sc.log_window()
    oga, ogk, oloss = oracle.rollout_grad(sc.obj_off, f64({q: v[0] for q, v in lw.items()}), sc.accel,
                                          sc.curvature, sc.controlled, f64(lw), T, sc.dt, dl.cpu().numpy())
    assert within(loss.detach().cpu().numpy(), oloss, atol=1e-3, rtol=1e-4).all()
    ga, gk = a.grad.cpu().numpy(), k.grad.cpu().numpy()
    for s in range(sc.num_scenarios):
        cols = slice(sc.obj_off[s], sc.obj_off[s + 1])
        for name, g, o in (("accel", ga, oga), ("curvature", gk, ogk)):
            assert_grad_close(g[:, cols], o[:, cols], "%s s=%d" % (name, s))
    assert (ga[:, sc.controlled == 0] == 0).all()
    assert np.abs(oga).max() > 0.1                  # the gradient is not trivially zero


def test_adjoint_scenario_without_controlled_objects():
    """A scenario with no controlled object contributes nothing: its
    gradients are zero and the other scenarios' match the oracle."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _grad_scene(T=9)
    sc.controlled[sc.obj_off[1]:sc.obj_off[2]] = 0
    ds = wm.upload(sc, dev)
    T = sc.steps
    a = ds.act_seq.accel.clone().requires_grad_(True)
    k = ds.act_seq.curvature.clone().requires_grad_(True)
    loss = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, None, T, sc.dt, 4, None)
    loss.sum().backward()
    torch.cuda.synchronize()
    lw = sc.log_window()
    oga, ogk, _ = oracle.rollout_grad(sc.obj_off, f64({q: v[0] for q, v in lw.items()}), sc.accel, sc.curvature,
                                      sc.controlled, f64(lw), T, sc.dt)
    ga, gk = a.grad.cpu().numpy(), k.grad.cpu().numpy()
    c1 = slice(sc.obj_off[1], sc.obj_off[2])
    assert (ga[:, c1] == 0).all() and (gk[:, c1] == 0).all()
    for s in (0, 2, 3):
        cols = slice(sc.obj_off[s], sc.obj_off[s + 1])
        for name, g, o in (("accel", ga, oga), ("curvature", gk, ogk)):
            assert_grad_close(g[:, cols], o[:, cols], "%s s=%d" % (name, s))


def test_adjoint_checkpoint_interval_invariance():
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _grad_scene(T=17)
    ds = wm.upload(sc, dev)
    T = sc.steps
    grads = []
    for K in (1, 5, 17):
        a = ds.act_seq.accel.clone().requires_grad_(True)
        k = ds.act_seq.curvature.clone().requires_grad_(True)
        loss = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, None, T, sc.dt, K, None)
        loss.sum().backward()
        grads.append((a.grad.clone(), k.grad.clone(), loss.detach().clone()))
    for g in grads[1:]:
        assert torch.equal(g[0], grads[0][0]) and torch.equal(g[1], grads[0][1])
        assert torch.equal(g[2], grads[0][2])


def test_adjoint_many_objects():
    """Scenarios of 800..820 objects: the adjoint then stages one step at a
    time in LDS (several blocks per checkpoint segment) and splits each
    controlled object's partners over 64 lanes.  Gradient against the oracle,
    and identical for checkpoint intervals 1, 3 and 7."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(3, scenarios=2, objects=(800, 820), rg_points=(240, 480), steps=7, object_box=60)
    ds = wm.upload(sc, dev)
    T = sc.steps
    grads = []
    for K in (3, 1, 7):
        a = ds.act_seq.accel.clone().requires_grad_(True)
        k = ds.act_seq.curvature.clone().requires_grad_(True)
        loss = wm.RolloutLoss.apply(a, k, ds.batch, ds.init, ds.act_seq.controlled, ds.log_seq, None, T, sc.dt, K, None)
        loss.sum().backward()
        torch.cuda.synchronize()
        grads.append((a.grad.clone(), k.grad.clone()))
    for g in grads[1:]:
        assert torch.equal(g[0], grads[0][0]) and torch.equal(g[1], grads[0][1])
    lw = sc.log_window()
    oga, ogk, _ = oracle.rollout_grad(sc.obj_off, f64({q: v[0] for q, v in lw.items()}), sc.accel, sc.curvature,
                                      sc.controlled, f64(lw), T, sc.dt)
    ga, gk = grads[0][0].cpu().numpy(), grads[0][1].cpu().numpy()
    for s in range(sc.num_scenarios):
        cols = slice(sc.obj_off[s], sc.obj_off[s + 1])
        for name, g, o in (("accel", ga, oga), ("curvature", gk, ogk)):
            assert_grad_close(g[:, cols], o[:, cols], "%s s=%d" % (name, s))
    assert np.abs(oga).max() > 0.1


def _observe_both(ds, st, rg, E, k, obj=False, rows=4):
    """The observation of one state row `st` (a State of [n]) through both
    forms: wm_observe (one row: one work-group per ego over every point) and
    wm_observe_seq over `rows` copies of the row (the block-pruned form, whose
    later rows start from the previous row's bound).  Returns (rg_idx,
    rg_feat, obj_feat or None) as numpy arrays, once per row of each form."""
    import torch
    from paper_2310_08710_amd import wm
    dev = st.x.device
    S, maxN = ds.batch.num_scenarios, ds.batch.max_objects
    slots = S * E
    idx = torch.empty((rows, slots * k), dtype=torch.int32, device=dev)
    rf = torch.empty((rows, slots * k * 4), device=dev)
    of = torch.empty((rows, slots * maxN * 8), device=dev) if obj else None
    wm.observe(ds.batch, st, rg, ds.ego, E, k, idx[0], rf[0], of[0] if obj else None)
    torch.cuda.synchronize()
    out = [(idx[0].cpu().numpy().copy(), rf[0].cpu().numpy().copy(), of[0].cpu().numpy().copy() if obj else None)]
    rep = wm.State(*[getattr(st, f).reshape(1, -1).repeat(rows, 1).contiguous()
                     for f in wm.STATE_FIELDS + ("valid",)])
    wm.observe_seq(ds.batch, rep, rows, rg, ds.ego, E, k, idx, rf, of)
    torch.cuda.synchronize()
    for r in range(rows):
        out.append((idx[r].cpu().numpy(), rf[r].cpu().numpy(), of[r].cpu().numpy() if obj else None))
    return out


@pytest.mark.parametrize("k", [1, 64, 333, 1024])
def test_observe_topk_and_frames(k):
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4, scenarios=3, objects=(4, 40), rg_points=(700, 3000), steps=2, rg_invalid_frac=0.05,
                          invalid_frac=0.1)
    # quantise some points to a 0.5 m grid so that exact binary32 key ties occur
    sc.rg["x"][::3] = np.round(sc.rg["x"][::3] * 2) / 2
    sc.rg["y"][::3] = np.round(sc.rg["y"][::3] * 2) / 2
    ds = wm.upload(sc, dev)
    S, E = sc.num_scenarios, sc.ego.shape[1]
    maxN = ds.batch.max_objects
    st = sc.state_at(synth.T0)
    o_idx, o_rf, o_of = oracle.observe(sc.obj_off, sc.rg_off, f64(st), f64(sc.rg), sc.ego, k, maxN)
    for gi, grf, gof in _observe_both(ds, ds.init, ds.rg, E, k, obj=True):
        np.testing.assert_array_equal(gi.reshape(S, E, k), o_idx)     # bit-exact
        assert within(grf.reshape(S, E, k, 4), o_rf).all()
        g_of = gof.reshape(S, E, maxN, 8)
        ok = within(g_of, o_of)
        ok[..., 2] = np.abs(((g_of[..., 2] - o_of[..., 2] + math.pi) % (2 * math.pi)) - math.pi) <= 1e-5
        assert ok.all()


@pytest.mark.parametrize("k", [1000, 1024])
def test_observe_selection_inside_one_bin(k):
    """Selections decided inside one radix bin of the squared distance: in
    scenario 0, 2,500 road points share one location 3 m from ego 0, so more
    than 1,024 binary32 keys are exactly equal at the k-th place and the
    lowest indices must win; in scenario 1, 4,000 points lie on a ring of
    radius 9.85..10.15 m around ego 0 (d2 in [97, 103], one bin of the first
    11-bit digit); in scenario 2, 2,000 points lie on a ring 0.25 mm thick, so
    the keys share the first two digits and many are equal."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4, scenarios=3, objects=(8, 40), rg_points=(6000, 8000), steps=2, rg_invalid_frac=0.02)
    st = sc.state_at(synth.T0)
    rng = np.random.default_rng(11)
    for s, m in ((0, 2500), (1, 4000), (2, 2000)):
        p0, p1 = sc.rg_off[s], sc.rg_off[s + 1]
        at = p0 + rng.choice(p1 - p0, m, replace=False)     # spread over the index range
        g = sc.ego[s, 0]
        ex, ey = float(st["x"][g]), float(st["y"][g])
        if s == 0:
            rad, ang = np.full(m, 3.0), np.full(m, 0.7)
        elif s == 1:
            rad, ang = rng.uniform(9.85, 10.15, m), rng.uniform(-np.pi, np.pi, m)
        else:
            rad, ang = rng.uniform(10.0, 10.00025, m), rng.uniform(-np.pi, np.pi, m)
        sc.rg["x"][at] = (ex + rad * np.cos(ang)).astype(np.float32)
        sc.rg["y"][at] = (ey + rad * np.sin(ang)).astype(np.float32)
        sc.rg["valid"][at] = 1
    ds = wm.upload(sc, dev)
    S, E = sc.num_scenarios, sc.ego.shape[1]
    maxN = ds.batch.max_objects
    o_idx, o_rf, _ = oracle.observe(sc.obj_off, sc.rg_off, f64(st), f64(sc.rg), sc.ego, k, maxN)
    # the constructed groups do decide the k-th place of ego 0
    for s in range(S):
        assert (o_idx[s, 0] >= 0).all()
    for gi, grf, _ in _observe_both(ds, ds.init, ds.rg, E, k):
        np.testing.assert_array_equal(gi.reshape(S, E, k), o_idx)     # bit-exact
        assert within(grf.reshape(S, E, k, 4), o_rf).all()


def test_observe_when_the_sampled_bound_misleads():
    """Every 16th road point (the ones the kernel samples to bound the k-th
    distance) lies within 5 m of ego 0 and every other point 60..80 m away:
    the bound then admits fewer than k points, and the selection must fall
    back to every point.  Indices bit-exact against the oracle."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4, scenarios=2, objects=(8, 16), rg_points=(8000, 9000), steps=2)
    st = sc.state_at(synth.T0)
    rng = np.random.default_rng(13)
    for s in range(sc.num_scenarios):
        p0, p1 = sc.rg_off[s], sc.rg_off[s + 1]
        g = sc.ego[s, 0]
        j = np.arange(p1 - p0)
        rad = np.where(j % 16 == 0, rng.uniform(0.5, 5.0, j.size), rng.uniform(60.0, 80.0, j.size))
        ang = rng.uniform(-np.pi, np.pi, j.size)
        sc.rg["x"][p0:p1] = (st["x"][g] + rad * np.cos(ang)).astype(np.float32)
        sc.rg["y"][p0:p1] = (st["y"][g] + rad * np.sin(ang)).astype(np.float32)
        sc.rg["valid"][p0:p1] = 1
    ds = wm.upload(sc, dev)
    S, E, k = sc.num_scenarios, sc.ego.shape[1], 1000
    o_idx, o_rf, _ = oracle.observe(sc.obj_off, sc.rg_off, f64(st), f64(sc.rg), sc.ego, k, ds.batch.max_objects)
    # ego 0 sees its 500-odd near points first, then far ones
    assert ((o_idx[:, 0, :400] % 16) == 0).all() and ((o_idx[:, 0, -100:] % 16) != 0).any()
    for gi, grf, _ in _observe_both(ds, ds.init, ds.rg, E, k):
        np.testing.assert_array_equal(gi.reshape(S, E, k), o_idx)
        assert within(grf.reshape(S, E, k, 4), o_rf).all()


def test_observe_small_and_odd_point_counts():
    """Scenarios of 0, 1, 2, 3, 5, 4,097 and 6,143 road points (the last round
    of the 1024-thread work-group is partial; loads past a scenario's end are
    clamped), k = 4 and k = 1000, so that k exceeds the valid points of some
    scenarios; some points invalid.  Again with the road-graph arrays 4 bytes
    past a 16-byte boundary."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    counts = [0, 1, 2, 3, 5, 4097, 6143]
    sc = synth.make_scene(4, scenarios=len(counts), objects=(3, 9), rg_points=(24, 24), steps=2)
    rng = np.random.default_rng(5)
    P = np.asarray(counts)
    sc.rg_off = np.concatenate([[0], np.cumsum(P)]).astype(np.int32)
    tot = int(P.sum())
    sc.rg = {"x": rng.uniform(-60, 60, tot).astype(np.float32), "y": rng.uniform(-60, 60, tot).astype(np.float32),
             "dir_x": np.ones(tot, np.float32), "dir_y": np.zeros(tot, np.float32),
             "type": np.ones(tot, np.int8), "valid": (rng.random(tot) > 0.1).astype(np.uint8)}
    sc.rg["valid"][int(P[0])] = 1
    st = sc.state_at(synth.T0)
    ds = wm.upload(sc, dev)
    S, E = sc.num_scenarios, sc.ego.shape[1]
    maxN = ds.batch.max_objects

    def shifted(t):
        # the same values at an address 4 bytes past a 16-byte boundary
        buf = torch.empty(t.numel() + 16, dtype=t.dtype, device=dev)
        off = 4 // t.element_size()
        buf[off:off + t.numel()] = t
        return buf[off:off + t.numel()]

    rg_odd = wm.Roadgraph(*(shifted(getattr(ds.rg, f)) for f in ("x", "y", "dir_x", "dir_y", "type", "valid")))
    assert rg_odd.x.data_ptr() % 16 == 4
    for k in (4, 1000):
        o_idx, o_rf, _ = oracle.observe(sc.obj_off, sc.rg_off, f64(st), f64(sc.rg), sc.ego, k, maxN)
        for rg in (ds.rg, rg_odd):
            for gi, grf, _ in _observe_both(ds, ds.init, rg, E, k):
                np.testing.assert_array_equal(gi.reshape(S, E, k), o_idx, err_msg="k=%d" % k)
                assert within(grf.reshape(S, E, k, 4), o_rf).all(), k


def test_observe_every_step_of_a_sequence():
    """wm_observe_seq over the logged rows equals the oracle's observation of
    each row (indices bit-exact); over a fused rollout's trajectory it equals
    one wm_observe call per row."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    k = 200
    sc = synth.make_scene(4, scenarios=3, objects=(4, 40), rg_points=(700, 3000), steps=6, rg_invalid_frac=0.05,
                          invalid_frac=0.1)
    ds = wm.upload(sc, dev)
    S, E = sc.num_scenarios, sc.ego.shape[1]
    maxN, n, T = ds.batch.max_objects, sc.total_objects, sc.steps
    R = T + 1
    idx = torch.empty((R, S * E * k), dtype=torch.int32, device=dev)
    rf = torch.empty((R, S * E * k * 4), device=dev)
    of = torch.empty((R, S * E * maxN * 8), device=dev)
    wm.observe_seq(ds.batch, ds.log_seq, R, ds.rg, ds.ego, E, k, idx, rf, of)
    torch.cuda.synchronize()
    lw = sc.log_window()
    for t in range(R):
        o_idx, o_rf, o_of = oracle.observe(sc.obj_off, sc.rg_off, f64({q: v[t] for q, v in lw.items()}), f64(sc.rg),
                                           sc.ego, k, maxN)
        np.testing.assert_array_equal(idx[t].cpu().numpy().reshape(S, E, k), o_idx, err_msg="row %d" % t)
        assert within(rf[t].cpu().numpy().reshape(S, E, k, 4), o_rf).all(), t
        g_of = of[t].cpu().numpy().reshape(S, E, maxN, 8)
        ok = within(g_of, o_of)
        ok[..., 2] = np.abs(((g_of[..., 2] - o_of[..., 2] + math.pi) % (2 * math.pi)) - math.pi) <= 1e-5
        assert ok.all(), t
    # the rollout's own trajectory: one launch equals one call per row
    ws = ds.batch.workspace(T, 0)
    traj = wm.State.empty((T, n), dev)
    wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, traj=traj)
    idx2 = torch.empty((T, S * E * k), dtype=torch.int32, device=dev)
    of2 = torch.empty((T, S * E * maxN * 8), device=dev)
    wm.observe_seq(ds.batch, traj, T, ds.rg, ds.ego, E, k, idx2, None, of2)
    one = torch.empty((S * E * k,), dtype=torch.int32, device=dev)
    of1 = torch.empty((S * E * maxN * 8,), device=dev)
    for t in range(T):
        wm.observe(ds.batch, traj.row(t), ds.rg, ds.ego, E, k, one, None, of1)
        torch.cuda.synchronize()
        assert torch.equal(one, idx2[t]) and torch.equal(of1, of2[t]), t


def test_prepared_steps_equal_plain_steps():
    """wm_step_prepared after one wm_roadgraph_prepare gives the same states
    and metrics as wm_step, which compacts the road edges at every call."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _ragged(T=8)
    ds = wm.upload(sc, dev)
    traj, met = _run_plain(ds, sc, dev)
    n, T = sc.total_objects, sc.steps
    t2 = wm.State.empty((T, n), dev)
    m2 = wm.Metrics.empty((T, n), dev)
    ws = ds.batch.workspace()
    wm.roadgraph_prepare(ds.batch, ds.rg, ws)
    cur = ds.init
    for t in range(1, T + 1):
        act = wm.Action(ds.act_seq.accel[t - 1], ds.act_seq.curvature[t - 1], ds.act_seq.controlled)
        wm.step_prepared(ds.batch, cur, act, ds.log_seq.row(t), ds.rg, sc.dt, t2.row(t - 1), m2.row(t - 1), ws)
        cur = t2.row(t - 1)
    torch.cuda.synchronize()
    for f in synth.STATE_FIELDS + ("valid",):
        assert torch.equal(getattr(traj, f), getattr(t2, f)), f
    for f in wm.Metrics.FIELDS:
        assert torch.equal(getattr(met, f), getattr(m2, f)), f


def test_largest_scenario_fused_equals_plain_and_oracle():
    """Scenarios with the largest supported object count (1024): the fused
    rollout (units of 64 objects, all 1024 partners in LDS) equals the plain
    steps and matches the oracle."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(2, scenarios=2, objects=(1024, 1024), rg_points=(2000, 2400), steps=3, object_box=100,
                          invalid_frac=0.05, on_road_frac=0.3)
    assert int(np.diff(sc.obj_off).max()) == 1024
    ds = wm.upload(sc, dev)
    traj, met, loss, _ = _run_fused(ds, sc, dev)
    ptraj, pmet = _run_plain(ds, sc, dev)
    for f in synth.STATE_FIELDS + ("valid",):
        assert torch.equal(getattr(traj, f), getattr(ptraj, f)), f
    for f in wm.Metrics.FIELDS:
        assert torch.equal(getattr(met, f), getattr(pmet, f)), f
    T = sc.steps
    lw = sc.log_window()
    init = f64({k: v[0] for k, v in lw.items()})
    ref = oracle.rollout(sc.obj_off, sc.rg_off, init, sc.accel, sc.curvature, sc.controlled, f64(lw), f64(sc.rg), T,
                         sc.dt)
    gm = {f: getattr(met, f).cpu().numpy() for f in METRICS}
    compare_rollout(traj.numpy(), gm, loss.cpu().numpy(), ref, sc.obj_off, sc.rg_off, f64(sc.rg))


@pytest.mark.gpu
def test_fused_rollout_exact_scan_of_tied_corners():
    """A tiny stationary object whose four corners all sit within a millimetre
    of (302, 201), where four road-edge points in four different 32-point
    blocks lie at distance 5: every corner has three or more candidate blocks
    within the band, so the fused rollout takes its exact scan for all four
    corners at every step, and the object's off-road margin comes only from
    that path.  The scene sits away from the origin, so that |corner|^2 (the
    offset between the scan's expanded form and the squared distance) is much
    larger than the band.  Compared with the oracle step by step (playback,
    so the states are the logged ones)."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    P, T = 320, 3
    xy = np.stack([1300.0 + np.arange(P), 1200.0 + 0.5 * np.arange(P)], 1)
    ring = [(305, 205), (299, 197), (306, 204), (298, 198)]          # distance 5 from (302, 201)
    positions = (10, 160, 230, 300)
    for k, pos in enumerate(positions):
        xy[pos] = ring[k]
    ang = np.arange(P) * 0.1
    rg = {"x": xy[:, 0], "y": xy[:, 1], "dir_x": np.cos(ang), "dir_y": np.sin(ang),
          "type": np.ones(P, np.int8), "valid": np.ones(P, np.uint8)}
    n = 2
    row = {"x": np.array([302.0, 330.0]), "y": np.array([201.0, 160.0]), "yaw": np.array([0.0, 0.7]),
           "vx": np.zeros(n), "vy": np.zeros(n), "length": np.array([0.002, 4.5]),
           "width": np.array([0.002, 1.9]), "valid": np.ones(n, np.uint8)}
    obj_off = np.array([0, n], np.int32)
    rg_off = np.array([0, P], np.int32)
    batch = wm.Batch.from_offsets(obj_off, rg_off, dev)

    def rows(v, dtype):
        return torch.tensor(np.tile(np.asarray(v), (T + 1, 1)), dtype=dtype, device=dev)

    log = wm.State(*[rows(row[f], torch.float32) for f in wm.STATE_FIELDS], rows(row["valid"], torch.uint8))
    init = wm.State(*[getattr(log, f)[0].clone() for f in wm.STATE_FIELDS], log.valid[0].clone())
    act = wm.Action(torch.zeros((T, n), device=dev), torch.zeros((T, n), device=dev),
                    torch.zeros(n, dtype=torch.uint8, device=dev))
    met = wm.Metrics.empty((T, n), dev)
    traj = wm.State.empty((T, n), dev)
    ws = batch.workspace(T, 0)
    wm.rollout(batch, init, act, log, wm.Roadgraph.from_numpy(rg, dev), T, 0.1, ws, traj=traj, metrics=met)
    torch.cuda.synchronize()
    ref = oracle.offroad(obj_off, rg_off, row, rg)
    for t in range(T):
        np.testing.assert_array_equal(met.offroad[t].cpu().numpy(), ref["offroad"])
        np.testing.assert_allclose(met.offroad_margin[t].cpu().numpy(), ref["margin"], rtol=1e-5, atol=1e-4)
    assert met.offroad_margin[0, 0].item() != wm.NO_VALUE


@pytest.mark.gpu
def test_autotune_cache_file(tmp_path, monkeypatch):
    """With WM_TUNE_CACHE set, wm_autotune appends its pick to the file, and a
    matching line (same device kind and batch bucket) is taken without timing:
    a planted line for this batch's bucket is returned as is."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = _ragged(T=4)
    ds = wm.upload(sc, dev)
    T = sc.steps
    ws = ds.batch.workspace(T, 0)
    prop = torch.cuda.get_device_properties(0)
    tag = "%s %d" % (prop.gcnArchName.split(":")[0], prop.multi_processor_count)
    ob = max(int(sc.max_objects - 1).bit_length(), 0)
    pb = max(int(sc.max_rg_points - 1).bit_length(), 0)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("WM_TUNE_CACHE", str(path))
    picked = wm.autotune(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws)
    lines = path.read_text().splitlines()
    assert len(lines) == 1
    assert lines[0].split() == ["wm-tune", "3"] + tag.split() + [str(ob), str(pb), str(picked[0]), str(picked[1])]
    planted = (128, 2) if tuple(picked) != (128, 2) else (64, 4)
    path.write_text("wm-tune 3 %s %d %d %d %d\n" % (tag, ob, pb, planted[0], planted[1]))
    assert tuple(wm.autotune(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws)) == planted
    assert len(path.read_text().splitlines()) == 1   # taken, not timed and appended


def test_pruned_scans_with_boxes_in_global_memory():
    """Scenarios of 55,000-60,000 road points (about 37,000 road-edge points,
    more than 256 chunks of 128): the pruned scans then read the chunk and
    block boxes from global memory instead of LDS.  The per-step off-road
    with the pruned scan (tuning 64 x 8) equals the scan of every point
    (tuning 256 x 4, 1024 threads) bit for bit and agrees with the oracle;
    the fused rollout equals the plain steps bit for bit."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4, scenarios=2, objects=(20, 70), rg_points=(55000, 60000), steps=3,
                          rg_invalid_frac=0.02, object_box=40, on_road_frac=0.5)
    edges = [int(((sc.rg["type"][a:b] == synth.TYPE_ROAD_EDGE) & (sc.rg["valid"][a:b] != 0)).sum())
             for a, b in zip(sc.rg_off[:-1], sc.rg_off[1:])]
    assert min(edges) > 256 * 128, edges
    ds = wm.upload(sc, dev)
    n = sc.total_objects
    ws = ds.batch.workspace()
    res = {}
    for tune in ((64, 8), (256, 4)):
        off = torch.empty(n, dtype=torch.uint8, device=dev)
        mg = torch.empty(n, device=dev)
        near = torch.empty((n, 4), dtype=torch.int32, device=dev)
        wm.offroad(ds.batch, ds.init, ds.rg, ws, off, mg, near, tune=tune)
        torch.cuda.synchronize()
        res[tune] = (off, mg, near)
    for a, b in zip(res[(64, 8)], res[(256, 4)]):
        assert torch.equal(a, b)
    ref = oracle.offroad(sc.obj_off, sc.rg_off, f64(sc.state_at(synth.T0)), f64(sc.rg))
    off, mg, _ = res[(64, 8)]
    ties = compare_offroad(off.cpu().numpy(), mg.cpu().numpy(), ref, "global boxes")
    assert ties <= n // 20
    traj, met, _, _ = _run_fused(ds, sc, dev)
    ptraj, pmet = _run_plain(ds, sc, dev)
    assert torch.equal(traj.x, ptraj.x)
    for f in ("offroad", "offroad_margin", "collision", "overlap_margin"):
        assert torch.equal(getattr(met, f), getattr(pmet, f)), f


def test_observe_one_row_of_many_egos():
    """One row of 320 scenarios x 8 egos (2,560 observations, more than two
    per resident work-group slot of an MI355X): the one-row call takes the
    block form with several egos per work-group.  Indices bit-exact and
    features within tolerance against the oracle, with exact key ties from
    points quantised to a 0.5 m grid.  Objects here lie up to 200 m apart:
    an ego-frame position is a difference of binary32 products of that
    size, so its tolerance grows with the coordinates (8 ulp of their sum)."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(4, scenarios=320, objects=(8, 24), rg_points=(600, 1500), steps=2, rg_invalid_frac=0.05,
                          invalid_frac=0.05)
    sc.rg["x"][::3] = np.round(sc.rg["x"][::3] * 2) / 2
    sc.rg["y"][::3] = np.round(sc.rg["y"][::3] * 2) / 2
    ds = wm.upload(sc, dev)
    S, E, k = sc.num_scenarios, sc.ego.shape[1], 200
    assert S * E >= 2048
    maxN = ds.batch.max_objects
    st = sc.state_at(synth.T0)
    idx = torch.empty(S * E * k, dtype=torch.int32, device=dev)
    rf = torch.empty(S * E * k * 4, device=dev)
    of = torch.empty(S * E * maxN * 8, device=dev)
    wm.observe(ds.batch, ds.init, ds.rg, ds.ego, E, k, idx, rf, of)
    torch.cuda.synchronize()
    o_idx, o_rf, o_of = oracle.observe(sc.obj_off, sc.rg_off, f64(st), f64(sc.rg), sc.ego, k, maxN)
    np.testing.assert_array_equal(idx.cpu().numpy().reshape(S, E, k), o_idx)
    assert within(rf.cpu().numpy().reshape(S, E, k, 4), o_rf).all()
    g_of = of.cpu().numpy().reshape(S, E, maxN, 8)
    ok = within(g_of, o_of)
    ok[..., 2] = np.abs(((g_of[..., 2] - o_of[..., 2] + math.pi) % (2 * math.pi)) - math.pi) <= 1e-5
    # coordinates of each ego and of each scenario's objects (0 past the end)
    ax, ay = np.abs(st["x"].astype(np.float64)), np.abs(st["y"].astype(np.float64))
    obj = np.zeros((S, maxN), np.int64)
    has = np.zeros((S, maxN), bool)
    for sc_i in range(S):
        cnt = sc.obj_off[sc_i + 1] - sc.obj_off[sc_i]
        obj[sc_i, :cnt] = sc.obj_off[sc_i] + np.arange(cnt)
        has[sc_i, :cnt] = True
    scale = (ax[sc.ego] + ay[sc.ego])[:, :, None] + np.where(has, ax[obj] + ay[obj], 0.0)[:, None, :]
    tol = 1e-5 + 8 * 2.0 ** -24 * scale
    for c in (0, 1):
        ok[..., c] = np.abs(g_of[..., c] - o_of[..., c]) <= tol
    assert ok.all(), np.argwhere(~ok)[:5]
