"""GPU parity of the fused rollout with IDM sim agents (Sec. 3.5) against the
oracle's own IDM rollout from the same inputs.  An IDM step takes discrete
decisions (which pose first touches which object, whether the path end is
reached); a scenario is compared up to the first step whose decision margin
(reported by the oracle) falls within the band the measured state difference
allows, and every step before that must match to the state tolerance, with
collision and off-road masks exact outside their bands.

With the default parameters many agents meet a path-end decision at a margin
of about 1e-6 m: logged objects held at the generator's 0.5 m/s speed floor
cover exactly 1.5 m in 3 s, and an agent starting at 0.5 m/s under a free-road
acceleration of 2 m/s^2 also covers 1.5 m in its first 10 steps.  Those
scenarios stop being compared there, so the default-parameter case requires
half of the object-steps; the cases with a_max = 1.7 m/s^2 (a parameter of the
call) avoid the coincidence and require 90%."""
import numpy as np
import pytest

import oracle
from helpers import (BAND, assert_traj_close, compare_collision, compare_offroad, device, f64, scenario_band,
                     state_delta, within)
from paper_2310_08710_amd import synth

pytestmark = pytest.mark.gpu

FIELDS = synth.STATE_FIELDS + ("valid",)


def _scene(seed_base=1000, T=30):
    return synth.make_scene(2, seed_base=seed_base, scenarios=8, objects=(8, 48), rg_points=(2000, 4000), steps=T,
                            controlled_per_scenario=4, object_box=50.0, invalid_frac=0.05)


def _gpu_idm(sc, idm=None, controlled=None):
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    if controlled is not None:
        sc.controlled = controlled
    ds = wm.upload(sc, dev)
    n, T = sc.total_objects, sc.steps
    ws = ds.batch.workspace(T, 0)
    traj = wm.State.empty((T, n), dev)
    met = wm.Metrics.empty((T, n), dev)
    wm.rollout_idm(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, idm=idm, traj=traj, metrics=met)
    torch.cuda.synchronize()
    return ds, traj, met


@pytest.mark.parametrize("seed,large,a_max,min_frac", [(1000, False, None, 0.5), (1000, False, 1.7, 0.9),
                                                      (3000, False, 1.7, 0.9), (5000, True, 1.7, 0.9)])
def test_idm_rollout_matches_oracle(seed, large, a_max, min_frac):
    # large: scenarios above 256 objects take the lead search without the
    # per-agent candidate masks
    sc = _scene(seed) if not large else synth.make_scene(
        2, seed_base=seed, scenarios=2, objects=(260, 300), rg_points=(2000, 3000), steps=12,
        controlled_per_scenario=4, object_box=120.0, invalid_frac=0.05)
    _, traj, met = _gpu_idm(sc, idm=None if a_max is None else {"max_accel": a_max})
    T, n = sc.steps, sc.total_objects
    lw = f64(sc.log_window())
    init = {k: v[0] for k, v in lw.items()}
    rg = f64(sc.rg)
    ref = oracle.rollout_idm(sc.obj_off, sc.rg_off, init, sc.accel, sc.curvature, sc.controlled, lw, rg, T,
                             sc.dt, idm=None if a_max is None else {"a_max": a_max})
    g = traj.numpy()
    gm = {f: getattr(met, f).cpu().numpy() for f in ("collision", "overlap_margin", "offroad", "offroad_margin",
                                                       "log_div")}
    off = np.asarray(sc.obj_off)
    agents = ~np.isinf(ref["idm_margin"]).all(axis=0)
    assert agents.sum() > n // 2
    live = np.ones(sc.num_scenarios, bool)      # scenarios still compared
    compared = 0
    offroad_seen = set()
    prev_delta = np.zeros(n)
    for t in range(T):
        # the decisions of step t+1 were taken from the states of step t
        # (row t-1); stop a scenario when one of them is within the band
        for s in range(sc.num_scenarios):
            sl = slice(off[s], off[s + 1])
            if live[s] and off[s + 1] > off[s]:
                band = BAND + 2.0 * prev_delta[sl].max() + 1e-4
                if ref["idm_margin"][t, sl].min() < band:
                    live[s] = False
        cols = np.concatenate([np.arange(off[s], off[s + 1]) for s in range(sc.num_scenarios) if live[s]] +
                              [np.zeros(0, int)])
        if cols.size == 0:
            break
        gt = {k: v[t, cols] for k, v in g.items()}
        ot = {k: v[t, cols] for k, v in ref["traj"].items()}
        assert_traj_close(gt, ot, "t=%d" % t)
        delta = state_delta(gt, ot)
        sub_off = np.concatenate([[0], np.cumsum([off[s + 1] - off[s] for s in range(sc.num_scenarios) if live[s]])])
        band = scenario_band(delta, sub_off)
        compare_collision(gm["collision"][t, cols], gm["overlap_margin"][t, cols], ref["collision"][t, cols],
                          ref["overlap_margin"][t, cols], "t=%d" % t, band=band)
        # off-road of the IDM-driven states: the oracle's metric of its own
        # state row, with its per-corner tie information, on the live columns
        sub_rg = np.concatenate([[0], np.cumsum([sc.rg_off[s + 1] - sc.rg_off[s]
                                                 for s in range(sc.num_scenarios) if live[s]])])
        rows = np.concatenate([np.arange(sc.rg_off[s], sc.rg_off[s + 1]) for s in range(sc.num_scenarios)
                               if live[s]] + [np.zeros(0, int)])
        r = oracle.offroad(sub_off, sub_rg, ot, {k: v[rows] for k, v in rg.items()}, band=float(band.max()))
        np.testing.assert_array_equal(r["offroad"], ref["offroad"][t, cols], err_msg="oracle offroad t=%d" % t)
        compare_offroad(gm["offroad"][t, cols], gm["offroad_margin"][t, cols], r, "t=%d" % t, band=band)
        offroad_seen.update(np.unique(gm["offroad"][t, cols]).tolist())
        ld = gm["log_div"][t, cols]
        assert (within(ld, ref["log_div"][t, cols]) | (np.abs(ld - ref["log_div"][t, cols]) <= delta + 1e-5)).all()
        prev_delta[cols] = delta
        compared += cols.size
    assert compared >= min_frac * T * n, (compared, T * n)
    assert offroad_seen == {0, 1}                 # both mask values were compared
    # the agents did react
    moved = np.abs(ref["traj"]["x"][:, agents] - lw["x"][1:, agents]).max()
    assert moved > 0.5


def test_idm_without_agents_is_the_plain_rollout():
    import torch
    from paper_2310_08710_amd import wm
    sc = _scene(T=12)
    ctrl = np.ones_like(sc.controlled)
    ds, traj, met = _gpu_idm(sc, controlled=ctrl)
    n, T = sc.total_objects, sc.steps
    ws = ds.batch.workspace(T, 0)
    t2 = wm.State.empty((T, n), ds.init.x.device)
    m2 = wm.Metrics.empty((T, n), ds.init.x.device)
    wm.rollout(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, traj=t2, metrics=m2)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert torch.equal(getattr(traj, f), getattr(t2, f)), f
    for f in ("collision", "offroad", "overlap_margin", "offroad_margin", "log_div", "infeasible", "reward"):
        assert torch.equal(getattr(met, f), getattr(m2, f)), f


def test_idm_tunings_agree():
    import torch
    from paper_2310_08710_amd import wm
    sc = _scene(T=10)
    ds, traj, met = _gpu_idm(sc)
    n, T = sc.total_objects, sc.steps
    ws = ds.batch.workspace(T, 0)
    for tune in ((64, 2), (128, 2), (64, 8)):
        t2 = wm.State.empty((T, n), ds.init.x.device)
        m2 = wm.Metrics.empty((T, n), ds.init.x.device)
        wm.rollout_idm(ds.batch, ds.init, ds.act_seq, ds.log_seq, ds.rg, T, sc.dt, ws, traj=t2, metrics=m2,
                       tune=tune)
        torch.cuda.synchronize()
        for f in FIELDS:
            assert torch.equal(getattr(traj, f), getattr(t2, f)), (tune, f)
        assert torch.equal(met.offroad_margin, m2.offroad_margin)
