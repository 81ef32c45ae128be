"""GPU parity of the delta action space (App. A.1) and of discretized actions
(Sec. 5.2, Expert), through the C ABI."""
import numpy as np
import pytest

import oracle
from helpers import assert_state_close, device, f64, within
from paper_2310_08710_amd import synth

pytestmark = pytest.mark.gpu


def test_delta_step_and_inverse():
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(2, scenarios=6, objects=(1, 70), rg_points=(240, 480), steps=2, invalid_frac=0.1)
    ds = wm.upload(sc, dev)
    n = sc.total_objects
    rng = np.random.default_rng(9)
    d = rng.uniform(-2, 2, (3, n)).astype(np.float32)
    ctrl = (rng.random(n) < 0.7).astype(np.uint8)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    nxt = wm.State.empty(n, dev)
    wm.step_delta(ds.batch, ds.init, T(d[0]), T(d[1]), T(d[2]), T(ctrl), ds.log_seq.row(1), sc.dt, nxt)
    torch.cuda.synchronize()
    lw = sc.log_window()
    ref = oracle.delta_forward(f64({q: v[0] for q, v in lw.items()}), d[0], d[1], d[2], ctrl,
                               f64({q: v[1] for q, v in lw.items()}), sc.dt)
    g = nxt.numpy()
    # vx = (x' - x)/dt: the rounding of x' (|x| <= 128 m, ulp 7.6e-6) is divided by dt
    assert_state_close({k: v for k, v in g.items() if k not in ("vx", "vy")} | {"vx": ref["vx"], "vy": ref["vy"]},
                       ref, "delta step")
    for f in ("vx", "vy"):
        assert within(g[f], ref[f], atol=2 * 7.63e-6 / sc.dt).all(), f
    # inverse on logged transitions
    dx, dy, dyaw = (torch.empty(n, device=dev) for _ in range(3))
    v = torch.empty(n, dtype=torch.uint8, device=dev)
    wm.inverse_delta(ds.batch, ds.log_seq.row(0), ds.log_seq.row(1), dx, dy, dyaw, v)
    torch.cuda.synchronize()
    ox, oy, ot, ov = oracle.delta_inverse(f64({q: w[0] for q, w in lw.items()}), f64({q: w[1] for q, w in lw.items()}))
    np.testing.assert_array_equal(v.cpu().numpy(), ov)
    for gv, o in ((dx, ox), (dy, oy), (dyaw, ot)):
        assert within(gv.cpu().numpy(), o).all()


@pytest.mark.parametrize("lo,hi,bins", [(-6.0, 6.0, 13), (-0.3, 0.3, 31), (-1.0, 1.0, 5), (0.0, 1.0, 2)])
def test_discretize_bit_exact(lo, hi, bins):
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    rng = np.random.default_rng(10)
    step = (hi - lo) / (bins - 1)
    v = np.concatenate([rng.uniform(lo - 1, hi + 1, 20000), lo + step * (np.arange(bins) + 0.5),   # half-way
                        lo + step * np.arange(bins), [np.inf, -np.inf, 1e30, -1e30]]).astype(np.float32)
    idx = torch.empty(v.size, dtype=torch.int32, device=dev)
    snp = torch.empty(v.size, device=dev)
    wm.discretize(torch.from_numpy(v).to(dev), lo, hi, bins, idx, snp)
    torch.cuda.synchronize()
    oi, os_ = oracle.discretize(v, lo, hi, bins)
    np.testing.assert_array_equal(idx.cpu().numpy(), oi)
    np.testing.assert_array_equal(snp.cpu().numpy(), os_)


def test_discrete_expert_actions():
    """Expert actions (inverse kinematics on the logs) discretized into a 13 x
    31 grid: indices agree with the oracle's except where the two continuous
    inverses straddle a bin boundary within their tolerance."""
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    sc = synth.make_scene(1, scenarios=8, rg_points=(240, 240), steps=2)
    ds = wm.upload(sc, dev)
    n = sc.total_objects
    a, k = torch.empty(n, device=dev), torch.empty(n, device=dev)
    wm.inverse_action(ds.batch, ds.log_seq.row(0), ds.log_seq.row(1), sc.dt, a, k)
    ia, ik = torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev)
    wm.discretize(a, -6.0, 6.0, 13, ia)
    wm.discretize(k, -0.3, 0.3, 31, ik)
    torch.cuda.synchronize()
    lw = sc.log_window()
    oa, ok_, _ = oracle.bicycle_inverse(f64({q: w[0] for q, w in lw.items()}), f64({q: w[1] for q, w in lw.items()}),
                                        sc.dt)
    for g, o, lo, hi, bins, tol in ((ia, oa, -6.0, 6.0, 13, 2e-4), (ik, ok_, -0.3, 0.3, 31, 2e-5)):
        oi, _ = oracle.discretize(o, lo, hi, bins)
        u = (o - lo) * (bins - 1) / (hi - lo)
        near = np.abs(u - np.floor(u) - 0.5) < tol * (bins - 1) / (hi - lo)
        np.testing.assert_array_equal(g.cpu().numpy()[~near], oi[~near])
        assert (~near).mean() > 0.99
