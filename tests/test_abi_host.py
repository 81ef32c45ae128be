"""The C-ABI library loads on a machine without a GPU, exports every function
that include/wm.h declares, and rejects bad host-visible arguments before
touching the device (no call here reaches a launch)."""
import ctypes as C
import os
import re

import pytest

from paper_2310_08710_amd import wm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(wm.LIB_PATH), reason="libwm.so not built")

FAKE = 0x100000  # never dereferenced: every call below fails validation first


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 11
    lib = wm.lib()
    for name in names:
        assert hasattr(lib, name), name


def _batch(S=2, n=10, P=100, max_obj=6, max_rg=60):
    return wm.CBatch(S, n, P, max_obj, max_rg, FAKE, FAKE)


def _state(null_field=None):
    vals = [FAKE] * 8
    if null_field is not None:
        vals[null_field] = None
    return wm.CState(*vals)


def _rg():
    return wm.CRoadgraph(*([FAKE] * 6))


def _act():
    return wm.CAction(FAKE, FAKE, FAKE)


def _msg():
    return wm.lib().wm_last_error_message().decode()


def step(batch=None, cur=None, act=None, log=None, rg=None, dt=0.1, nxt=None, m=None, ws=None, ws_bytes=0):
    b = batch if batch is not None else _batch()
    cur = cur if cur is not None else _state()
    nxt = nxt if nxt is not None else wm.CState(*([FAKE + 64] * 8))
    return wm.lib().wm_step(C.byref(b), C.byref(cur), C.byref(act if act is not None else _act()),
                            C.byref(log if log is not None else _state()), C.byref(rg) if rg is not None else None,
                            dt, C.byref(nxt), C.byref(m) if m is not None else None, ws, ws_bytes, None)


def test_error_strings():
    for code in range(7):
        assert wm.error_string(code)
    assert "unknown" in wm.error_string(99)


def test_workspace_bytes_pure_host():
    b = _batch()
    n0 = wm.lib().wm_workspace_bytes(C.byref(b), 0, 0)
    n1 = wm.lib().wm_workspace_bytes(C.byref(b), 80, 10)
    assert 0 < n0 < n1
    bad = _batch(S=0)
    assert wm.lib().wm_workspace_bytes(C.byref(bad), 0, 0) == 0


def test_step_validation():
    assert wm.lib().wm_step(None, None, None, None, None, 0.1, None, None, None, 0, None) == wm.WM_ERR_NULL
    assert step(batch=_batch(S=0)) == wm.WM_ERR_RANGE
    assert step(batch=_batch(max_obj=20)) == wm.WM_ERR_SHAPE                  # max > total
    assert step(batch=wm.CBatch(1, 2000, 10, 1100, 10, FAKE, FAKE)) == wm.WM_ERR_UNSUPPORTED
    assert step(batch=wm.CBatch(1, 10, 10, 10, 10, None, FAKE)) == wm.WM_ERR_NULL
    assert step(cur=_state(null_field=3)) == wm.WM_ERR_NULL
    assert "cur" in _msg()
    assert step(act=wm.CAction(FAKE, None, FAKE)) == wm.WM_ERR_NULL
    for dt in (0.0, -0.1, float("nan"), float("inf")):
        assert step(dt=dt) == wm.WM_ERR_RANGE
    assert step(nxt=_state()) == wm.WM_ERR_RANGE                              # next aliases cur
    m = wm.CMetrics(None, FAKE, None, None, None)
    assert step(rg=_rg(), m=m) == wm.WM_ERR_WORKSPACE                          # offroad needs workspace
    assert "workspace" in _msg()
    assert step(rg=_rg(), m=m, ws=FAKE, ws_bytes=16) == wm.WM_ERR_WORKSPACE
    assert step(rg=wm.CRoadgraph(FAKE, FAKE, None, FAKE, FAKE, FAKE), m=m) == wm.WM_ERR_NULL


def test_step_noalloc_validation():
    """The device-scratch step validates like wm_step and rejects a batch
    whose off-road workspace exceeds its WM_NOALLOC_SCRATCH_BYTES (64 MiB)
    before any device call."""
    lib = wm.lib()
    m = wm.CMetrics(None, FAKE, None, None, None)

    def call(batch=None, cur=None, rg=None, m=None, dt=0.1):
        b = batch if batch is not None else _batch()
        c = cur if cur is not None else _state()
        return lib.wm_step_noalloc(C.byref(b), C.byref(c), C.byref(_act()), C.byref(_state()),
                                   C.byref(rg) if rg is not None else None, dt,
                                   C.byref(wm.CState(*([FAKE + 64] * 8))), C.byref(m) if m is not None else None,
                                   None)

    assert lib.wm_step_noalloc(None, None, None, None, None, 0.1, None, None, None) == wm.WM_ERR_NULL
    assert call(batch=_batch(S=0)) == wm.WM_ERR_RANGE
    assert call(cur=_state(null_field=2)) == wm.WM_ERR_NULL
    assert call(dt=0.0) == wm.WM_ERR_RANGE
    # 3 million road points: 24 bytes of workspace per point slot > 64 MiB
    big = wm.CBatch(4, 400, 3000000, 100, 750000, FAKE, FAKE)
    assert lib.wm_workspace_bytes(C.byref(big), 0, 0) > 64 << 20
    assert call(batch=big, rg=_rg(), m=m) == wm.WM_ERR_UNSUPPORTED
    assert "wm_step_noalloc" in _msg() and "scratch" in _msg()


def test_step_observe_validation():
    """The closed-loop step validates the step's and the observation's
    arguments before any launch."""
    lib = wm.lib()
    m = wm.CMetrics(FAKE, FAKE, None, None, None)

    def call(batch=None, cur=None, rg="fake", ego=FAKE, E=8, k=100, idx=FAKE, dt=0.1, ws=FAKE, ws_bytes=1 << 30):
        b = batch if batch is not None else _batch()
        c = cur if cur is not None else _state()
        r = _rg() if rg == "fake" else rg
        return lib.wm_step_observe(C.byref(b), C.byref(c), C.byref(_act()), C.byref(_state()),
                                   C.byref(r) if r is not None else None, dt,
                                   C.byref(wm.CState(*([FAKE + 64] * 8))), C.byref(m), ego, E, k, idx, None, None,
                                   ws, ws_bytes, None)

    assert call(rg=None) == wm.WM_ERR_NULL
    assert call(ego=None) == wm.WM_ERR_NULL
    assert call(idx=None) == wm.WM_ERR_NULL
    assert call(E=0) == wm.WM_ERR_RANGE
    assert call(k=0) == wm.WM_ERR_RANGE
    assert call(k=2000) == wm.WM_ERR_UNSUPPORTED
    assert call(batch=wm.CBatch(1, 10, 40000, 10, 40000, FAKE, FAKE)) == wm.WM_ERR_UNSUPPORTED   # > 32768 points
    assert call(cur=_state(null_field=0)) == wm.WM_ERR_NULL
    assert call(dt=-1.0) == wm.WM_ERR_RANGE
    assert call(ws=None) == wm.WM_ERR_WORKSPACE                      # off-road metrics read the prepared edges
    assert call(ws_bytes=8) == wm.WM_ERR_WORKSPACE


def test_offroad_and_tuning_validation():
    L = wm.lib()
    b, s, r = _batch(), _state(), _rg()
    need = L.wm_workspace_bytes(C.byref(b), 0, 0)
    for U, G in ((32, 4), (64, 3), (256, 8), (128, 32)):
        t = wm.CTuning(U, G)
        rc = L.wm_offroad(C.byref(b), C.byref(s), C.byref(r), FAKE, FAKE, None, C.byref(t), FAKE, need, None)
        assert rc == wm.WM_ERR_RANGE, (U, G)
    rc = L.wm_offroad(C.byref(b), C.byref(s), None, FAKE, FAKE, None, None, FAKE, need, None)
    assert rc == wm.WM_ERR_NULL
    rc = L.wm_offroad(C.byref(b), C.byref(s), C.byref(r), FAKE, FAKE, None, None, FAKE, need - 1, None)
    assert rc == wm.WM_ERR_WORKSPACE


def test_observe_validation():
    L = wm.lib()
    b, s, r = _batch(), _state(), _rg()
    assert L.wm_observe(C.byref(b), C.byref(s), C.byref(r), FAKE, 0, 10, FAKE, None, None, None) == wm.WM_ERR_RANGE
    assert L.wm_observe(C.byref(b), C.byref(s), C.byref(r), FAKE, 8, 0, FAKE, None, None, None) == wm.WM_ERR_RANGE
    assert L.wm_observe(C.byref(b), C.byref(s), C.byref(r), FAKE, 8, 2000, FAKE, None, None,
                        None) == wm.WM_ERR_UNSUPPORTED
    big = wm.CBatch(1, 10, 40000, 10, 40000, FAKE, FAKE)
    assert L.wm_observe(C.byref(big), C.byref(s), C.byref(r), FAKE, 8, 10, FAKE, None, None,
                        None) == wm.WM_ERR_UNSUPPORTED
    assert L.wm_observe(C.byref(b), C.byref(s), C.byref(r), None, 8, 10, FAKE, None, None, None) == wm.WM_ERR_NULL


def test_rollout_validation():
    L = wm.lib()
    b, s, a, r = _batch(), _state(), _act(), _rg()
    need = L.wm_workspace_bytes(C.byref(b), 80, 10)

    def roll(T=80, dt=0.1, K=10, ck=None, ws_bytes=need, tune=None, act=a):
        return L.wm_rollout(C.byref(b), C.byref(s), C.byref(act), C.byref(s), C.byref(r), T, dt, K,
                            C.byref(ck) if ck is not None else None, None, None, None,
                            C.byref(tune) if tune is not None else None, FAKE, ws_bytes, None)

    assert roll(T=0) == wm.WM_ERR_RANGE
    assert roll(dt=0.0) == wm.WM_ERR_RANGE
    assert roll(K=-1) == wm.WM_ERR_RANGE
    assert roll(K=0, ck=_state()) == wm.WM_ERR_RANGE
    assert roll(ck=_state(null_field=7)) == wm.WM_ERR_NULL
    assert roll(ws_bytes=need - 1) == wm.WM_ERR_WORKSPACE
    assert roll(tune=wm.CTuning(64, 5)) == wm.WM_ERR_RANGE
    assert roll(act=wm.CAction(None, FAKE, FAKE)) == wm.WM_ERR_NULL
    bb = wm.CBatch(1, 30000000, 10, 1000, 10, FAKE, FAKE)
    assert L.wm_rollout(C.byref(bb), C.byref(s), C.byref(a), C.byref(s), None, 80, 0.1, 0, None, None, None, None,
                        None, FAKE, 1 << 40, None) == wm.WM_ERR_UNSUPPORTED

    def back(K=10, dloss=FAKE, ga=FAKE, ws_bytes=need, ck=s):
        return L.wm_rollout_backward(C.byref(b), C.byref(s), C.byref(a), C.byref(s), 80, 0.1, K,
                                     C.byref(ck) if ck is not None else None, dloss, ga, FAKE, FAKE, ws_bytes, None)

    assert back(K=0) == wm.WM_ERR_RANGE
    assert back(dloss=None) == wm.WM_ERR_NULL
    assert back(ga=None) == wm.WM_ERR_NULL
    assert back(ck=None) == wm.WM_ERR_NULL
    assert back(ws_bytes=0) == wm.WM_ERR_WORKSPACE


def test_inverse_and_overlap_validation():
    L = wm.lib()
    b, s = _batch(), _state()
    assert L.wm_inverse_action(C.byref(b), C.byref(s), C.byref(s), 0.1, None, FAKE, None, None) == wm.WM_ERR_NULL
    assert L.wm_inverse_action(C.byref(b), C.byref(s), C.byref(s), -1.0, FAKE, FAKE, None, None) == wm.WM_ERR_RANGE
    assert L.wm_overlap(C.byref(b), C.byref(s), None, FAKE, None, None, None, None) == wm.WM_ERR_NULL
    # nothing requested: a no-op that never launches
    assert L.wm_overlap(C.byref(b), C.byref(s), None, None, None, None, None, None) == wm.WM_OK


def _idm(**kw):
    p = dict(wm.IDM_DEFAULT)
    p.update(kw)
    return wm.CIdm(*[float(p[k]) for k in ("desired_speed", "min_gap", "time_headway", "max_accel",
                                           "comfort_decel", "exponent", "max_brake", "lookahead_step")],
                   int(p["lookahead_poses"]))


@pytest.mark.parametrize("bad", [{"desired_speed": 0.0}, {"max_brake": -1.0}, {"lookahead_step": float("nan")},
                                 {"lookahead_poses": 0}, {"lookahead_poses": 65}, {"min_gap": -0.5},
                                 {"time_headway": float("inf")}])
def test_idm_rollout_rejects_bad_parameters(bad):
    b = _batch()
    p = _idm(**bad)
    rc = wm.lib().wm_rollout_idm(C.byref(b), C.byref(_state()), C.byref(_act()), C.byref(_state()), None, 10, 0.1,
                                 C.byref(p), None, None, None, FAKE, 1 << 30, None)
    assert rc == 2, _msg()     # WM_ERR_RANGE
    assert "idm" in _msg()
    rc = wm.lib().wm_rollout_idm(C.byref(b), C.byref(_state()), C.byref(_act()), C.byref(_state()), None, 10, 0.1,
                                 None, None, None, None, FAKE, 1 << 30, None)
    assert rc == 1             # WM_ERR_NULL


# The boundary's calls as the scope table of this build names them: the
# step, the inverse, the two metrics, the observation, the rollout and its
# adjoint, the rollout's workspace query and the two error reporters.
BOUNDARY_CALLS = ("wm_step", "wm_inverse_action", "wm_overlap", "wm_offroad", "wm_observe", "wm_rollout",
                  "wm_rollout_backward", "wm_rollout_workspace_bytes", "wm_error_string", "wm_last_error_message")


def test_boundary_calls_are_declared_and_exported():
    names = declared_functions()
    lib = wm.lib()
    for name in BOUNDARY_CALLS:
        assert name in names, name
        assert hasattr(lib, name), name
    b = _batch()
    for T, K in ((0, 0), (80, 10), (7, 3)):
        assert lib.wm_rollout_workspace_bytes(C.byref(b), T, K) == lib.wm_workspace_bytes(C.byref(b), T, K)


def _cpu_batch(counts=(3, 4), points=(10, 12)):
    import numpy as np
    obj_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    rg_off = np.concatenate([[0], np.cumsum(points)]).astype(np.int32)
    return wm.Batch.from_offsets(obj_off, rg_off, "cpu")


def _cpu_state(n, dtype=None):
    import torch
    st = wm.State.empty((n,), "cpu")
    if dtype is not None:
        st.x = st.x.to(dtype)
    return st


def test_binding_rejects_short_or_mistyped_tensors():
    """Sizes and dtypes are checked in the binding before any pointer reaches
    the library (a short tensor would otherwise be written past its end)."""
    import torch
    b = _cpu_batch()
    n, P = b.total_objects, b.total_rg_points
    act = wm.Action(torch.zeros(n), torch.zeros(n), torch.ones(n, dtype=torch.uint8))
    rg = wm.Roadgraph(torch.zeros(P), torch.zeros(P), torch.zeros(P), torch.zeros(P),
                      torch.zeros(P, dtype=torch.int8), torch.ones(P, dtype=torch.uint8))
    good = _cpu_state(n)
    with pytest.raises(ValueError, match="next.x has 6 elements"):
        wm.step(b, good, act, good, None, 0.1, _cpu_state(n - 1))
    with pytest.raises(ValueError, match="dtype"):
        wm.step(b, _cpu_state(n, torch.float64), act, good, None, 0.1, _cpu_state(n))
    short_act = wm.Action(torch.zeros(n), torch.zeros(n - 2), act.controlled)
    with pytest.raises(ValueError, match="curvature"):
        wm.step(b, good, short_act, good, None, 0.1, _cpu_state(n))
    with pytest.raises(ValueError, match="metrics.offroad_margin"):
        wm.step(b, good, act, good, rg, 0.1, _cpu_state(n), wm.Metrics(offroad_margin=torch.zeros(n - 1)))
    short_rg = wm.Roadgraph(rg.x[:-1], rg.y, rg.dir_x, rg.dir_y, rg.type, rg.valid)
    with pytest.raises(ValueError, match="rg.x"):
        wm.offroad(b, good, short_rg, torch.zeros(64, dtype=torch.uint8), margin=torch.zeros(n))
    with pytest.raises(ValueError, match="nearest"):
        wm.offroad(b, good, rg, torch.zeros(64, dtype=torch.uint8), nearest=torch.zeros(4 * n - 1, dtype=torch.int32))
    ego = torch.zeros(2 * 2, dtype=torch.int32)
    with pytest.raises(ValueError, match="rg_idx"):
        wm.observe(b, good, rg, ego, 2, 5, torch.zeros(2 * 2 * 5 - 1, dtype=torch.int32))
    with pytest.raises(ValueError, match="obj_feat"):
        wm.observe(b, good, rg, ego, 2, 5, torch.zeros(20, dtype=torch.int32),
                   obj_feat=torch.zeros(2 * 2 * 4 * 8 - 1))
    T = 3
    seq_act = wm.Action(torch.zeros(T * n), torch.zeros(T * n), act.controlled)
    log = _cpu_state((T + 1) * n)
    ws = torch.zeros(64, dtype=torch.uint8)
    with pytest.raises(ValueError, match="traj.y"):
        tr = _cpu_state(T * n)
        tr.y = tr.y[:-1]
        wm.rollout(b, good, seq_act, log, None, T, 0.1, ws, traj=tr)
    with pytest.raises(ValueError, match="log_seq"):
        wm.rollout(b, good, seq_act, _cpu_state(T * n), None, T, 0.1, ws)
    with pytest.raises(ValueError, match="loss"):
        wm.rollout(b, good, seq_act, log, None, T, 0.1, ws, loss=torch.zeros(1))
    with pytest.raises(ValueError, match="grad_curvature"):
        wm.rollout_backward(b, good, seq_act, log, T, 0.1, 2, _cpu_state(2 * n), torch.ones(2), torch.zeros(T * n),
                            torch.zeros(T * n - 1), ws)
    with pytest.raises(ValueError, match="batch.obj_off"):
        bad = wm.Batch(b.obj_off.to(torch.int64), b.rg_off, 2, n, P, 4, 12)
        wm.step(bad, good, act, good, None, 0.1, _cpu_state(n))


def test_scan_counts_validation():
    """wm_rollout_scan_counts rejects NULL pointers and a workspace that ends
    before its counters, before touching the device."""
    lib = wm.lib()
    b = _batch()
    out = (C.c_uint64 * 3)()
    assert lib.wm_rollout_scan_counts(C.byref(b), None, 1 << 20, out, None) == wm.WM_ERR_NULL
    assert lib.wm_rollout_scan_counts(C.byref(b), FAKE, 1 << 20, None, None) == wm.WM_ERR_NULL
    assert lib.wm_rollout_scan_counts(C.byref(b), FAKE, 16, out, None) == wm.WM_ERR_WORKSPACE
    assert lib.wm_rollout_scan_counts(None, FAKE, 1 << 20, out, None) == wm.WM_ERR_NULL
