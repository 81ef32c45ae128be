"""wm_step_noalloc, the step whose workspace is the library's device-resident
array, against wm_step with a caller workspace (same kernels): identical
successor states and metrics on two calls in a row, the second on a smaller
batch than the first, so that it runs over what the first left in the
array."""
import numpy as np
import pytest

from helpers import device
from paper_2310_08710_amd import synth

pytestmark = pytest.mark.gpu

MET_FIELDS = ("collision", "offroad", "overlap_margin", "offroad_margin", "log_div", "infeasible", "reward")


def _step(sc, noalloc):
    import torch
    from paper_2310_08710_amd import wm
    dev = device()
    ds = wm.upload(sc, dev)
    n = sc.total_objects
    act = wm.Action(ds.act_seq.accel[0].contiguous(), ds.act_seq.curvature[0].contiguous(), ds.act_seq.controlled)
    nxt = wm.State.empty(n, dev)
    met = wm.Metrics.empty(n, dev)
    if noalloc:
        wm.step_noalloc(ds.batch, ds.init, act, ds.log_seq.row(1), ds.rg, sc.dt, nxt, met)
    else:
        ws = ds.batch.workspace()
        wm.step(ds.batch, ds.init, act, ds.log_seq.row(1), ds.rg, sc.dt, nxt, met, ws)
    torch.cuda.synchronize()
    return nxt.numpy(), {f: getattr(met, f).cpu().numpy() for f in MET_FIELDS}


def test_step_noalloc_equals_step_on_two_calls():
    from paper_2310_08710_amd import wm
    big = synth.make_scene(1, scenarios=24, objects=(100, 128), rg_points=(20000, 30000), steps=2, object_box=30,
                           on_road_frac=0.5, invalid_frac=0.05, rg_invalid_frac=0.02)
    small = synth.make_scene(2, scenarios=5, objects=(1, 40), rg_points=(24, 3000), steps=2, object_box=20,
                             on_road_frac=0.6, invalid_frac=0.1)
    for name, sc in (("24 scenarios", big), ("5 smaller scenarios", small)):
        print("wm_step_noalloc vs wm_step:", name, sc.total_objects, "objects", sc.total_rg_points, "road points",
              flush=True)
        assert wm.Batch.from_offsets(sc.obj_off, sc.rg_off, "cpu").workspace_bytes() <= 64 << 20
        g_st, g_met = _step(sc, True)
        r_st, r_met = _step(sc, False)
        for f, v in r_st.items():
            np.testing.assert_array_equal(g_st[f], v, err_msg="%s: state %s" % (name, f))
        for f, v in r_met.items():
            np.testing.assert_array_equal(g_met[f], v, err_msg="%s: metric %s" % (name, f))
        # the scenes exercise both values of the masks
        assert g_met["offroad"].any() and not g_met["offroad"].all(), name
        assert g_met["collision"].any() and not g_met["collision"].all(), name
