"""Synthetic scene generator: determinism, layout and road-edge orientation."""
import numpy as np

from paper_2310_08710_amd import synth


def test_deterministic_and_prefix_stable():
    a = synth.make_scene(2, scenarios=6, rg_points=(500, 3000))
    b = synth.make_scene(2, scenarios=6, rg_points=(500, 3000))
    c = synth.make_scene(2, scenarios=3, rg_points=(500, 3000))
    for k in a.log:
        assert a.log[k].tobytes() == b.log[k].tobytes()
    for k in a.rg:
        assert a.rg[k].tobytes() == b.rg[k].tobytes()
    n3 = c.total_objects
    np.testing.assert_array_equal(a.log["x"][:, :n3], c.log["x"])
    np.testing.assert_array_equal(a.rg["x"][:c.total_rg_points], c.rg["x"])


def test_layout_and_ranges():
    sc = synth.make_scene(2, scenarios=20, rg_points=(240, 5000))
    counts = np.diff(sc.obj_off)
    pcounts = np.diff(sc.rg_off)
    assert counts.min() >= 8 and counts.max() <= 128
    assert pcounts.min() >= 240 and pcounts.max() <= 5000
    assert sc.log["x"].shape == (synth.T0 + 80 + 1, sc.total_objects)
    assert sc.accel.shape == (80, sc.total_objects)
    for f in synth.STATE_FIELDS:
        assert sc.log[f].dtype == np.float32 and sc.log[f].flags.c_contiguous
    x0 = sc.log["x"][0]
    assert np.abs(x0).max() <= 100
    L = sc.log["length"][0]
    assert L.min() >= 4 and L.max() <= 5.5
    # logged speed never drops below 0.5 m/s after the first interval
    sp = np.hypot(sc.log["vx"], sc.log["vy"])
    assert sp[1:].min() >= 0.5 - 1e-4
    # padding: floor(P/24) points per polyline, the rest invalid
    for s in range(sc.num_scenarios):
        v = sc.rg["valid"][sc.rg_off[s]:sc.rg_off[s + 1]]
        assert v.sum() == (pcounts[s] // 24) * 24
    np.testing.assert_allclose(np.hypot(sc.rg["dir_x"], sc.rg["dir_y"])[sc.rg["valid"] == 1], 1.0, atol=1e-5)


def test_road_lies_left_of_every_edge():
    sc = synth.make_scene(1, scenarios=2, rg_points=(2400, 2400))
    for s in range(2):
        base = sc.rg_off[s]
        per = 2400 // 24
        for lane in range(8):
            c0 = base + lane * 3 * per
            center = np.stack([sc.rg["x"][c0:c0 + per], sc.rg["y"][c0:c0 + per]], 1).astype(float)
            for e, rev in ((1, False), (2, True)):
                e0 = c0 + e * per
                assert (sc.rg["type"][e0:e0 + per] == synth.TYPE_ROAD_EDGE).all()
                ex = np.stack([sc.rg["x"][e0:e0 + per], sc.rg["y"][e0:e0 + per]], 1).astype(float)
                d = np.stack([sc.rg["dir_x"][e0:e0 + per], sc.rg["dir_y"][e0:e0 + per]], 1).astype(float)
                cc = center[::-1] if rev else center
                side = d[:, 0] * (cc[:, 1] - ex[:, 1]) - d[:, 1] * (cc[:, 0] - ex[:, 0])
                assert (side[:-1] > 1.0).mean() > 0.95   # the lane center is on the left


def test_config_shapes():
    sc = synth.make_scene(0)
    assert sc.num_scenarios == 1 and sc.total_objects == 16 and sc.total_rg_points == 1000 and sc.steps == 10
    assert sc.controlled.all()
    sc3 = synth.make_scene(3, scenarios=2, rg_points=(240, 240), steps=3)
    assert sc3.controlled.reshape(2, 128)[:, :8].all() and not sc3.controlled.reshape(2, 128)[:, 8:].any()
    np.testing.assert_array_equal(sc3.ego, np.array([np.arange(8), 128 + np.arange(8)]))
