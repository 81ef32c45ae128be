"""Pins of the oracle's off-road metric (Sec. 3.4, Off-Road: on the road when
left of the oriented road edge) against a straight-edge closed form, a
point-in-polygon brute force on a lane corridor, exact ties and
invariances."""
import math

import numpy as np

import oracle


def _rg(xy, dirs, types=None, valid=None):
    xy = np.asarray(xy, float)
    dirs = np.asarray(dirs, float)
    P = xy.shape[0]
    return {"x": xy[:, 0], "y": xy[:, 1], "dir_x": dirs[:, 0], "dir_y": dirs[:, 1],
            "type": np.ones(P, np.int8) if types is None else np.asarray(types, np.int8),
            "valid": np.ones(P, np.uint8) if valid is None else np.asarray(valid, np.uint8)}


def _objs(x, y, yaw, length, width, valid=None):
    n = len(x)
    return {"x": np.asarray(x, float), "y": np.asarray(y, float), "yaw": np.asarray(yaw, float),
            "vx": np.zeros(n), "vy": np.zeros(n), "length": np.asarray(length, float),
            "width": np.asarray(width, float),
            "valid": np.ones(n, np.uint8) if valid is None else np.asarray(valid, np.uint8)}


def test_straight_edge_closed_form():
    # Edge along +x through y = 0, road on the left (y > 0).  Away from the
    # ends, the nearest point is straight below/above the corner, so the corner
    # margin is -y_corner and the object margin is -(lowest corner y) =
    # -y + (l/2)|sin yaw| + (w/2)|cos yaw|.
    xs = np.arange(-400, 401) * 0.5
    rg = _rg(np.stack([xs, np.zeros_like(xs)], 1), np.tile([1.0, 0.0], (xs.size, 1)))
    rng = np.random.default_rng(20)
    n = 300
    x, y = rng.uniform(-150, 150, n), rng.uniform(-20, 20, n)
    yaw, L, W = rng.uniform(-math.pi, math.pi, n), rng.uniform(3, 6, n), rng.uniform(1.5, 2.5, n)
    off = np.array([0, n], np.int32)
    r = oracle.offroad(off, np.array([0, xs.size], np.int32), _objs(x, y, yaw, L, W), rg)
    expect = -y + 0.5 * L * np.abs(np.sin(yaw)) + 0.5 * W * np.abs(np.cos(yaw))
    # corners whose foot point lies between two samples are still exact: the
    # side value does not depend on which sample of a straight edge is nearest
    np.testing.assert_allclose(r["margin"], expect, atol=1e-9)
    np.testing.assert_array_equal(r["offroad"], (expect > 0).astype(np.uint8))


def _corridor(rng):
    """One lane: a gently curving center line with edges offset 1.8 m; right
    edge in the lane direction, left edge reversed.  Returns (roadgraph,
    polygon [right..., reversed left...])."""
    n = 400
    h = np.cumsum(np.r_[0.2, rng.uniform(-0.01, 0.01, n - 2)])
    pts = np.zeros((n, 2))
    pts[1:] = np.cumsum(0.5 * np.stack([np.cos(h), np.sin(h)], 1), 0)
    d = np.zeros_like(pts)
    d[:-1] = (pts[1:] - pts[:-1]) / np.linalg.norm(pts[1:] - pts[:-1], axis=1, keepdims=True)
    d[-1] = d[-2]
    nrm = np.stack([-d[:, 1], d[:, 0]], 1)
    right, left = pts - 1.8 * nrm, (pts + 1.8 * nrm)[::-1]

    def dirs(p):
        q = np.zeros_like(p)
        q[:-1] = (p[1:] - p[:-1]) / np.linalg.norm(p[1:] - p[:-1], axis=1, keepdims=True)
        q[-1] = q[-2]
        return q

    xy = np.concatenate([pts, right, left])
    dd = np.concatenate([d, dirs(right), dirs(left)])
    types = np.r_[np.zeros(n), np.ones(2 * n)]
    return _rg(xy, dd, types), np.concatenate([right, left]), pts


def _inside(poly, p):
    """Even-odd ray casting."""
    x, y = p
    inside = False
    for i in range(len(poly)):
        (x1, y1), (x2, y2) = poly[i], poly[(i + 1) % len(poly)]
        if (y1 > y) != (y2 > y):
            xc = x1 + (y - y1) * (x2 - x1) / (y2 - y1)
            if xc > x:
                inside = not inside
    return inside


def test_corridor_matches_point_in_polygon():
    rng = np.random.default_rng(21)
    rg, poly, center = _corridor(rng)
    P = rg["x"].size
    # tiny boxes so that each corner is (almost) a probe point
    m = 1500
    base = center[rng.integers(20, center.shape[0] - 20, m)]
    xy = base + rng.normal(0, 2.5, (m, 2))
    objs = _objs(xy[:, 0], xy[:, 1], rng.uniform(-3, 3, m), np.full(m, 0.02), np.full(m, 0.02))
    r = oracle.offroad(np.array([0, m], np.int32), np.array([0, P], np.int32), objs, rg)
    checked = 0
    for i in range(m):
        for k in range(4):
            s = r["corner_margin"][i, k]
            if abs(s) < 0.5:
                continue
            c, sn = math.cos(objs["yaw"][i]), math.sin(objs["yaw"][i])
            sl, sw = ((1, 1), (1, -1), (-1, -1), (-1, 1))[k]
            p = (xy[i, 0] + sl * 0.01 * c - sw * 0.01 * sn, xy[i, 1] + sl * 0.01 * sn + sw * 0.01 * c)
            assert (s > 0) == (not _inside(poly, p)), (i, k, s)
            checked += 1
    assert checked > 3000
    assert 0 < r["offroad"].mean() < 1


def test_exact_tie_goes_to_lowest_index():
    # Box yaw 0 centred at the origin, 4 x 2: corner FL = (2, 1) exactly.  Two
    # edge points at distance 5 (3-4-5 triangle) lie on opposite sides.
    fl = (2.0, 1.0)
    pts = [(fl[0] + 3, fl[1] + 4), (fl[0] - 3, fl[1] - 4), (50.0, 50.0)]
    dirs = [(1.0, 0.0), (1.0, 0.0), (1.0, 0.0)]
    objs = _objs([0.0], [0.0], [0.0], [4.0], [2.0])
    off, roff = np.array([0, 1], np.int32), np.array([0, 3], np.int32)
    r = oracle.offroad(off, roff, objs, _rg(pts, dirs))
    assert r["nearest"][0, 0] == 0
    assert r["corner_margin"][0, 0] == 4.0          # corner below the point at y+4
    r2 = oracle.offroad(off, roff, objs, _rg([pts[1], pts[0], pts[2]], dirs))
    assert r2["nearest"][0, 0] == 0 and r2["corner_margin"][0, 0] == -4.0
    assert r["ambiguous"][0, 0] == 1 and r2["ambiguous"][0, 0] == 1
    assert r["tied"][0, 0] == 1 and r2["tied"][0, 0] == 1


def test_same_side_tie_is_tied_not_ambiguous():
    # two points at distance 5 from the front-left corner (2, 1), both above
    # it with direction +x: same side, so the mask is decided (s = 4 for
    # either) but the nearest index (lowest wins) is a tie
    fl = (2.0, 1.0)
    pts = [(fl[0] + 3, fl[1] + 4), (fl[0] - 3, fl[1] + 4), (50.0, 50.0)]
    dirs = [(1.0, 0.0)] * 3
    objs = _objs([0.0], [0.0], [0.0], [4.0], [2.0])
    off, roff = np.array([0, 1], np.int32), np.array([0, 3], np.int32)
    r = oracle.offroad(off, roff, objs, _rg(pts, dirs))
    assert r["nearest"][0, 0] == 0 and r["corner_margin"][0, 0] == 4.0
    assert r["ambiguous"][0, 0] == 0 and r["tied"][0, 0] == 1
    # moved 1 cm closer to point 1: unique beyond a 1 mm band, tied within 5 cm
    objs2 = _objs([-0.006], [0.008], [0.0], [4.0], [2.0])
    r = oracle.offroad(off, roff, objs2, _rg(pts, dirs), band=1e-3)
    assert r["nearest"][0, 0] == 1 and r["tied"][0, 0] == 0
    r = oracle.offroad(off, roff, objs2, _rg(pts, dirs), band=5e-2)
    assert r["tied"][0, 0] == 1


def test_filters_type_validity_and_empty():
    pts = [(0.0, -1.0), (0.0, 10.0), (0.0, -0.5)]
    dirs = [(1.0, 0.0)] * 3
    objs = _objs([0.0, 5.0], [2.0, 5.0], [0.0, 0.0], [0.2, 0.2], [0.2, 0.2], valid=[1, 0])
    off, roff = np.array([0, 2], np.int32), np.array([0, 3], np.int32)
    # point 2 is the nearest but is a lane center, point 0 is invalid
    r = oracle.offroad(off, roff, objs, _rg(pts, dirs, types=[1, 1, 0], valid=[0, 1, 1]))
    assert (r["nearest"][0] == 1).all() and r["offroad"][0] == 1
    assert r["margin"][1] == oracle.NO_VALUE and (r["nearest"][1] == -1).all() and r["offroad"][1] == 0
    r = oracle.offroad(off, roff, objs, _rg(pts, dirs, types=[0, 0, 0]))
    assert r["margin"][0] == oracle.NO_VALUE and r["offroad"][0] == 0


def test_rigid_motion_and_point_order_invariance():
    from paper_2310_08710_amd import synth
    sc = synth.make_scene(0, on_road_frac=0.6, object_box=20)
    st = sc.state_at(synth.T0)
    st64 = {k: v.astype(np.float64) if v.dtype != np.uint8 else v for k, v in st.items()}
    rg = {k: v.astype(np.float64) if v.dtype == np.float32 else v for k, v in sc.rg.items()}
    r = oracle.offroad(sc.obj_off, sc.rg_off, st64, rg)
    phi, tx, ty = 2.3, -40.0, 15.0
    c, s = math.cos(phi), math.sin(phi)
    rot = lambda x, y: (c * x - s * y, s * x + c * y)  # noqa: E731
    st2 = dict(st64)
    st2["x"], st2["y"] = [u + t for u, t in zip(rot(st64["x"], st64["y"]), (tx, ty))]
    st2["yaw"] = st64["yaw"] + phi
    rg2 = dict(rg)
    rg2["x"], rg2["y"] = [u + t for u, t in zip(rot(rg["x"], rg["y"]), (tx, ty))]
    rg2["dir_x"], rg2["dir_y"] = rot(rg["dir_x"], rg["dir_y"])
    r2 = oracle.offroad(sc.obj_off, sc.rg_off, st2, rg2)
    np.testing.assert_allclose(r2["margin"], r["margin"], atol=1e-9)
    perm = np.random.default_rng(22).permutation(rg["x"].size)
    rg3 = {k: v[perm] for k, v in rg.items()}
    r3 = oracle.offroad(sc.obj_off, sc.rg_off, st64, rg3)
    np.testing.assert_allclose(r3["margin"], r["margin"], atol=1e-12)
    np.testing.assert_array_equal(perm[r3["nearest"]], r["nearest"])
