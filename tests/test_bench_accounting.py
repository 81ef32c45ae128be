"""The bench's count of the adjoint's evaluated pair terms (the work its
roofline figure is taken on), on small hand-placed scenes on the CPU: an
object is never its own partner, partners beyond the distance bound do not
count, partners within it do."""
import math
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_2310_08710_amd import wm  # noqa: E402


def _scene(xs, ys, T, length=4.0, width=2.0):
    """One scenario; the objects stand still at (xs, ys) for T + 1 rows."""
    n = len(xs)
    rows = T + 1
    x = torch.tensor(np.tile(np.asarray(xs, np.float32), (rows, 1)))
    y = torch.tensor(np.tile(np.asarray(ys, np.float32), (rows, 1)))
    z = torch.zeros((rows, n))
    ln = torch.full((rows, n), length)
    wd = torch.full((rows, n), width)
    log = wm.State(x, y, z.clone(), z.clone(), z.clone(), ln, wd, torch.ones((rows, n), dtype=torch.uint8))
    init = wm.State(*[getattr(log, f)[0].clone() for f in wm.STATE_FIELDS], log.valid[0].clone())
    traj = wm.State(*[getattr(log, f)[1:].clone() for f in wm.STATE_FIELDS], log.valid[1:].clone())
    off = torch.tensor([0, n], dtype=torch.int32)
    return off, init, log, traj


def test_far_apart_objects_count_nothing():
    T = 5
    off, init, log, traj = _scene([0.0, 100.0, 200.0], [0.0, 0.0, 0.0], T)
    ctrl = torch.tensor([1, 1, 0], dtype=torch.uint8)
    ops, near, tested = bench.adjoint_executed_ops(off, ctrl, init, log, traj, T)
    assert near == 0                      # no partner within the bound, never itself
    assert tested == T * 2 * 2            # partners other than itself
    assert ops == T * (bench.ADJ_OPS_PER_TEST * 2 * 3 + bench.ADJ_OPS_PER_OBJECT * 2) + bench.ADJ_OPS_PER_PAIR * near


def test_bound_edge():
    # reach r = half length + half width = 3 m each; the bound counts a pair
    # when d <= sqrt(2) (r_i + r_j + gap)
    T = 3
    edge = math.sqrt(2.0) * (3.0 + 3.0 + bench.ADJ_CULL_GAP)
    off, init, log, traj = _scene([0.0, edge - 0.05, -(edge + 0.05)], [0.0, 0.0, 0.0], T)
    ctrl = torch.tensor([1, 0, 0], dtype=torch.uint8)
    _, near, _ = bench.adjoint_executed_ops(off, ctrl, init, log, traj, T)
    assert near == T                      # only the object just inside


def test_uncontrolled_objects_come_from_the_log():
    # the controlled object's trajectory moves it next to object 1 after the
    # first step; the log keeps it far away
    T = 4
    off, init, log, traj = _scene([0.0, 500.0], [0.0, 0.0], T)
    traj.x[1:, 0] = 495.0
    ctrl = torch.tensor([1, 0], dtype=torch.uint8)
    _, near, _ = bench.adjoint_executed_ops(off, ctrl, init, log, traj, T)
    assert near == T - 1


def test_algorithmic_adjoint_pairs():
    """The method's count of the adjoint's pairs: unordered pairs of valid
    objects with a controlled member, 8 x 127 - 28 = 988 per step at 128
    objects with 8 controlled; invalid objects take part in none."""
    off = np.array([0, 128, 256], np.int32)
    ctrl = np.zeros(256, np.uint8)
    ctrl[0:8] = 1
    ctrl[128:136] = 1
    valid = np.ones(256, np.uint8)
    ops, pairs = bench.adjoint_algorithmic_ops(off, ctrl, valid, 80)
    assert pairs == 2 * 988 * 80
    assert ops == bench.ADJ_ALG_OPS_PER_PAIR * pairs
    # every object controlled: all N (N - 1) / 2 pairs
    _, pairs = bench.adjoint_algorithmic_ops(off[:2], np.ones(128, np.uint8), valid[:128], 1)
    assert pairs == 128 * 127 // 2
    # an invalid controlled object and an invalid partner drop out
    valid[0] = 0
    valid[100] = 0
    _, pairs = bench.adjoint_algorithmic_ops(off[:2], ctrl[:128], valid[:128], 1)
    assert pairs == 7 * 125 - 21          # 126 valid objects, 7 of them controlled


class _Scene:
    def __init__(self, counts):
        self.obj_off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)


def test_rollout_executed_ops():
    """The fused rollout's executed work from its counts: 512 corner-point
    pairs (32 points x 16 corners) at 6 ops per folded block, 10 ops per box
    test, and the same overlap, dynamics and displacement terms as the
    algorithmic count."""
    sc = _Scene([3, 5])
    ops, pairs = bench.rollout_executed_ops(sc, 2, (0, 0, 0))
    rest = 2 * (3 * (20 * 2 + 35) + 5 * (20 * 4 + 35))
    assert pairs == 0 and ops == rest
    ops, pairs = bench.rollout_executed_ops(sc, 2, (7, 11, 13))
    assert pairs == 7 * 512
    assert ops == 6 * 7 * 512 + 10 * (11 + 13) + rest
