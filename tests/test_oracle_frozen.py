"""Pins of the oracle's frozen-decision surrogate (the function the adjoint differentiates).

* Replaying the recorded choices at the recorded parameters reproduces the base run.
* The loss does not change when a row of M, or the pass weights, are scaled by a positive
  factor (the advection direction is a normalised gradient), so by Euler's theorem
  sum_b M[l][b] dL/dM[l][b] = 0 for every l and sum_k a_k dL/da_k = 0.
* Central differences converge: steps 1e-5 and 1e-6 agree.
"""

import numpy as np

import oracle as O
import workloads


def _case():
    w = workloads.scaled("clustered", n_edges=60, grid=64, groups=3, n_iters=3, seed=5)
    p = O.params_for(w)
    off, xy = O.initial_state(w.node_xy, w.src, w.dst, p)
    rec, offT, xyT = O.record_run(off, xy, w.group, w.M, p, 3)
    return w, p, xy, rec, offT, xyT


def test_frozen_replay_reproduces_base_run():
    w, p, xy, rec, offT, xyT = _case()
    L = O.frozen_loss(xy, w.M, p.a(), rec, w.group, p)
    assert abs(L - O.ink(offT, xyT)) <= 1e-9 * L


def test_scaling_invariance_and_euler_identities():
    w, p, xy, rec, _, _ = _case()
    M = w.M.astype(np.float64)
    L = O.frozen_loss(xy, M, p.a(), rec, w.group, p)
    M2 = M.copy()
    M2[1] *= 3.0
    assert abs(O.frozen_loss(xy, M2, p.a(), rec, w.group, p) - L) <= 1e-9 * L
    assert abs(O.frozen_loss(xy, M, 2.5 * p.a(), rec, w.group, p) - L) <= 1e-9 * L
    B = M.shape[0]
    G = np.array([[O.frozen_fd(xy, M, p.a(), rec, w.group, p, "M", (l, b), 1e-6)
                   for b in range(B)] for l in range(B)])
    rows = (G * M).sum(1)
    scale = np.abs(G * M).sum(1)
    assert (np.abs(rows) <= 1e-5 * scale + 1e-8).all(), (rows, scale)


def test_central_differences_converge():
    w, p, xy, rec, _, _ = _case()
    for which, idx in [("M", (0, 1)), ("a", 0), ("x", (5, 1))]:
        g5 = O.frozen_fd(xy, w.M, p.a(), rec, w.group, p, which, idx, 1e-5)
        g6 = O.frozen_fd(xy, w.M, p.a(), rec, w.group, p, which, idx, 1e-6)
        assert abs(g5 - g6) <= 1e-4 * max(abs(g6), 1e-3), (which, g5, g6)


def test_frozen_state_replays_base_run_and_linear_loss():
    w, p, xy, rec, offT, xyT = _case()
    xs = O.frozen_state(xy, w.M, p.a(), rec, w.group, p)
    np.testing.assert_array_equal(offT, rec[-1]["s_off"])
    assert np.abs(xs - xyT).max() <= 1e-9
    # the linear loss of weights cT is the weighted sum of the final coordinates
    c = np.zeros_like(xs)
    c[7, 0], c[11, 1] = 2.0, -0.5
    L = O.frozen_loss(xy, w.M, p.a(), rec, w.group, p, c)
    assert abs(L - (2.0 * xyT[7, 0] - 0.5 * xyT[11, 1])) <= 1e-9 * (1 + abs(L))
    # end points never move, so the gradient of an end point's final coordinate with
    # respect to the same end point is 1 beside what it does through the interior
    end = int(offT[1]) - 1                     # last point of edge 0 in the final layout
    c = np.zeros_like(xs)
    c[end, 0] = 1.0
    start_end = 1                              # edge 0's last point in the two-point start
    g = O.frozen_fd(xy, w.M, p.a(), rec, w.group, p, "x", (start_end, 0), 1e-6, c)
    assert abs(g - 1.0) <= 1e-6
