"""Parity at the full size of the measured workload: 1 000 000 edges of the 3D-stack graph,
8 groups, 1024x1024x8 maps, first radius 32 px, the point buffers sized as the benchmark
sizes them (capacity factor 10) and the default kernel variants.

* From the straight edges (the benchmark's own first iteration): sample counts per edge
  bit-exact, sample positions within 1e-4 px on a seeded sample of 4 M points and at every
  end point (bit-exact there), the histogram stack equal to the oracle's splat of its FP64
  samples except for samples within 1e-4 px of a pixel edge (where FP32 rounding of the
  sample may cross it).
* From the oracle's samples rounded to FP32, given to both sides: histogram and all int64
  box sums bit-exact over the whole stack, the density within 1e-5 of the bilinear scale
  (as in the small stage tests), every halving decision one of the valid outcomes (> 99 %
  equal), and the new positions within 1e-4 px (plus the gradient-direction conditioning)
  on a seeded sample of 2 M points whose decisions and neighbours' decisions agree.
"""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_EDGES, GRID, GROUPS, CAPACITY = 1_000_000, 1024, 8, 10.0


@pytest.fixture(scope="module")
def full():
    w = workloads.stack3d(n_edges=N_EDGES, grid=GRID, groups=GROUPS)
    p = O.params_for(w)
    o0, x0 = O.initial_state(w.node_xy, w.src, w.dst, p)
    ro, rs, _ = O.resample(o0, x0, p.delta)
    return w, p, ro, rs


def _maps(hb, b, kind, B, pass_=0):
    return np.stack([b.map(kind, g, pass_) for g in range(B)])


def test_fullsize_first_iteration(hb, full):
    w, p, ro, rs = full
    B = w.n_groups
    with hb.Bundler(0) as b:
        b.set_workload(w, capacity_factor=CAPACITY)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = _maps(hb, b, hb.HB_MAP_HIST, B).astype(np.int64)
    np.testing.assert_array_equal(off_s, ro)
    N = len(rs)
    rng = np.random.default_rng(2024)
    idx = rng.integers(0, N, 4_000_000)
    err = np.abs(xy_s[idx].astype(np.float64) - rs[idx]).max(1)
    assert (err <= 1e-4 + PT.F32_ULP_AT(xy_s[idx]).max(1)).all(), err.max()
    ends = np.concatenate([ro[:-1], ro[1:] - 1])
    np.testing.assert_array_equal(xy_s[ends], rs[ends].astype(np.float32))
    href = O.splat(ro, rs, w.group, B, w.grid_w, w.grid_h)
    assert hist.sum() == href.sum() == N
    assert np.abs(hist - href).sum() <= 2 * PT.near_pixel_edge(rs).sum()


def test_fullsize_given_samples(hb, full):
    w, p, ro, rs = full
    B, W, H, P = w.n_groups, w.grid_w, w.grid_h, w.passes
    xs = rs.astype(np.float32)
    with hb.Bundler(0) as b:
        b.set_workload(w, capacity_factor=CAPACITY)
        b.set_points(ro, xs)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN | hb.HB_RUN_RECORD_DECISIONS)
        off_n, xy_n = b.points(hb.HB_POINTS_STATE)
        jacc = b.decisions().astype(np.int64)
        hist = _maps(hb, b, hb.HB_MAP_HIST, B).astype(np.int64)
        S = np.stack([_maps(hb, b, hb.HB_MAP_BOX, B, k + 1) for k in range(P)])
        rho = _maps(hb, b, hb.HB_MAP_DENSITY, B).astype(np.float64)
    np.testing.assert_array_equal(off_n, ro)
    x64 = xs.astype(np.float64)
    del rs
    ref = O.iterate(ro, x64, w.group, w.M.astype(np.float64), p, 0, skip_resample=True)

    np.testing.assert_array_equal(hist, ref["hist"])
    np.testing.assert_array_equal(S, ref["S"])
    r = ref["r"]
    aw = p.a()
    c = float((2 * r + 1) ** 2)
    Sbar = sum(aw[k] * ref["S"][k].astype(np.float64) / c ** (k + 1) for k in range(P))
    bound = 1e-5 * np.tensordot(np.abs(w.M.astype(np.float64)), Sbar, 1) + 1e-300
    assert (np.abs(rho - ref["rho"]) <= bound).all()
    del S, Sbar, bound

    adv = ref["adv"]
    ok = PT.acceptable(jacc, adv["jacc"], adv["jfirm"], adv["amb"])
    assert ok.all(), f"{(~ok).sum()} invalid decisions"
    agree = jacc == adv["jacc"]
    assert agree.mean() > 0.99
    nb = agree.copy()
    nb[1:] &= agree[:-1]
    nb[:-1] &= agree[1:]
    ends = np.concatenate([ro[:-1], ro[1:] - 1])
    np.testing.assert_array_equal(xy_n[ends], xs[ends])

    # positions on a sample of interior points whose own and neighbours' decisions agree
    interior = np.ones(len(xs), bool)
    interior[ends] = False
    cand = np.flatnonzero(nb & interior)
    rng = np.random.default_rng(2025)
    idx = np.sort(rng.choice(cand, size=min(2_000_000, len(cand)), replace=False))
    grad = ref["grad"]
    h = p.bandwidth(0)
    tpt = np.empty((3, len(idx)))
    for k, j in enumerate((idx - 1, idx, idx + 1)):
        cond = PT.direction_condition(grad, w.group[np.searchsorted(ro, j, side="right") - 1], x64[j])
        tpt[k] = 1e-4 + np.where(np.isfinite(cond), h * 1e-6 * cond, 0.0)
    ty = 0.5 * tpt[1] + 0.25 * (tpt[0] + tpt[2]) + 2 * PT.F32_ULP_AT(xy_n[idx]).max(1)
    err = np.abs(xy_n[idx].astype(np.float64) - ref["xy"][idx]).max(1)
    assert (err <= ty).all(), f"max err {err.max()} px"
    assert np.percentile(err, 99) <= 1e-4, np.percentile(err, 99)



def test_fullsize_widths(hb, full):
    """Width encoding of the polylines after 3 iterations at full size, by properties that
    hold at any size: densities non-negative, the largest one gets w_max, and on a seeded
    sample of 4 M points each width is the log-scale map of its own density (FP64 check of
    the FP32 result); the maps rebuilt from the polylines hold every point once."""
    w, p, ro, rs = full
    w_min, w_max = 0.5, 6.0
    with hb.Bundler(0) as b:
        b.set_workload(w, capacity_factor=CAPACITY)
        b.run(3)
        n = hb.hb_get_num_points(b.ctx)
        dens, widths = b.point_widths(3, w_min, w_max, True)
        hist = _maps(hb, b, hb.HB_MAP_HIST, w.n_groups).astype(np.int64)
    assert len(dens) == len(widths) == n
    assert hist.sum() == n
    assert (dens >= 0).all()
    dmax = float(dens.max())
    assert dmax > 0
    assert widths[int(np.argmax(dens))] == np.float32(w_max)
    rng = np.random.default_rng(2026)
    idx = rng.integers(0, n, 4_000_000)
    want = w_min + (w_max - w_min) * np.log1p(dens[idx].astype(np.float64)) / np.log1p(dmax)
    err = np.abs(widths[idx].astype(np.float64) - want)
    assert err.max() <= 1e-5 * (w_max - w_min), err.max()
