"""GPU-vs-oracle parity of the directed-graph steps (Section 3, the pipeline; Section 5):
the normal push of interior samples after resampling and the orientation slices of the
edges. Orientation slices are integers: bit-exact. Pushed samples: within 1e-4 px (FP32
storage of an FP64 position). Multi-iteration runs: point counts, ink and drift statistics
within 1 %.
"""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _f32_pixels(node_xy, src, dst, W, H, bbox=(0.0, 0.0, 1.0, 1.0)):
    """End points in pixel units, rounded to FP32 the way positions are stored."""
    p = O.Params(grid_w=W, grid_h=H, radii=[1], bbox=bbox)
    _, xy = O.initial_state(node_xy, src, dst, p)
    return xy.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("W,H,seed", [(300, 200, 31), (256, 256, 32), (1024, 96, 33)])
def test_orientation_groups_parity(hb, W, H, seed):
    rng = np.random.default_rng(seed)
    # random nodes plus nodes on a 1/8 lattice, so that axis-parallel and diagonal edges
    # (the slice borders) occur many times
    lattice = (rng.integers(0, 9, (400, 2)) / 8.0).astype(np.float32)
    nodes = np.concatenate([rng.random((600, 2)).astype(np.float32), lattice])
    E = 5000
    src = rng.integers(0, len(nodes), E).astype(np.int32)
    dst = rng.integers(0, len(nodes), E).astype(np.int32)
    dst[:200] = src[:200]                      # coincident end points: slice 0
    with hb.Bundler(0) as b:
        b.set_params(W, H, [1])
        b.set_graph(nodes, src, dst)
        got = b.orientation_groups()
        got_dev = b.orientation_groups(device="cuda:0").cpu().numpy()
    xy = _f32_pixels(nodes, src, dst, W, H)
    ref = O.orientation(xy[1::2] - xy[0::2])
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got_dev, ref)
    assert set(np.unique(ref)) == {0, 1, 2, 3}
    d = xy[1::2] - xy[0::2]
    ties = (np.abs(d[:, 0]) == np.abs(d[:, 1])) & (d[:, 0] != 0)
    if W == H:
        assert ties.sum() > 20                 # the slice borders were exercised


def test_orientation_groups_errors_and_empty(hb):
    with hb.Bundler(0) as b:
        b.set_params(32, 32, [2])
        with pytest.raises(hb.HBError) as ei:
            b.orientation_groups()
        assert ei.value.status == hb.HB_ESTATE
        b.set_graph(np.zeros((1, 2), np.float32), np.zeros(0, np.int32), np.zeros(0, np.int32))
        assert b.orientation_groups().shape == (0,)


@pytest.mark.parametrize("E,W,H,delta,doff,seed", [(800, 128, 96, 1.0, 0.75, 41),
                                                    (300, 512, 512, 4.0, -2.0, 42)])
def test_directed_offset_resample_parity(hb, E, W, H, delta, doff, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=90, step=4.0)
    group = np.zeros(E, np.int32)
    nodes = rng.random((16, 2)).astype(np.float32)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2], delta=delta, directed_offset=doff)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32),
                    rng.integers(0, 16, E).astype(np.int32))
        b.set_groups(group, np.ones((1, 1), np.float32))
        b.set_points(off, xy)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = b.map(hb.HB_MAP_HIST, 0).astype(np.int64)
    x64 = xy.astype(np.float64)
    ro, rs, _, seg = O.resample(off, x64, delta, want_seg=True)
    rp = O.directed_offset(off, x64, ro, seg, rs, doff)
    np.testing.assert_array_equal(off_s, ro)
    err = np.abs(xy_s.astype(np.float64) - rp).max(1)
    assert (err <= 1e-4 + PT.F32_ULP_AT(xy_s).max(1)).all(), err.max()
    # the push happened: interior samples are |doff| away from the unpushed ones
    interior = np.ones(len(rs), bool)
    interior[ro[:-1]] = False
    interior[ro[1:] - 1] = False
    mv = np.hypot(*(xy_s.astype(np.float64) - rs)[interior].T)
    assert np.abs(mv - abs(doff)).max() <= 2e-4
    ends = np.concatenate([ro[:-1], ro[1:] - 1])
    np.testing.assert_array_equal(xy_s[ends], xy[np.concatenate([off[:-1], off[1:] - 1])])
    href = O.splat(ro, rp, group, 1, W, H)[0]
    assert hist.sum() == href.sum() == len(rp)
    assert np.abs(hist - href).sum() <= 2 * PT.near_pixel_edge(rp).sum()


@pytest.mark.parametrize("every", [False, True])
def test_directed_push_once_or_every_iteration_closed_form(hb, every):
    """A straight horizontal edge and its reversed copy with the advection made negligible
    (h = 1e-12 px) and no Laplacian smoothing: after T iterations their middles sit at
    +-|d| from the line when the push follows the first sampling only, and at +-T|d| when
    it follows every resampling (the oracle's closed form, here through the library)."""
    W, T, d = 128, 4, 0.75
    node = np.array([[8.25 / W, 60.5 / W], [120.25 / W, 60.5 / W]], np.float32)
    with hb.Bundler(0) as b:
        b.set_params(W, W, [4], h_max=1e-12, smooth_weight=0.0, directed_offset=d,
                     directed_mode=hb.HB_DIRECTED_EVERY_ITER if every else hb.HB_DIRECTED_ONCE)
        b.set_graph(node, np.array([0, 1], np.int32), np.array([1, 0], np.int32))
        b.set_groups(np.zeros(2, np.int32), np.ones((1, 1), np.float32))
        b.run(T)
        off, xy = b.points(hb.HB_POINTS_STATE)
    p = O.Params(grid_w=W, grid_h=W, radii=[4], directed_offset=d, h_max=1e-12,
                 smooth_weight=0.0, directed_every=every)
    roff, rxy, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                         np.ones((1, 1)), p, T)
    np.testing.assert_array_equal(off, roff)
    assert np.abs(xy.astype(np.float64) - rxy).max() <= 1e-4
    k = T if every else 1
    a, bb = xy[off[0]:off[1]].astype(np.float64), xy[off[1]:off[2]].astype(np.float64)
    mid = np.abs(a[:, 0] - 64.0) < 30.0
    np.testing.assert_allclose(a[mid, 1] - 60.5, k * d, atol=1e-4)
    mid = np.abs(bb[:, 0] - 64.0) < 30.0
    np.testing.assert_allclose(bb[mid, 1] - 60.5, -k * d, atol=1e-4)


@pytest.mark.parametrize("every", [False, True])
def test_directed_offset_end_to_end_tiny(hb, every):
    """The tiny workload with a 1 px push (0.4 % of the 256 px drawing), orientation slices
    as groups and the Eq. 4 interaction, against the oracle over 7 iterations, with the push
    after the first sampling only and after every resampling. (Later iterations of this run
    are chaotic: rounding the oracle's own polylines to FP32 after every iteration moves its
    ink by 0.14 % at the 9th and 0.5 % at the 10th, against <= 0.02 % up to the 7th.)"""
    w = workloads.tiny()
    n_iters = 7
    doff = 1.0
    xy0 = _f32_pixels(w.node_xy, w.src, w.dst, w.grid_w, w.grid_h, w.bbox)
    group = O.orientation(xy0[1::2] - xy0[0::2])
    M = workloads.interaction_eq4(4, 0.25)
    with hb.Bundler(0) as b:
        b.set_params(w.grid_w, w.grid_h, w.radii, delta=w.delta, passes=w.passes, lam=w.lam,
                     bbox=w.bbox, directed_offset=doff,
                     directed_mode=hb.HB_DIRECTED_EVERY_ITER if every else hb.HB_DIRECTED_ONCE)
        b.set_graph(w.node_xy, w.src, w.dst, w.weight)
        np.testing.assert_array_equal(b.orientation_groups(), group)
        b.set_groups(group, M)
        b.run(1)
        off1, xy1 = b.points(hb.HB_POINTS_SAMPLES)
        b.run(n_iters - 1)
        counts = b.iter_counts(n_iters - 1)
        off, xy = b.points(hb.HB_POINTS_STATE)
        ink = b.ink()
    p = O.params_for(w)
    p.directed_offset = doff
    p.directed_every = every
    o0, x0 = O.initial_state(w.node_xy, w.src, w.dst, p)
    r0 = O.iterate(o0, x0, group, M.astype(np.float64), p, 0, keep_maps=False)
    np.testing.assert_array_equal(off1, r0["off"])
    assert np.abs(xy1 - r0["samples"]).max() <= 1e-4
    roff, rxy, rcounts = O.run(w.node_xy, w.src, w.dst, group, M.astype(np.float64), p,
                               n_iters)
    assert PT.relclose(ink, O.ink(roff, rxy), 0.01)
    for a, b_ in zip(counts, rcounts[1:]):
        assert PT.relclose(a, b_, 0.01)
    ds, dr = PT.drift_stats(off, xy), PT.drift_stats(roff, rxy)
    for k in ("mean", "p50", "p90", "p99"):
        assert abs(ds[k] - dr[k]) <= 0.01 * dr[k], (k, ds[k], dr[k])


def test_directed_offset_rejected_by_checkpointed_forward(hb):
    w = workloads.scaled("uniform", n_edges=200, grid=64, groups=1, n_iters=2, seed=5)
    with hb.Bundler(0) as b:
        b.set_workload(w, directed_offset=0.5)
        with pytest.raises(hb.HBError) as ei:
            hb.hb_forward_ckpt(b.ctx, 1)
        assert ei.value.status == hb.HB_EINVAL
        b.run(1)                               # the plain iteration takes it
