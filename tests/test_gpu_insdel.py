"""GPU-vs-oracle parity of the insert/delete resampling (Section 3, the pipeline: points
created where consecutive points are too far apart, removed where too close). Both sides
compute in FP64 with the same order of operations from the same FP32 points, so point counts
are bit-exact and the points agree to the FP32 rounding; multi-iteration runs within 1 %."""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("E,W,H,delta,dmin,seed", [(800, 128, 96, 1.0, 0.0, 71),
                                                    (300, 512, 512, 4.0, 1.5, 72),
                                                    (1200, 200, 150, 2.0, 0.25, 73)])
def test_insdel_resample_parity(hb, E, W, H, delta, dmin, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=150, step=1.0)
    group = np.zeros(E, np.int32)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2], delta=delta, resample_mode=hb.HB_RESAMPLE_INSERT_DELETE,
                     delta_min=dmin)
        nodes = rng.random((16, 2)).astype(np.float32)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32),
                    rng.integers(0, 16, E).astype(np.int32))
        b.set_groups(group, np.ones((1, 1), np.float32))
        b.set_points(off, xy)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = b.map(hb.HB_MAP_HIST, 0).astype(np.int64)
    ro, rs = O.resample_insdel(off, xy.astype(np.float64), dmin if dmin > 0 else 0.5 * delta, delta)
    np.testing.assert_array_equal(off_s, ro)
    err = np.abs(xy_s.astype(np.float64) - rs).max(1)
    assert (err <= PT.F32_ULP_AT(xy_s).max(1)).all(), err.max()
    href = O.splat(ro, rs, group, 1, W, H)[0]
    assert hist.sum() == len(rs)
    assert np.abs(hist - href).sum() <= 2 * PT.near_pixel_edge(rs, 1e-5).sum()
    # the removal happened: fewer points than a uniform resampling at delta / 4 would make,
    # and no gap above delta
    gaps = np.hypot(*np.diff(xy_s.astype(np.float64), axis=0).T)
    inner = np.ones(len(gaps), bool)
    inner[off_s[1:-1] - 1] = False
    assert gaps[inner].max() <= delta * (1 + 1e-6)


def test_insdel_end_to_end_tiny(hb):
    """The tiny workload with the insert/delete resampling, 6 iterations, against the oracle."""
    w = workloads.tiny()
    n_iters = 6
    with hb.Bundler(0) as b:
        b.set_workload(w, resample_mode=hb.HB_RESAMPLE_INSERT_DELETE)
        b.run(1)
        off1, xy1 = b.points(hb.HB_POINTS_SAMPLES)
        b.run(n_iters - 1)
        counts = b.iter_counts(n_iters - 1)
        off, xy = b.points(hb.HB_POINTS_STATE)
        ink = b.ink()
    p = O.params_for(w)
    p.insert_delete = True
    o0, x0 = O.initial_state(w.node_xy, w.src, w.dst, p)
    r0 = O.iterate(o0, x0, w.group, w.M, p, 0, keep_maps=False)
    np.testing.assert_array_equal(off1, r0["off"])
    assert np.abs(xy1 - r0["samples"]).max() <= 1e-4
    roff, rxy, rcounts = O.run(w.node_xy, w.src, w.dst, w.group, w.M, p, n_iters)
    assert PT.relclose(ink, O.ink(roff, rxy), 0.01)
    for a, b_ in zip(counts, rcounts[1:]):
        assert PT.relclose(a, b_, 0.01)
    ds, dr = PT.drift_stats(off, xy), PT.drift_stats(roff, rxy)
    for k in ("mean", "p50", "p90", "p99"):
        assert abs(ds[k] - dr[k]) <= 0.01 * dr[k], (k, ds[k], dr[k])


def test_insdel_and_uniform_batched_equal_alone(hb):
    ws = workloads.batched(n_graphs=4, first_seed=500, e_min=300, e_max=4000, n_iters=3,
                           sides=(64, 128, 256), max_groups=4)
    modes = [(hb.HB_RESAMPLE_INSERT_DELETE, hb.HB_SPLAT_POINTS), (hb.HB_RESAMPLE_UNIFORM, hb.HB_SPLAT_POINTS),
             (hb.HB_RESAMPLE_INSERT_DELETE, hb.HB_SPLAT_STRIP), (hb.HB_RESAMPLE_UNIFORM, hb.HB_SPLAT_STRIP)]
    alone = []
    for w, (rm, sm) in zip(ws, modes):
        with hb.Bundler(0) as b:
            b.set_workload(w, resample_mode=rm, splat_mode=sm)
            b.run(3)
            alone.append((b.points(), [b.map(hb.HB_MAP_HIST, g) for g in range(w.n_groups)]))
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for b, w, (rm, sm) in zip(bs, ws, modes):
            b.set_workload(w, resample_mode=rm, splat_mode=sm)
        hb.batch_run(bs, 3)
        for b, w, ((o, x), hs) in zip(bs, ws, alone):
            o2, x2 = b.points()
            np.testing.assert_array_equal(o2, o)
            np.testing.assert_array_equal(x2, x)
            for g in range(w.n_groups):
                np.testing.assert_array_equal(b.map(hb.HB_MAP_HIST, g), hs[g])
    finally:
        for b in bs:
            b.close()


def test_insdel_errors(hb):
    w = workloads.scaled("uniform", n_edges=200, grid=64, groups=1, n_iters=2, seed=5)
    with hb.Bundler(0) as b:
        with pytest.raises(hb.HBError) as ei:
            b.set_workload(w, resample_mode=hb.HB_RESAMPLE_INSERT_DELETE, directed_offset=0.5)
        assert ei.value.status == hb.HB_EINVAL
        b.set_workload(w, resample_mode=hb.HB_RESAMPLE_INSERT_DELETE)
        with pytest.raises(hb.HBError) as ei:
            hb.hb_forward_ckpt(b.ctx, 1)
        assert ei.value.status == hb.HB_EINVAL
        b.run(2)
        assert b.points()[0][-1] > 0
