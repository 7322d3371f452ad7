"""GPU-vs-oracle parity of the line-strip splat (the rasterised drawing of Eq. 1 that the
paper's implementation uses, Section 4): histograms of the drawn strips are integers and
must match bit for bit for identical samples; the box passes on them too. Resampled runs
and multi-iteration runs follow the usual tolerances (1e-4 px samples, 1 % statistics)."""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("E,W,H,B,weighted,seed", [(1500, 100, 72, 3, False, 51),
                                                    (600, 257, 130, 1, True, 52),
                                                    (2000, 320, 200, 5, True, 53),
                                                    (400, 64, 64, 8, False, 54)])
def test_strip_histogram_parity_given_samples(hb, E, W, H, B, weighted, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    weight = rng.integers(1, 7, E).astype(np.int32) if weighted else None
    M = workloads.interaction_eq4(B, 0.25) if B > 1 else np.ones((1, 1), np.float32)
    r = 3
    with hb.Bundler(0) as b:
        b.set_params(W, H, [r], splat_mode=hb.HB_SPLAT_STRIP)
        nodes = rng.random((16, 2)).astype(np.float32)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32),
                    rng.integers(0, 16, E).astype(np.int32), weight)
        b.set_groups(group, M)
        b.set_points(off, xy)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN)
        hist = np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)
        S3 = np.stack([b.map(hb.HB_MAP_BOX, g, 3) for g in range(B)])
    ref = O.splat_strip(off, xy.astype(np.float64), group, B, W, H, weight)
    np.testing.assert_array_equal(hist, ref)
    np.testing.assert_array_equal(S3, O.box_chain(ref, 3, r)[2])
    # the strip draws more than the points (every point's pixel at least once)
    assert hist.sum() > (len(xy) if weight is None else 0)


@pytest.mark.parametrize("E,W,H,delta,seed", [(800, 128, 96, 1.0, 55), (300, 512, 512, 4.0, 56)])
def test_strip_resampled_parity(hb, E, W, H, delta, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=90, step=4.0)
    group = np.zeros(E, np.int32)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2], delta=delta, splat_mode=hb.HB_SPLAT_STRIP)
        nodes = rng.random((16, 2)).astype(np.float32)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32),
                    rng.integers(0, 16, E).astype(np.int32))
        b.set_groups(group, np.ones((1, 1), np.float32))
        b.set_points(off, xy)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = b.map(hb.HB_MAP_HIST, 0).astype(np.int64)
    ro, rs, _ = O.resample(off, xy.astype(np.float64), delta)
    np.testing.assert_array_equal(off_s, ro)
    assert np.abs(xy_s.astype(np.float64) - rs).max() <= 1e-4 + 2e-4
    href = O.splat_strip(ro, rs, group, 1, W, H)[0]
    # identical except around samples within 1e-4 px of a pixel edge: each of those moves
    # the pixels of its two segments (at most ceil(delta) + 2 each)
    near = PT.near_pixel_edge(rs).sum()
    assert np.abs(hist - href).sum() <= 2 * 2 * (int(np.ceil(delta)) + 2) * near


def test_strip_end_to_end_tiny(hb):
    """The tiny workload with the line-strip splat, 6 iterations, against the oracle."""
    w = workloads.tiny()
    n_iters = 6
    with hb.Bundler(0) as b:
        b.set_workload(w, splat_mode=hb.HB_SPLAT_STRIP)
        b.run(1)
        off1, xy1 = b.points(hb.HB_POINTS_SAMPLES)
        b.run(n_iters - 1)
        counts = b.iter_counts(n_iters - 1)
        off, xy = b.points(hb.HB_POINTS_STATE)
        ink = b.ink()
    p = O.params_for(w)
    p.strip_splat = True
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


def test_strip_and_point_graphs_batched_equal_alone(hb):
    ws = workloads.batched(n_graphs=4, first_seed=400, e_min=300, e_max=4000, n_iters=3,
                           sides=(64, 128, 256), max_groups=4)
    modes = [hb.HB_SPLAT_STRIP, hb.HB_SPLAT_POINTS, hb.HB_SPLAT_STRIP, hb.HB_SPLAT_POINTS]
    alone = []
    for w, m in zip(ws, modes):
        with hb.Bundler(0) as b:
            b.set_workload(w, splat_mode=m)
            b.run(3)
            alone.append((b.points(), [b.map(hb.HB_MAP_HIST, g) for g in range(w.n_groups)]))
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for b, w, m in zip(bs, ws, modes):
            b.set_workload(w, splat_mode=m)
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


def test_strip_errors(hb):
    # long given segments: more drawn pixels than the entry buffer holds -> HB_EOVERFLOW
    rng = np.random.default_rng(57)
    E = 40
    with hb.Bundler(0) as b:
        b.set_params(1024, 1024, [2], splat_mode=hb.HB_SPLAT_STRIP)
        # coincident nodes: the first sample count, hence the buffer capacity, stays small
        nodes = np.full((16, 2), 0.5, np.float32)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32), rng.integers(0, 16, E).astype(np.int32))
        b.set_groups(np.zeros(E, np.int32), np.ones((1, 1), np.float32))
        off = np.arange(0, 2 * E + 1, 2).astype(np.int64)
        xy = np.tile(np.array([[3.5, 3.5], [1020.5, 1000.5]], np.float32), (E, 1))
        b.set_points(off, xy)
        with pytest.raises(hb.HBError) as ei:
            b.run(1, hb.HB_RUN_SAMPLES_GIVEN)
        assert ei.value.status == hb.HB_EOVERFLOW
    w = workloads.scaled("uniform", n_edges=200, grid=64, groups=1, n_iters=2, seed=5)
    with hb.Bundler(0) as b:
        b.set_workload(w, splat_mode=hb.HB_SPLAT_STRIP)
        with pytest.raises(hb.HBError) as ei:
            hb.hb_forward_ckpt(b.ctx, 1)
        assert ei.value.status == hb.HB_EINVAL
        b.run(2)
        assert b.points()[0][-1] > 0
