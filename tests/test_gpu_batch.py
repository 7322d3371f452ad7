"""Batched form: many graphs of uneven size, group count and grid in one launch per stage;
hipGraph capture and replay; the autotuner's trial runs leave the polylines unchanged."""

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def small_batch(n=6, seed=200):
    return workloads.batched(n_graphs=n, first_seed=seed, e_min=300, e_max=6000, n_iters=4,
                             sides=(64, 128, 256), max_groups=5)


def snapshot(hb, b, w):
    off, xy = b.points()
    maps = [b.map(hb.HB_MAP_HIST, g) for g in range(w.n_groups)]
    maps += [b.map(hb.HB_MAP_BOX, g, 3) for g in range(w.n_groups)]
    return off, xy, maps


def assert_same(a, c):
    np.testing.assert_array_equal(a[0], c[0])
    np.testing.assert_array_equal(a[1], c[1])
    for x, y in zip(a[2], c[2]):
        np.testing.assert_array_equal(x, y)


def test_batch_equals_individual_runs(hb):
    ws = small_batch()
    assert len({w.grid_w for w in ws}) > 1 and len({w.n_groups for w in ws}) > 1
    alone = []
    for w in ws:
        with hb.Bundler(0) as b:
            b.set_workload(w)
            b.run(3)
            alone.append(snapshot(hb, b, w))
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for b, w in zip(bs, ws):
            b.set_workload(w)
        hb.batch_run(bs, 2)
        hb.batch_run(bs, 1)
        for b, w, ref in zip(bs, ws, alone):
            assert_same(snapshot(hb, b, w), ref)
            assert b.iteration == 3
    finally:
        for b in bs:
            b.close()


def test_batch_grows_point_buffers_per_graph(hb):
    ws = small_batch(4, seed=300)
    alone = []
    for w in ws:
        with hb.Bundler(0) as b:
            b.set_workload(w, capacity_factor=8.0)
            b.run(4)
            alone.append(snapshot(hb, b, w))
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for b, w in zip(bs, ws):
            b.set_workload(w, capacity_factor=1.1)
        hb.batch_run(bs, 4)
        for b, w, ref in zip(bs, ws, alone):
            assert_same(snapshot(hb, b, w), ref)
    finally:
        for b in bs:
            b.close()


def test_graph_replay_matches_eager(hb):
    w = workloads.scaled("zipf", n_edges=4000, grid=256, groups=3, n_iters=3, seed=21)
    with hb.Bundler(0) as b:
        b.set_workload(w)
        b.run(2)
        ref2 = snapshot(hb, b, w)
        b.run(1)
        ref3 = snapshot(hb, b, w)
    with hb.Bundler(0) as b, hb.Bundler(0) as other:
        other.set_workload(w)
        for rep in range(3):
            b.set_workload(w)
            b.run(2, hb.HB_RUN_GRAPH)           # captured on the first pass, replayed after
            assert_same(snapshot(hb, b, w), ref2)
            other.run(1)                        # eager work between the replays
            b.run(1)
            assert_same(snapshot(hb, b, w), ref3)


def test_batch_graph_replay_matches_eager(hb):
    ws = small_batch(3, seed=400)
    refs = []
    for w in ws:
        with hb.Bundler(0) as b:
            b.set_workload(w)
            b.run(2)
            refs.append(snapshot(hb, b, w))
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for rep in range(3):
            for b, w in zip(bs, ws):
                b.set_workload(w)
            hb.batch_run(bs, 2, hb.HB_RUN_GRAPH)
            for b, w, ref in zip(bs, ws, refs):
                assert_same(snapshot(hb, b, w), ref)
    finally:
        for b in bs:
            b.close()


def test_autotune_restores_polylines_and_tuning_is_bit_identical(hb):
    ws = small_batch(3, seed=500)
    bs = [hb.Bundler(0) for _ in ws]
    try:
        for b, w in zip(bs, ws):
            b.set_workload(w)
        hb.batch_run(bs, 1)
        before = [b.points() for b in bs]
        choice = hb.autotune(bs, 1)
        assert choice[0] in (1, 2, 4) and choice[1] in (1, 2, 4)
        assert choice[2] in (64, 128, 256) and choice[3] in (4, 16, 64) and 14 <= choice[4] <= 17
        for b, ref in zip(bs, before):
            off, xy = b.points()
            np.testing.assert_array_equal(off, ref[0])
            np.testing.assert_array_equal(xy, ref[1])
            assert b.iteration == 1 and b.tuning() == choice[:2]
            assert hb.hb_get_tiling(b.ctx) == choice[2:]
        hb.batch_run(bs, 2)
        tuned = [b.points() for b in bs]
    finally:
        for b in bs:
            b.close()
    # every kernel variant and launch shape computes the same bits
    for (ru, au), tiling in [((1, 1), (16, 1, 12)), ((4, 4), (1024, 64, 20)), ((2, 2), (64, 4, 14))]:
        for w, ref in zip(ws, tuned):
            with hb.Bundler(0) as b:
                b.set_workload(w)
                b.tuning(ru, au)
                hb.hb_set_tiling(b.ctx, *tiling)
                assert hb.hb_get_tiling(b.ctx) == tiling
                b.run(3)
                off, xy = b.points()
                np.testing.assert_array_equal(off, ref[0])
                np.testing.assert_array_equal(xy, ref[1])
    with hb.Bundler(0) as b:
        for bad in [(100, 4, 16), (128, 128, 16), (128, 4, 11), (2048, 4, 16)]:
            with pytest.raises(hb.HBError) as ei:
                hb.hb_set_tiling(b.ctx, *bad)
            assert ei.value.status == hb.HB_EINVAL


def test_resample_chunk_counts_give_the_same_bits(hb):
    """The resampling sums its arclengths in blocks of 64 segments whatever its chunk count
    (64, 128 or 256 segments per trip), so its three kernels give the same polylines bit for
    bit; a 0.25 px spacing makes polylines of many chunks."""
    w = workloads.scaled("clustered", n_edges=2000, grid=512, groups=3, n_iters=3, seed=31,
                         delta=0.25)
    ref = None
    for ru in (2, 1, 4):
        with hb.Bundler(0) as b:
            b.set_workload(w)
            b.tuning(ru, 2)
            b.run(3)
            off, xy = b.points()
        if ref is None:
            ref = (off, xy)
            assert np.diff(off).max() > 1000
        else:
            np.testing.assert_array_equal(off, ref[0])
            np.testing.assert_array_equal(xy, ref[1])


def test_batch_argument_errors(hb):
    w = small_batch(1, seed=600)[0]
    with hb.Bundler(0) as a, hb.Bundler(0) as c:
        a.set_workload(w)
        with pytest.raises(hb.HBError) as ei:
            hb.batch_run([a, c], 1)                 # c has no graph
        assert ei.value.status == hb.HB_ESTATE
        with pytest.raises(hb.HBError) as ei:
            hb.batch_run([a, a], 1)
        assert ei.value.status == hb.HB_EINVAL
        with pytest.raises(hb.HBError):
            hb.batch_run([a], 1, hb.HB_RUN_SAMPLES_GIVEN)


@pytest.mark.parametrize("mode", ["strip", "insdel", "sigma"])
def test_graph_replay_matches_eager_in_variant_modes(hb, mode):
    """The captured iteration holds the kernels of the chosen modes (line strips, insert/delete
    resampling, per-pass radii) and replays them like eager runs, with eager work between."""
    w = workloads.scaled("clustered", n_edges=3000, grid=256, groups=2, n_iters=3, seed=22)
    kw = {"strip": dict(splat_mode=hb.HB_SPLAT_STRIP),
          "insdel": dict(resample_mode=hb.HB_RESAMPLE_INSERT_DELETE),
          "sigma": dict(sigmas=[3.7, 2.9])}[mode]
    with hb.Bundler(0) as b:
        b.set_workload(w, **kw)
        b.run(2)
        ref = snapshot(hb, b, w)
    with hb.Bundler(0) as b, hb.Bundler(0) as other:
        other.set_workload(w)
        for rep in range(3):
            b.set_workload(w, **kw)
            b.run(2, hb.HB_RUN_GRAPH)
            assert_same(snapshot(hb, b, w), ref)
            other.run(1)
