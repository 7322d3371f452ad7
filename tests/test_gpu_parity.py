"""GPU-vs-oracle parity of the bundling iteration, through the C ABI.

Stage parity feeds both sides the same seeded inputs: histograms and int64 box sums must
match bit for bit, the FP32 density stack within 1e-5 relative (of sum_b |M[l][b]| Sbar_b),
and one-iteration point positions within 1e-4 px. Halving decisions are compared where
they are unique; where the FP64 oracle's density margin is within the ambiguity band the
GPU's choice must be one of the valid outcomes, and the positions are checked for it.
"""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _bundler(hb, W, H, radii, E, group, M, seed=0, **kw):
    b = hb.Bundler(0)
    b.set_params(W, H, radii, **kw)
    rng = np.random.default_rng(seed)
    nodes = rng.random((16, 2)).astype(np.float32)
    src = rng.integers(0, 16, E).astype(np.int32)
    dst = ((src + 1) % 16).astype(np.int32)
    b.set_graph(nodes, src, dst)
    b.set_groups(group, M)
    return b


def _gpu_maps(hb, b, B, P):
    hist = np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)
    S = np.stack([np.stack([b.map(hb.HB_MAP_BOX, g, k + 1) for g in range(B)]) for k in range(P)])
    rho = np.stack([b.map(hb.HB_MAP_DENSITY, g) for g in range(B)]).astype(np.float64)
    grad = np.stack([b.map(hb.HB_MAP_GRAD, g) for g in range(B)]).astype(np.float64)
    return hist, S, rho, grad


STAGE_CASES = [
    # E, W, H, B, r, pass weights, seed
    (1500, 100, 72, 3, 3, None, 1),
    (600, 257, 130, 1, 8, None, 2),
    (400, 64, 64, 8, 2, [0.2, 0.3, 0.5], 3),
    (2000, 320, 200, 5, 6, None, 4),
    # a small grid whose height leaves three rows in the last strip of four (H = 4k + 3)
    (300, 37, 23, 2, 2, None, 5),
]


@pytest.mark.parametrize("E,W,H,B,r,a,seed", STAGE_CASES)
def test_stage_parity_given_samples(hb, E, W, H, B, r, a, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    M = workloads.interaction_eq4(B, 0.25) if B > 1 else np.ones((1, 1), np.float32)
    if B > 2:
        M = M + np.float32(0.05) * rng.random((B, B)).astype(np.float32)
    P = 3
    with _bundler(hb, W, H, [r], E, group, M, seed, pass_weights=a) as b:
        b.set_points(off, xy)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN | hb.HB_RUN_RECORD_DECISIONS)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        off_n, xy_n = b.points(hb.HB_POINTS_STATE)
        jacc = b.decisions().astype(np.int64)
        hist, S, rho, grad = _gpu_maps(hb, b, B, P)

    np.testing.assert_array_equal(off_s, off)
    np.testing.assert_array_equal(xy_s, xy)
    np.testing.assert_array_equal(off_n, off)

    p = O.Params(grid_w=W, grid_h=H, radii=[r], pass_weights=a)
    x64 = xy.astype(np.float64)
    ref = O.iterate(off, x64, group, M.astype(np.float64), p, 0, skip_resample=True)

    # histograms and box sums: bit-exact
    np.testing.assert_array_equal(hist, ref["hist"])
    np.testing.assert_array_equal(S, ref["S"])
    assert hist.sum() == len(xy)

    # density: within 1e-5 of sum_b |M[l][b]| Sbar_b
    aw = p.a()
    c = float((2 * r + 1) ** 2)
    Sbar = sum(aw[k] * ref["S"][k].astype(np.float64) / c ** (k + 1) for k in range(P))
    bound = 1e-5 * np.tensordot(np.abs(M.astype(np.float64)), Sbar, 1) + 1e-300
    assert (np.abs(rho - ref["rho"]) <= bound).all()

    # gradient: FP32 rounding of an FP64 value, relative to the layer's density scale
    scale = np.abs(ref["rho"]).max(axis=(1, 2))[:, None, None, None]
    assert (np.abs(grad - ref["grad"]) <= 1e-6 * scale + 1e-6 * np.abs(ref["grad"])).all()

    # decisions: unique where unambiguous, valid otherwise
    adv = ref["adv"]
    ok = PT.acceptable(jacc, adv["jacc"], adv["jfirm"], adv["amb"])
    assert ok.all(), f"{(~ok).sum()} invalid decisions"
    agree = jacc == adv["jacc"]
    assert agree.mean() > 0.99

    # positions: 1e-4 px, plus the conditioning of the interpolated gradient direction
    h = p.bandwidth(0)
    cond = PT.interp_condition(ref["grad"], group, off, x64)
    tdir = np.where(np.isfinite(cond), h * 1e-6 * cond, 0.0)
    tpt = 1e-4 + tdir + 2 * PT.F32_ULP_AT(xy_n).max(1)
    ty = tpt.copy()
    ty[1:-1] = 0.5 * tpt[1:-1] + 0.25 * (tpt[:-2] + tpt[2:])
    nb = agree.copy()
    nb[1:] &= agree[:-1]
    nb[:-1] &= agree[1:]
    err = np.abs(xy_n.astype(np.float64) - ref["xy"]).max(1)
    assert (err[nb] <= ty[nb]).all(), f"max err {err[nb].max()} px"
    assert np.percentile(err[nb], 99) <= 1e-4, np.percentile(err[nb], 99)
    # the rest: the GPU's (valid) decisions, replayed on the oracle's directions
    jj = np.where(jacc == -2, -1, jacc)
    yalt = PT.laplace(off, PT.candidate(x64, adv["dir"], h, jj, W, H))
    erra = np.abs(xy_n.astype(np.float64) - yalt).max(1)
    assert (erra[~nb] <= ty[~nb]).all(), f"max err {erra[~nb].max()} px"
    # end points bit-exact
    ends = np.concatenate([off[:-1], off[1:] - 1])
    np.testing.assert_array_equal(xy_n[ends], xy[ends])


@pytest.mark.parametrize("E,W,H,B,r,a,seed", [STAGE_CASES[0], STAGE_CASES[2]])
def test_fixed_step_parity_given_samples(hb, E, W, H, B, r, a, seed):
    """The original fixed step (max_halvings = -1): every interior point moves by h along
    the normalised gradient, no decisions, against the oracle's fixed step."""
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    M = workloads.interaction_eq4(B, 0.25) if B > 1 else np.ones((1, 1), np.float32)
    with _bundler(hb, W, H, [r], E, group, M, seed, pass_weights=a, max_halvings=-1) as b:
        b.set_points(off, xy)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN | hb.HB_RUN_RECORD_DECISIONS)
        off_n, xy_n = b.points(hb.HB_POINTS_STATE)
        jacc = b.decisions().astype(np.int64)
    p = O.Params(grid_w=W, grid_h=H, radii=[r], pass_weights=a, max_halvings=-1)
    x64 = xy.astype(np.float64)
    ref = O.iterate(off, x64, group, M.astype(np.float64), p, 0, skip_resample=True)
    ends = np.zeros(len(xy), bool)
    ends[off[:-1]] = ends[off[1:] - 1] = True
    np.testing.assert_array_equal(jacc[ends], -2)
    np.testing.assert_array_equal(jacc[~ends], 0)
    np.testing.assert_array_equal(ref["adv"]["jacc"][~ends], 0)
    h = p.bandwidth(0)
    cond = PT.interp_condition(ref["grad"], group, off, x64)
    tdir = np.where(np.isfinite(cond), h * 1e-6 * cond, 0.0)
    tpt = 1e-4 + tdir + 2 * PT.F32_ULP_AT(xy_n).max(1)
    ty = tpt.copy()
    ty[1:-1] = 0.5 * tpt[1:-1] + 0.25 * (tpt[:-2] + tpt[2:])
    err = np.abs(xy_n.astype(np.float64) - ref["xy"]).max(1)
    assert (err <= ty).all(), f"max err {err.max()} px"
    assert np.percentile(err, 99) <= 1e-4
    np.testing.assert_array_equal(xy_n[ends], xy[ends])


def _given_hist(hb, W, H, off, xy, group, B, weight=None, seed=0):
    """Histogram the GPU builds from given samples (one iteration with HB_RUN_SAMPLES_GIVEN)."""
    E = len(off) - 1
    rng = np.random.default_rng(seed)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2])
        nodes = rng.random((16, 2)).astype(np.float32)
        src = rng.integers(0, 16, E).astype(np.int32)
        b.set_graph(nodes, src, ((src + 1) % 16).astype(np.int32), weight)
        b.set_groups(group, np.eye(B, dtype=np.float32))
        b.set_points(off, xy)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN)
        return np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)


@pytest.mark.parametrize("W,H,B,E,heavy,seed", [
    (200, 130, 3, 700, 30000, 21), (64, 64, 1, 700, 30000, 22), (1000, 65, 2, 12, 1 << 20, 23)])
def test_weighted_histogram_parity(hb, W, H, B, E, heavy, seed):
    """Edge weights: each sample adds its edge's weight; ragged tiles at the right and
    bottom borders; weights up to the largest accepted one (the int32 range check bounds
    the sample count times the largest weight)."""
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H, step=3.0)
    group = rng.integers(0, B, E).astype(np.int32)
    weight = rng.integers(1, 9, E).astype(np.int32)
    if E < 50:
        weight[:] = np.minimum(heavy - 1 - np.arange(E), hb.HB_MAX_EDGE_WEIGHT)
    else:
        weight[::97] = heavy
    assert int(np.diff(off).sum()) * int(weight.max()) < 2 ** 31
    hist = _given_hist(hb, W, H, off, xy, group, B, weight, seed)
    ref = O.splat(off, xy.astype(np.float64), group, B, W, H, weight)
    np.testing.assert_array_equal(hist, ref)
    assert hist.sum() == int((np.diff(off) * weight.astype(np.int64)).sum())


def test_histogram_hot_tile(hb):
    """About 240 000 samples in one 64 x 64 tile (several LDS work items of one tile) plus
    a sparse background: bit-exact against the oracle's splat."""
    rng = np.random.default_rng(24)
    W = H = 256
    E_hot, E_bg = 4000, 500
    c = rng.integers(60, 64, E_hot)
    off_h = np.concatenate([[0], np.cumsum(c)]).astype(np.int64)
    xy_h = rng.uniform([128.0, 64.0], [191.99, 127.99], (int(off_h[-1]), 2))
    off_b, xy_b = PT.random_polylines(rng, E_bg, W, H)
    off = np.concatenate([off_h, off_b[1:] + off_h[-1]])
    xy = np.concatenate([xy_h, xy_b]).astype(np.float32)
    E = E_hot + E_bg
    group = np.zeros(E, np.int32)
    hist = _given_hist(hb, W, H, off, xy, group, 1)
    ref = O.splat(off, xy.astype(np.float64), group, 1, W, H)
    np.testing.assert_array_equal(hist, ref)
    assert hist[0, 64:128, 128:192].sum() >= 240000


def test_edge_weight_limits(hb):
    nodes = np.random.default_rng(0).random((4, 2)).astype(np.float32)
    src, dst = np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    with hb.Bundler(0) as b:
        b.set_params(32, 32, [2])
        for bad in (0, -3, hb.HB_MAX_EDGE_WEIGHT + 1):
            with pytest.raises(hb.HBError) as ei:
                b.set_graph(nodes, src, dst, np.array([1, bad], np.int32))
            assert ei.value.status == hb.HB_EINVAL
        b.set_graph(nodes, src, dst, np.array([1, hb.HB_MAX_EDGE_WEIGHT], np.int32))


def test_edge_sample_limit(hb):
    """An edge that would get 2^31 samples or more is refused with HB_EOVERFLOW before any
    point work (the point kernels index the samples of one edge with 32-bit integers)."""
    nodes = np.array([[0.05, 0.5], [0.95, 0.5]], np.float32)
    with hb.Bundler(0) as b:
        b.set_params(1024, 1024, [2], delta=4e-7)   # 921.6 px / 4e-7 px > 2^31 samples
        with pytest.raises(hb.HBError) as ei:
            b.set_graph(nodes, np.array([0], np.int32), np.array([1], np.int32))
        assert ei.value.status == hb.HB_EOVERFLOW
        # the context stays usable: the same edge at a sane spacing runs
        b.set_params(1024, 1024, [2], delta=1.0)
        b.set_graph(nodes, np.array([0], np.int32), np.array([1], np.int32))
        b.set_groups(np.zeros(1, np.int32), np.ones((1, 1), np.float32))
        b.run(1)
        assert 900 < b.points()[0][-1] < 950   # about 922 samples of the 921.6 px edge


@pytest.mark.parametrize("E,W,H,delta,seed", [(800, 128, 96, 1.0, 5), (300, 512, 512, 4.0, 6)])
def test_resample_parity(hb, E, W, H, delta, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=90, step=4.0)
    group = np.zeros(E, np.int32)
    with _bundler(hb, W, H, [2], E, group, np.ones((1, 1), np.float32), seed, delta=delta) as b:
        b.set_points(off, xy)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = b.map(hb.HB_MAP_HIST, 0).astype(np.int64)
    ro, rs, lens = O.resample(off, xy.astype(np.float64), delta)
    np.testing.assert_array_equal(off_s, ro)
    err = np.abs(xy_s.astype(np.float64) - rs).max(1)
    assert (err <= 1e-4 + PT.F32_ULP_AT(xy_s).max(1)).all(), err.max()
    ends = np.concatenate([ro[:-1], ro[1:] - 1])
    np.testing.assert_array_equal(xy_s[ends], xy[np.concatenate([off[:-1], off[1:] - 1])])
    # histogram of the samples: exact except where a sample sits within 1e-4 of a pixel edge
    href = O.splat(ro, rs, group, 1, W, H)[0]
    assert hist.sum() == href.sum() == len(rs)
    assert np.abs(hist - href).sum() <= 2 * PT.near_pixel_edge(rs).sum()


@pytest.mark.parametrize("E,W,H,B,delta,weighted,seed", [
    (900, 300, 200, 3, 1.0, False, 31),
    (400, 256, 256, 1, 4.0, True, 32),
    (400, 520, 390, 2, 61.0, False, 33),
    (400, 520, 390, 2, 80.0, True, 34),
])
def test_resampled_histogram_is_splat_of_samples(hb, E, W, H, B, delta, weighted, seed):
    """The histogram of an iteration with the uniform resampling must equal the splat of the
    GPU's own samples exactly (the tile counts made during the resampling, the binning and
    the tile histograms): several layers, weights, ragged border tiles, and sample spacings
    from 1 px to more than a tile (80 px: consecutive samples two tiles apart)."""
    rng = np.random.default_rng(seed)
    if delta > 8:
        off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=4, step=150.0)
    else:
        off, xy = PT.random_polylines(rng, E, W, H, n_min=2, n_max=90, step=4.0)
    group = rng.integers(0, B, E).astype(np.int32)
    weight = rng.integers(1, 6, E).astype(np.int32) if weighted else None
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2], delta=delta)
        nodes = rng.random((16, 2)).astype(np.float32)
        src = rng.integers(0, 16, E).astype(np.int32)
        b.set_graph(nodes, src, ((src + 1) % 16).astype(np.int32), weight)
        b.set_groups(group, np.eye(B, dtype=np.float32))
        b.set_points(off, xy)
        b.run(1)
        off_s, xy_s = b.points(hb.HB_POINTS_SAMPLES)
        hist = np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)
    ref = O.splat(off_s, xy_s.astype(np.float64), group, B, W, H, weight)
    np.testing.assert_array_equal(hist, ref)
    # the largest tile step between consecutive samples of one edge: one tile at most below
    # 64 px spacing, two in the 80 px case
    tu = np.clip(np.floor(xy_s[:, 0]), 0, W - 1).astype(np.int64) >> 6
    tv = np.clip(np.floor(xy_s[:, 1]), 0, H - 1).astype(np.int64) >> 6
    inner = np.ones(len(xy_s) - 1, bool)
    inner[off_s[1:-1] - 1] = False
    step = np.maximum(np.abs(np.diff(tu)), np.abs(np.diff(tv)))[inner].max()
    assert (step > 1) == (delta > 64), step


def test_end_to_end_tiny_config(hb):
    """The tiny configuration (2 000 edges, 256x256, r = 8, 10 iterations) against the oracle."""
    w = workloads.tiny()
    p = O.params_for(w)
    with hb.Bundler(0) as b:
        b.set_workload(w)
        b.run(1)
        off1, xy1 = b.points(hb.HB_POINTS_SAMPLES)
        b.run(w.n_iters - 1)
        counts = b.iter_counts(w.n_iters - 1)
        off, xy = b.points(hb.HB_POINTS_STATE)
        ink = b.ink()
    o0, x0 = O.initial_state(w.node_xy, w.src, w.dst, p)
    r0 = O.iterate(o0, x0, w.group, w.M, p, 0, keep_maps=False)
    np.testing.assert_array_equal(off1, r0["off"])
    assert np.abs(xy1 - r0["samples"]).max() <= 1e-4
    roff, rxy, rcounts = O.run(w.node_xy, w.src, w.dst, w.group, w.M, p, w.n_iters)
    assert PT.relclose(ink, O.ink(roff, rxy), 0.01)
    assert PT.relclose(O.ink(off, xy.astype(np.float64)), ink, 1e-9)
    for a, b_ in zip(counts, rcounts[1:]):
        assert PT.relclose(a, b_, 0.01)
    ds, dr = PT.drift_stats(off, xy), PT.drift_stats(roff, rxy)
    for k in ("mean", "p50", "p90", "p99"):
        assert abs(ds[k] - dr[k]) <= 0.01 * dr[k], (k, ds[k], dr[k])


def test_run_is_deterministic(hb):
    w = workloads.scaled("zipf", n_edges=3000, grid=256, groups=4, n_iters=3, seed=11)
    outs = []
    for _ in range(2):
        with hb.Bundler(0) as b:
            b.set_workload(w)
            b.run(3)
            outs.append((b.points(), [b.map(hb.HB_MAP_HIST, g) for g in range(4)],
                         [b.map(hb.HB_MAP_BOX, g, 3) for g in range(4)]))
    (o1, x1), h1, s1 = outs[0]
    (o2, x2), h2, s2 = outs[1]
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_array_equal(x1, x2)
    for a, c in zip(h1 + s1, h2 + s2):
        np.testing.assert_array_equal(a, c)


def test_capacity_growth_matches_large_capacity(hb):
    w = workloads.scaled("clustered", n_edges=1500, grid=256, groups=2, n_iters=6, seed=12)
    res = []
    for cf in (1.1, 8.0):
        with hb.Bundler(0) as b:
            b.set_workload(w, capacity_factor=cf)
            b.run(6)
            res.append(b.points())
    np.testing.assert_array_equal(res[0][0], res[1][0])
    np.testing.assert_array_equal(res[0][1], res[1][1])


def test_edge_cases(hb):
    # no edges
    with hb.Bundler(0) as b:
        b.set_params(32, 32, [2])
        b.set_graph(np.zeros((1, 2), np.float32), np.zeros(0, np.int32), np.zeros(0, np.int32))
        b.set_groups(np.zeros(0, np.int32), np.ones((1, 1), np.float32))
        b.run(2)
        off, xy = b.points()
        assert off.tolist() == [0] and xy.shape == (0, 2)
        assert (b.map(hb.HB_MAP_HIST, 0) == 0).all()
    # coincident end points, and a lone horizontal edge on a pixel-centre row (y = 32.5):
    # its density is symmetric about the row, so it never leaves it
    nodes = np.array([[0.25, 0.25], [0.25, 0.25], [0.1, 32.5 / 64], [0.9, 32.5 / 64]], np.float32)
    with hb.Bundler(0) as b:
        b.set_params(64, 64, [2, 1])
        b.set_graph(nodes, np.array([0, 2], np.int32), np.array([1, 3], np.int32))
        b.set_groups(np.array([0, 1], np.int32), np.eye(2, dtype=np.float32))
        b.run(3)
        off, xy = b.points()
        assert off[1] - off[0] == 2
        np.testing.assert_array_equal(xy[0], xy[1])
        np.testing.assert_array_equal(xy[off[1]], (nodes[2].astype(np.float64) * 64).astype(np.float32))
        assert (xy[off[1]:, 1] == np.float32(32.5)).all()
    # many groups, few edges, tiny grid
    rng = np.random.default_rng(13)
    E = 200
    with hb.Bundler(0) as b:
        b.set_params(5, 3, [1])
        b.set_graph(rng.random((40, 2)).astype(np.float32), rng.integers(0, 40, E).astype(np.int32),
                    rng.integers(0, 40, E).astype(np.int32))
        b.set_groups(rng.integers(0, 64, E).astype(np.int32), np.eye(64, dtype=np.float32))
        b.run(2)
        off, xy = b.points()
        assert (xy[:, 0] <= 5).all() and (xy[:, 1] <= 3).all()


def test_api_errors_on_device(hb):
    with hb.Bundler(0) as b:
        with pytest.raises(hb.HBError) as ei:
            b.run(1)
        assert ei.value.status == hb.HB_ESTATE
        b.set_params(32, 32, [2])
        nodes = np.random.default_rng(0).random((4, 2)).astype(np.float32)
        with pytest.raises(hb.HBError) as ei:
            b.set_graph(nodes, np.array([0, 5], np.int32), np.array([1, 2], np.int32))
        assert ei.value.status == hb.HB_EINVAL
        b.set_graph(nodes, np.array([0, 1], np.int32), np.array([1, 2], np.int32))
        with pytest.raises(hb.HBError) as ei:
            b.set_groups(np.array([0, 2], np.int32), np.eye(2, dtype=np.float32))
        assert ei.value.status == hb.HB_EINVAL
        b.set_groups(np.array([0, 1], np.int32), np.eye(2, dtype=np.float32))
        with pytest.raises(hb.HBError):
            b.map(hb.HB_MAP_HIST, 0)
        b.run(1)
        with pytest.raises(hb.HBError):
            b.map(hb.HB_MAP_BOX, 0, 4)
        with pytest.raises(hb.HBError):
            b.set_points(np.array([0, 1, 3], np.int64), np.zeros((3, 2), np.float32))
        with pytest.raises(hb.HBError):
            b.decisions()


def test_allocation_failure_is_an_error_code(hb, monkeypatch):
    """A failed device allocation (simulated through HB_TEST_FAIL_ALLOC, which makes every
    allocation of the library fail) returns HB_ENOMEM without aborting; once allocations
    succeed again the same context sets the graph and runs."""
    w = workloads.scaled("uniform", n_edges=200, grid=64, groups=2, n_iters=1, seed=5)
    with hb.Bundler(0) as b:
        b.set_params(w.grid_w, w.grid_h, w.radii)
        monkeypatch.setenv("HB_TEST_FAIL_ALLOC", "1")
        with pytest.raises(hb.HBError) as ei:
            b.set_graph(w.node_xy, w.src, w.dst)
        assert ei.value.status == hb.HB_ENOMEM
        assert "allocation" in hb.hb_last_error(b.ctx)
        monkeypatch.delenv("HB_TEST_FAIL_ALLOC")
        b.set_graph(w.node_xy, w.src, w.dst)
        b.set_groups(w.group, w.M)
        b.run(1)
        off, xy = b.points()
        assert off[-1] == len(xy) > 0


def test_int32_count_bound_per_tile(hb):
    """The int32 histogram is guarded tile by tile: a tile whose entries times the largest
    edge weight could pass 2^31 gives HB_EOVERFLOW, while a graph whose total N w passes
    2^32 but whose tiles stay below the bound runs, with the histogram equal to the oracle's
    (int64) splat."""
    rng = np.random.default_rng(17)
    wmax = hb.HB_MAX_EDGE_WEIGHT
    # spread: 4000 short edges over a 1024^2 grid, about 90 samples per 64x64 tile
    E = 4000
    start = rng.uniform(0.02, 0.98, (E, 2))
    ang = rng.uniform(0, 2 * np.pi, E)
    end = np.clip(start + 5.0 / 1024 * np.stack([np.cos(ang), np.sin(ang)], 1), 0.0, 1.0)
    nodes = np.concatenate([start, end]).astype(np.float32)
    src = np.arange(E, dtype=np.int32)
    dst = (E + np.arange(E)).astype(np.int32)
    weight = np.full(E, wmax, np.int32)
    with hb.Bundler(0) as b:
        b.set_params(1024, 1024, [2])
        b.set_graph(nodes, src, dst, weight)
        b.set_groups(np.zeros(E, np.int32), np.ones((1, 1), np.float32))
        b.run(1)
        off, xy = b.points(hb.HB_POINTS_SAMPLES)
        hist = b.map(hb.HB_MAP_HIST, 0).astype(np.int64)
    assert float(len(xy)) * wmax > 2.0 ** 32
    ref = O.splat(off, xy.astype(np.float64), np.zeros(E, np.int32), 1, 1024, 1024, weight)[0]
    np.testing.assert_array_equal(hist, ref)
    # crowded: 300 edges of about 20 px inside one 64 x 64 tile (more than 2^31 / wmax entries)
    E = 300
    start = rng.uniform(130.0 / 1024, 140.0 / 1024, (E, 2))
    end = start + 14.0 / 1024
    nodes = np.concatenate([start, end]).astype(np.float32)
    src = np.arange(E, dtype=np.int32)
    dst = (E + np.arange(E)).astype(np.int32)
    with hb.Bundler(0) as b:
        b.set_params(1024, 1024, [2])
        b.set_graph(nodes, src, dst, np.full(E, wmax, np.int32))
        b.set_groups(np.zeros(E, np.int32), np.ones((1, 1), np.float32))
        with pytest.raises(hb.HBError) as ei:
            b.run(1)
        assert ei.value.status == hb.HB_EOVERFLOW
