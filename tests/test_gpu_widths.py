"""GPU-vs-oracle parity of the width encoding (Section 3.4): the maps of the polylines taken
as samples, the density of each point's own layer at the point and the width it gets on a
linear or logarithmic scale. The densities agree within 1e-5 of the bilinear sum of |rho|
(FP32 map and FP32 interpolation against FP64); the widths within 3e-5 of the width range
(both relative errors of a density and of the largest one) plus FP32 rounding."""

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


def _run(hb, off, xy, group, M, W, H, radii, it, w_min, w_max, log_scale, strip=False, weight=None,
         device=None):
    B = M.shape[0]
    E = len(off) - 1
    with hb.Bundler(0) as b:
        b.set_params(W, H, radii, splat_mode=hb.HB_SPLAT_STRIP if strip else hb.HB_SPLAT_POINTS)
        rng = np.random.default_rng(0)
        nodes = rng.random((8, 2)).astype(np.float32)
        b.set_graph(nodes, rng.integers(0, 8, E).astype(np.int32), rng.integers(0, 8, E).astype(np.int32),
                    weight)
        b.set_groups(group, M)
        b.set_points(off, xy)
        dens, widths = b.point_widths(it, w_min, w_max, log_scale, device)
        if device is not None:
            dens, widths = dens.cpu().numpy(), widths.cpu().numpy()
        hist = np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)
    return dens, widths, hist


def _reference(off, xy, group, M, W, H, radii, it, w_min, w_max, log_scale, strip=False, weight=None):
    p = O.Params(grid_w=W, grid_h=H, radii=list(radii))
    p.strip_splat = strip
    x64 = xy.astype(np.float64)
    rho = O.maps_of(off, x64, group, M.astype(np.float64), p, it, weight)
    dens, widths = O.point_widths(off, x64, group, rho, w_min, w_max, log_scale)
    dabs, _ = O.point_widths(off, x64, group, np.abs(rho), 0.0, 1.0)
    if strip:
        hist = O.splat_strip(off, x64, group, M.shape[0], W, H, weight)
    else:
        hist = O.splat(off, x64, group, M.shape[0], W, H, weight)
    return dens, widths, dabs, hist


def _check(got, ref, w_min, w_max):
    dens, widths, hist = got
    rdens, rwidths, dabs, rhist = ref
    np.testing.assert_array_equal(hist, rhist)
    assert dens.shape == rdens.shape and widths.shape == rwidths.shape
    assert (dens >= 0).all()
    bound = 1e-5 * dabs + 1e-30
    bad = np.abs(dens.astype(np.float64) - rdens) > bound
    assert not bad.any(), (np.flatnonzero(bad)[:5], dens[bad][:5], rdens[bad][:5])
    tol = 3e-5 * (w_max - w_min) + 2e-7 * max(w_max, 1.0)
    err = np.abs(widths.astype(np.float64) - rwidths)
    assert err.max() <= tol, (err.max(), tol)
    assert (widths >= np.float32(w_min)).all() and (widths <= np.float32(w_max)).all()


@pytest.mark.parametrize("E,W,H,B,radii,it,log_scale,seed", [
    (1200, 100, 72, 3, [4, 3], 1, False, 91),     # ragged tiles, several layers, iteration 1 radius
    (900, 257, 130, 1, [6], 0, True, 92),         # one layer, logarithmic scale
    (700, 64, 64, 2, [2, 5, 1], 2, True, 93),
])
def test_widths_points(hb, E, W, H, B, radii, it, log_scale, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    M = workloads.interaction_eq4(B, 0.25) if B > 1 else np.ones((1, 1), np.float32)
    got = _run(hb, off, xy, group, M, W, H, radii, it, 0.5, 6.0, log_scale)
    _check(got, _reference(off, xy, group, M, W, H, radii, it, 0.5, 6.0, log_scale), 0.5, 6.0)


@pytest.mark.parametrize("log_scale", [False, True])
def test_widths_strip(hb, log_scale):
    rng = np.random.default_rng(94)
    E, W, H, B = 800, 150, 90, 2
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    M = workloads.interaction_eq4(B, 0.25)
    got = _run(hb, off, xy, group, M, W, H, [3], 0, 1.0, 8.0, log_scale, strip=True)
    _check(got, _reference(off, xy, group, M, W, H, [3], 0, 1.0, 8.0, log_scale, strip=True), 1.0, 8.0)


def test_widths_weighted_device_ptrs(hb):
    """Integer edge weights in the splat; outputs in device memory."""
    import torch
    rng = np.random.default_rng(95)
    E, W, H = 600, 96, 80
    off, xy = PT.random_polylines(rng, E, W, H)
    group = np.zeros(E, np.int32)
    M = np.ones((1, 1), np.float32)
    weight = rng.integers(1, 7, E).astype(np.int32)
    got = _run(hb, off, xy, group, M, W, H, [3], 0, 0.25, 4.0, False, weight=weight,
               device=torch.device("cuda:0"))
    ref = _reference(off, xy, group, M, W, H, [3], 0, 0.25, 4.0, False, weight=weight)
    _check(got, ref, 0.25, 4.0)


def test_widths_degenerate(hb):
    """A zero interaction matrix (no density anywhere) gives w_min everywhere; w_min = w_max
    gives that width everywhere; the largest density gets w_max."""
    rng = np.random.default_rng(96)
    E, W, H = 300, 64, 48
    off, xy = PT.random_polylines(rng, E, W, H)
    group = np.zeros(E, np.int32)
    dens, widths, _ = _run(hb, off, xy, group, np.zeros((1, 1), np.float32), W, H, [2], 0, 0.5, 3.0, False)
    assert (dens == 0).all() and (widths == np.float32(0.5)).all()
    _, widths, _ = _run(hb, off, xy, group, np.ones((1, 1), np.float32), W, H, [2], 0, 2.0, 2.0, True)
    assert (widths == np.float32(2.0)).all()
    dens, widths, _ = _run(hb, off, xy, group, np.ones((1, 1), np.float32), W, H, [2], 0, 1.0, 5.0, False)
    assert widths[np.argmax(dens)] == np.float32(5.0)
    # no edges: nothing to encode, in both splat modes
    for mode in (hb.HB_SPLAT_POINTS, hb.HB_SPLAT_STRIP):
        with hb.Bundler(0) as b:
            b.set_params(32, 32, [2], splat_mode=mode)
            b.set_graph(np.zeros((1, 2), np.float32), np.zeros(0, np.int32), np.zeros(0, np.int32))
            b.set_groups(np.zeros(0, np.int32), np.ones((1, 1), np.float32))
            d0, w0 = b.point_widths(0, 1.0, 2.0)
            assert d0.shape == (0,) and w0.shape == (0,)
            assert (b.map(hb.HB_MAP_HIST, 0) == 0).all()


def test_widths_invalid(hb):
    rng = np.random.default_rng(97)
    E, W, H = 50, 32, 32
    off, xy = PT.random_polylines(rng, E, W, H, n_max=10)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [2])
        b.set_graph(rng.random((4, 2)).astype(np.float32), np.zeros(E, np.int32), np.ones(E, np.int32))
        b.set_groups(np.zeros(E, np.int32), np.ones((1, 1), np.float32))
        b.set_points(off, xy)
        for args in [(-1, 0.5, 2.0, False), (0, -0.5, 2.0, False), (0, 3.0, 2.0, False),
                     (0, float("nan"), 2.0, False), (0, 0.5, float("inf"), False)]:
            with pytest.raises(hb.HBError) as ei:
                b.point_widths(*args)
            assert ei.value.status == hb.HB_EINVAL
        n = hb.hb_get_num_points(b.ctx)
        d = np.empty(n, np.float32)
        w = np.empty(n, np.float32)
        st = hb.load().hb_point_widths(b.ctx, 0, 0.5, 2.0, 2, d.ctypes.data, w.ctypes.data, n, 0)
        assert st == hb.HB_EINVAL
        st = hb.load().hb_point_widths(b.ctx, 0, 0.5, 2.0, 0, d.ctypes.data, w.ctypes.data, n - 1, 0)
        assert st == hb.HB_EINVAL
        d2, w2 = b.point_widths(0, 0.5, 2.0)         # the context still works
        assert w2.shape == (n,)
