"""Pins of the FP64 oracle against closed forms, brute force and invariants.

Each pin is computed independently of the oracle's own code (numpy/scipy brute
force or a closed form), so that a plausible mistake in the oracle (a dropped term,
a wrong sign, an off-by-one window, a transposed operand) fails at least one test.
"""

import math

import numpy as np
import pytest
import scipy.ndimage
import scipy.signal

import oracle as O


def rng(seed=0):
    return np.random.default_rng(seed)


# ------------------------------------------------------------------ resampling (Sec. 2.1, 3)

def test_resample_straight_axis_closed_form():
    off = np.array([0, 2], np.int64)
    xy = np.array([[10.25, 20.5], [110.25, 20.5]])
    o, s, _ = O.resample(off, xy, 1.0)
    assert o[-1] == 101
    np.testing.assert_array_equal(s[:, 1], 20.5)
    np.testing.assert_allclose(s[:, 0], 10.25 + np.arange(101), atol=1e-12)


def test_resample_diagonal_closed_form():
    off = np.array([0, 2], np.int64)
    xy = np.array([[0.0, 0.0], [30.0, 40.0]])
    o, s, lens = O.resample(off, xy, 1.0)
    assert lens[0] == 50.0 and o[-1] == 51
    k = np.arange(51)
    np.testing.assert_allclose(s, np.stack([0.6 * k, 0.8 * k], 1), atol=1e-12)


@pytest.mark.parametrize("L,delta,n", [(37.0, 1.0, 38), (37.0, 4.0, 11), (0.0, 1.0, 2),
                                       (0.3, 1.0, 2), (1.0, 1.0, 2), (2.5, 1.0, 4)])
def test_sample_count(L, delta, n):
    off = np.array([0, 2], np.int64)
    xy = np.array([[5.0, 7.0], [5.0 + L, 7.0]])
    o, s, _ = O.resample(off, xy, delta)
    assert o[-1] == n
    np.testing.assert_array_equal(s[0], xy[0])
    np.testing.assert_array_equal(s[-1], xy[1])


def _np_resample(p, delta):
    seg = np.hypot(*np.diff(p, axis=0).T)
    C = np.concatenate([[0.0], np.cumsum(seg)])
    L = C[-1]
    n = max(1, math.ceil(L / delta)) + 1
    s = np.arange(n) * L / (n - 1)
    return np.stack([np.interp(s, C, p[:, 0]), np.interp(s, C, p[:, 1])], 1)


def test_resample_matches_numpy_interp_on_random_polylines():
    g = rng(1)
    polys = [np.cumsum(g.normal(0, 3, (int(m), 2)), 0) + 100 for m in g.integers(2, 40, 50)]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])]).astype(np.int64)
    o, s, _ = O.resample(off, np.concatenate(polys), 1.0)
    for e, p in enumerate(polys):
        ref = _np_resample(p, 1.0)
        got = s[o[e]:o[e + 1]]
        assert got.shape == ref.shape
        np.testing.assert_allclose(got, ref, atol=1e-9)
        np.testing.assert_array_equal(got[0], p[0])
        np.testing.assert_array_equal(got[-1], p[-1])


def test_resample_idempotent_on_straight_polylines():
    g = rng(2)
    t = np.sort(g.random(30))
    t[0], t[-1] = 0.0, 1.0
    # collinear, uneven spacing, length 100.5 (away from an integer: counts are then
    # unambiguous; at integer lengths the FP64 sum may land on either side)
    p = np.stack([3.0 + 80.4 * t, 5.0 + 60.3 * t], 1)
    off = np.array([0, 30], np.int64)
    o1, s1, _ = O.resample(off, p, 1.0)
    o2, s2, _ = O.resample(o1, s1, 1.0)
    assert o1[-1] == 102 and o2[-1] == 102
    np.testing.assert_allclose(s2, s1, atol=1e-9)


# ------------------------------------------------------------------ splat (Eq. 1 / Eq. 3)

def _np_splat(off, xy, group, B, W, H, weight=None):
    h = np.zeros((B, H, W), np.int64)
    E = len(off) - 1
    eid = np.repeat(np.arange(E), np.diff(off))
    w = np.ones(E, np.int64) if weight is None else weight.astype(np.int64)
    u = np.clip(np.floor(xy[:, 0]), 0, W - 1).astype(np.int64)
    v = np.clip(np.floor(xy[:, 1]), 0, H - 1).astype(np.int64)
    np.add.at(h, (group[eid], v, u), w[eid])
    return h


def _random_points(g, E, W, H, B):
    counts = g.integers(2, 30, E)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    xy = np.stack([g.uniform(-2, W + 2, off[-1]), g.uniform(-2, H + 2, off[-1])], 1)
    group = g.integers(0, B, E).astype(np.int32)
    return off, xy, group


def test_splat_matches_bruteforce_and_mass():
    g = rng(3)
    W, H, B, E = 37, 29, 3, 200
    off, xy, group = _random_points(g, E, W, H, B)
    weight = g.integers(1, 5, E).astype(np.int32)
    h = O.splat(off, xy, group, B, W, H, weight)
    np.testing.assert_array_equal(h, _np_splat(off, xy, group, B, W, H, weight))
    assert h.sum() == (np.diff(off) * weight).sum()


def test_splat_pixel_boundaries_and_clamp():
    off = np.array([0, 5], np.int64)
    xy = np.array([[5.0, 3.0], [4.999999, 3.0], [16.0, 0.0], [-0.5, 15.9], [15.99, -3.0]])
    h = O.splat(off, xy, np.zeros(1, np.int32), 1, 16, 16)
    assert h[0, 3, 5] == 1 and h[0, 3, 4] == 1 and h[0, 0, 15] == 2 and h[0, 15, 0] == 1


def test_splat_permutation_and_transpose():
    g = rng(4)
    W = H = 32
    off, xy, group = _random_points(g, 100, W, H, 2)
    h = O.splat(off, xy, group, 2, W, H)
    perm = g.permutation(100)
    cnt = np.diff(off)[perm]
    off2 = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    xy2 = np.concatenate([xy[off[e]:off[e + 1]] for e in perm])
    np.testing.assert_array_equal(O.splat(off2, xy2, group[perm], 2, W, H), h)
    ht = O.splat(off, xy[:, ::-1], group, 2, W, H)
    np.testing.assert_array_equal(ht, h.transpose(0, 2, 1))


# ------------------------------------------------------------------ box chain (Sec. 3.1)

@pytest.mark.parametrize("W,H,r", [(17, 11, 1), (20, 20, 3), (16, 9, 4), (8, 8, 7)])
def test_box_brute_integral_scipy_agree(W, H, r):
    m = rng(5).integers(0, 1000, (H, W)).astype(np.int64)
    ref = scipy.signal.convolve2d(m, np.ones((2 * r + 1, 2 * r + 1), np.int64), mode="same")
    np.testing.assert_array_equal(O.box_brute(m, r), ref)
    np.testing.assert_array_equal(O.box_integral(m, r), ref)


def test_integral_image_corner_is_total():
    m = rng(6).integers(0, 50, (13, 21)).astype(np.int64)
    I = O.integral_image(m)
    assert I[-1, -1] == m.sum()
    np.testing.assert_array_equal(I[1:, 1:], m.cumsum(0).cumsum(1))
    assert (I[0] == 0).all() and (I[:, 0] == 0).all()


@pytest.mark.parametrize("P,r", [(1, 2), (3, 2), (3, 4), (2, 5)])
def test_box_chain_impulse_closed_form(P, r):
    W = H = 2 * P * r + 9
    c = W // 2
    hist = np.zeros((1, H, W), np.int64)
    hist[0, c, c] = 1
    S = O.box_chain(hist, P, r)
    S2 = O.box_chain(hist, P, r, brute=True)
    np.testing.assert_array_equal(S, S2)
    k = np.ones(1, np.int64)
    for _ in range(P):
        k = np.convolve(k, np.ones(2 * r + 1, np.int64))     # coefficients of (1+z+..+z^2r)^P
    ref = np.zeros((H, W), np.int64)
    ref[c - P * r:c + P * r + 1, c - P * r:c + P * r + 1] = np.outer(k, k)
    np.testing.assert_array_equal(S[-1, 0], ref)
    if P >= 1:
        first = np.zeros((H, W), np.int64)
        first[c - r:c + r + 1, c - r:c + r + 1] = 1
        np.testing.assert_array_equal(S[0, 0], first)
    # mass and per-axis variance of P passes: sigma^2 = P r (r+1) / 3
    assert S[-1, 0].sum() == (2 * r + 1) ** (2 * P)
    d = np.arange(W) - c
    prof = S[-1, 0].sum(0).astype(np.float64)
    var = (prof * d ** 2).sum() / prof.sum()
    assert abs(var - O.sigma(r, P) ** 2) < 1e-9


def test_box_chain_mass_conserved_away_from_border():
    P, r, W = 3, 3, 48
    hist = np.zeros((2, W, W), np.int64)
    g = rng(7)
    inner = slice(P * r + 1, W - P * r - 1)
    hist[:, inner, inner] = g.integers(0, 9, hist[:, inner, inner].shape)
    S = O.box_chain(hist, P, r)
    np.testing.assert_array_equal(S[-1].sum((1, 2)), hist.sum((1, 2)) * (2 * r + 1) ** (2 * P))


# ------------------------------------------------------------------ density stack (Eq. 3 / Eq. 4)

def test_density_preserves_constant_maps_in_interior():
    P, r, W = 3, 2, 40
    hist = np.full((1, W, W), 7, np.int64)
    S = O.box_chain(hist, P, r)
    rho = O.density(S, r, np.array([0, 0, 1.0]), np.ones((1, 1)))
    m = P * r
    np.testing.assert_allclose(rho[0, m:W - m, m:W - m], 7.0, rtol=1e-15)
    rho1 = O.density(S, r, np.array([1.0, 0, 0]), np.ones((1, 1)))
    np.testing.assert_allclose(rho1[0, r:W - r, r:W - r], 7.0, rtol=1e-15)


def _float_box(m, r, P):
    k = np.ones((2 * r + 1, 2 * r + 1)) / (2 * r + 1) ** 2
    for _ in range(P):
        m = scipy.signal.convolve2d(m, k, mode="same")
    return m


def test_density_equals_mixing_before_smoothing():
    """Eq. 3 mixes at the histogram and smooths afterwards; the oracle mixes after smoothing."""
    g = rng(8)
    B, W, H, P, r = 3, 24, 20, 3, 2
    hist = g.integers(0, 20, (B, H, W)).astype(np.int64)
    M = g.normal(0, 1, (B, B))
    rho = O.density(O.box_chain(hist, P, r), r, np.array([0, 0, 1.0]), M)
    for l in range(B):
        mixed = np.tensordot(M[l], hist.astype(np.float64), axes=1)
        np.testing.assert_allclose(rho[l], _float_box(mixed, r, P), rtol=1e-10, atol=1e-10)


def test_density_identity_and_permutation():
    g = rng(9)
    B, W, P, r = 4, 16, 3, 1
    hist = g.integers(0, 20, (B, W, W)).astype(np.int64)
    S = O.box_chain(hist, P, r)
    a = np.array([0.2, 0.3, 0.5])
    rho_I = O.density(S, r, a, np.eye(B))
    for b in range(B):
        rho_b = O.density(O.box_chain(hist[b:b + 1], P, r), r, a, np.ones((1, 1)))
        np.testing.assert_array_equal(rho_I[b], rho_b[0])
    M = g.normal(0, 1, (B, B))
    perm = g.permutation(B)
    rho = O.density(S, r, a, M)
    rho_p = O.density(O.box_chain(hist[perm], P, r), r, a, M[np.ix_(perm, perm)])
    np.testing.assert_allclose(rho_p, rho[perm], rtol=1e-14, atol=1e-14)


def test_eq4_fixture():
    import os
    import workloads
    path = os.path.join(os.path.dirname(__file__), "golden", "eq4_interaction.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    for B, alpha, diag, off in rows:
        M = workloads.interaction_eq4(int(B), float(alpha))
        assert M[0, 0] == np.float32(float(diag))
        assert M[0, 1] == np.float32(float(off))


# ------------------------------------------------------------------ gradient and bilinear

def test_gradient_of_linear_map_is_exact_inside():
    W, H = 12, 9
    v, u = np.mgrid[0:H, 0:W]
    rho = (3.0 + 0.75 * u - 1.25 * v)[None].astype(np.float64)
    g = O.gradient(rho)
    np.testing.assert_allclose(g[0, 1:-1, 1:-1, 0], 0.75, rtol=1e-15)
    np.testing.assert_allclose(g[0, 1:-1, 1:-1, 1], -1.25, rtol=1e-15)
    # zero outside the grid
    np.testing.assert_allclose(g[0, 4, 0, 0], 0.5 * (rho[0, 4, 1] - 0.0))
    np.testing.assert_allclose(g[0, H - 1, 5, 1], 0.5 * (0.0 - rho[0, H - 2, 5]))


def test_bilinear_reproduces_linear_functions_and_scipy():
    W, H = 10, 7
    v, u = np.mgrid[0:H, 0:W]
    m = 2.0 + 0.5 * u + 0.25 * v
    g = rng(10)
    for x, y in g.uniform(0.5, [W - 0.5, H - 0.5], (50, 2)):
        assert abs(O.bilinear(m, x, y) - (2.0 + 0.5 * (x - 0.5) + 0.25 * (y - 0.5))) < 1e-12
    r = g.random((H, W))
    for x, y in g.uniform(-1, [W + 1, H + 1], (80, 2)):
        ref = scipy.ndimage.map_coordinates(r, [[y - 0.5], [x - 0.5]], order=1, mode="nearest")[0]
        assert abs(O.bilinear(r, x, y) - ref) < 1e-12
    assert O.bilinear(r, 3.5, 2.5) == r[2, 3]


# ------------------------------------------------------------------ advection (Eq. 5 + halving)

def _bump(W, c, P, r):
    hist = np.zeros((1, W, W), np.int64)
    hist[0, c, c] = 1000
    S = O.box_chain(hist, P, r)
    rho = O.density(S, r, np.array([0, 0, 1.0]), np.ones((1, 1)))
    return rho, O.gradient(rho)


def test_advect_accepts_only_non_lower_density_and_end_points_fixed():
    g = rng(11)
    W, B = 48, 2
    hist = g.integers(0, 5, (B, W, W)).astype(np.int64)
    rho = O.density(O.box_chain(hist, 3, 3), 3, np.array([0, 0, 1.0]), np.array([[1, -.1], [-.1, 1]]))
    grad = O.gradient(rho)
    off, xy, group = _random_points(g, 60, W, W, B)
    xy = np.clip(xy, 0, W - 1 / 256)
    res = O.advect(off, xy, group, rho, grad, h=6.0)
    moved = res["jacc"] >= 0
    assert moved.sum() > 0.5 * len(xy) - 2 * 60
    for i in np.nonzero(moved)[0]:
        e = np.searchsorted(off, i, side="right") - 1
        m = rho[group[e]]
        # independent bilinear (scipy, pixel centres at +1/2, nearest-edge clamping)
        r0 = scipy.ndimage.map_coordinates(m, [[xy[i, 1] - .5], [xy[i, 0] - .5]], order=1, mode="nearest")[0]
        r1 = scipy.ndimage.map_coordinates(m, [[res["xy"][i, 1] - .5], [res["xy"][i, 0] - .5]], order=1, mode="nearest")[0]
        assert r1 >= r0 - 1e-12 * abs(r0)
        step = np.hypot(*(res["xy"][i] - xy[i]))
        assert step <= 6.0 / 2 ** res["jacc"][i] + 1e-9
    ends = np.concatenate([off[:-1], off[1:] - 1])
    np.testing.assert_array_equal(res["xy"][ends], xy[ends])
    assert (res["jacc"][ends] == -2).all()


def test_advect_flat_map_does_not_move():
    W = 32
    rho = np.full((1, W, W), 5.0)
    grad = O.gradient(rho)     # zero inside, non-zero only on the border pixels
    off = np.array([0, 3], np.int64)
    xy = np.array([[10.2, 10.7], [15.3, 16.1], [20.0, 20.0]])
    res = O.advect(off, xy, np.zeros(1, np.int32), rho, grad, h=4.0)
    np.testing.assert_array_equal(res["xy"], xy)
    assert res["jacc"][1] == 0


@pytest.mark.parametrize("x,h", [(26.5, 2.0), (26.5, 12.0), (27.25, 3.0), (36.0, 9.0), (38.0, 40.0), (31.0, 5.0)])
def test_advect_toward_isolated_bump_closed_form(x, h):
    """On the row through a symmetric bump the gradient points at the peak and the halving
    loop accepts the first step that does not end farther from the peak than it started."""
    W, c, P, r = 64, 32, 3, 3
    rho, grad = _bump(W, c, P, r)
    y = c + 0.5
    off = np.array([0, 3], np.int64)
    xy = np.array([[1.0, 1.0], [x, y], [60.0, 60.0]])
    res = O.advect(off, xy, np.zeros(1, np.int32), rho, grad, h=h, K=8)
    peak = c + 0.5
    sgn = 1.0 if peak > x else -1.0
    expect = x
    for j in range(9):
        cand = x + sgn * h / 2 ** j
        if abs(cand - peak) <= abs(x - peak):
            expect = cand
            break
    assert res["xy"][1, 1] == y
    assert abs(res["xy"][1, 0] - expect) < 1e-12
    assert res["dir"][1, 0] == pytest.approx(sgn) and res["dir"][1, 1] == 0.0


@pytest.mark.parametrize("x,h", [(26.5, 2.0), (26.5, 12.0), (36.0, 9.0), (31.0, 5.0), (40.0, 45.0)])
def test_fixed_step_moves_by_h_closed_form(x, h):
    """The original step (K = -1) moves every interior point by exactly h toward the peak of
    a symmetric bump, overshooting it where h is larger than the distance, clamped only at
    the grid border; end points stay."""
    W, c, P, r = 64, 32, 3, 3
    rho, grad = _bump(W, c, P, r)
    y = c + 0.5
    off = np.array([0, 3], np.int64)
    xy = np.array([[1.0, 1.0], [x, y], [60.0, 60.0]])
    res = O.advect(off, xy, np.zeros(1, np.int32), rho, grad, h=h, K=-1)
    sgn = 1.0 if c + 0.5 > x else -1.0
    expect = min(max(x + sgn * h, 0.0), W - 1 / 256)
    assert abs(res["xy"][1, 0] - expect) < 1e-12 and res["xy"][1, 1] == y
    assert res["jacc"][1] == 0
    np.testing.assert_array_equal(res["xy"][[0, 2]], xy[[0, 2]])


def test_fixed_step_displacement_is_h_times_direction():
    """On random maps every interior point moves by h d with d the unit direction of the
    scipy-interpolated gradient (where no clamp applies), and the halving version agrees
    wherever its first try is accepted."""
    g = rng(12)
    W, B = 48, 2
    hist = g.integers(0, 5, (B, W, W)).astype(np.int64)
    rho = O.density(O.box_chain(hist, 3, 3), 3, np.array([0, 0, 1.0]), np.eye(B))
    grad = O.gradient(rho)
    off, xy = _random_points(g, 40, W, W, B)[:2]
    group = g.integers(0, B, 40).astype(np.int32)
    xy = np.clip(xy, 8, W - 8)
    h = 3.0
    res = O.advect(off, xy, group, rho, grad, h=h, K=-1)
    hal = O.advect(off, xy, group, rho, grad, h=h, K=8)
    ends = np.zeros(len(xy), bool)
    ends[off[:-1]] = ends[off[1:] - 1] = True
    for i in np.nonzero(~ends)[0]:
        e = np.searchsorted(off, i, side="right") - 1
        gx = scipy.ndimage.map_coordinates(grad[group[e], :, :, 0], [[xy[i, 1] - .5], [xy[i, 0] - .5]], order=1, mode="nearest")[0]
        gy = scipy.ndimage.map_coordinates(grad[group[e], :, :, 1], [[xy[i, 1] - .5], [xy[i, 0] - .5]], order=1, mode="nearest")[0]
        n = math.hypot(gx, gy)
        d = np.array([gx, gy]) / max(n, 1e-6)
        np.testing.assert_allclose(res["xy"][i], xy[i] + h * d, atol=1e-9)
        if hal["jacc"][i] == 0:
            np.testing.assert_allclose(hal["xy"][i], res["xy"][i], atol=1e-12)
    np.testing.assert_array_equal(res["xy"][ends], xy[ends])


# ------------------------------------------------------------------ Laplacian

def test_laplacian_fixed_points_and_zigzag():
    j = np.arange(12, dtype=np.float64)
    off = np.array([0, 12, 24], np.int64)
    line = np.stack([1.0 + 2.0 * j, -3.0 + 0.5 * j], 1)
    zig = np.stack([j, (-1.0) ** j], 1)
    out = O.laplacian(off, np.concatenate([line, zig]), s=0.3, passes=1)
    np.testing.assert_allclose(out[:12], line, atol=1e-12)
    np.testing.assert_allclose(out[13:23, 1], (-1.0) ** j[1:11] * (1 - 2 * 0.3), atol=1e-12)
    np.testing.assert_allclose(out[13:23, 0], j[1:11], atol=1e-12)
    np.testing.assert_array_equal(out[[0, 11, 12, 23]], np.concatenate([line, zig])[[0, 11, 12, 23]])


def test_ink_of_known_polylines():
    off = np.array([0, 2, 5], np.int64)
    xy = np.array([[0, 0], [3, 4], [0, 0], [1, 0], [1, 1]], np.float64)
    assert O.ink(off, xy) == 7.0


# ------------------------------------------------------------------ whole iterations

def _params(W, radii, **kw):
    return O.Params(grid_w=W, grid_h=W, radii=radii, **kw)


def test_straight_horizontal_edge_stays_on_its_row():
    W = 64
    p = _params(W, [4])
    node = np.array([[10.25 / W, 30.5 / W], [50.75 / W, 30.5 / W]], np.float32)
    off, xy, counts = O.run(node, np.array([0]), np.array([1]), np.zeros(1, np.int32),
                            np.ones((1, 1)), p, 5)
    np.testing.assert_array_equal(xy[:, 1], 30.5)
    # points slide along the line only (toward the edge's own density peak at its middle),
    # end points stay, and the result is mirror-symmetric about the midpoint x = 30.5
    assert xy[0, 0] == 10.25 and xy[-1, 0] == 50.75
    assert xy[:, 0].min() >= 10.25 and xy[:, 0].max() <= 50.75
    np.testing.assert_allclose(xy[:, 0] + xy[::-1, 0], 61.0, atol=1e-6)
    assert counts[0] == 42


def test_two_parallel_edges_attract():
    W = 64
    p = _params(W, [4])
    node = np.array([[10, 28.5], [54, 28.5], [10, 33.5], [54, 33.5]], np.float32) / W
    off, xy, _ = O.run(node, np.array([0, 2]), np.array([1, 3]), np.zeros(2, np.int32),
                       np.ones((1, 1)), p, 4)
    mid0 = xy[off[0]:off[1]][len(xy[off[0]:off[1]]) // 2, 1]
    mid1 = xy[off[1]:off[2]][len(xy[off[1]:off[2]]) // 2, 1]
    assert mid1 - mid0 < 5.0 - 1.0


def test_identity_interaction_equals_independent_runs():
    g = rng(12)
    W = 64
    p = _params(W, [3, 2])
    node = g.random((40, 2)).astype(np.float32)
    src, dst = np.arange(0, 20), np.arange(20, 40)
    group = (np.arange(20) % 2).astype(np.int32)
    off, xy, _ = O.run(node, src, dst, group, np.eye(2), p, 2)
    for b in range(2):
        sel = np.nonzero(group == b)[0]
        o2, x2, _ = O.run(node, src[sel], dst[sel], np.zeros(len(sel), np.int32), np.ones((1, 1)), p, 2)
        mine = np.concatenate([xy[off[e]:off[e + 1]] for e in sel])
        np.testing.assert_array_equal(mine, x2)


def test_transposed_input_gives_transposed_output():
    g = rng(13)
    W = 64
    p = _params(W, [3])
    node = g.random((30, 2)).astype(np.float32)
    src, dst = np.arange(15), np.arange(15, 30)
    grp = np.zeros(15, np.int32)
    off, xy, _ = O.run(node, src, dst, grp, np.ones((1, 1)), p, 3)
    off_t, xy_t, _ = O.run(node[:, ::-1].copy(), src, dst, grp, np.ones((1, 1)), p, 3)
    np.testing.assert_array_equal(off, off_t)
    np.testing.assert_allclose(xy_t[:, ::-1], xy, atol=1e-9)


def test_schedule_values():
    p = _params(256, [8])
    assert abs(p.hmax() - 2 * math.sqrt(3 * 8 * 9 / 3)) < 1e-12
    h = [p.bandwidth(i) for i in range(10)]
    np.testing.assert_allclose(h, [16.97056 * 0.9 ** i for i in range(10)], rtol=1e-6)


# ------------------------------------------------------------------ directed graphs (Sec. 3)

def _pushed(off, xy, delta, d):
    o, s, _, seg = O.resample(off, xy, delta, want_seg=True)
    return o, s, seg, O.directed_offset(off, xy, o, seg, s, d)


def test_directed_offset_straight_edges_closed_form():
    # the same horizontal edge in both directions: the interior samples of the rightward
    # edge move to y + d (left normal of +x is +y), those of the leftward one to y - d
    off = np.array([0, 2, 4], np.int64)
    xy = np.array([[10.25, 20.5], [110.25, 20.5], [110.25, 20.5], [10.25, 20.5]])
    d = 2.5
    o, s, seg, out = _pushed(off, xy, 1.0, d)
    assert o[1] == 101 and o[2] == 202
    a, b = out[:101], out[101:]
    np.testing.assert_array_equal(a[1:-1, 1], 20.5 + d)
    np.testing.assert_array_equal(b[1:-1, 1], 20.5 - d)
    np.testing.assert_allclose(a[:, 0], 10.25 + np.arange(101), atol=1e-12)
    np.testing.assert_allclose(b[:, 0], 110.25 - np.arange(101), atol=1e-12)
    # the two directions part by 2|d|; end points stay
    assert np.all(a[1:-1, 1] - b[::-1][1:-1, 1] == 2 * d)
    np.testing.assert_array_equal(out[[0, 100, 101, 201]], xy[[0, 1, 2, 3]])


def test_directed_offset_distance_side_and_identity_on_random_polylines():
    g = rng(21)
    polys = [np.cumsum(g.normal(0, 3, (int(m), 2)), 0) + 100 for m in g.integers(2, 40, 60)]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])]).astype(np.int64)
    xy = np.concatenate(polys)
    d = -1.75
    o, s, seg, out = _pushed(off, xy, 1.0, d)
    np.testing.assert_array_equal(O.directed_offset(off, xy, o, seg, s, 0.0), s)
    interior = np.ones(len(s), bool)
    interior[o[:-1]] = False
    interior[o[1:] - 1] = False
    np.testing.assert_array_equal(out[~interior], s[~interior])
    # every interior sample moved by |d|, perpendicular to its segment, on the side given
    # by the sign of d (cross product of the segment direction and the move)
    eid = np.repeat(np.arange(len(polys)), np.diff(o))[interior]
    j = seg[interior]
    p0 = xy[off[eid] + j]
    p1 = xy[off[eid] + j + 1]
    e = p1 - p0
    mv = out[interior] - s[interior]
    np.testing.assert_allclose(np.hypot(mv[:, 0], mv[:, 1]), abs(d), atol=1e-12)
    ln = np.hypot(e[:, 0], e[:, 1])
    np.testing.assert_allclose((e[:, 0] * mv[:, 1] - e[:, 1] * mv[:, 0]) / ln, d, atol=1e-12)
    np.testing.assert_allclose((e[:, 0] * mv[:, 0] + e[:, 1] * mv[:, 1]) / ln, 0.0, atol=1e-12)


def test_directed_offset_commutes_with_quarter_turn():
    g = rng(22)
    polys = [np.cumsum(g.normal(0, 4, (int(m), 2)), 0) for m in g.integers(2, 20, 30)]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])]).astype(np.int64)
    xy = np.concatenate(polys)
    turn = lambda a: np.stack([-a[:, 1], a[:, 0]], 1)     # exact 90-degree rotation
    o, s, seg, out = _pushed(off, xy, 1.0, 0.8)
    o2, s2, seg2, out2 = _pushed(off, turn(xy), 1.0, 0.8)
    np.testing.assert_array_equal(o, o2)
    np.testing.assert_allclose(out2, turn(out), atol=1e-9)


def test_directed_run_keeps_opposite_edges_mirrored():
    # two copies of one edge in opposite directions: pushed to opposite sides, then
    # advected in a density that is symmetric about their common line, so the two final
    # polylines are mirror images of each other about that line
    W = 64
    p = _params(W, [4], directed_offset=1.25)   # pushed rows stay off pixel borders
    node = np.array([[10.25 / W, 30.5 / W], [50.75 / W, 30.5 / W]], np.float32)
    off, xy, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                       np.ones((1, 1)), p, 3)
    a, b = xy[off[0]:off[1]], xy[off[1]:off[2]][::-1]
    assert len(a) == len(b)
    np.testing.assert_allclose(a[:, 0], b[:, 0], atol=1e-9)
    np.testing.assert_allclose(a[:, 1] + b[:, 1], 61.0, atol=1e-9)
    assert (a[1:-1, 1] != 30.5).any()
    # with no push the two copies coincide and stay on the row
    off0, xy0, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                         np.ones((1, 1)), _params(W, [4]), 3)
    np.testing.assert_array_equal(xy0[:, 1], 30.5)


@pytest.mark.parametrize("every", [False, True])
def test_directed_push_once_or_every_iteration(every):
    # Section 3's pipeline pushes once after the first sampling and then loops from the
    # resampling, which interpolates along the pushed polyline and so keeps the offset.
    # With the advection made negligible (h = 1e-12 px) and no Laplacian smoothing, the
    # middle of a straight horizontal edge therefore sits at exactly |d| from its line after
    # any number of iterations, and its reversed copy at -d: the two part by 2|d|, once.
    # Pushing after every resampling instead stacks the offsets: T|d| after T iterations.
    W, T, d = 128, 4, 0.75
    p = _params(W, [4], directed_offset=d, h_max=1e-12, smooth_weight=0.0,
                directed_every=every)
    node = np.array([[8.25 / W, 60.5 / W], [120.25 / W, 60.5 / W]], np.float32)
    off, xy, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                       np.ones((1, 1)), p, T)
    a, b = xy[off[0]:off[1]], xy[off[1]:off[2]]
    k = T if every else 1
    mid_a = np.abs(a[:, 0] - 64.0) < 30.0
    mid_b = np.abs(b[:, 0] - 64.0) < 30.0
    np.testing.assert_allclose(a[mid_a, 1] - 60.5, k * d, atol=1e-9)
    np.testing.assert_allclose(b[mid_b, 1] - 60.5, -k * d, atol=1e-9)
    # the interior never goes past the middle's offset; the end points stay
    assert np.abs(a[1:-1, 1] - 60.5).max() <= k * d + 1e-9
    np.testing.assert_array_equal(a[[0, -1], 1], 60.5)
    np.testing.assert_array_equal(b[[0, -1], 1], 60.5)
    # one iteration is the same in both readings (the first sampling is pushed)
    p1 = _params(W, [4], directed_offset=d, h_max=1e-12, smooth_weight=0.0,
                 directed_every=not every)
    o1, x1, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                      np.ones((1, 1)), p1, 1)
    o2, x2, _ = O.run(node, np.array([0, 1]), np.array([1, 0]), np.zeros(2, np.int32),
                      np.ones((1, 1)), p, 1)
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_array_equal(x1, x2)


# ------------------------------------------------------------------ orientation bins (Sec. 5)

def test_orientation_axes_diagonals_and_zero():
    dirs = np.array([[1, 0], [1, 1], [0, 1], [-1, 1], [-1, 0], [-1, -1], [0, -1], [1, -1],
                     [0, 0], [3.5, 0], [0, 0.25]], np.float64)
    # slices [90k - 45, 90k + 45): 45 -> 1, 135 -> 2, 225 -> 3, 315 -> 0
    np.testing.assert_array_equal(O.orientation(dirs), [0, 1, 1, 2, 2, 3, 3, 0, 0, 0, 1])


def test_orientation_matches_atan2_and_quarter_turns():
    g = rng(23)
    v = g.normal(0, 1, (20000, 2)) * g.choice([1e-3, 1.0, 1e3], (20000, 1))
    ang = np.degrees(np.arctan2(v[:, 1], v[:, 0])) % 360.0
    away = np.abs(((ang + 45.0) % 90.0) - 45.0) > 1e-6      # not within 1e-6 deg of a border
    ref = (np.floor((ang + 45.0) / 90.0).astype(np.int64) % 4)
    got = O.orientation(v)
    np.testing.assert_array_equal(got[away], ref[away])
    assert away.mean() > 0.999
    turn = np.stack([-v[:, 1], v[:, 0]], 1)                  # +90 degrees, exact
    np.testing.assert_array_equal(O.orientation(turn), (got + 1) % 4)
    np.testing.assert_array_equal(O.orientation(-v), (got + 2) % 4)


# ------------------------------------------------------------------ line-strip splat (Eq. 1 drawn)

def _textbook_bresenham(x0, y0, x1, y1):
    """All-octant integer Bresenham (error accumulator), both end pixels included."""
    dx, dy = abs(x1 - x0), -abs(y1 - y0)
    sx, sy = (1 if x0 < x1 else -1), (1 if y0 < y1 else -1)
    err = dx + dy
    pts = []
    while True:
        pts.append((x0, y0))
        if x0 == x1 and y0 == y1:
            return pts
        e2 = 2 * err
        if e2 >= dy:
            err += dy
            x0 += sx
        if e2 <= dx:
            err += dx
            y0 += sy


def _strip_pixels(p0, p1, W=64, H=64):
    off = np.array([0, 2], np.int64)
    xy = np.array([p0, p1], np.float64) + 0.5          # pixel centres
    h = O.splat_strip(off, xy, np.zeros(1, np.int32), 1, W, H)[0]
    v, u = np.nonzero(h)
    return h, set(zip(u.tolist(), v.tolist()))


def test_strip_segments_match_textbook_bresenham_without_ties():
    g = rng(31)
    checked = 0
    for _ in range(400):
        x0, y0, x1, y1 = (int(c) for c in g.integers(0, 64, 4))
        n = max(abs(x1 - x0), abs(y1 - y0))
        minor = abs(y1 - y0) if abs(x1 - x0) >= abs(y1 - y0) else abs(x1 - x0)
        # a rounding tie: t * minor / n at exactly half an integer for some t
        if n and any((2 * t * minor) % (2 * n) == n for t in range(n)):
            continue
        h, got = _strip_pixels((x0, y0), (x1, y1))
        ref = _textbook_bresenham(x0, y0, x1, y1)
        assert got == set(ref)
        assert h.sum() == len(ref) == n + 1 and h.max() == 1
        checked += 1
    assert checked > 200


def test_strip_is_connected_and_counts_each_drawn_pixel():
    g = rng(32)
    for _ in range(100):
        x0, y0, x1, y1 = (int(c) for c in g.integers(0, 64, 4))
        h, got = _strip_pixels((x0, y0), (x1, y1))
        n = max(abs(x1 - x0), abs(y1 - y0))
        assert h.sum() == n + 1 and (x0, y0) in got and (x1, y1) in got
        # 8-connected digital line: one pixel per step of the major coordinate
        major = 0 if abs(x1 - x0) >= abs(y1 - y0) else 1
        coords = sorted(got, key=lambda q: q[major] * (1 if (x1 - x0, y1 - y0)[major] >= 0 else -1))
        for a, b in zip(coords, coords[1:]):
            assert abs(a[0] - b[0]) <= 1 and abs(a[1] - b[1]) <= 1 and abs(a[major] - b[major]) == 1


def test_strip_mass_and_dominates_point_splat():
    g = rng(33)
    W, H, B, E = 48, 40, 3, 120
    off, xy, group = _random_points(g, E, W, H, B)
    weight = g.integers(1, 5, E).astype(np.int32)
    hs = O.splat_strip(off, xy, group, B, W, H, weight)
    hp = O.splat(off, xy, group, B, W, H, weight)
    u = np.clip(np.floor(xy[:, 0]), 0, W - 1).astype(np.int64)
    v = np.clip(np.floor(xy[:, 1]), 0, H - 1).astype(np.int64)
    mass = 0
    for e in range(E):
        du, dv = np.diff(u[off[e]:off[e + 1]]), np.diff(v[off[e]:off[e + 1]])
        mass += int(weight[e]) * (1 + int(np.maximum(np.abs(du), np.abs(dv)).sum()))
    assert hs.sum() == mass
    # every point's pixel is drawn (segments start on it, the strip ends on the last one);
    # points sharing a pixel with their predecessor draw it once
    E_ids = np.repeat(np.arange(E), np.diff(off))
    first = np.ones(len(xy), bool)
    same = (u[1:] == u[:-1]) & (v[1:] == v[:-1]) & (E_ids[1:] == E_ids[:-1])
    first[1:] = ~same
    hp_runs = np.zeros_like(hp)
    np.add.at(hp_runs, (group[E_ids[first]], v[first], u[first]), weight[E_ids[first]])
    assert (hs >= hp_runs).all()


def test_strip_straight_row_closed_form():
    off = np.array([0, 3], np.int64)
    xy = np.array([[2.5, 7.25], [9.75, 7.5], [20.1, 7.9]])
    h = O.splat_strip(off, xy, np.zeros(1, np.int32), 1, 32, 16)[0]
    ref = np.zeros((16, 32), np.int64)
    ref[7, 2:21] = 1
    np.testing.assert_array_equal(h, ref)
    # a fold: the strip goes right and back, so pixels between the turns count twice
    xy2 = np.array([[2.5, 3.5], [10.5, 3.5], [5.5, 3.5]])
    h2 = O.splat_strip(off, xy2, np.zeros(1, np.int32), 1, 32, 16)[0]
    ref2 = np.zeros((16, 32), np.int64)
    ref2[3, 2:11] += 1          # 2..9 from the first segment, 10 starts the second
    ref2[3, 6:10] += 1          # 10 -> 6 drawn by the second segment (10 already counted)
    ref2[3, 5] += 1             # the last point
    np.testing.assert_array_equal(h2, ref2)


# ------------------------------------------------------------------ grouping (Sec. 5)

def _blobs(seed, k, n_per, dim, spread=0.02):
    g = rng(seed)
    centres = g.uniform(0.1, 0.9, (k, dim))
    X = np.concatenate([c + spread * g.normal(size=(n_per, dim)) for c in centres])
    return X[g.permutation(len(X))].astype(np.float32)


@pytest.mark.parametrize("k,dim,seed", [(4, 2, 41), (8, 4, 42), (5, 1, 43)])
def test_kmeans_matches_sklearn_lloyd(k, dim, seed):
    import sklearn.cluster
    X = _blobs(seed, k + 2, 300, dim, spread=0.05)
    init = X[O.init_indices(seed, k, 0, len(X))].astype(np.float64)
    labels, cen, inertia, rounds = O.kmeans(X, init, max_iters=300)
    km = sklearn.cluster.KMeans(n_clusters=k, init=init, n_init=1, algorithm="lloyd",
                                max_iter=300, tol=0.0).fit(X.astype(np.float64))
    assert rounds < 300
    np.testing.assert_array_equal(labels, km.labels_)
    np.testing.assert_allclose(cen, km.cluster_centers_, rtol=1e-10, atol=1e-12)
    assert abs(inertia - km.inertia_) <= 1e-9 * km.inertia_


def test_kmeans_fixed_point_and_permutation():
    X = _blobs(44, 6, 120, 2, spread=0.08)
    init = X[:6].astype(np.float64)
    labels, cen, inertia, _ = O.kmeans(X, init, max_iters=500)
    # a converged Lloyd run: every point is nearest to its own centre, every centre the mean
    d = ((X[:, None, :].astype(np.float64) - cen[None]) ** 2).sum(2)
    np.testing.assert_array_equal(labels, d.argmin(1))
    for c in range(6):
        np.testing.assert_allclose(cen[c], X[labels == c].astype(np.float64).mean(0), rtol=1e-12)
    assert abs(inertia - d.min(1).sum()) <= 1e-12 * inertia
    perm = rng(45).permutation(len(X))
    l2, c2, i2, _ = O.kmeans(X[perm], init, max_iters=500)
    np.testing.assert_array_equal(l2, labels[perm])
    np.testing.assert_allclose(c2, cen, rtol=1e-12)


@pytest.mark.parametrize("k,dim,seed", [(3, 2, 46), (7, 4, 47)])
def test_davies_bouldin_matches_sklearn(k, dim, seed):
    import sklearn.metrics
    X = _blobs(seed, k, 200, dim, spread=0.07)
    labels = rng(seed).integers(0, k, len(X)).astype(np.int32)
    ref = sklearn.metrics.davies_bouldin_score(X.astype(np.float64), labels)
    assert abs(O.davies_bouldin(X, labels, k) - ref) <= 1e-10 * ref
    l, _, _, _ = O.kmeans(X, X[O.init_indices(seed, k, 0, len(X))], max_iters=300)
    ref = sklearn.metrics.davies_bouldin_score(X.astype(np.float64), l)
    assert abs(O.davies_bouldin(X, l, k) - ref) <= 1e-10 * ref


def test_draw_is_splitmix64_and_init_indices_distinct():
    # SplitMix64 reference values: the published generator seeded with 0 (state advanced by
    # the golden gamma before each output) produces these first outputs
    ref = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [O.draw(0, 0, -1, 4096 + t) for t in range(3)] == ref
    idx = O.init_indices(123, 16, 7, 20)
    assert len(set(idx.tolist())) == 16 and idx.min() >= 0 and idx.max() < 20


def test_choose_groups_finds_separated_blobs():
    X = _blobs(48, 6, 150, 2, spread=0.01)
    B, labels, db = O.choose_groups(X, kmin=4, kmax=9, restarts=100, seed=3, max_iters=200)
    assert B == 6
    assert db.argmin() == 6 - 4 and len(np.unique(labels)) == 6


# ------------------------------------------------------------------ insert/delete resampling

def test_insdel_closed_forms():
    off = np.array([0, 4, 8], np.int64)
    xy = np.array([[0, 0], [0.2, 0], [0.5, 0], [3.0, 0],       # 0.2 and 0.5 too close: removed
                   [0, 1], [0.7, 1], [2.9, 1], [3.0, 1]], np.float64)   # 2.9 -> 3.0 too close
    o, s = O.resample_insdel(off, xy, 0.5, 1.0)
    np.testing.assert_array_equal(o, [0, 4, 10])
    np.testing.assert_allclose(s[:4], [[0, 0], [1, 0], [2, 0], [3, 0]], atol=1e-15)
    # kept 0, 0.7, 3.0 (2.9 is 2.2 from 0.7: kept too), gaps 0.7 (1 part), 2.2 (3 parts), 0.1
    o2, s2 = O.resample_insdel(np.array([0, 4], np.int64), xy[4:], 0.5, 1.0)
    exp = [0.0, 0.7, 0.7 + 2.2 / 3, 0.7 + 4.4 / 3, 2.9, 3.0]
    np.testing.assert_allclose(s2[:, 0], exp, atol=1e-12)
    np.testing.assert_array_equal(s2[:, 1], 1.0)


def test_insdel_invariants_on_random_polylines():
    g = rng(51)
    polys = [np.cumsum(g.normal(0, 1.2, (int(m), 2)), 0) + 50 for m in g.integers(2, 60, 80)]
    off = np.concatenate([[0], np.cumsum([len(p) for p in polys])]).astype(np.int64)
    xy = np.concatenate(polys)
    dmin, dmax = 0.5, 1.0
    o, s = O.resample_insdel(off, xy, dmin, dmax)
    for e, p in enumerate(polys):
        q = s[o[e]:o[e + 1]]
        np.testing.assert_array_equal(q[0], p[0])
        np.testing.assert_array_equal(q[-1], p[-1])
        gaps = np.hypot(*np.diff(q, axis=0).T)
        assert (gaps <= dmax * (1 + 1e-12)).all()
        # kept points: the interior input points at least dmin from their predecessor
        dpred = np.hypot(*np.diff(p, axis=0).T)
        kept = set(map(tuple, p[1:-1][dpred[:-1] >= dmin].tolist()))
        out = set(map(tuple, q.tolist()))
        assert kept <= out
        removed = p[1:-1][dpred[:-1] < dmin]
        for r in removed:
            assert tuple(r.tolist()) not in out or tuple(r.tolist()) in kept


def test_insdel_fixed_point_and_two_point_edges():
    # a uniform polyline with spacing in [dmin, dmax] is unchanged
    t = np.arange(0, 41) * 0.8
    p = np.stack([10 + 0.6 * t, 20 + 0.8 * t], 1)
    o, s = O.resample_insdel(np.array([0, 41], np.int64), p, 0.5, 1.0)
    np.testing.assert_array_equal(s, p)
    # straight two-point edges: the uniform resampling with delta = dmax
    g = rng(52)
    ends = g.uniform(0, 200, (30, 2, 2))
    off = np.arange(0, 61, 2).astype(np.int64)
    xy = ends.reshape(-1, 2)
    o1, s1 = O.resample_insdel(off, xy, 0.5, 1.0)
    o2, s2, _ = O.resample(off, xy, 1.0)
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_allclose(s1, s2, atol=1e-9)


# ------------------------------------------------------------------ box widths for a real sigma

@pytest.mark.parametrize("P", [2, 3, 4])
def test_kovesi_radii_equal_when_sigma_is_reachable(P):
    for r in range(1, 41):
        s = math.sqrt(P * r * (r + 1) / 3.0)
        assert O.kovesi_radii(s, P) == [r] * P


@pytest.mark.parametrize("P", [3, 4])
def test_kovesi_radii_closest_two_width_mix(P):
    for sig in np.linspace(1.0, 60.0, 237):
        rr = O.kovesi_radii(sig, P)
        assert rr == sorted(rr) and max(rr) - min(rr) <= 1
        ach = sum(r * (r + 1) / 3.0 for r in rr)
        rl = min(rr)
        # brute force over the mixes of radius rl and rl + 1 (m passes of rl first)
        best = min(abs(m * rl * (rl + 1) / 3.0 + (P - m) * (rl + 1) * (rl + 2) / 3.0 - sig * sig)
                   for m in range(P + 1))
        assert abs(ach - sig * sig) <= best + 1e-9
        assert abs(math.sqrt(ach) - sig) <= 0.08 * sig + 0.6


def test_box_chain_radii_impulse_variance_and_scipy():
    W = H = 101
    h = np.zeros((1, H, W), np.int64)
    h[0, 50, 50] = 1
    rr = [3, 4, 4]
    S = O.box_chain_radii(h, rr)
    out = S[-1, 0].astype(np.float64)
    assert out.sum() == np.prod([(2 * r + 1) ** 2 for r in rr])
    u = np.arange(W) - 50
    var = (out.sum(0) * u * u).sum() / out.sum()
    assert abs(var - sum(r * (r + 1) / 3.0 for r in rr)) < 1e-9
    g = rng(61)
    m = g.integers(0, 5, (1, 37, 45)).astype(np.int64)
    S2 = O.box_chain_radii(m, [1, 2, 3])
    ref = m[0].astype(np.float64)
    for k, r in enumerate([1, 2, 3]):
        ref = scipy.signal.convolve2d(ref, np.ones((2 * r + 1, 2 * r + 1)), mode="same")
        np.testing.assert_array_equal(S2[k, 0], np.rint(ref).astype(np.int64))
    np.testing.assert_array_equal(O.box_chain_radii(m, [2, 2, 2]), O.box_chain(m, 3, 2))
    a = np.array([0.2, 0.3, 0.5])
    M = np.ones((1, 1))
    np.testing.assert_allclose(O.density_radii(O.box_chain(m, 3, 2), [2, 2, 2], a, M),
                               O.density(O.box_chain(m, 3, 2), 2, a, M), rtol=1e-15)


# ------------------------------------------------------------------ width encoding (Sec. 3.4)

def test_point_widths_closed_form_on_a_linear_map():
    W, H = 40, 30
    u = np.arange(W) + 0.5
    rho = np.broadcast_to(0.25 * u[None, :], (H, W)).astype(np.float64)[None].copy()
    off = np.array([0, 5], np.int64)
    xy = np.array([[2.0, 5.0], [10.0, 7.5], [20.25, 9.0], [30.5, 3.0], [39.5, 12.0]])
    dens, w = O.point_widths(off, xy, np.zeros(1, np.int32), rho, 1.0, 5.0)
    # bilinear on a linear map is exact inside; the last point clamps to the border column
    np.testing.assert_allclose(dens, 0.25 * np.minimum(xy[:, 0], W - 0.5), rtol=1e-12)
    np.testing.assert_allclose(w, 1.0 + 4.0 * dens / dens.max(), rtol=1e-12)
    assert w.max() == 5.0
    dl, wl = O.point_widths(off, xy, np.zeros(1, np.int32), rho, 1.0, 5.0, log_scale=True)
    np.testing.assert_allclose(wl, 1.0 + 4.0 * np.log1p(dens) / np.log1p(dens.max()), rtol=1e-12)
    # the log scale lifts the small densities, keeps the order and the end values
    assert (np.diff(wl[np.argsort(dens)]) >= 0).all() and (wl >= w - 1e-12).all()


def test_point_widths_zero_and_negative_density():
    rho = -np.ones((2, 8, 8))
    rho[1, 4, 4] = 3.0
    off = np.array([0, 2, 4], np.int64)
    xy = np.array([[4.5, 4.5], [1.5, 1.5], [4.5, 4.5], [0.5, 7.5]])
    dens, w = O.point_widths(off, xy, np.array([0, 1], np.int32), rho, 0.5, 2.0)
    np.testing.assert_array_equal(dens, [0.0, 0.0, 3.0, 0.0])
    np.testing.assert_array_equal(w, [0.5, 0.5, 2.0, 0.5])
    d0, w0 = O.point_widths(off, xy, np.array([0, 0], np.int32), rho, 0.5, 2.0)
    np.testing.assert_array_equal(w0, 0.5)
