"""Comparison helpers for GPU-vs-oracle parity tests (test code; no method arithmetic
beyond what a check needs)."""

import numpy as np

import oracle as O

F32_ULP_AT = lambda x: np.spacing(np.abs(np.asarray(x, np.float32)).astype(np.float32)).astype(np.float64)


def random_polylines(rng, E, W, H, n_min=2, n_max=150, step=1.5):
    """Random-walk polylines inside [0, W) x [0, H) as float32 (sample sets or states)."""
    counts = rng.integers(n_min, n_max + 1, E)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    pts = []
    for c in counts:
        start = rng.uniform([2, 2], [W - 2, H - 2])
        walk = start + np.cumsum(rng.normal(0, step, (c, 2)), 0)
        walk[:, 0] = np.clip(walk[:, 0], 0.0, W - 1e-3)
        walk[:, 1] = np.clip(walk[:, 1], 0.0, H - 1e-3)
        pts.append(walk)
    xy = np.concatenate(pts).astype(np.float32)
    return off, xy


def near_pixel_edge(xy, tol=1e-4):
    f = np.abs(xy - np.round(xy))
    return (f < tol).any(axis=1)


def acceptable(g, jacc, jfirm, amb):
    """True where the GPU's halving index g is one of the valid outcomes of the oracle's
    decision: the oracle's own, any try whose density margin is within the ambiguity band
    before the first unambiguous acceptance, or that acceptance (no move if none)."""
    g = g.astype(np.int64)
    ok = g == jacc
    bit = np.where(g >= 0, (amb.astype(np.int64) >> np.clip(g, 0, 31)) & 1, 0).astype(bool)
    ok |= (g >= 0) & bit & ((jfirm < 0) | (g < jfirm))
    ok |= (g == jfirm)
    return ok


def candidate(x, d, h, j, W, H):
    """Position after an accepted try j (-1: no move), clamped like the method."""
    x = np.asarray(x, np.float64)
    m = np.where(j >= 0, h * np.exp2(-np.maximum(j, 0).astype(np.float64)), 0.0)
    c = x + m[:, None] * d
    c[:, 0] = np.clip(c[:, 0], 0.0, W - 1.0 / 256)
    c[:, 1] = np.clip(c[:, 1], 0.0, H - 1.0 / 256)
    return np.where((j >= 0)[:, None], c, x)


def laplace(off, xa, s=0.5):
    y = xa.copy()
    E = len(off) - 1
    interior = np.ones(len(xa), bool)
    interior[off[:-1]] = False
    interior[off[1:] - 1] = False
    idx = np.nonzero(interior)[0]
    y[idx] = (1 - s) * xa[idx] + 0.5 * s * (xa[idx - 1] + xa[idx + 1])
    return y


def interp_condition(grad, group, off, xy):
    """Condition number of the bilinear gradient direction at each point of the polylines
    (off, xy) in its edge's layer (see direction_condition)."""
    eid = np.repeat(np.arange(len(off) - 1), np.diff(off))
    return direction_condition(grad, np.asarray(group)[eid], xy)


def direction_condition(grad, lay, xy):
    """Condition number of the bilinear gradient direction at the points xy of layers lay:
    sum_i w_i |g_i| / |sum_i w_i g_i| (inf where the gradient vanishes)."""
    B, H, W, _ = grad.shape
    xy = np.asarray(xy, np.float64)
    fx = np.clip(xy[:, 0] - 0.5, -1, W)
    fy = np.clip(xy[:, 1] - 0.5, -1, H)
    u0 = np.floor(fx).astype(np.int64)
    v0 = np.floor(fy).astype(np.int64)
    tx, ty = fx - u0, fy - v0
    uu = [np.clip(u0, 0, W - 1), np.clip(u0 + 1, 0, W - 1)]
    vv = [np.clip(v0, 0, H - 1), np.clip(v0 + 1, 0, H - 1)]
    flat = grad.reshape(-1, 2)
    base = np.asarray(lay, np.int64) * H
    num = np.zeros(len(xy))
    vec = np.zeros((len(xy), 2))
    for w, a, b in (((1 - tx) * (1 - ty), 0, 0), (tx * (1 - ty), 1, 0), ((1 - tx) * ty, 0, 1),
                    (tx * ty, 1, 1)):
        gv = flat[(base + vv[b]) * W + uu[a]]
        num += w * np.abs(gv).sum(1)
        vec += w[:, None] * gv
    den = np.abs(vec).sum(1)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, num / den, np.inf)


def drift_stats(off, xy, n_ref=32):
    """Per edge: resample to n_ref points by arclength; drift = distance to the matching point
    of the straight segment between the end points. Returns mean, p50, p90, p99."""
    E = len(off) - 1
    drifts = []
    for e in range(E):
        p = np.asarray(xy[off[e]:off[e + 1]], np.float64)
        seg = np.hypot(*np.diff(p, axis=0).T)
        C = np.concatenate([[0.0], np.cumsum(seg)])
        if C[-1] <= 0:
            continue
        s = np.linspace(0, C[-1], n_ref)
        q = np.stack([np.interp(s, C, p[:, 0]), np.interp(s, C, p[:, 1])], 1)
        t = np.linspace(0, 1, n_ref)[:, None]
        straight = p[0] + t * (p[-1] - p[0])
        drifts.append(np.hypot(*(q - straight).T))
    d = np.concatenate(drifts) if drifts else np.zeros(1)
    return {"mean": d.mean(), "p50": np.percentile(d, 50), "p90": np.percentile(d, 90),
            "p99": np.percentile(d, 99)}


def relclose(a, b, rel):
    return abs(a - b) <= rel * max(abs(a), abs(b), 1e-12)


def check_stage(ref, p, off, xy, group, M, maps, jacc, xy_n, agree_min=0.99):
    """One iteration from the samples (off, xy) against the oracle's record ``ref`` of the
    same iteration (O.iterate with skip_resample): histograms and box sums bit-exact, the
    density within 1e-5 of sum_b |M[l][b]| Sbar_b, the gradient within 1e-6 of the layer's
    density scale, halving decisions equal or valid within the ambiguity band, new positions
    within 1e-4 px + 2 FP32 ulps + the conditioning of the interpolated direction (points
    whose own and neighbours' decisions agree), the others within the same bound of the
    oracle replaying the GPU's valid decisions, end points bit-exact."""
    hist, S, rho, grad = maps
    W, H = p.grid_w, p.grid_h
    P = len(S)
    np.testing.assert_array_equal(hist, ref["hist"])
    np.testing.assert_array_equal(S, ref["S"])
    aw = p.a()
    r = ref["r"]
    c = float((2 * r + 1) ** 2)
    Sbar = sum(aw[k] * ref["S"][k].astype(np.float64) / c ** (k + 1) for k in range(P))
    bound = 1e-5 * np.tensordot(np.abs(np.asarray(M, np.float64)), Sbar, 1) + 1e-300
    assert (np.abs(rho - ref["rho"]) <= bound).all()
    scale = np.abs(ref["rho"]).max(axis=(1, 2))[:, None, None, None]
    assert (np.abs(grad - ref["grad"]) <= 1e-6 * scale + 1e-6 * np.abs(ref["grad"])).all()
    adv = ref["adv"]
    ok = acceptable(jacc, adv["jacc"], adv["jfirm"], adv["amb"])
    assert ok.all(), f"{(~ok).sum()} invalid decisions"
    agree = jacc == adv["jacc"]
    assert agree.mean() > agree_min, agree.mean()
    x64 = xy.astype(np.float64)
    h = ref["h"]
    cond = interp_condition(ref["grad"], group, off, x64)
    tdir = np.where(np.isfinite(cond), h * 1e-6 * cond, 0.0)
    tpt = 1e-4 + tdir + 2 * F32_ULP_AT(xy_n).max(1)
    ty = tpt.copy()
    ty[1:-1] = 0.5 * tpt[1:-1] + 0.25 * (tpt[:-2] + tpt[2:])
    nb = agree.copy()
    nb[1:] &= agree[:-1]
    nb[:-1] &= agree[1:]
    err = np.abs(xy_n.astype(np.float64) - ref["xy"]).max(1)
    assert (err[nb] <= ty[nb]).all(), f"max err {err[nb].max()} px"
    assert np.percentile(err[nb], 99) <= 1e-4, np.percentile(err[nb], 99)
    jj = np.where(jacc == -2, -1, jacc)
    yalt = laplace(off, candidate(x64, adv["dir"], h, jj, W, H))
    erra = np.abs(xy_n.astype(np.float64) - yalt).max(1)
    assert (erra[~nb] <= ty[~nb]).all()
    ends = np.concatenate([off[:-1], off[1:] - 1])
    np.testing.assert_array_equal(xy_n[ends], xy[ends])
