"""GPU-vs-oracle parity of the box chain for a real sigma (P passes of two odd widths by
Kovesi's rule, one radius per pass): the int64 box passes are bit-exact, the density within
the usual 1e-5 relative bound, multi-iteration runs within 1 %."""

import math

import numpy as np
import pytest

import oracle as O
import workloads
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("E,W,H,B,sig,seed", [(1500, 100, 72, 3, 3.7, 81), (600, 257, 130, 1, 9.1, 82),
                                               (800, 64, 64, 2, 1.2, 83)])
def test_sigma_stage_parity_given_samples(hb, E, W, H, B, sig, seed):
    rng = np.random.default_rng(seed)
    off, xy = PT.random_polylines(rng, E, W, H)
    group = rng.integers(0, B, E).astype(np.int32)
    M = workloads.interaction_eq4(B, 0.25) if B > 1 else np.ones((1, 1), np.float32)
    rr = O.kovesi_radii(sig, 3)
    assert len(set(rr)) > 1                         # two widths (one of radius 0 for 1.2)
    with hb.Bundler(0) as b:
        b.set_params(W, H, [1], sigmas=[sig])
        nodes = rng.random((16, 2)).astype(np.float32)
        b.set_graph(nodes, rng.integers(0, 16, E).astype(np.int32), rng.integers(0, 16, E).astype(np.int32))
        b.set_groups(group, M)
        b.set_points(off, xy)
        b.run(1, hb.HB_RUN_SAMPLES_GIVEN)
        hist = np.stack([b.map(hb.HB_MAP_HIST, g) for g in range(B)]).astype(np.int64)
        S = np.stack([np.stack([b.map(hb.HB_MAP_BOX, g, k + 1) for g in range(B)]) for k in range(3)])
        rho = np.stack([b.map(hb.HB_MAP_DENSITY, g) for g in range(B)]).astype(np.float64)
    ref_h = O.splat(off, xy.astype(np.float64), group, B, W, H)
    np.testing.assert_array_equal(hist, ref_h)
    ref_S = O.box_chain_radii(ref_h, rr)
    np.testing.assert_array_equal(S, ref_S)
    a = np.array([0.0, 0.0, 1.0])
    ref_rho = O.density_radii(ref_S, rr, a, M.astype(np.float64))
    c = np.cumprod([(2 * r + 1) ** 2 for r in rr]).astype(np.float64)
    bound = 1e-5 * np.tensordot(np.abs(M.astype(np.float64)), ref_S[2].astype(np.float64) / c[2], 1) + 1e-300
    assert (np.abs(rho - ref_rho) <= bound).all()


def test_sigma_end_to_end_tiny(hb):
    """The tiny workload with a real sigma schedule (10 px decaying to 5 px), 6 iterations."""
    w = workloads.tiny()
    n_iters = 6
    sig = [10.0 * 0.5 ** (i / 5.0) for i in range(n_iters)]
    with hb.Bundler(0) as b:
        b.set_params(w.grid_w, w.grid_h, w.radii, delta=w.delta, passes=w.passes, lam=w.lam,
                     bbox=w.bbox, sigmas=sig)
        b.set_graph(w.node_xy, w.src, w.dst, w.weight)
        b.set_groups(w.group, w.M)
        b.run(n_iters)
        counts = b.iter_counts(n_iters)
        off, xy = b.points(hb.HB_POINTS_STATE)
        ink = b.ink()
    p = O.params_for(w)
    p.sigmas = sig
    roff, rxy, rcounts = O.run(w.node_xy, w.src, w.dst, w.group, w.M, p, n_iters)
    assert PT.relclose(ink, O.ink(roff, rxy), 0.01)
    for a, b_ in zip(counts, rcounts):
        assert PT.relclose(a, b_, 0.01)
    ds, dr = PT.drift_stats(off, xy), PT.drift_stats(roff, rxy)
    for k in ("mean", "p50", "p90", "p99"):
        assert abs(ds[k] - dr[k]) <= 0.01 * dr[k], (k, ds[k], dr[k])


def test_sigma_rejected_by_checkpointed_forward(hb):
    w = workloads.scaled("uniform", n_edges=200, grid=64, groups=1, n_iters=2, seed=5)
    with hb.Bundler(0) as b:
        b.set_workload(w, sigmas=[2.2])
        with pytest.raises(hb.HBError) as ei:
            hb.hb_forward_ckpt(b.ctx, 1)
        assert ei.value.status == hb.HB_EINVAL
        b.run(1)
