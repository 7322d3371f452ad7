"""The allocation-free Davies-Bouldin entry point against hb_davies_bouldin: two calls in a
row on one context (the second on fewer points, fewer clusters and another dimension, so the
shared scratch array holds the first call's values when the second starts), device inputs,
indices equal within 1e-10 relative (FP64 sums in another fixed order); out-of-range labels
rejected."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(seed, n, dim, k):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0, 500, (k, dim))
    lab = rng.integers(0, k, n)
    X = (centres[lab] + rng.normal(0, 20, (n, dim))).astype(np.float32)
    return X, lab.astype(np.int32)


def test_noalloc_davies_bouldin_matches_allocating_call(hb):
    import torch
    dev = torch.device("cuda:0")
    with hb.Bundler(0) as b:
        for seed, n, dim, k in [(1, 70001, 4, 16), (2, 3001, 2, 5)]:
            print(f"noalloc case seed={seed} n={n} dim={dim} k={k}", flush=True)
            X, lab = _case(seed, n, dim, k)
            Xd = torch.from_numpy(X).to(dev)
            ld = torch.from_numpy(lab).to(dev)
            got = hb.hb_davies_bouldin_noalloc(b.ctx, Xd, ld, k)
            ref = hb.hb_davies_bouldin(b.ctx, Xd, ld, k)
            ref_host = hb.hb_davies_bouldin(b.ctx, X, lab, k)
            assert ref == ref_host
            assert got > 0
            assert abs(got - ref) <= 1e-10 * abs(ref), (got, ref)
        bad = ld.clone()
        bad[17] = k
        with pytest.raises(hb.HBError) as ei:
            hb.hb_davies_bouldin_noalloc(b.ctx, Xd, bad, k)
        assert ei.value.status == hb.HB_EINVAL
        # host arrays are refused by the binding, k out of range by the library
        with pytest.raises(ValueError):
            hb.hb_davies_bouldin_noalloc(b.ctx, X, lab, k)
        with pytest.raises(hb.HBError) as ei:
            hb.hb_davies_bouldin_noalloc(b.ctx, Xd, ld, 65)
        assert ei.value.status == hb.HB_EINVAL
        # the context still works after the errors
        assert abs(hb.hb_davies_bouldin_noalloc(b.ctx, Xd, ld, k) - ref) <= 1e-10 * abs(ref)
