"""GPU-vs-oracle parity of the grouping step (Section 5): edge features, Lloyd's k-means,
the Davies-Bouldin index and the choice of B over random restarts. Labels are decided in
FP64 with the same order of operations on both sides: bit-exact from equal centres; centre
sums are reduced in another order on the GPU, so later rounds may flip a point whose two
nearest centres are within 1e-9 (relative) of each other; centres, inertia and index agree
within 1e-10 relative."""

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu


def _blobs(seed, k, n_per, dim, spread):
    g = np.random.default_rng(seed)
    centres = g.uniform(0.1, 0.9, (k, dim)) * 256
    X = np.concatenate([c + spread * 256 * g.normal(size=(n_per, dim)) for c in centres])
    return X[g.permutation(len(X))].astype(np.float32)


def _same_partition(a, b):
    """Labels equal up to a renumbering of the clusters."""
    pairs = set(zip(a.tolist(), b.tolist()))
    return len(pairs) == len(set(a.tolist())) == len(set(b.tolist()))


def test_edge_features_parity(hb):
    w = workloads.scaled("clustered", n_edges=3000, grid=512, groups=1, n_iters=1, seed=61)
    p = O.params_for(w)
    with hb.Bundler(0) as b:
        b.set_workload(w)
        for kind, name in ((hb.HB_FEAT_ORIGIN, "origin"), (hb.HB_FEAT_DESTINATION, "destination"),
                           (hb.HB_FEAT_ORIGIN_DESTINATION, "od"), (hb.HB_FEAT_LENGTH, "length")):
            got = b.edge_features(kind)
            np.testing.assert_array_equal(got, O.edge_features(w.node_xy, w.src, w.dst, p, name))


@pytest.mark.parametrize("n_per,dim,k,seed", [(3000, 4, 8, 62), (2500, 2, 5, 63), (1700, 1, 3, 64)])
def test_kmeans_parity(hb, n_per, dim, k, seed):
    X = _blobs(seed, k + 2, n_per, dim, 0.04)
    init = X[O.init_indices(seed, k, 0, len(X))].astype(np.float64)
    with hb.Bundler(0) as b:
        l1, c1, i1, r1 = b.kmeans(X, init, max_iters=1)
        lf, cf, inf_, rf = b.kmeans(X, init, max_iters=500)
        import torch
        ld, cd, idd, rd = b.kmeans(torch.from_numpy(X).cuda(), init, max_iters=500)
    o1, oc1, oi1, or1 = O.kmeans(X, init, max_iters=1)
    # one round from equal centres: labels bit-exact; centres and inertia up to summation order
    np.testing.assert_array_equal(l1, o1)
    np.testing.assert_allclose(c1, oc1, rtol=1e-12, atol=1e-9)
    assert abs(i1 - oi1) <= 1e-12 * oi1 and r1 == or1 == 1
    of, ocf, oif, orf = O.kmeans(X, init, max_iters=500)
    d = ((X[:, None, :].astype(np.float64) - ocf[None]) ** 2).sum(2)
    ds = np.sort(d, 1)
    amb = (ds[:, 1] - ds[:, 0]) <= 1e-9 * ds[:, 1] if k > 1 else np.zeros(len(X), bool)
    assert (lf == of)[~amb].all() and (lf != of).sum() <= amb.sum()
    np.testing.assert_allclose(cf, ocf, rtol=1e-10, atol=1e-7)
    assert abs(inf_ - oif) <= 1e-10 * oif and rf == orf
    np.testing.assert_array_equal(ld.cpu().numpy(), lf)
    np.testing.assert_array_equal(cd, cf)


def test_davies_bouldin_parity_and_errors(hb):
    X = _blobs(65, 6, 2000, 3, 0.05)
    g = np.random.default_rng(66)
    lab_r = g.integers(0, 6, len(X)).astype(np.int32)
    lab_k, _, _, _ = O.kmeans(X, X[O.init_indices(66, 6, 0, len(X))], max_iters=300)
    with hb.Bundler(0) as b:
        for lab in (lab_r, lab_k):
            got = b.davies_bouldin(X, lab, 6)
            ref = O.davies_bouldin(X, lab, 6)
            assert abs(got - ref) <= 1e-10 * ref
        # a label outside [0, k) is an argument error, never an out-of-bounds read
        bad = lab_k.copy()
        bad[17] = 6
        with pytest.raises(hb.HBError) as ei:
            b.davies_bouldin(X, bad, 6)
        assert ei.value.status == hb.HB_EINVAL
        with pytest.raises(hb.HBError):
            b.kmeans(X[:3], X[:4].astype(np.float64))       # fewer points than centres
        assert b.davies_bouldin(X, np.zeros(len(X), np.int32), 1) == 0.0


def test_choose_groups_parity(hb):
    X = _blobs(67, 6, 500, 2, 0.012)
    with hb.Bundler(0) as b:
        B, lab, db = b.choose_groups(X, kmin=4, kmax=9, restarts=30, seed=5, max_iters=200)
    oB, olab, odb = O.choose_groups(X, kmin=4, kmax=9, restarts=30, seed=5, max_iters=200)
    assert B == oB == 6
    np.testing.assert_allclose(db, odb, rtol=1e-9)
    assert _same_partition(lab, olab)


def test_grouped_workload_runs(hb):
    """Groups chosen on the GPU from origin-destination features feed the bundling run."""
    w = workloads.scaled("zipf", n_edges=4000, grid=256, groups=1, n_iters=2, seed=68)
    with hb.Bundler(0) as b:
        b.set_workload(w)
        X = b.edge_features(hb.HB_FEAT_ORIGIN_DESTINATION)
        B, lab, db = b.choose_groups(X, kmin=4, kmax=6, restarts=5, seed=1, max_iters=50)
        assert 4 <= B <= 6 and lab.min() >= 0 and lab.max() < B
        b.set_groups(lab, workloads.interaction_eq4(B, 0.25))
        b.run(2)
        assert b.points()[0][-1] > 2 * w.n_edges
