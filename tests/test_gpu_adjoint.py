"""Hand-written adjoint of the bundling iterations against the FP64 oracle.

The oracle gradient is the central difference (step 1e-6) of the oracle's frozen-decision
surrogate, whose choices come from the oracle's own base run. Gradients with respect to
the interaction matrix, the pass weights and sampled point coordinates must agree within
1e-3 relative, with an absolute floor of 1e-6 times the largest gradient entry.
"""

import numpy as np
import pytest

import oracle as O
import workloads

pytestmark = pytest.mark.gpu


def _setup(hb, w, a=None):
    b = hb.Bundler(0)
    kw = {} if a is None else {"pass_weights": list(a)}
    b.set_workload(w, **kw)
    return b


CASES = [(5, None, 1), (5, None, 2), (6, [0.2, 0.3, 0.5], 2)]


@pytest.mark.parametrize("seed,a,T", CASES)
def test_gradients_match_oracle_finite_differences(hb, seed, a, T):
    """Both sides make the same discrete choices over these horizons (checked through the
    sample counts and the loss); the oracle gradient is then the derivative of the same
    function."""
    w = workloads.scaled("clustered", n_edges=60, grid=64, groups=3, n_iters=3, seed=seed)
    p = O.params_for(w)
    if a is not None:
        p.pass_weights = list(a)
    with _setup(hb, w, a) as b:
        n0 = hb.hb_get_num_points(b.ctx)
        hb.hb_forward_ckpt(b.ctx, T)
        counts = b.iter_counts(T)
        loss, dM, da, dx = hb.hb_backward(b.ctx, w.n_groups, w.passes, n0)
        loss2, dM2, da2, dx2 = hb.hb_backward(b.ctx, w.n_groups, w.passes, n0)
    # bit-reproducible
    assert loss == loss2
    np.testing.assert_array_equal(dM, dM2)
    np.testing.assert_array_equal(da, da2)
    np.testing.assert_array_equal(dx, dx2)

    off, xy = O.initial_state(w.node_xy, w.src, w.dst, p)
    rec, offT, xyT = O.record_run(off, xy, w.group, w.M, p, T)
    assert [int(r["s_off"][-1]) for r in rec] == list(map(int, counts))
    assert abs(loss - O.ink(offT, xyT)) <= 1e-6 * loss

    M = w.M.astype(np.float64)
    fd = lambda which, idx, st=1e-6: O.frozen_fd(xy, M, p.a(), rec, w.group, p, which, idx, st)
    B = w.n_groups
    gM = np.array([[fd("M", (l, bb)) for bb in range(B)] for l in range(B)])
    ga = np.array([fd("a", k) for k in range(3)])
    rng = np.random.default_rng(seed)
    coords = []
    for i in rng.choice(len(xy), 40, replace=False):
        for c in range(2):
            g6, g5 = fd("x", (i, c)), fd("x", (i, c), 1e-5)
            if abs(g6 - g5) <= 1e-5 * max(abs(g6), 1e-3):      # not on a kink
                coords.append((i, c, g6))
            if len(coords) == 16:
                break
        if len(coords) == 16:
            break
    assert len(coords) == 16
    gx = np.array([g for _, _, g in coords])
    got = np.array([dx[i, c] for i, c, _ in coords])

    scale = max(np.abs(gM).max(), np.abs(ga).max(), np.abs(gx).max())
    floor = 1e-6 * scale
    np.testing.assert_allclose(dM, gM, rtol=1e-3, atol=floor)
    np.testing.assert_allclose(da, ga, rtol=1e-3, atol=floor)
    np.testing.assert_allclose(got, gx, rtol=1e-3, atol=floor)
    # Euler identities (scale invariance of the normalised advection direction)
    rows = (dM.astype(np.float64) * M).sum(1)
    assert (np.abs(rows) <= 1e-4 * np.abs(dM * M).sum(1) + floor).all()
    assert abs((da.astype(np.float64) * p.a()).sum()) <= 1e-4 * np.abs(da * p.a()).sum() + floor


def test_longer_horizon_euler_identities_and_reproducibility(hb):
    w = workloads.scaled("zipf", n_edges=2000, grid=256, groups=4, n_iters=5, seed=12)
    with _setup(hb, w) as b:
        n0 = hb.hb_get_num_points(b.ctx)
        hb.hb_forward_ckpt(b.ctx, 5)
        loss, dM, da, dx = hb.hb_backward(b.ctx, w.n_groups, w.passes, n0)
        ink = b.ink()
        hb.hb_forward_ckpt(b.ctx, 1)      # checkpoints replaced; state moved on
    assert loss == ink
    M = w.M.astype(np.float64)
    rows = (dM.astype(np.float64) * M).sum(1)
    assert (np.abs(rows) <= 1e-4 * np.abs(dM * M).sum(1)).all()
    assert np.isfinite(dx).all() and np.abs(dx).max() > 0


def test_autograd_function_matches_backward(hb):
    import torch
    w = workloads.scaled("zipf", n_edges=80, grid=64, groups=2, n_iters=2, seed=8)
    params = dict(grid_w=w.grid_w, grid_h=w.grid_h, radii=w.radii, delta=w.delta, passes=w.passes,
                  lam=w.lam)
    dev = torch.device("cuda:0")
    with hb.Bundler(0) as b:
        b.set_workload(w)
        off, xy = b.points()
        xy0 = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
        M = torch.tensor(w.M, dtype=torch.float32, requires_grad=True)
        a = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float32, requires_grad=True)
        loss = hb.bundle_ink(xy0, M, a, b, off, w.group, 2, params)
        loss.backward()
        # the same run through the C calls, from the same start iteration
        b.set_points(off, xy)
        b.iteration = 0
        hb.hb_forward_ckpt(b.ctx, 2)
        l2, dM, da, dx = hb.hb_backward(b.ctx, 2, 3, len(xy))
    assert float(loss.detach()) == l2
    np.testing.assert_array_equal(M.grad.numpy(), dM)
    np.testing.assert_array_equal(a.grad.numpy(), da)
    np.testing.assert_array_equal(xy0.grad.cpu().numpy(), dx)


def test_autograd_twice_same_loss_and_stale_node_rejected(hb):
    """The forward sets its start iteration itself, so two calls on one context give the same
    loss and gradients; a graph node whose checkpoints were replaced by a later forward
    refuses its backward (HB_ESTATE) instead of returning the later run's gradients."""
    import torch
    w = workloads.scaled("zipf", n_edges=80, grid=64, groups=2, n_iters=2, seed=8)
    params = dict(grid_w=w.grid_w, grid_h=w.grid_h, radii=w.radii, delta=w.delta, passes=w.passes,
                  lam=w.lam)
    dev = torch.device("cuda:0")
    with hb.Bundler(0) as b:
        b.set_workload(w)
        off, xy = b.points()
        grads = []
        losses = []
        for _ in range(2):
            xy0 = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
            M = torch.tensor(w.M, dtype=torch.float32, requires_grad=True)
            a = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float32, requires_grad=True)
            loss = hb.bundle_ink(xy0, M, a, b, off, w.group, 2, params)
            loss.backward()
            losses.append(float(loss.detach()))
            grads.append((M.grad.numpy().copy(), a.grad.numpy().copy(), xy0.grad.cpu().numpy()))
        assert losses[0] == losses[1]
        for g1, g2 in zip(*grads):
            np.testing.assert_array_equal(g1, g2)
        # two forwards, then the backward of the first
        xa = torch.tensor(xy, dtype=torch.float32, device=dev, requires_grad=True)
        Ma = torch.tensor(w.M, dtype=torch.float32, requires_grad=True)
        aa = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float32, requires_grad=True)
        first = hb.bundle_ink(xa, Ma, aa, b, off, w.group, 2, params)
        second = hb.bundle_ink(xa.detach().clone().requires_grad_(True), Ma.detach().clone(),
                               aa.detach().clone(), b, off, w.group, 2, params)
        with pytest.raises(hb.HBError) as ei:
            first.backward()
        assert ei.value.status == hb.HB_ESTATE
        second.backward()                     # the current checkpoints still work


def test_caller_loss_gradient_matches_oracle(hb):
    """A loss of the final polylines other than ink: L = sum(c * xy_T) with fixed random c,
    its gradient given to hb_backward (host and device forms, and through autograd), against
    the oracle's central differences of the same loss on its frozen surrogate."""
    import torch
    w = workloads.scaled("clustered", n_edges=60, grid=64, groups=3, n_iters=2, seed=5)
    p = O.params_for(w)
    T = 2
    with _setup(hb, w) as b:
        off0, xy0h = b.points()
        n0 = len(xy0h)
        gen = hb.hb_forward_ckpt(b.ctx, T)
        offT, xyT = b.points()
        c = np.random.default_rng(3).normal(size=xyT.shape).astype(np.float32)
        _, dM, da, dx = hb.hb_backward(b.ctx, w.n_groups, w.passes, n0, dL_dxy_T=c, generation=gen)
        dev = torch.device("cuda:0")
        _, dMd, dad, dxd = hb.hb_backward(b.ctx, w.n_groups, w.passes, n0,
                                          dL_dxy_T=torch.from_numpy(c).to(dev), device=dev)
        with pytest.raises(hb.HBError) as ei:      # wrong length
            hb.hb_backward(b.ctx, w.n_groups, w.passes, n0, dL_dxy_T=c[:-1])
        assert ei.value.status == hb.HB_EINVAL
        with pytest.raises(hb.HBError) as ei:      # an older generation
            hb.hb_backward(b.ctx, w.n_groups, w.passes, n0, dL_dxy_T=c, generation=gen - 1)
        assert ei.value.status == hb.HB_ESTATE
        # autograd: the polylines output with the same linear loss
        params = dict(grid_w=w.grid_w, grid_h=w.grid_h, radii=w.radii, delta=w.delta,
                      passes=w.passes, lam=w.lam)
        xt = torch.tensor(xy0h, dtype=torch.float32, device=dev, requires_grad=True)
        Mt = torch.tensor(w.M, dtype=torch.float32, requires_grad=True)
        at = torch.tensor([0.0, 0.0, 1.0], dtype=torch.float32, requires_grad=True)
        xyt, offt, _ = hb.bundle_polylines(xt, Mt, at, b, off0, w.group, T, params)
        np.testing.assert_array_equal(offt.cpu().numpy(), offT)
        (torch.from_numpy(c).to(dev) * xyt).sum().backward()
    np.testing.assert_array_equal(dMd, dM)
    np.testing.assert_array_equal(dad, da)
    np.testing.assert_array_equal(dxd.cpu().numpy(), dx)
    np.testing.assert_array_equal(Mt.grad.numpy(), dM)
    np.testing.assert_array_equal(at.grad.numpy(), da)
    np.testing.assert_array_equal(xt.grad.cpu().numpy(), dx)

    off, xy = O.initial_state(w.node_xy, w.src, w.dst, p)
    rec, offR, xyR = O.record_run(off, xy, w.group, w.M, p, T)
    np.testing.assert_array_equal(offR, offT)
    cT = c.astype(np.float64)
    M = w.M.astype(np.float64)
    fd = lambda which, idx, st=1e-6: O.frozen_fd(xy, M, p.a(), rec, w.group, p, which, idx, st, cT)
    B = w.n_groups
    gM = np.array([[fd("M", (l, bb)) for bb in range(B)] for l in range(B)])
    ga = np.array([fd("a", k) for k in range(3)])
    rng = np.random.default_rng(4)
    coords = []
    for i in rng.permutation(len(xy)):
        for cc in range(2):
            g6, g5 = fd("x", (i, cc)), fd("x", (i, cc), 1e-5)
            if abs(g6 - g5) <= 1e-5 * max(abs(g6), 1e-3):      # not on a kink
                coords.append((i, cc, g6))
        if len(coords) >= 16:
            break
    assert len(coords) >= 16
    gx = np.array([g for _, _, g in coords])
    got = np.array([dx[i, cc] for i, cc, _ in coords])
    scale = max(np.abs(gM).max(), np.abs(ga).max(), np.abs(gx).max())
    floor = 1e-6 * scale
    np.testing.assert_allclose(dM, gM, rtol=1e-3, atol=floor)
    np.testing.assert_allclose(da, ga, rtol=1e-3, atol=floor)
    np.testing.assert_allclose(got, gx, rtol=1e-3, atol=floor)


def test_backward_needs_fresh_checkpoints(hb):
    w = workloads.scaled("uniform", n_edges=40, grid=64, groups=1, n_iters=2, seed=9)
    with _setup(hb, w) as b:
        with pytest.raises(hb.HBError) as ei:
            hb.hb_backward(b.ctx, 1, 3, 80)
        assert ei.value.status == hb.HB_ESTATE
        hb.hb_forward_ckpt(b.ctx, 2)
        b.run(1)
        with pytest.raises(hb.HBError):
            hb.hb_backward(b.ctx, 1, 3, 80)


def test_checkpointed_forward_matches_plain_run(hb):
    """The checkpointed forward writes straight into its checkpoints; its polylines, sample
    counts and ink equal a plain run's bit for bit."""
    w = workloads.scaled("zipf", n_edges=3000, grid=256, groups=4, n_iters=3, seed=21)
    res = []
    for ckpt in (False, True):
        with _setup(hb, w) as b:
            if ckpt:
                hb.hb_forward_ckpt(b.ctx, 3)
            else:
                b.run(3)
            res.append((b.points(), b.iter_counts(3), b.ink(), b.iteration))
    (o1, x1), c1, i1, t1 = res[0]
    (o2, x2), c2, i2, t2 = res[1]
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(c1, c2)
    assert i1 == i2 and t1 == t2 == 3
