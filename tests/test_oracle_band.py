"""Pins of the advection's ambiguity band (Section 3.3, step halving, and the reading that a
try whose density margin is within amb_tol * (|rho(x)| + |rho(x')|) of zero may go either way
in finite precision).

The maps are built so that every try lands on a known value: the gradient map is the
constant (1, 0), so the direction is exactly +x; the point sits on a pixel centre of its row,
and the first six tries (steps 32, 16, 8, 4, 2, 1 px) land on pixel centres of the same row,
where the bilinear sample is the pixel's own value. The expected decision record of every
case below is written out by hand from the definition of the band, so a wrong band factor, a
strict instead of a non-strict comparison, a loop that runs past the first firm acceptance or
a wrong number of tries fails one of them.
"""

import numpy as np
import pytest

import oracle as O
from tests.parity import acceptable

W, H = 80, 8
X0 = 40.5            # start: centre of pixel 40
STEP = 32.0          # h; tries at +32, +16, +8, +4, +2, +1 px land on pixels 72, 56, 48, 44, 42, 41
PIX = [72, 56, 48, 44, 42, 41]


def _maps(rows):
    """rows: {v: (rho at the start, [rho at the six pixel-centre tries])}; other pixels 0."""
    rho = np.zeros((1, H, W))
    for v, (r0, vals) in rows.items():
        rho[0, v, 40] = r0
        for u, val in zip(PIX, vals):
            rho[0, v, u] = val
    grad = np.zeros((1, H, W, 2))
    grad[..., 0] = 1.0
    return rho, grad


def _run(rows, K=8, amb_tol=1e-5):
    rho, grad = _maps(rows)
    vs = sorted(rows)
    # one edge per case: end point, the probed point, end point
    off = np.arange(0, 3 * len(vs) + 1, 3, dtype=np.int64)
    xy = []
    for v in vs:
        xy += [[0.5, 0.5], [X0, v + 0.5], [0.5, 0.5]]
    res = O.advect(off, np.array(xy), np.zeros(len(vs), np.int32), rho, grad, h=STEP, K=K,
                   amb_tol=amb_tol)
    mid = np.arange(1, 3 * len(vs), 3)
    return {v: (int(res["jacc"][i]), int(res["jfirm"][i]), int(res["amb"][i]), res["xy"][i])
            for v, i in zip(vs, mid)}


R = 1000.0


def rel(*d):
    return [R * (1.0 + x) for x in d]


def test_band_records_written_out_by_hand():
    rows = {
        # firm accept at the first try: nothing ambiguous
        1: (R, rel(1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3)),
        # every try firmly lower (the last three tries interpolate between pixels 40 and 41,
        # margins -0.5e-3 R, -0.25e-3 R, -0.125e-3 R): no move, nothing firm
        2: (R, rel(-1e-3, -1e-3, -1e-3, -1e-3, -1e-3, -1e-3)),
        # firm reject, ambiguous reject, ambiguous accept, firm accept; the two zero margins
        # after the firm accept would be ambiguous but are never tried
        3: (R, rel(-1e-3, -1.5e-5, 1.5e-5, 1e-3, 0.0, 0.0)),
        # the band edge: |margin| = 2.01e-5 R is outside tol (|r0| + |r1|) (about 2.0e-5 R),
        # 1.99e-5 R inside
        4: (R, rel(-2.01e-5, -1.99e-5, 2.01e-5, 0.0, 0.0, 0.0)),
        # every try an ambiguous accept (the last three interpolated: 5e-7, 2.5e-7, 1.25e-7
        # relative): accepted at the first try, no firm acceptance, all K + 1 bits set
        5: (R, rel(1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6)),
        # ambiguous rejects up to a firm accept at the fifth try
        6: (R, rel(-1e-6, -1e-6, -1e-6, -1e-6, 1e-3, 0.0)),
    }
    got = _run(rows)
    expect = {1: (0, 0, 0b0), 2: (-1, -1, 0b0), 3: (2, 3, 0b0110), 4: (2, 2, 0b010),
              5: (0, -1, 0b111111111), 6: (4, 4, 0b01111)}
    for v, (jacc, jfirm, amb) in expect.items():
        assert got[v][:3] == (jacc, jfirm, amb), (v, got[v][:3], (jacc, jfirm, amb))
    # the moved point is the first accepted try, on the row
    np.testing.assert_array_equal(got[1][3], [X0 + 32.0, 1.5])
    np.testing.assert_array_equal(got[2][3], [X0, 2.5])
    np.testing.assert_array_equal(got[3][3], [X0 + 8.0, 3.5])
    np.testing.assert_array_equal(got[5][3], [X0 + 32.0, 5.5])
    np.testing.assert_array_equal(got[6][3], [X0 + 2.0, 6.5])


@pytest.mark.parametrize("K,bits", [(0, 0b1), (2, 0b111), (5, 0b111111), (8, 0b111111111)])
def test_band_has_exactly_one_bit_per_try(K, bits):
    """All tries ambiguous: K + 1 bits (tries j = 0..K), first try accepted, none firm."""
    got = _run({2: (R, rel(1e-6, 1e-6, 1e-6, 1e-6, 1e-6, 1e-6))}, K=K)
    assert got[2][:3] == (0, -1, bits)


def test_band_edge_is_inclusive():
    """With tol = 2^-16, r0 = 2^16 - 1 and r1 = 2^16 + 1 the margin 2 equals the band
    2^-16 (r0 + r1) exactly in FP64: the try is ambiguous (non-strict comparison). The next
    try is a firm accept."""
    r0 = 65535.0
    got = _run({3: (r0, [65537.0, r0 + 1000.0, r0, r0, r0, r0])}, amb_tol=2.0 ** -16)
    assert got[3][:3] == (0, 1, 0b1)
    # a zero map: margin 0 = band 0 at every try
    got = _run({4: (0.0, [0.0] * 6)})
    assert got[4][:3] == (0, -1, 0b111111111)


def test_fixed_step_records_no_band():
    got = _run({3: (R, rel(-1e-3, -1.5e-5, 1.5e-5, 1e-3, 0.0, 0.0))}, K=-1)
    assert got[3][:3] == (0, 0, 0)
    np.testing.assert_array_equal(got[3][3], [X0 + 32.0, 3.5])


def test_acceptable_outcomes_follow_the_band():
    """GPU decisions that the parity tests accept for the records above: the oracle's, any
    ambiguous try before the first firm accept, or that accept (no move when none is firm)."""
    cases = {
        # (jacc, jfirm, amb): outcomes -1..8 that are valid
        (2, 3, 0b0110): {1, 2, 3},
        (-1, -1, 0b0): {-1},
        (0, 0, 0b0): {0},
        (0, -1, 0b111111111): {-1, 0, 1, 2, 3, 4, 5, 6, 7, 8},
        (4, 4, 0b01111): {0, 1, 2, 3, 4},
        (2, 2, 0b010): {1, 2},
    }
    for (jacc, jfirm, amb), valid in cases.items():
        g = np.arange(-1, 9)
        ok = acceptable(g, np.full(10, jacc), np.full(10, jfirm), np.full(10, amb, np.uint32))
        assert set(g[ok].tolist()) == valid, ((jacc, jfirm, amb), g[ok])
    # end points: only -2
    ok = acceptable(np.array([-2, -1, 0]), np.full(3, -2), np.full(3, -2), np.zeros(3, np.uint32))
    assert ok.tolist() == [True, False, False]
