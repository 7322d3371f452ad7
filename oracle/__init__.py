"""FP64 CPU oracle of the 3D-density-histogram edge-bundling iteration (arXiv 1504.02687).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the GPU library and its Python binding never do.
It shares no code with the GPU path. The arithmetic lives in ``oracle.c`` (plain
loops, one function per step of the method); this module marshals numpy arrays and
strings the steps together in the paper's order (Section 3, Fig. 1):

    resample -> splat (Eq. 1/3) -> box chain (Section 3.1) -> density stack (Eq. 3/4)
    -> gradient -> advection with step halving (Eq. 5) -> Laplacian smoothing.

Functions without an independent pin are marked "parity unpinned" in their docstring.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (FP contraction off so the source order is the arithmetic)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared",
               "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, f64, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint32
        sig = {
            "orc_num_threads": (ctypes.c_int, []),
            "orc_set_threads": (None, [ctypes.c_int]),
            "orc_sigma": (f64, [ctypes.c_int, ctypes.c_int]),
            "orc_bandwidth": (f64, [ctypes.c_int, f64, f64]),
            "orc_polyline_length": (f64, [P, i64]),
            "orc_sample_count": (i64, [f64, f64]),
            "orc_resample_counts": (i64, [i64, P, P, f64, P, P]),
            "orc_resample": (None, [i64, P, P, P, P, P, P]),
            "orc_directed_offset": (None, [i64, P, P, P, P, f64, P]),
            "orc_insdel_counts": (i64, [i64, P, P, f64, f64, P]),
            "orc_insdel": (None, [i64, P, P, f64, f64, P, P]),
            "orc_orientation": (None, [i64, P, P]),
            "orc_resample_frozen": (None, [i64, P, P, P, P, P]),
            "orc_advect_frozen": (None, [i64, P, P, P, i32, i32, P, f64, P, f64, P]),
            "orc_splat": (None, [i64, P, P, P, P, i32, i32, i32, P]),
            "orc_splat_strip": (None, [i64, P, P, P, P, i32, i32, i32, P]),
            "orc_box_brute": (None, [i32, i32, P, i32, P]),
            "orc_integral_image": (None, [i32, i32, P, P]),
            "orc_box_integral": (None, [i32, i32, P, i32, P]),
            "orc_box_chain": (None, [i32, i32, i32, i32, i32, P, P, i32]),
            "orc_density": (None, [i32, i32, i32, i32, i32, P, P, P, P]),
            "orc_gradient": (None, [i32, i32, i32, P, P]),
            "orc_kovesi_radii": (None, [f64, i32, P]),
            "orc_box_chain_radii": (None, [i32, i32, i32, i32, P, P, P, i32]),
            "orc_density_radii": (None, [i32, i32, i32, i32, P, P, P, P, P]),
            "orc_bilinear": (f64, [i32, i32, P, i32, i32, f64, f64]),
            "orc_advect": (None, [i64, P, P, P, i32, i32, i32, P, P, f64, i32, f64, f64,
                                  P, P, P, P, P]),
            "orc_laplacian": (None, [i64, P, P, f64, i32, P]),
            "orc_ink": (f64, [i64, P, P]),
            "orc_sqdist": (f64, [P, P, i32]),
            "orc_point_widths": (None, [i64, P, P, P, i32, i32, P, f64, f64, i32, P, P]),
            "orc_kmeans": (i32, [i64, i32, P, i32, P, i32, P, P]),
            "orc_davies_bouldin": (f64, [i64, i32, P, i32, P]),
            "orc_draw": (ctypes.c_uint64, [ctypes.c_uint64, i32, i32, i64]),
            "orc_init_indices": (None, [ctypes.c_uint64, i32, i32, i64, P]),
            "orc_choose_groups": (i32, [i64, i32, P, i32, i32, i32, ctypes.c_uint64, i32, P, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------------- parameters

@dataclasses.dataclass
class Params:
    """Parameters of the method (Sections 3.1-3.3 and 5); defaults are the paper's."""

    grid_w: int
    grid_h: int
    radii: List[int]
    delta: float = 1.0          # sampling step (px)
    passes: int = 3             # box passes (Section 3.1: three)
    h_max: Optional[float] = None   # None: 2 sigma(r_0) (Section 3.3, Fig. 2)
    lam: float = 0.9            # bandwidth decay (Fig. 2)
    eps: float = 1e-6           # Eq. 5 epsilon
    max_halvings: int = 8       # K
    smooth_weight: float = 0.5  # Laplacian weight s
    smooth_passes: int = 1
    pass_weights: Optional[List[float]] = None   # a_k; None: only the last pass
    amb_tol: float = 1e-5       # decision margin treated as ambiguous in parity checks
    bbox: tuple = (0.0, 0.0, 1.0, 1.0)
    directed_offset: float = 0.0    # push of interior samples along the left normal (px)
    directed_every: bool = False    # push after every resampling instead of the first only
    strip_splat: bool = False       # histogram of the drawn line strips instead of the points
    insert_delete: bool = False     # insert/delete resampling instead of the uniform one
    delta_min: Optional[float] = None   # removal spacing of insert/delete (None: delta / 2)
    sigmas: Optional[List[float]] = None   # sigma per iteration: per-pass radii by Kovesi's rule

    def radius(self, it: int) -> int:
        return int(self.radii[min(it, len(self.radii) - 1)])

    def pass_radii(self, it: int) -> List[int]:
        """Box radius of every pass of iteration it (equal radii, or Kovesi's for a sigma)."""
        if self.sigmas:
            return kovesi_radii(self.sigmas[min(it, len(self.sigmas) - 1)], self.passes)
        return [self.radius(it)] * self.passes

    def a(self) -> np.ndarray:
        if self.pass_weights is None:
            a = np.zeros(self.passes)
            a[-1] = 1.0
            return a
        return _c(self.pass_weights, np.float64)

    def hmax(self) -> float:
        if self.h_max is not None and self.h_max > 0:
            return float(self.h_max)
        if self.sigmas:
            return 2.0 * float(self.sigmas[0])
        return 2.0 * sigma(self.radius(0), self.passes)

    def bandwidth(self, it: int) -> float:
        return float(lib().orc_bandwidth(it, self.hmax(), self.lam))


def params_for(w) -> Params:
    """Parameters of a ``workloads.Workload``."""
    return Params(grid_w=w.grid_w, grid_h=w.grid_h, radii=list(w.radii), delta=w.delta,
                  passes=w.passes, lam=w.lam, bbox=tuple(w.bbox))


def sigma(r: int, passes: int) -> float:
    return float(lib().orc_sigma(r, passes))


# ----------------------------------------------------------------------- steps

def initial_state(node_xy, src, dst, p: Params):
    """Two-point polylines (source, target) in pixel units (FP64)."""
    xy = np.asarray(node_xy, dtype=np.float64)
    x0, y0, x1, y1 = p.bbox
    px = (xy[:, 0] - x0) / (x1 - x0) * p.grid_w
    py = (xy[:, 1] - y0) / (y1 - y0) * p.grid_h
    pts = np.stack([px, py], axis=1)
    E = len(src)
    out = np.empty((E, 2, 2), dtype=np.float64)
    out[:, 0] = pts[np.asarray(src)]
    out[:, 1] = pts[np.asarray(dst)]
    off = np.arange(0, 2 * E + 1, 2, dtype=np.int64)
    return off, out.reshape(-1, 2)


def polyline_length(xy) -> float:
    xy = _c(xy, np.float64)
    return float(lib().orc_polyline_length(_p(xy), xy.shape[0]))


def sample_count(L: float, delta: float) -> int:
    return int(lib().orc_sample_count(L, delta))


def resample(off, xy, delta, want_seg=False):
    """Uniform-arclength resampling of every polyline; returns (off_out, xy_out, lens) and,
    with want_seg, the segment index of every sample (-1 at end points)."""
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    E = off.shape[0] - 1
    counts = np.empty(E, np.int64)
    lens = np.empty(E, np.float64)
    N = lib().orc_resample_counts(E, _p(off), _p(xy), delta, _p(counts), _p(lens))
    off_out = np.zeros(E + 1, np.int64)
    np.cumsum(counts, out=off_out[1:])
    assert off_out[-1] == N
    xy_out = np.empty((N, 2), np.float64)
    seg = np.empty(N, np.int64) if want_seg else None
    lib().orc_resample(E, _p(off), _p(xy), _p(off_out), _p(lens), _p(xy_out), _p(seg))
    if want_seg:
        return off_out, xy_out, lens, seg
    return off_out, xy_out, lens


def resample_insdel(off, xy, dmin, dmax):
    """Insert/delete resampling: interior points closer than dmin to their input predecessor
    removed, gaps between kept points cut into parts of at most dmax. Returns (off, xy)."""
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    E = off.shape[0] - 1
    counts = np.empty(E, np.int64)
    N = lib().orc_insdel_counts(E, _p(off), _p(xy), float(dmin), float(dmax), _p(counts))
    off_out = np.zeros(E + 1, np.int64)
    np.cumsum(counts, out=off_out[1:])
    assert off_out[-1] == N
    out = np.empty((N, 2), np.float64)
    lib().orc_insdel(E, _p(off), _p(xy), float(dmin), float(dmax), _p(off_out), _p(out))
    return off_out, out


def directed_offset(off_in, xy_in, off_out, seg, xy, d):
    """Samples xy (from resample with want_seg) pushed by d px along the left normal of the
    input segment each lies on; end points unchanged (Section 3, the pipeline)."""
    off_in = _c(off_in, np.int64)
    xy_in = _c(xy_in, np.float64)
    off_out = _c(off_out, np.int64)
    seg = _c(seg, np.int64)
    out = np.array(xy, dtype=np.float64, copy=True, order="C")
    lib().orc_directed_offset(off_in.shape[0] - 1, _p(off_in), _p(xy_in), _p(off_out), _p(seg),
                              float(d), _p(out))
    return out


def orientation(dxy):
    """Orientation slice in [0, 4) of every direction (dx, dy): slice k holds the angles in
    [90k - 45, 90k + 45) degrees (Section 5)."""
    dxy = _c(np.reshape(dxy, (-1, 2)), np.float64)
    out = np.empty(dxy.shape[0], np.int32)
    lib().orc_orientation(dxy.shape[0], _p(dxy), _p(out))
    return out


def splat(off, xy, group, B, W, H, weight=None):
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    group = _c(group, np.int32)
    weight = None if weight is None else _c(weight, np.int32)
    hist = np.empty((B, H, W), np.int64)
    lib().orc_splat(off.shape[0] - 1, _p(off), _p(xy), _p(group), _p(weight), B, W, H, _p(hist))
    return hist


def splat_strip(off, xy, group, B, W, H, weight=None):
    """Line-strip (rasterised) histogram: each polyline drawn through the pixels of its
    points, every drawn pixel adding the edge weight (the paper's Bresenham drawing)."""
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    group = _c(group, np.int32)
    weight = None if weight is None else _c(weight, np.int32)
    hist = np.empty((B, H, W), np.int64)
    lib().orc_splat_strip(off.shape[0] - 1, _p(off), _p(xy), _p(group), _p(weight), B, W, H,
                          _p(hist))
    return hist


def box_brute(m, r):
    m = _c(m, np.int64)
    H, W = m.shape
    out = np.empty_like(m)
    lib().orc_box_brute(W, H, _p(m), r, _p(out))
    return out


def integral_image(m):
    m = _c(m, np.int64)
    H, W = m.shape
    out = np.empty((H + 1, W + 1), np.int64)
    lib().orc_integral_image(W, H, _p(m), _p(out))
    return out


def box_integral(m, r):
    m = _c(m, np.int64)
    H, W = m.shape
    out = np.empty_like(m)
    lib().orc_box_integral(W, H, _p(m), r, _p(out))
    return out


def kovesi_radii(sig: float, passes: int) -> List[int]:
    out = np.empty(passes, np.int32)
    lib().orc_kovesi_radii(float(sig), passes, _p(out))
    return out.tolist()


def box_chain_radii(hist, radii, brute=False):
    """S[k, b] = pass k+1 of the box chain with radius radii[k] on group b (int64, exact)."""
    hist = _c(hist, np.int64)
    B, H, W = hist.shape
    rr = _c(radii, np.int32)
    S = np.empty((len(rr), B, H, W), np.int64)
    lib().orc_box_chain_radii(B, W, H, len(rr), _p(rr), _p(hist), _p(S), 1 if brute else 0)
    return S


def density_radii(S, radii, a, M):
    S = _c(S, np.int64)
    P, B, H, W = S.shape
    rr = _c(radii, np.int32)
    a = _c(a, np.float64)
    M = _c(M, np.float64)
    rho = np.empty((B, H, W), np.float64)
    lib().orc_density_radii(B, W, H, P, _p(rr), _p(S), _p(a), _p(M), _p(rho))
    return rho


def box_chain(hist, passes, r, brute=False):
    """S[k, b] = pass k+1 of the box chain on group b (int64, exact)."""
    hist = _c(hist, np.int64)
    B, H, W = hist.shape
    S = np.empty((passes, B, H, W), np.int64)
    lib().orc_box_chain(B, W, H, passes, r, _p(hist), _p(S), 1 if brute else 0)
    return S


def density(S, r, a, M):
    S = _c(S, np.int64)
    P, B, H, W = S.shape
    a = _c(a, np.float64)
    M = _c(M, np.float64)
    rho = np.empty((B, H, W), np.float64)
    lib().orc_density(B, W, H, P, r, _p(S), _p(a), _p(M), _p(rho))
    return rho


def gradient(rho):
    rho = _c(rho, np.float64)
    B, H, W = rho.shape
    g = np.empty((B, H, W, 2), np.float64)
    lib().orc_gradient(B, W, H, _p(rho), _p(g))
    return g


def bilinear(m, x, y, comp=0):
    """Bilinear sample of a [H, W] or [H, W, C] map at pixel-unit position (x, y)."""
    m = _c(m, np.float64)
    H, W = m.shape[:2]
    stride = 1 if m.ndim == 2 else m.shape[2]
    return float(lib().orc_bilinear(W, H, _p(m), stride, comp, float(x), float(y)))


def advect(off, xy, group, rho, grad, h, K=8, eps=1e-6, amb_tol=1e-5):
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    group = _c(group, np.int32)
    rho = _c(rho, np.float64)
    grad = _c(grad, np.float64)
    B, H, W = rho.shape
    N = xy.shape[0]
    out = np.empty((N, 2), np.float64)
    jacc = np.empty(N, np.int32)
    jfirm = np.empty(N, np.int32)
    amb = np.empty(N, np.uint32)
    d = np.empty((N, 2), np.float64)
    lib().orc_advect(off.shape[0] - 1, _p(off), _p(xy), _p(group), B, W, H, _p(rho), _p(grad),
                     h, K, eps, amb_tol, _p(out), _p(jacc), _p(jfirm), _p(amb), _p(d))
    return {"xy": out, "jacc": jacc, "jfirm": jfirm, "amb": amb, "dir": d}


def laplacian(off, xy, s=0.5, passes=1):
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    out = np.empty_like(xy)
    lib().orc_laplacian(off.shape[0] - 1, _p(off), _p(xy), s, passes, _p(out))
    return out


def ink(off, xy) -> float:
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    return float(lib().orc_ink(off.shape[0] - 1, _p(off), _p(xy)))


# ----------------------------------------------------------------------- width encoding (3.4)

def point_widths(off, xy, group, rho, w_min, w_max, log_scale=False):
    """Per point: the density of its edge's layer at the point (>= 0) and the line width
    w_min + (w_max - w_min) f(rho) / f(rho_max), f linear or log1p. Returns (dens, widths)."""
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    group = _c(group, np.int32)
    rho = _c(rho, np.float64)
    B, H, W = rho.shape
    N = xy.shape[0]
    dens = np.empty(N, np.float64)
    widths = np.empty(N, np.float64)
    lib().orc_point_widths(off.shape[0] - 1, _p(off), _p(xy), _p(group), W, H, _p(rho), float(w_min),
                           float(w_max), 1 if log_scale else 0, _p(dens), _p(widths))
    return dens, widths


def maps_of(off, xy, group, M, p: "Params", it: int, weight=None):
    """The density stack of the polylines (off, xy) taken as samples, with the box radii of
    iteration it (histogram, box passes, density; no advection)."""
    B = int(np.asarray(M).shape[0])
    if p.strip_splat:
        hist = splat_strip(off, xy, group, B, p.grid_w, p.grid_h, weight)
    else:
        hist = splat(off, xy, group, B, p.grid_w, p.grid_h, weight)
    rr = p.pass_radii(it)
    S = box_chain_radii(hist, rr)
    return density_radii(S, rr, p.a(), M)


# ----------------------------------------------------------------------- grouping (Section 5)

def edge_features(node_xy, src, dst, p: "Params", kind: str):
    """Per-edge features in grid (pixel) units, FP32: "origin" (x_s, y_s), "destination"
    (x_t, y_t), "od" (x_s, y_s, x_t, y_t) or "length" (|x_t - x_s|)."""
    _, xy = initial_state(node_xy, src, dst, p)
    xy = xy.astype(np.float32)
    a, b = xy[0::2], xy[1::2]
    if kind == "origin":
        return np.ascontiguousarray(a)
    if kind == "destination":
        return np.ascontiguousarray(b)
    if kind == "od":
        return np.ascontiguousarray(np.concatenate([a, b], 1))
    if kind == "length":
        d = b.astype(np.float64) - a.astype(np.float64)
        return np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]).astype(np.float32)[:, None]
    raise ValueError(kind)


def kmeans(X, centers, max_iters=100):
    """Lloyd's k-means from the given centres (FP64); returns labels, centres, inertia, rounds."""
    X = _c(X, np.float32)
    n, dim = X.shape
    cen = np.array(centers, dtype=np.float64, order="C", copy=True)
    k = cen.shape[0]
    labels = np.empty(n, np.int32)
    inertia = ctypes.c_double()
    rounds = lib().orc_kmeans(n, dim, _p(X), k, _p(cen), max_iters, _p(labels), ctypes.byref(inertia))
    return labels, cen, float(inertia.value), int(rounds)


def davies_bouldin(X, labels, k):
    X = _c(X, np.float32)
    labels = _c(labels, np.int32)
    return float(lib().orc_davies_bouldin(X.shape[0], X.shape[1], _p(X), int(k), _p(labels)))


def draw(seed, B, r, t):
    return int(lib().orc_draw(seed, B, r, t))


def init_indices(seed, k, r, n):
    idx = np.empty(k, np.int64)
    lib().orc_init_indices(seed, k, r, n, _p(idx))
    return idx


def choose_groups(X, kmin=4, kmax=16, restarts=100, seed=0, max_iters=100):
    """B in [kmin, kmax] of the lowest Davies-Bouldin index (Section 5); returns (B, labels,
    db per B)."""
    X = _c(X, np.float32)
    n, dim = X.shape
    labels = np.empty(n, np.int32)
    db = np.empty(kmax - kmin + 1, np.float64)
    B = lib().orc_choose_groups(n, dim, _p(X), kmin, kmax, restarts, seed, max_iters, _p(labels), _p(db))
    return int(B), labels, db


# ----------------------------------------------------------------------- iteration

def iterate(off, xy, group, M, p: Params, it: int, weight=None, skip_resample=False,
            keep_maps=True):
    """One bundling iteration (Fig. 1) from the polyline state (off, xy).

    Returns a dict with the samples, histogram, box passes, density, gradient, the
    advection record and the new polyline state.
    """
    B = int(np.asarray(M).shape[0])
    W, H = p.grid_w, p.grid_h
    r = p.radius(it)
    if skip_resample:
        s_off, s_xy = _c(off, np.int64), _c(xy, np.float64)
    elif p.insert_delete:
        dmin = p.delta_min if p.delta_min is not None else 0.5 * p.delta
        s_off, s_xy = resample_insdel(off, xy, dmin, p.delta)
    elif p.directed_offset != 0.0 and (it == 0 or p.directed_every):
        # Section 3, the pipeline: the push follows the first sampling (iteration 0); the
        # loop then restarts from the resampling. The other reading pushes every iteration.
        s_off, s_xy, _, seg = resample(off, xy, p.delta, want_seg=True)
        s_xy = directed_offset(off, xy, s_off, seg, s_xy, p.directed_offset)
    else:
        s_off, s_xy, _ = resample(off, xy, p.delta)
    if p.strip_splat:
        hist = splat_strip(s_off, s_xy, group, B, W, H, weight)
    else:
        hist = splat(s_off, s_xy, group, B, W, H, weight)
    if p.sigmas:
        rr = p.pass_radii(it)
        S = box_chain_radii(hist, rr)
        rho = density_radii(S, rr, p.a(), M)
    else:
        S = box_chain(hist, p.passes, r)
        rho = density(S, r, p.a(), M)
    g = gradient(rho)
    h = p.bandwidth(it)
    adv = advect(s_off, s_xy, group, rho, g, h, p.max_halvings, p.eps, p.amb_tol)
    new_xy = laplacian(s_off, adv["xy"], p.smooth_weight, p.smooth_passes)
    out = {"off": s_off, "samples": s_xy, "adv": adv, "xy": new_xy, "h": h, "r": r}
    if keep_maps:
        out.update(hist=hist, S=S, rho=rho, grad=g)
    return out


def run(node_xy, src, dst, group, M, p: Params, n_iters: int, weight=None):
    """T iterations from the straight edges; returns the final state and point counts."""
    off, xy = initial_state(node_xy, src, dst, p)
    counts = []
    for it in range(n_iters):
        res = iterate(off, xy, group, M, p, it, weight, keep_maps=False)
        off, xy = res["off"], res["xy"]
        counts.append(int(off[-1]))
    return off, xy, counts


# ----------------------------------------------------------------------- frozen surrogate

def record_run(off, xy, group, M, p: Params, n_iters: int, it0: int = 0, weight=None):
    """Base run from the polylines (off, xy): per iteration, the discrete choices that the
    frozen surrogate replays (sample offsets, segment indices, histograms, decisions)."""
    if p.directed_offset != 0.0 or p.strip_splat or p.insert_delete or p.sigmas:
        raise ValueError("the frozen surrogate covers the point splat without a directed offset")
    rec = []
    off = _c(off, np.int64)
    xy = _c(xy, np.float64)
    B = int(np.asarray(M).shape[0])
    for t in range(n_iters):
        it = it0 + t
        s_off, s_xy, _, seg = resample(off, xy, p.delta, want_seg=True)
        hist = splat(s_off, s_xy, group, B, p.grid_w, p.grid_h, weight)
        r = p.radius(it)
        S = box_chain(hist, p.passes, r)
        g = gradient(density(S, r, p.a(), M))
        adv = advect(s_off, s_xy, group, density(S, r, p.a(), M), g, p.bandwidth(it),
                     p.max_halvings, p.eps, p.amb_tol)
        rec.append({"in_off": off, "s_off": s_off, "seg": seg, "S": S, "jacc": adv["jacc"],
                    "jfirm": adv["jfirm"], "amb": adv["amb"], "h": p.bandwidth(it), "r": r})
        off, xy = s_off, laplacian(s_off, adv["xy"], p.smooth_weight, p.smooth_passes)
    return rec, off, xy


def frozen_loss(xy0, M, a, rec, group, p: Params, cT=None):
    """Loss of the polylines after the recorded iterations, replayed with the frozen choices,
    as a function of the starting positions xy0, the interaction matrix M and the pass
    weights a (all FP64): their ink, or, with weights cT [N_T, 2], the linear loss
    sum(cT * xy_T) of the final points."""
    xy = frozen_state(xy0, M, a, rec, group, p)
    if cT is not None:
        return float((np.asarray(cT, np.float64) * xy).sum())
    return ink(rec[-1]["s_off"], xy)


def frozen_state(xy0, M, a, rec, group, p: Params):
    """Final polylines (layout rec[-1]["s_off"]) of the frozen replay of the recorded
    iterations from xy0, M and a (FP64)."""
    xy = _c(xy0, np.float64)
    group = _c(group, np.int32)
    a = _c(a, np.float64)
    M = _c(M, np.float64)
    for r in rec:
        in_off, s_off, seg = r["in_off"], r["s_off"], r["seg"]
        E = in_off.shape[0] - 1
        sx = np.empty((s_off[-1], 2), np.float64)
        lib().orc_resample_frozen(E, _p(in_off), _p(xy), _p(s_off), _p(seg), _p(sx))
        g = gradient(density(r["S"], r["r"], a, M))
        B, H, W, _ = g.shape
        ax = np.empty_like(sx)
        jacc = _c(r["jacc"], np.int32)
        lib().orc_advect_frozen(E, _p(s_off), _p(sx), _p(group), W, H, _p(g), r["h"], _p(jacc),
                                p.eps, _p(ax))
        xy = laplacian(s_off, ax, p.smooth_weight, p.smooth_passes)
    return xy


def frozen_fd(xy0, M, a, rec, group, p: Params, which: str, index, step: float, cT=None):
    """Central finite difference of frozen_loss (ink, or the linear loss of weights cT) in
    one parameter: which is "M" (index (l, b)), "a" (index k) or "x" (index (point,
    coordinate))."""
    def f(delta):
        x, m, aa = np.array(xy0, np.float64), np.array(M, np.float64), np.array(a, np.float64)
        if which == "M":
            m[index] += delta
        elif which == "a":
            aa[index] += delta
        else:
            x[index] += delta
        return frozen_loss(x, m, aa, rec, group, p, cT)
    return (f(step) - f(-step)) / (2.0 * step)
