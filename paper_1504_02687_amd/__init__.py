"""Python binding of the MI355X edge-bundling library (``libhb.so``, C ABI in ``include/hb.h``).

Argument marshalling only: every step of the bundling iteration runs in the HIP kernels of
``libhb.so``. Arrays may be numpy arrays (host) or torch CUDA tensors (device, passed with
``HB_DEVICE_PTRS``); torch is only used for device memory and the current stream. If the
library has not been built, ``load()`` raises: there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhb.so")

HB_OK, HB_EINVAL, HB_ENOMEM, HB_EDEVICE, HB_ESTATE, HB_EOVERFLOW, HB_EINTERNAL = 0, -1, -2, -3, -4, -5, -6
HB_DEVICE_PTRS = 1
HB_RUN_SAMPLES_GIVEN, HB_RUN_RECORD_DECISIONS, HB_RUN_ASYNC, HB_RUN_GRAPH = 1, 2, 4, 8
HB_POINTS_STATE, HB_POINTS_SAMPLES = 0, 1
HB_MAP_HIST, HB_MAP_BOX, HB_MAP_DENSITY, HB_MAP_GRAD = 0, 1, 2, 3
HB_SPLAT_POINTS, HB_SPLAT_STRIP = 0, 1
HB_RESAMPLE_UNIFORM, HB_RESAMPLE_INSERT_DELETE = 0, 1
HB_DIRECTED_ONCE, HB_DIRECTED_EVERY_ITER = 0, 1
HB_FEAT_ORIGIN, HB_FEAT_DESTINATION, HB_FEAT_ORIGIN_DESTINATION, HB_FEAT_LENGTH = 0, 1, 2, 3
HB_KMEANS_MAX_K, HB_KMEANS_MAX_DIM = 64, 8
_FEAT_DIM = {0: 2, 1: 2, 2: 4, 3: 1}
HB_MAX_GROUPS, HB_MAX_PASSES = 64, 8
HB_MAX_EDGE_WEIGHT = (1 << 20) - 1

STATUS_NAMES = {0: "HB_OK", -1: "HB_EINVAL", -2: "HB_ENOMEM", -3: "HB_EDEVICE",
                -4: "HB_ESTATE", -5: "HB_EOVERFLOW",
                -6: "HB_EINTERNAL"}


class HBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class hb_params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("grid_w", ctypes.c_int32),
        ("grid_h", ctypes.c_int32),
        ("bbox", ctypes.c_float * 4),
        ("delta_px", ctypes.c_float),
        ("box_passes", ctypes.c_int32),
        ("n_radii", ctypes.c_int32),
        ("radius_per_iter", ctypes.POINTER(ctypes.c_int32)),
        ("h_max_px", ctypes.c_float),
        ("lambda_", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("max_halvings", ctypes.c_int32),
        ("smooth_weight", ctypes.c_float),
        ("smooth_passes", ctypes.c_int32),
        ("pass_weights", ctypes.POINTER(ctypes.c_float)),
        ("capacity_factor", ctypes.c_float),
        ("directed_offset_px", ctypes.c_float),
        ("splat_mode", ctypes.c_int32),
        ("resample_mode", ctypes.c_int32),
        ("delta_min_px", ctypes.c_float),
        ("n_sigmas", ctypes.c_int32),
        ("sigma_per_iter", ctypes.POINTER(ctypes.c_float)),
        ("directed_mode", ctypes.c_int32),
    ]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "hb_default_params": (None, [ctypes.POINTER(hb_params), ctypes.c_int32, ctypes.c_int32]),
    "hb_validate_params": (ctypes.c_int32, [ctypes.POINTER(hb_params)]),
    "hb_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p]),
    "hb_destroy": (None, [ctypes.c_void_p]),
    "hb_set_params": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(hb_params)]),
    "hb_set_graph": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "hb_set_groups": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_uint32]),
    "hb_orientation_groups": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]),
    "hb_edge_features": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int64,
                                          ctypes.c_uint32]),
    "hb_kmeans": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32),
                                   ctypes.c_uint32]),
    "hb_davies_bouldin": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                           ctypes.c_uint32]),
    "hb_davies_bouldin_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                                   ctypes.POINTER(ctypes.c_double)]),
    "hb_choose_groups": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                          ctypes.c_void_p, ctypes.c_uint32]),
    "hb_point_widths": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                         ctypes.c_uint32]),
    "hb_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32]),
    "hb_sync": (ctypes.c_int32, [ctypes.c_void_p]),
    "hb_get_num_points": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "hb_get_points": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_uint32]),
    "hb_set_points": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_uint32]),
    "hb_get_map": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]),
    "hb_get_decisions": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]),
    "hb_get_iter_counts": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "hb_get_ink": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
    "hb_get_iteration": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)]),
    "hb_set_iteration": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "hb_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "hb_version": (ctypes.c_char_p, []),
    "hb_set_profiling": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "hb_batch_run": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint32]),
    "hb_forward_ckpt": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32,
                                         ctypes.POINTER(ctypes.c_int64)]),
    "hb_backward": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_double), ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]),
    "hb_get_ckpt_decisions": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]),
    "hb_get_ckpt_points": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32]),
    "hb_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]),
    "hb_set_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]),
    "hb_set_tiling": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "hb_get_tiling": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "hb_get_tuning": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "hb_get_stage_times": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_int32, ctypes.c_int32]),
}

STAGES = ["scan", "clear", "resample_splat", "box", "density_grad", "advect_smooth", "bin"]


def load():
    """Load libhb.so (built in-tree by ``build()``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python -m paper_1504_02687_amd.build)")
        # torch ships its own HIP runtime: load it first, so that libhb binds to that same
        # runtime and torch's device tensors and streams are valid in libhb's calls (a second
        # runtime loaded beside an initialised one leaves torch without devices)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols() -> Sequence[str]:
    return list(_SIGS)


# ------------------------------------------------------------------ marshalling

def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _arr(x, dtype):
    """(pointer, keepalive, is_device) of a numpy array or torch tensor with the given dtype."""
    if x is None:
        return None, None, False
    if _is_torch(x):
        import torch
        tdt = {np.float32: torch.float32, np.int32: torch.int32, np.int64: torch.int64,
               np.int8: torch.int8, np.float64: torch.float64}[np.dtype(dtype).type]
        if x.dtype != tdt or not x.is_contiguous():
            x = x.to(tdt).contiguous()
        return x.data_ptr(), x, x.is_cuda
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data, a, False


def _check(ctx, st):
    if st != HB_OK:
        msg = load().hb_last_error(ctx)
        raise HBError(st, msg.decode() if msg else "")


def _flags(*devs):
    d = [v for v in devs if v is not None]
    if any(d) and not all(d):
        raise ValueError("mix of host and device arrays in one call")
    return HB_DEVICE_PTRS if d and all(d) else 0


# ------------------------------------------------------------------ the C calls

def hb_default_params(grid_w: int, grid_h: int) -> hb_params:
    p = hb_params()
    load().hb_default_params(ctypes.byref(p), grid_w, grid_h)
    return p


def hb_validate_params(p: hb_params) -> int:
    return int(load().hb_validate_params(ctypes.byref(p)))


def hb_create(device: int = 0, stream: Optional[int] = None):
    ctx = ctypes.c_void_p()
    st = load().hb_create(ctypes.byref(ctx), device, ctypes.c_void_p(stream) if stream else None)
    _check(None, st)
    return ctx


def hb_destroy(ctx) -> None:
    load().hb_destroy(ctx)


def hb_set_params(ctx, p: hb_params) -> None:
    _check(ctx, load().hb_set_params(ctx, ctypes.byref(p)))


def hb_set_graph(ctx, node_xy, src, dst, weight=None) -> None:
    pn, kn, dn = _arr(node_xy, np.float32)
    ps, ks, ds = _arr(src, np.int32)
    pd, kd, dd = _arr(dst, np.int32)
    pw, kw, dw = _arr(weight, np.int32)
    flags = _flags(dn, ds, dd, dw if weight is not None else None)
    n_nodes = int(kn.shape[0])
    _check(ctx, load().hb_set_graph(ctx, n_nodes, pn, int(ks.shape[0]), ps, pd, pw, flags))


def hb_set_groups(ctx, group, M) -> None:
    pg, kg, dg = _arr(group, np.int32)
    pm, km, dm = _arr(M, np.float32)
    B = int(km.shape[0])
    _check(ctx, load().hb_set_groups(ctx, B, pg, pm, _flags(dg, dm)))


def hb_orientation_groups(ctx, n_edges: int, device=None):
    """Orientation slice in [0, 4) of every edge (int32 numpy array, or a torch tensor on
    ``device``)."""
    if device is not None:
        import torch
        out = torch.empty(n_edges, dtype=torch.int32, device=device)
        _check(ctx, load().hb_orientation_groups(ctx, ctypes.c_void_p(out.data_ptr()), HB_DEVICE_PTRS))
        return out
    out = np.empty(n_edges, np.int32)
    _check(ctx, load().hb_orientation_groups(ctx, out.ctypes.data, 0))
    return out


def hb_edge_features(ctx, kind: int, n_edges: int) -> np.ndarray:
    """Edge property `kind` (HB_FEAT_*) of every edge, float32 [E, dim]."""
    dim = _FEAT_DIM[int(kind)]
    out = np.empty((n_edges, dim), np.float32)
    _check(ctx, load().hb_edge_features(ctx, int(kind), out.ctypes.data, out.size, 0))
    return out


def _points(X):
    px, kx, dx = _arr(X, np.float32)
    n, dim = (int(kx.shape[0]), int(kx.shape[1])) if kx.ndim == 2 else (int(kx.shape[0]), 1)
    return px, kx, dx, n, dim


def hb_kmeans(ctx, X, centers, max_iters: int = 100):
    """Lloyd's k-means from `centers` [k, dim]; returns (labels int32 [n], centres float64,
    inertia, rounds). X may be a numpy array or a CUDA tensor (labels then on the device)."""
    px, kx, dx, n, dim = _points(X)
    cen = np.array(centers, dtype=np.float64, order="C", copy=True).reshape(-1, dim)
    k = int(cen.shape[0])
    if dx:
        import torch
        labels = torch.empty(n, dtype=torch.int32, device=kx.device)
        pl = labels.data_ptr()
    else:
        labels = np.empty(n, np.int32)
        pl = labels.ctypes.data
    inertia, rounds = ctypes.c_double(), ctypes.c_int32()
    _check(ctx, load().hb_kmeans(ctx, px, n, dim, k, cen.ctypes.data, int(max_iters), pl,
                                 ctypes.byref(inertia), ctypes.byref(rounds), _flags(dx)))
    return labels, cen, float(inertia.value), int(rounds.value)


def hb_davies_bouldin(ctx, X, labels, k: int) -> float:
    px, kx, dx, n, dim = _points(X)
    pl, kl, dl = _arr(labels, np.int32)
    out = ctypes.c_double()
    _check(ctx, load().hb_davies_bouldin(ctx, px, n, dim, int(k), pl, ctypes.byref(out), _flags(dx, dl)))
    return float(out.value)


def hb_davies_bouldin_noalloc(ctx, X, labels, k: int) -> float:
    """hb_davies_bouldin without device allocation; X [n, dim] float32 and labels [n] int32
    must be torch tensors on the context's GPU."""
    px, kx, dx, n, dim = _points(X)
    pl, kl, dl = _arr(labels, np.int32)
    if not (dx and dl):
        raise ValueError("X and labels must be device tensors")
    out = ctypes.c_double()
    _check(ctx, load().hb_davies_bouldin_noalloc(ctx, px, n, dim, int(k), pl, ctypes.byref(out)))
    return float(out.value)


def hb_choose_groups(ctx, X, kmin: int = 4, kmax: int = 16, restarts: int = 100, seed: int = 0,
                     max_iters: int = 100):
    """B in [kmin, kmax] of the lowest Davies-Bouldin index; returns (B, labels, db per B)."""
    px, kx, dx, n, dim = _points(X)
    if dx:
        import torch
        labels = torch.empty(n, dtype=torch.int32, device=kx.device)
        pl = labels.data_ptr()
    else:
        labels = np.empty(n, np.int32)
        pl = labels.ctypes.data
    db = np.empty(kmax - kmin + 1, np.float64)
    B = ctypes.c_int32()
    _check(ctx, load().hb_choose_groups(ctx, px, n, dim, int(kmin), int(kmax), int(restarts),
                                        ctypes.c_uint64(int(seed)), int(max_iters), pl,
                                        ctypes.byref(B), db.ctypes.data, _flags(dx)))
    return int(B.value), labels, db


def hb_run(ctx, n_iters: int, flags: int = 0) -> None:
    _check(ctx, load().hb_run(ctx, n_iters, flags))


def hb_sync(ctx) -> None:
    _check(ctx, load().hb_sync(ctx))


def hb_get_num_points(ctx, which: int = HB_POINTS_STATE) -> int:
    n = ctypes.c_int64()
    _check(ctx, load().hb_get_num_points(ctx, which, ctypes.byref(n)))
    return int(n.value)


def hb_point_widths(ctx, it: int, w_min: float, w_max: float, log_scale: bool = False, device=None):
    """Density at every point of the current polylines and its line width (Section 3.4);
    returns (dens, widths), float32 [N] numpy arrays, or torch tensors on ``device``."""
    n = hb_get_num_points(ctx, HB_POINTS_STATE)
    args = (int(it), float(w_min), float(w_max), 1 if log_scale else 0)
    if device is not None:
        import torch
        dens = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        widths = torch.empty(max(n, 1), dtype=torch.float32, device=device)
        _check(ctx, load().hb_point_widths(ctx, *args, ctypes.c_void_p(dens.data_ptr()),
                                           ctypes.c_void_p(widths.data_ptr()), n, HB_DEVICE_PTRS))
        return dens[:n], widths[:n]
    dens = np.empty(max(n, 1), np.float32)
    widths = np.empty(max(n, 1), np.float32)
    _check(ctx, load().hb_point_widths(ctx, *args, dens.ctypes.data, widths.ctypes.data, n, 0))
    return dens[:n], widths[:n]


def hb_get_points(ctx, which: int = HB_POINTS_STATE, n_edges: Optional[int] = None, device=None):
    """Offsets [E+1] (int64) and xy [N, 2] (float32) as numpy arrays, or torch tensors on
    ``device`` when given."""
    n = hb_get_num_points(ctx, which)
    if n_edges is None:
        raise ValueError("n_edges is required")
    if device is not None:
        import torch
        off = torch.empty(n_edges + 1, dtype=torch.int64, device=device)
        xy = torch.empty((n, 2), dtype=torch.float32, device=device)
        _check(ctx, load().hb_get_points(ctx, which, off.data_ptr(), xy.data_ptr(), n, HB_DEVICE_PTRS))
        return off, xy
    off = np.empty(n_edges + 1, np.int64)
    xy = np.empty((n, 2), np.float32)
    _check(ctx, load().hb_get_points(ctx, which, off.ctypes.data, xy.ctypes.data, n, 0))
    return off, xy


def hb_set_points(ctx, offsets, xy) -> None:
    po, ko, do = _arr(offsets, np.int64)
    px, kx, dx = _arr(xy, np.float32)
    n = int(kx.shape[0])
    _check(ctx, load().hb_set_points(ctx, po, px, n, _flags(do, dx)))


def hb_get_map(ctx, kind: int, group: int, grid_w: int, grid_h: int, pass_: int = 0):
    dtype, extra = {HB_MAP_HIST: (np.int32, ()), HB_MAP_BOX: (np.int64, ()),
                    HB_MAP_DENSITY: (np.float32, ()), HB_MAP_GRAD: (np.float32, (2,))}[kind]
    out = np.empty((grid_h, grid_w) + extra, dtype)
    _check(ctx, load().hb_get_map(ctx, kind, group, pass_, out.ctypes.data, out.nbytes, 0))
    return out


def hb_get_decisions(ctx) -> np.ndarray:
    n = hb_get_num_points(ctx, HB_POINTS_SAMPLES)
    out = np.empty(n, np.int8)
    _check(ctx, load().hb_get_decisions(ctx, out.ctypes.data, n, 0))
    return out


def hb_get_iter_counts(ctx, n_iters: int) -> np.ndarray:
    out = np.zeros(max(1, n_iters), np.int64)
    _check(ctx, load().hb_get_iter_counts(ctx, out.ctypes.data, len(out)))
    return out[:n_iters]


def hb_get_ink(ctx) -> float:
    v = ctypes.c_double()
    _check(ctx, load().hb_get_ink(ctx, ctypes.byref(v)))
    return float(v.value)


def hb_get_iteration(ctx) -> int:
    v = ctypes.c_int32()
    _check(ctx, load().hb_get_iteration(ctx, ctypes.byref(v)))
    return int(v.value)


def hb_set_iteration(ctx, it: int) -> None:
    _check(ctx, load().hb_set_iteration(ctx, it))


def hb_last_error(ctx=None) -> str:
    m = load().hb_last_error(ctx)
    return m.decode() if m else ""


def hb_version() -> str:
    return load().hb_version().decode()


def hb_set_profiling(ctx, enable: bool) -> None:
    _check(ctx, load().hb_set_profiling(ctx, 1 if enable else 0))


def hb_get_stage_times(ctx, reset: bool = False):
    """{stage: (total ms, launches)} accumulated while profiling was enabled."""
    n = len(STAGES)
    ms = np.zeros(n, np.float64)
    cnt = np.zeros(n, np.int64)
    _check(ctx, load().hb_get_stage_times(ctx, ms.ctypes.data, cnt.ctypes.data, n, 1 if reset else 0))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(STAGES)}


def _ctx_array(ctxs):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    return arr


def hb_batch_run(ctxs, n_iters: int, flags: int = 0) -> None:
    arr = _ctx_array(ctxs)
    _check(ctxs[0], load().hb_batch_run(arr, len(ctxs), n_iters, flags))


def hb_autotune(ctxs, n_iters: int = 1):
    """(resample chunks, advect chunks, column rows, tile-count sets, log2 item entries)."""
    arr = _ctx_array(ctxs)
    choice = (ctypes.c_int32 * 5)()
    _check(ctxs[0], load().hb_autotune(arr, len(ctxs), n_iters, choice))
    return tuple(int(v) for v in choice)


def hb_set_tuning(ctx, resample_chunks: int, advect_chunks: int) -> None:
    _check(ctx, load().hb_set_tuning(ctx, resample_chunks, advect_chunks))


def hb_get_tuning(ctx):
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, load().hb_get_tuning(ctx, ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def hb_set_tiling(ctx, col_rows: int, sets_max: int, item_entries_log2: int) -> None:
    _check(ctx, load().hb_set_tiling(ctx, col_rows, sets_max, item_entries_log2))


def hb_get_tiling(ctx):
    a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(ctx, load().hb_get_tiling(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return int(a.value), int(b.value), int(c.value)


# ------------------------------------------------------------------ convenience

def make_params(grid_w: int, grid_h: int, radii: Sequence[int], *, delta: float = 1.0,
                passes: int = 3, h_max: float = 0.0, lam: float = 0.9, eps: float = 1e-6,
                max_halvings: int = 8, smooth_weight: float = 0.5,
                pass_weights: Optional[Sequence[float]] = None, bbox=(0.0, 0.0, 1.0, 1.0),
                capacity_factor: float = 2.0, directed_offset: float = 0.0,
                splat_mode: int = 0, resample_mode: int = 0, delta_min: float = 0.0,
                sigmas: Optional[Sequence[float]] = None, directed_mode: int = 0):
    """hb_params plus the arrays it points to (keep both alive until hb_set_params)."""
    p = hb_default_params(grid_w, grid_h)
    r = (ctypes.c_int32 * len(radii))(*[int(v) for v in radii])
    p.radius_per_iter = ctypes.cast(r, ctypes.POINTER(ctypes.c_int32))
    p.n_radii = len(radii)
    p.delta_px = delta
    p.box_passes = passes
    p.h_max_px = h_max
    p.lambda_ = lam
    p.eps = eps
    p.max_halvings = max_halvings
    p.smooth_weight = smooth_weight
    for i in range(4):
        p.bbox[i] = bbox[i]
    p.capacity_factor = capacity_factor
    p.directed_offset_px = directed_offset
    p.directed_mode = directed_mode
    p.splat_mode = splat_mode
    p.resample_mode = resample_mode
    p.delta_min_px = delta_min
    keep = [r]
    if sigmas:
        sg = (ctypes.c_float * len(sigmas))(*[float(v) for v in sigmas])
        p.sigma_per_iter = ctypes.cast(sg, ctypes.POINTER(ctypes.c_float))
        p.n_sigmas = len(sigmas)
        keep.append(sg)
    if pass_weights is not None:
        a = (ctypes.c_float * passes)(*[float(v) for v in pass_weights])
        p.pass_weights = ctypes.cast(a, ctypes.POINTER(ctypes.c_float))
        keep.append(a)
    return p, keep


class Bundler:
    """One library context on one GPU (owns an ``hb_ctx``)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self.ctx = hb_create(device, stream)
        self.n_edges = 0
        self.grid = (0, 0)

    def close(self):
        if self.ctx is not None:
            hb_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, grid_w, grid_h, radii, **kw):
        p, keep = make_params(grid_w, grid_h, radii, **kw)
        hb_set_params(self.ctx, p)
        del keep
        self.grid = (grid_w, grid_h)

    def set_graph(self, node_xy, src, dst, weight=None):
        hb_set_graph(self.ctx, node_xy, src, dst, weight)
        self.n_edges = int(len(src))

    def set_groups(self, group, M):
        hb_set_groups(self.ctx, group, M)

    def orientation_groups(self, device=None):
        return hb_orientation_groups(self.ctx, self.n_edges, device)

    def edge_features(self, kind):
        return hb_edge_features(self.ctx, kind, self.n_edges)

    def kmeans(self, X, centers, max_iters=100):
        return hb_kmeans(self.ctx, X, centers, max_iters)

    def davies_bouldin(self, X, labels, k):
        return hb_davies_bouldin(self.ctx, X, labels, k)

    def choose_groups(self, X, kmin=4, kmax=16, restarts=100, seed=0, max_iters=100):
        return hb_choose_groups(self.ctx, X, kmin, kmax, restarts, seed, max_iters)

    def point_widths(self, it, w_min, w_max, log_scale=False, device=None):
        return hb_point_widths(self.ctx, it, w_min, w_max, log_scale, device)

    def set_workload(self, w, **kw):
        """Parameters, graph and groups of a ``workloads.Workload``."""
        self.set_params(w.grid_w, w.grid_h, w.radii, delta=w.delta, passes=w.passes, lam=w.lam,
                        bbox=w.bbox, **kw)
        self.set_graph(w.node_xy, w.src, w.dst, w.weight)
        self.set_groups(w.group, w.M)

    def run(self, n_iters, flags=0):
        hb_run(self.ctx, n_iters, flags)

    def sync(self):
        hb_sync(self.ctx)

    def points(self, which=HB_POINTS_STATE, device=None):
        return hb_get_points(self.ctx, which, self.n_edges, device)

    def set_points(self, offsets, xy):
        hb_set_points(self.ctx, offsets, xy)

    def map(self, kind, group, pass_=0):
        return hb_get_map(self.ctx, kind, group, self.grid[0], self.grid[1], pass_)

    def decisions(self):
        return hb_get_decisions(self.ctx)

    def iter_counts(self, n):
        return hb_get_iter_counts(self.ctx, n)

    def ink(self):
        return hb_get_ink(self.ctx)

    def tuning(self, resample_chunks=None, advect_chunks=None):
        if resample_chunks is not None:
            hb_set_tuning(self.ctx, resample_chunks, advect_chunks)
        return hb_get_tuning(self.ctx)

    def profiling(self, enable=True):
        hb_set_profiling(self.ctx, enable)

    def stage_times(self, reset=False):
        return hb_get_stage_times(self.ctx, reset)

    @property
    def iteration(self):
        return hb_get_iteration(self.ctx)

    @iteration.setter
    def iteration(self, it):
        hb_set_iteration(self.ctx, it)


def batch_run(bundlers, n_iters: int, flags: int = 0) -> None:
    """Advance several ``Bundler`` contexts together (one launch per stage for all)."""
    hb_batch_run([b.ctx for b in bundlers], n_iters, flags)


def autotune(bundlers, n_iters: int = 1):
    return hb_autotune([b.ctx for b in bundlers], n_iters)


# ------------------------------------------------------------------ differentiable form

def hb_forward_ckpt(ctx, n_iters: int) -> int:
    """Checkpointed forward of n_iters iterations; returns the checkpoints' generation."""
    gen = ctypes.c_int64()
    _check(ctx, load().hb_forward_ckpt(ctx, n_iters, 0, ctypes.byref(gen)))
    return int(gen.value)


def hb_backward(ctx, n_groups: int, n_passes: int, n_points0: int, dL_dxy_T=None,
                generation: int = -1, device=None):
    """(loss, dL/dM [B, B], dL/da [P], dL/dxy0 [N0, 2]). dL_dxy_T: gradient of the caller's
    loss with respect to the final polylines ([N_T, 2] numpy array or torch tensor; None: the
    ink loss). dL/dxy0 is a numpy array, or a torch tensor on ``device`` when given (then a
    given dL_dxy_T must be a tensor on that device too)."""
    loss = ctypes.c_double()
    dM = np.zeros((n_groups, n_groups), np.float32)
    da = np.zeros(n_passes, np.float32)
    pg, keep, gdev = _arr(dL_dxy_T, np.float32)
    n_t = int(keep.shape[0]) if keep is not None else 0
    if device is not None:
        import torch
        dx = torch.zeros((n_points0, 2), dtype=torch.float32, device=device)
        px, xdev = dx.data_ptr(), True
    else:
        dx = np.zeros((n_points0, 2), np.float32)
        px, xdev = dx.ctypes.data, False
    flags = _flags(gdev if keep is not None else None, xdev)
    _check(ctx, load().hb_backward(ctx, generation, pg, n_t, ctypes.byref(loss), dM.ctypes.data,
                                   da.ctypes.data, px, n_points0, flags))
    return float(loss.value), dM, da, dx


def hb_get_ckpt_decisions(ctx, t: int, n_edges: int, n_samples: int):
    """(sample offsets [E+1], accepted halving per sample [N_t] int8) of checkpoint t."""
    off = np.empty(n_edges + 1, np.int64)
    jacc = np.empty(max(1, n_samples), np.int8)
    _check(ctx, load().hb_get_ckpt_decisions(ctx, t, off.ctypes.data, jacc.ctypes.data, n_samples, 0))
    return off, jacc[:n_samples]


def hb_get_ckpt_points(ctx, t: int, n_edges: int, n_points: int):
    off = np.empty(n_edges + 1, np.int64)
    xy = np.empty((n_points, 2), np.float32)
    _check(ctx, load().hb_get_ckpt_points(ctx, t, off.ctypes.data, xy.ctypes.data, n_points, 0))
    return off, xy


def _bundle_function():
    import torch

    class BundleFn(torch.autograd.Function):
        """The final polylines after ``n_iters`` bundling iterations started at iteration
        ``start_iter``, as a differentiable function of the polylines ``xy0`` (N0 x 2 on the
        context's device, layout ``offsets``), the interaction matrix ``M`` (B x B) and the pass
        weights ``a`` (P), with the discrete choices of the forward run held fixed. Returns
        (xy_T [N_T, 2] float32, offsets_T [E+1] int64, ink float64); the offsets are not
        differentiable, and a loss may use xy_T, the ink, or both. ``bundler`` must already
        hold the graph and its parameters; the forward pass sets M, a, the start iteration and
        the polylines (device to device), runs with per-iteration checkpoints and keeps their
        generation, and the backward pass calls the hand-written adjoint with the gradient of
        the loss, failing with HB_ESTATE if the checkpoints were replaced meanwhile."""

        @staticmethod
        def forward(ctx, xy0, M, a, bundler, offsets, group, n_iters, start_iter, params):
            ctx.set_materialize_grads(False)   # an output the loss does not use gets None
            dev = xy0.device
            if dev.type != "cuda":
                raise ValueError("xy0 must be a tensor on the context's GPU")
            bundler.set_params(**params, pass_weights=[float(v) for v in a.detach().cpu()])
            bundler.set_groups(group, M.detach().cpu().numpy())
            torch.cuda.current_stream(dev).synchronize()   # xy0 complete before the library reads it
            off_in = torch.as_tensor(np.asarray(offsets, np.int64), device=dev)
            bundler.set_points(off_in, xy0.detach().float().contiguous())
            bundler.iteration = int(start_iter)
            ctx.gen = hb_forward_ckpt(bundler.ctx, n_iters)
            off_t, xy_t = bundler.points(HB_POINTS_STATE, device=dev)
            ink = hb_get_ink(bundler.ctx)
            ctx.bundler = bundler
            ctx.shapes = (M.shape[0], a.shape[0], xy0.shape[0])
            ctx.devs = (dev, M.device, a.device)
            ctx.mark_non_differentiable(off_t)
            return xy_t, off_t, torch.tensor(ink, dtype=torch.float64, device=dev)

        @staticmethod
        def backward(ctx, g_xy, g_off, g_ink):
            import torch
            b = ctx.bundler
            dev = ctx.devs[0]
            gi = 0.0 if g_ink is None else float(g_ink)
            outs = []
            # the ink part through the fused ink gradient, the rest through dL/dxy_T
            if gi != 0.0:
                outs.append((gi, hb_backward(b.ctx, *ctx.shapes, generation=ctx.gen, device=dev)))
            if g_xy is not None:
                torch.cuda.current_stream(dev).synchronize()
                gt = g_xy.detach().float().contiguous()
                outs.append((1.0, hb_backward(b.ctx, *ctx.shapes, dL_dxy_T=gt,
                                              generation=ctx.gen, device=dev)))
            dx = torch.zeros(ctx.shapes[2], 2, dtype=torch.float32, device=dev)
            dM = np.zeros((ctx.shapes[0], ctx.shapes[0]), np.float32)
            da = np.zeros(ctx.shapes[1], np.float32)
            for wgt, (_, m, aa, x) in outs:
                dx += wgt * x
                dM += wgt * m
                da += wgt * aa
            return (dx, torch.from_numpy(dM).to(ctx.devs[1]), torch.from_numpy(da).to(ctx.devs[2]),
                    None, None, None, None, None, None)

    return BundleFn


_BUNDLE_FN = None


def bundle_polylines(xy0, M, a, bundler, offsets, group, n_iters, params, start_iter=0):
    """torch entry point of the differentiable form: (xy_T, offsets_T, ink) after n_iters
    iterations from iteration start_iter (see BundleFn)."""
    global _BUNDLE_FN
    if _BUNDLE_FN is None:
        _BUNDLE_FN = _bundle_function()
    return _BUNDLE_FN.apply(xy0, M, a, bundler, offsets, group, n_iters, start_iter, params)


def bundle_ink(xy0, M, a, bundler, offsets, group, n_iters, params, start_iter=0):
    """Ink of the final polylines as a differentiable function of xy0, M and a."""
    return bundle_polylines(xy0, M, a, bundler, offsets, group, n_iters, params, start_iter)[2]
