"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
validates parameters on the host (argument errors come back as codes, never aborts)."""

import ctypes
import os
import re

import pytest

import paper_1504_02687_amd as hb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hb_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(hb.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(hb.exported_symbols())


def test_default_params_are_the_papers():
    p = hb.hb_default_params(800, 600)
    assert p.struct_size == ctypes.sizeof(hb.hb_params)
    assert (p.grid_w, p.grid_h, p.box_passes, p.max_halvings, p.smooth_passes) == (800, 600, 3, 8, 1)
    assert p.lambda_ == pytest.approx(0.9) and p.delta_px == 1.0 and p.smooth_weight == 0.5
    assert p.radius_per_iter[0] == 600 // 32
    assert hb.hb_validate_params(p) == hb.HB_OK


@pytest.mark.parametrize("field,value", [
    ("grid_w", 1), ("grid_h", 9000), ("delta_px", 0.0), ("delta_px", float("nan")),
    ("box_passes", 0), ("box_passes", 9), ("lambda_", 0.0), ("lambda_", 1.5), ("eps", 0.0),
    ("max_halvings", -2), ("max_halvings", 31), ("smooth_weight", 1.5), ("smooth_passes", 2),
    ("capacity_factor", 1.05), ("h_max_px", float("inf")), ("struct_size", 4), ("n_radii", 0),
    ("directed_offset_px", 4.5), ("directed_offset_px", -4.5), ("directed_offset_px", float("nan")),
    ("splat_mode", 2), ("splat_mode", -1), ("resample_mode", 2), ("delta_min_px", 1.0),
    ("delta_min_px", -0.5),
])
def test_invalid_params_rejected(field, value):
    p, keep = hb.make_params(64, 64, [3])
    setattr(p, field, value)
    assert hb.hb_validate_params(p) == hb.HB_EINVAL
    assert hb.hb_last_error() != ""


def test_build_module_is_reachable():
    """The build step the entry point calls is the submodule, not a package attribute."""
    import importlib
    m = importlib.import_module("paper_1504_02687_amd.build")
    assert callable(m.build) and m.LIB.endswith("libhb.so")
    import __graft_entry__
    assert callable(__graft_entry__.build) and callable(__graft_entry__.smoke)


def test_fixed_step_mode_accepted():
    p, keep = hb.make_params(64, 64, [3], max_halvings=-1)
    assert hb.hb_validate_params(p) == hb.HB_OK


def test_sigma_schedule_checks():
    p, keep = hb.make_params(64, 64, [3], sigmas=[2.5, 1.0])
    assert hb.hb_validate_params(p) == hb.HB_OK
    for bad in ([0.0], [float("nan")], [40.0]):          # 40 px needs boxes wider than 64
        p, keep = hb.make_params(64, 64, [3], sigmas=bad)
        assert hb.hb_validate_params(p) == hb.HB_EINVAL, bad
    p, keep = hb.make_params(64, 64, [3])
    p.n_sigmas = 1                                      # NULL sigma list
    assert hb.hb_validate_params(p) == hb.HB_EINVAL


def test_directed_offset_range():
    # |offset| <= max(W, H) / 16: 4 px on a 64 x 32 grid
    for v in (0.0, 0.5, -4.0, 4.0):
        p, keep = hb.make_params(64, 32, [3], directed_offset=v)
        assert hb.hb_validate_params(p) == hb.HB_OK, v
    assert hb.hb_default_params(64, 64).directed_offset_px == 0.0


def test_radius_and_bbox_checks():
    p, keep = hb.make_params(64, 32, [16])          # 2r+1 = 33 > min(W, H) = 32
    assert hb.hb_validate_params(p) == hb.HB_EINVAL
    p, keep = hb.make_params(64, 32, [15, 3])
    assert hb.hb_validate_params(p) == hb.HB_OK
    p, keep = hb.make_params(64, 32, [3], bbox=(1.0, 0.0, 0.5, 1.0))
    assert hb.hb_validate_params(p) == hb.HB_EINVAL
    p, keep = hb.make_params(64, 32, [3], pass_weights=[0.1, float("nan"), 1.0])
    assert hb.hb_validate_params(p) == hb.HB_EINVAL


def test_null_arguments_return_codes():
    lib = hb.load()
    assert lib.hb_validate_params(None) == hb.HB_EINVAL
    assert lib.hb_set_params(None, None) == hb.HB_EINVAL
    assert lib.hb_run(None, 1, 0) == hb.HB_EINVAL
    assert lib.hb_sync(None) == hb.HB_EINVAL
    lib.hb_destroy(None)
    assert lib.hb_create(None, 0, None) == hb.HB_EINVAL


def test_create_without_device_reports_error():
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("a GPU is present")
    ctx = ctypes.c_void_p()
    st = hb.load().hb_create(ctypes.byref(ctx), 0, None)
    assert st == hb.HB_EDEVICE
    assert "device" in hb.hb_last_error().lower()


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "hb.h")).read()
    assert int(re.search(r"#define HB_MAX_EDGE_WEIGHT (\d+)", text).group(1)) == hb.HB_MAX_EDGE_WEIGHT
    assert int(re.search(r"HB_NUM_STAGES = (\d+)", text).group(1)) == len(hb.STAGES)
    for name in ("HB_EINVAL", "HB_ENOMEM", "HB_EDEVICE", "HB_ESTATE", "HB_EOVERFLOW", "HB_EINTERNAL"):
        v = int(re.search(name + r" = (-\d+)", text).group(1))
        assert getattr(hb, name) == v and hb.STATUS_NAMES[v] == name
