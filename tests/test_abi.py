"""The C-ABI library loads, exports every function include/itc_lattice.h declares,
and rejects bad arguments on the host before touching the device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "itc_lattice.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(itc_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def itc():
    from paper_1310_7114_amd import itc as m
    m.load()
    return m


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("itc_lattice_precompute", "itc_lattice_fit", "itc_lattice_divergence",
                 "itc_lattice_divergence_backward", "itc_lattice_plan_create", "itc_lattice_run_batched"):
        assert must in names


def test_library_exports_every_declared_symbol(itc):
    lib = itc.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding knows every declared function too
    assert set(declared_functions()) <= set(itc.SIGNATURES)


def test_desc_layout_matches_header(itc):
    # int32 H, W; int64 pitch; int32 x2; double x2; int32 x2  -> 48 bytes
    assert ctypes.sizeof(itc.Desc) == 48


def test_sizes_and_radius(itc):
    lib = itc.load()
    d = itc.make_desc(100, 130, 4.0)
    assert lib.itc_lattice_radius(ctypes.byref(d)) == 12
    # planes: ceil(130/16) = 9 panels of 16 columns x 100 rows
    assert lib.itc_lattice_plane_elems(ctypes.byref(d)) == 9 * 100 * 16
    planes = 3 * 9 * 100 * 16 * 4
    parts = 3 * 2 * 4          # ceil(130/64) strips x ceil(100/64) row groups x 4 slots, FP64
    assert itc.maps_bytes(d) == ((planes + 7) // 8 * 8 + 8 * parts + 255) // 256 * 256
    # 2048 x 2048: 128 panels; 32 strips x 32 row groups x 4 partials
    dl = itc.make_desc(2048, 2048, 6.0)
    assert itc.maps_bytes(dl) == (3 * 2048 * 2048 * 4 + 8 * 32 * 32 * 4 + 255) // 256 * 256
    d2 = itc.make_desc(10, 10, 2.0, radius=5)
    assert lib.itc_lattice_radius(ctypes.byref(d2)) == 5
    d3 = itc.make_desc(10, 10, 2.5)
    assert lib.itc_lattice_radius(ctypes.byref(d3)) == 8


@pytest.mark.parametrize("field,value,status", [
    ("height", 0, 2), ("width", -3, 2), ("pitch", 5, 2), ("sigma", 0.0, 2), ("sigma", float("nan"), 2),
    ("weight_dtype", 7, 2), ("real_dtype", 0, 2), ("radius", -1, 2), ("reserved", 1, 2),
    ("radius", 33, 3), ("sigma", 11.0, 3),
])
def test_bad_descriptors_rejected(itc, field, value, status):
    lib = itc.load()
    d = itc.make_desc(16, 16, 2.0)
    setattr(d, field, value)
    st = lib.itc_lattice_precompute(ctypes.byref(d), ctypes.c_void_p(256), ctypes.c_void_p(256),
                                    ctypes.c_void_p(256), None)
    assert st == status, lib.itc_last_error()
    assert lib.itc_last_error()  # a reason is given
    assert lib.itc_lattice_maps_bytes(ctypes.byref(d)) == 0


def test_f64_radius_limit(itc):
    lib = itc.load()
    d = itc.make_desc(16, 16, 2.0, real_dtype=__import__("torch").float64, radius=25)
    assert lib.itc_lattice_precompute(ctypes.byref(d), ctypes.c_void_p(256), ctypes.c_void_p(256),
                                      ctypes.c_void_p(256), None) == 3


def test_null_and_range_arguments(itc):
    lib = itc.load()
    P = ctypes.c_void_p(256)
    assert lib.itc_lattice_precompute(None, P, P, P, None) == 1
    d = itc.make_desc(16, 16, 2.0)
    assert lib.itc_lattice_precompute(ctypes.byref(d), None, P, P, None) == 1
    assert lib.itc_lattice_precompute(ctypes.byref(d), P, ctypes.c_void_p(260), P, None) == 2  # misaligned maps
    fit = lib.itc_lattice_fit
    assert fit(ctypes.byref(d), P, P, 0, P, 10, -1.0, P, None, None, None) == 2          # M = 0
    assert fit(ctypes.byref(d), P, P, 1025, P, 10, -1.0, P, None, None, None) == 3       # M too large
    assert fit(ctypes.byref(d), P, P, 4, P, -1, -1.0, P, None, None, None) == 2          # iters < 0
    assert fit(ctypes.byref(d), P, P, 4, P, 3, float("nan"), P, None, None, None) == 2   # theta NaN
    assert fit(ctypes.byref(d), P, None, 4, P, 3, -1.0, P, P, None, None) == 1           # trace needs s_x
    assert fit(ctypes.byref(d), None, P, 4, P, 3, -1.0, P, None, None, None) == 1
    assert lib.itc_lattice_divergence(ctypes.byref(d), P, P, 4, P, None, None) == 1
    assert lib.itc_lattice_fit_batched(None, P, P, -1.0, P, None, None, None, None, None) == 1
    assert lib.itc_lattice_plan_size(None) == -1
    lib.itc_lattice_plan_destroy(None)
    # autotuning hooks of the convolution's tile shapes
    assert lib.itc_lattice_plan_conv_classes(None) == -1
    assert lib.itc_lattice_plan_conv_class(None, 0, None, None, None, None) == 1
    assert lib.itc_lattice_plan_set_conv_shape(None, 0, 256, 0) == 1


def test_fit_wide_arguments(itc):
    import torch
    lib = itc.load()
    P = ctypes.c_void_p(256)
    wb = lib.itc_lattice_fit_wide_work_bytes
    assert wb(0) == 0 and wb(1025) == 0
    n = wb(500)
    assert n > 0 and n % 256 == 0 and n >= 500 * (2 * 16 + 2 * 32)   # positions and terms, double buffered
    fw = lib.itc_lattice_fit_wide
    d = itc.make_desc(16, 16, 2.0)
    args = lambda **k: dict(dict(d=ctypes.byref(d), maps=P, s_x=P, M=4, w=P, iters=3, theta=-1.0, out=P,  # noqa: E731
                                 trace=None, done=None, work=P, nb=wb(4), s=None), **k)
    call = lambda a: fw(*a.values())  # noqa: E731
    assert call(args(M=0)) == 2 and call(args(M=1025)) == 3 and call(args(iters=-1)) == 2
    assert call(args(theta=float("nan"))) == 2
    assert call(args(work=None)) == 1 and call(args(maps=None)) == 1
    assert call(args(s_x=None, trace=P)) == 1                          # the trace needs s_x
    assert call(args(nb=wb(4) - 1)) == 2                               # work buffer too small
    assert call(args(work=ctypes.c_void_p(512 + 64))) == 2            # misaligned work
    d64 = itc.make_desc(16, 16, 2.0, real_dtype=torch.float64)
    assert call(args(d=ctypes.byref(d64))) == 3                        # FP32 maps only


def test_literal_density_arguments(itc):
    lib = itc.load()
    P = ctypes.c_void_p(256)
    d = itc.make_desc(300, 360, 28.0, radius=1)   # recursive maps: any width
    wb = lib.itc_lattice_literal_density_work_bytes
    n = wb(ctypes.byref(d), 4, 56.0, 0)
    assert n > 0 and n % 256 == 0 and n < lib.itc_lattice_literal_work_bytes(ctypes.byref(itc.make_desc(300, 360, 5.0)), 4, 56.0, 0)
    assert wb(ctypes.byref(d), 4, 90.0, 0) == 0       # ceil(3 omega) beyond ITC_MAX_LITERAL_RADIUS
    assert wb(ctypes.byref(d), 0, 56.0, 0) == 0
    fd = lib.itc_lattice_literal_fit_density
    assert fd(ctypes.byref(d), None, 56.0, 0, 4, P, 5, -1.0, P, None, None, P, None) == 1   # maps NULL
    assert fd(ctypes.byref(d), P, 56.0, 0, 4, P, 5, -1.0, P, None, None, None, None) == 1   # work NULL
    assert fd(ctypes.byref(d), ctypes.c_void_p(512 + 4), 56.0, 0, 4, P, 5, -1.0, P, None, None, P, None) == 2
    assert fd(ctypes.byref(d), P, 0.0, 0, 4, P, 5, -1.0, P, None, None, P, None) == 2      # omega
    assert fd(ctypes.byref(d), P, 90.0, 0, 4, P, 5, -1.0, P, None, None, P, None) == 3     # window too wide
    d64 = itc.make_desc(300, 360, 28.0, real_dtype=__import__("torch").float64, radius=1)
    assert fd(ctypes.byref(d64), P, 56.0, 0, 4, P, 5, -1.0, P, None, None, P, None) == 3


def test_chamfer_arguments(itc):
    lib = itc.load()
    P = ctypes.c_void_p(256)
    ch = lib.itc_lattice_chamfer
    d = itc.make_desc(16, 16, 1.0)
    assert ch(None, P, 3, 4, P, None) == 1
    assert ch(ctypes.byref(d), None, 3, 4, P, None) == 1
    assert ch(ctypes.byref(d), P, 3, 4, None, None) == 1
    for a, b in ((0, 0), (3, 2), (3, 7), (65, 65), (-1, 1)):
        assert ch(ctypes.byref(d), P, a, b, P, None) == 2, (a, b)
    df = itc.make_desc(16, 16, 1.0, weight_dtype=__import__("torch").float32)
    assert ch(ctypes.byref(df), P, 3, 4, P, None) == 2             # binary images are ITC_U8
    dw = itc.make_desc(2, 16385, 1.0)
    assert ch(ctypes.byref(dw), P, 3, 4, P, None) == 3             # wider than ITC_MAX_CHAMFER_WIDTH
    dt = itc.make_desc(65536, 4, 1.0)
    assert ch(ctypes.byref(dt), P, 3, 4, P, None) == 3             # taller than ITC_MAX_CHAMFER_HEIGHT
    dp = itc.make_desc(4, 16, 1.0, pitch=8)
    assert ch(ctypes.byref(dp), P, 3, 4, P, None) == 2             # pitch < width
    assert lib.itc_lattice_chamfer_batched(None, P, 3, 4, P, None) == 1


def test_literal_arguments(itc):
    import torch
    lib = itc.load()
    P = ctypes.c_void_p(256)
    d = itc.make_desc(64, 70, 2.5)
    wb = lib.itc_lattice_literal_work_bytes
    n = wb(ctypes.byref(d), 16, 5.0, 0)
    assert n > 0 and n % 256 == 0 and n >= itc.maps_bytes(d)
    assert wb(ctypes.byref(d), 16, 0.0, 0) == 0           # omega must be > 0
    assert wb(ctypes.byref(d), 16, 100.0, 0) == 0         # ceil(3 omega) beyond ITC_MAX_LITERAL_RADIUS
    assert wb(ctypes.byref(d), 16, 2.0, 257) == 0
    assert wb(ctypes.byref(d), 0, 2.0, 0) == 0
    assert wb(None, 16, 2.0, 0) == 0
    fit = lib.itc_lattice_literal_fit
    assert fit(ctypes.byref(d), None, 5.0, 0, 16, P, 10, -1.0, P, None, None, P, None) == 1
    assert fit(ctypes.byref(d), P, 5.0, 0, 16, P, 10, -1.0, P, None, None, None, None) == 1
    assert fit(ctypes.byref(d), P, -1.0, 0, 16, P, 10, -1.0, P, None, None, P, None) == 2
    assert fit(ctypes.byref(d), P, 5.0, 0, 0, P, 10, -1.0, P, None, None, P, None) == 2
    assert fit(ctypes.byref(d), P, 5.0, 0, 16, P, -1, -1.0, P, None, None, P, None) == 2
    assert fit(ctypes.byref(d), P, 5.0, 0, 16, P, 10, float("nan"), P, None, None, P, None) == 2
    assert fit(ctypes.byref(d), P, 5.0, 0, 16, P, 10, -1.0, P, None, None, ctypes.c_void_p(264), None) == 2
    assert fit(ctypes.byref(d), P, 5.0, 300, 16, P, 10, -1.0, P, None, None, P, None) == 3
    d64 = itc.make_desc(64, 70, 2.5, real_dtype=torch.float64)
    assert fit(ctypes.byref(d64), P, 5.0, 0, 16, P, 10, -1.0, P, None, None, P, None) == 3


def test_label_arguments(itc):
    lib = itc.load()
    P = ctypes.c_void_p(256)
    d = itc.make_desc(16, 16, 1.0)
    assert lib.itc_lattice_label(ctypes.byref(d), None, 4, P, P, None) == 1
    assert lib.itc_lattice_label(ctypes.byref(d), P, 4, None, P, None) == 1
    assert lib.itc_lattice_label(ctypes.byref(d), P, 4, P, None, None) == 1
    assert lib.itc_lattice_label(ctypes.byref(d), P, 0, P, P, None) == 2
    assert lib.itc_lattice_label(ctypes.byref(d), P, 1025, P, P, None) == 3
    assert lib.itc_lattice_label_batched(None, P, P, P, None) == 1


def test_volume_arguments(itc):
    lib = itc.load()
    assert ctypes.sizeof(itc.VolumeDesc) == 56
    P = ctypes.c_void_p(256)
    d = itc.VolumeDesc(8, 9, 10, 0, 10, 90, 0, 0, 1.0, 2.0)
    n = lib.itc_volume_maps_bytes(ctypes.byref(d))
    # FP64 S_X partials: one per workgroup of the depth pass (64 columns x 4 rows x 8 slices)
    assert n == (4 * 720 * 4 + 8 * (1 * 3 * 1) + 255) // 256 * 256
    assert lib.itc_volume_work_bytes(ctypes.byref(d)) == (3 * 720 * 4 + 255) // 256 * 256
    bad = [("depth", 0, 2), ("row_pitch", 9, 2), ("slice_pitch", 80, 2), ("weight_dtype", 9, 2), ("reserved", 1, 2),
           ("sigma", 0.0, 2), ("radius", -1, 2), ("radius", 33, 3), ("sigma", 30.0, 3)]
    for field, value, status in bad:
        e = itc.VolumeDesc(8, 9, 10, 0, 10, 90, 0, 0, 1.0, 2.0)
        setattr(e, field, value)
        assert lib.itc_volume_maps_bytes(ctypes.byref(e)) == 0, field
        assert lib.itc_volume_precompute(ctypes.byref(e), P, P, P, P, None) == status, field
    assert lib.itc_volume_precompute(ctypes.byref(d), None, P, P, P, None) == 1
    assert lib.itc_volume_precompute(ctypes.byref(d), P, ctypes.c_void_p(260), P, P, None) == 2
    fit = lib.itc_volume_fit
    assert fit(ctypes.byref(d), P, P, 0, P, 5, -1.0, P, None, None, None) == 2
    assert fit(ctypes.byref(d), P, P, 1025, P, 5, -1.0, P, None, None, None) == 3
    assert fit(ctypes.byref(d), P, None, 4, P, 5, -1.0, P, None, None, None) == 1
    assert fit(ctypes.byref(d), P, P, 4, P, -2, -1.0, P, None, None, None) == 2


def test_plan_rejects_bad_batches(itc):
    lib = itc.load()
    h = ctypes.c_void_p()
    assert lib.itc_lattice_plan_create(None, ctypes.byref(h)) == 1
    n = 2
    descs = (itc.Desc * n)(itc.make_desc(8, 8, 1.0), itc.make_desc(8, 8, 1.0))
    z64 = (ctypes.c_int64 * n)(0, 0)
    ms = (ctypes.c_int32 * n)(4, 0)                       # M = 0 for image 1
    it = (ctypes.c_int32 * n)(3, 3)
    b = itc.Batch(n, descs, z64, z64, ms, z64, it)
    assert lib.itc_lattice_plan_create(ctypes.byref(b), ctypes.byref(h)) == 2
    assert b"image 1" in lib.itc_last_error()
    ms2 = (ctypes.c_int32 * n)(4, 4)
    moff = (ctypes.c_int64 * n)(0, 100)                   # misaligned map offset
    b2 = itc.Batch(n, descs, z64, moff, ms2, z64, it)
    assert lib.itc_lattice_plan_create(ctypes.byref(b2), ctypes.byref(h)) == 2
    descs[1].real_dtype = 2
    b3 = itc.Batch(n, descs, z64, z64, ms2, z64, it)
    assert lib.itc_lattice_plan_create(ctypes.byref(b3), ctypes.byref(h)) == 3
    assert lib.itc_lattice_plan_create(ctypes.byref(itc.Batch(0, descs, z64, z64, ms2, z64, it)),
                                       ctypes.byref(h)) == 2


def test_status_strings(itc):
    lib = itc.load()
    assert lib.itc_status_str(0) == b"ok"
    assert lib.itc_status_str(3) == b"unsupported size"
