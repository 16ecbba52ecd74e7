"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/rsv.h declares, and rejects bad arguments on the host before any launch."""
import ctypes as C
import os
import re

import pytest

from paper_1807_07433_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]
FAKE = 0x1000  # non-NULL, aligned; never dereferenced because validation fails first


def declared():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        names |= set(re.findall(r"\b(rsv_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("librsv.so is not built; run __graft_entry__.build()")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "rsv_cost_volume" in names and len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_header(lib):
    assert set(_lib.declared_symbols()) <= set(declared())


def test_status_strings_and_version(lib):
    for s in range(-7, 1):
        assert lib.rsv_status_string(s)
    assert lib.rsv_version() >= 100
    assert lib.rsv_last_hip_error() == 0


def _params(**kw):
    base = dict(D=32, block_radius=3, agg_radius=4, lr_threshold=1, gamma_d=3.0, gamma_r=0.1,
                sigma_min=0.01)
    base.update(kw)
    return _lib.Params(**base)


def _img(h=32, w=48, dtype=_lib.RSV_U8, pitch=None, data=FAKE):
    return _lib.Image(data, dtype, h, w, pitch if pitch is not None else w)


def test_warp_validation(lib):
    pl = _lib.Plane(1.0, 0.1, 0.0, 2.0)
    assert lib.rsv_warp(_img(data=None), pl, FAKE, None) == -1
    assert lib.rsv_warp(_img(), pl, None, None) == -1
    assert lib.rsv_warp(_img(dtype=7), pl, FAKE, None) == -4
    assert lib.rsv_warp(_img(h=0), pl, FAKE, None) == -2
    assert lib.rsv_warp(_img(pitch=10), pl, FAKE, None) == -2
    assert lib.rsv_warp(_img(dtype=_lib.RSV_F32, data=FAKE + 2), pl, FAKE, None) == -5
    assert lib.rsv_warp(_img(), pl, FAKE + 1, None) == -5


@pytest.mark.parametrize("kw,status", [
    (dict(D=0), -2), (dict(D=513), -2), (dict(block_radius=0), -3), (dict(block_radius=5), -3),
    (dict(sigma_min=-1.0), -3)])
def test_cost_validation(lib, kw, status):
    p = _params(**kw)
    assert lib.rsv_cost_volume(_img(), FAKE, C.byref(p), FAKE, FAKE, None) == status


def test_cost_validation_shapes_and_nulls(lib):
    p = _params()
    assert lib.rsv_cost_volume(_img(h=6), FAKE, C.byref(p), FAKE, FAKE, None) == -2
    assert lib.rsv_cost_volume(_img(), None, C.byref(p), FAKE, FAKE, None) == -1
    assert lib.rsv_cost_volume(_img(), FAKE, None, FAKE, FAKE, None) == -1
    assert lib.rsv_cost_volume(_img(), FAKE, C.byref(p), None, FAKE, None) == -1
    assert lib.rsv_cost_volume(_img(), FAKE, C.byref(p), FAKE, FAKE + 2, None) == -5


@pytest.mark.parametrize("kw,status", [
    (dict(agg_radius=0), -3), (dict(agg_radius=7), -3), (dict(gamma_d=0.0), -3),
    (dict(gamma_r=-1.0), -3), (dict(gamma_r=float("nan")), -3), (dict(D=-3), -2)])
def test_aggregate_validation(lib, kw, status):
    p = _params(**kw)
    assert lib.rsv_aggregate(FAKE, _img(), C.byref(p), FAKE + 64, None) == status


def test_aggregate_rejects_aliasing(lib):
    p = _params()
    assert lib.rsv_aggregate(FAKE, _img(), C.byref(p), FAKE, None) == -3


def test_select_validation(lib):
    p = _params()
    ok = [FAKE] * 6
    assert lib.rsv_select_subpixel(FAKE, FAKE, 0, 10, C.byref(p), *ok, None) == -2
    assert lib.rsv_select_subpixel(FAKE, FAKE, 70000, 70000, C.byref(p), *ok, None) == -2  # H*W > 2^31-1
    assert lib.rsv_select_subpixel(None, FAKE, 10, 10, C.byref(p), *ok, None) == -1
    bad = _params(lr_threshold=-1)
    assert lib.rsv_select_subpixel(FAKE, FAKE, 10, 10, C.byref(bad), *ok, None) == -3


def test_triangulate_validation(lib):
    pl = _lib.Plane(1.0, 0.1, 0.0, 2.0)
    cam = _lib.Camera(700.0, 0.12, 10.0, 10.0)
    assert lib.rsv_triangulate(None, FAKE, 10, 10, pl, cam, FAKE, FAKE, None) == -1
    assert lib.rsv_triangulate(FAKE, FAKE, 10, 10, pl, cam, None, None, None) == -1
    assert lib.rsv_triangulate(FAKE, FAKE, 10, 10, pl, _lib.Camera(0.0, 0.12, 1, 1), FAKE, FAKE,
                               None) == -3
    assert lib.rsv_triangulate(FAKE, FAKE, -1, 10, pl, cam, FAKE, FAKE, None) == -2


def test_selected_sum_validation(lib):
    assert lib.rsv_selected_cost_sum(None, FAKE, FAKE, 10, 10, 4, FAKE, None) == -1
    assert lib.rsv_selected_cost_sum(FAKE, FAKE, FAKE, 10, 10, 0, FAKE, None) == -2
    assert lib.rsv_selected_cost_sum(FAKE, FAKE, FAKE, 10, 10, 4, FAKE + 4, None) == -5


def test_adjoint_validation(lib):
    pl = _lib.Plane(1.0, 0.1, 0.0, 2.0)
    p = _params(D=16)
    f32 = _img(dtype=_lib.RSV_F32)
    # cost, plane stride, row stride, disp, mask, gl, gr, gp, loss, ws, stream
    args = [FAKE, 32 * 48, 48] + [FAKE] * 6 + [FAKE, None]
    assert lib.rsv_cost_adjoint_workspace_bytes(10, 20) == 800
    assert lib.rsv_cost_adjoint_workspace_bytes(0, 20) == 0
    assert lib.rsv_cost_adjoint(_img(), f32, pl, C.byref(p), *args) == -4     # u8 left
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(_params(D=257)), *args) == -2
    assert lib.rsv_cost_adjoint(f32, _img(h=31, dtype=_lib.RSV_F32), pl, C.byref(p), *args) == -2
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(_params(agg_radius=9)), *args) == -3
    a = list(args)
    a[9] = None                      # workspace
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(p), *a) == -1
    a = list(args)
    a[0] = None                      # cost
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(p), *a) == -1
    a = list(args)
    a[2] = 47                        # row stride shorter than a row
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(p), *a) == -2
    a = list(args)
    a[1] = 0                         # no plane stride
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(p), *a) == -2
    a = list(args)
    a[7] = FAKE + 4                  # grad_plane must be 8-byte aligned
    assert lib.rsv_cost_adjoint(f32, f32, pl, C.byref(p), *a) == -5


def test_selected_aggregate_sum_validation(lib):
    p = _params(D=16)
    f = lib.rsv_selected_aggregate_sum
    assert f(None, 32 * 48, 48, _img(), C.byref(p), FAKE, FAKE, FAKE, None) == -1
    assert f(FAKE, 32 * 48, 48, _img(), C.byref(p), None, FAKE, FAKE, None) == -1
    assert f(FAKE, 32 * 48, 47, _img(), C.byref(p), FAKE, FAKE, FAKE, None) == -2
    assert f(FAKE, 32 * 48, 48, _img(), C.byref(_params(agg_radius=0)), FAKE, FAKE, FAKE, None) == -3
    assert f(FAKE, 32 * 48, 48, _img(), C.byref(p), FAKE, FAKE, FAKE + 4, None) == -5
    assert f(FAKE, 32 * 48, 48, _img(dtype=7), C.byref(p), FAKE, FAKE, FAKE, None) == -4


@pytest.mark.parametrize("stride", [48 + 32 - 2, 2**31 // 32 + 1])
def test_cost_joint_validation(lib, stride):
    """row_stride must hold W + D - 1 centres and H * row_stride must fit 31 bits."""
    p = _params()
    assert lib.rsv_cost_volume_joint(_img(), FAKE, C.byref(p), FAKE, stride, None) == -2
    assert lib.rsv_cost_volume_joint(_img(), FAKE, C.byref(p), None, 128, None) == -1
    assert lib.rsv_cost_volume_joint(_img(), FAKE, C.byref(_params(D=0)), FAKE, 128, None) == -2
    assert lib.rsv_cost_volume_joint(_img(), FAKE, C.byref(p), FAKE + 2, 128, None) == -5


@pytest.mark.parametrize("ps,rs,status", [
    (32 * 48, 47, -2),            # row stride shorter than a row
    (0, 48, -2),                  # no plane stride
    (2**26 + 1, 48, -2),          # planes too far apart for 32-bit tile offsets
    (32 * 48, 2**22, -2)])        # rows too far apart
def test_aggregate_strided_validation(lib, ps, rs, status):
    p = _params()
    assert lib.rsv_aggregate_strided(FAKE, ps, rs, _img(), C.byref(p), FAKE + 4096, None) == status
    assert lib.rsv_aggregate_strided(None, 32 * 48, 48, _img(), C.byref(p), FAKE, None) == -1
    assert lib.rsv_aggregate_strided(FAKE, 32 * 48, 48, _img(), C.byref(_params(agg_radius=9)),
                                     FAKE + 4096, None) == -3


def test_argmax_and_select_ref_validation(lib):
    p = _params()
    assert lib.rsv_aggregate_argmax(FAKE, 32 * 48, 48, _img(), C.byref(p), None, None) == -1
    assert lib.rsv_aggregate_argmax(None, 32 * 48, 48, _img(), C.byref(p), FAKE, None) == -1
    assert lib.rsv_aggregate_argmax(FAKE, 32 * 48, 47, _img(), C.byref(p), FAKE + 4096, None) == -2
    assert lib.rsv_aggregate_argmax(FAKE, 32 * 48, 48, _img(), C.byref(_params(gamma_d=0.0)),
                                    FAKE + 4096, None) == -3
    assert lib.rsv_aggregate_argmax(FAKE, 32 * 48, 48, _img(), C.byref(p), FAKE + 2, None) == -5
    assert lib.rsv_select_subpixel_ref(FAKE, None, 32, 48, C.byref(p), FAKE, FAKE, FAKE, None, None) == -1
    assert lib.rsv_select_subpixel_ref(FAKE, FAKE, 0, 48, C.byref(p), FAKE, FAKE, FAKE, None, None) == -2
    assert lib.rsv_select_subpixel_ref(FAKE, FAKE, 32, 48, C.byref(_params(lr_threshold=-1)), FAKE, FAKE,
                                       FAKE, None, None) == -3
    # the full form still needs its target volume
    assert lib.rsv_select_subpixel(FAKE, None, 32, 48, C.byref(p), FAKE, FAKE, FAKE, FAKE, None, None) == -1


def test_aggregate_select_validation(lib):
    """rsv_aggregate_select rejects bad arguments before launching: nulls, alignment,
    strides, the radii the LDS-loaded tile cannot take, widths below 4, and select
    parameters."""
    p = _params()
    A, B, Cc, Dd = FAKE, FAKE + 4096, FAKE + 8192, FAKE + 12288
    f = lib.rsv_aggregate_select
    assert f(A, 32 * 48, 48, _img(), C.byref(p), None, B, Cc, Dd, None) == -1
    assert f(A, 32 * 48, 48, _img(), C.byref(p), B, None, Cc, Dd, None) == -1
    assert f(None, 32 * 48, 48, _img(), C.byref(p), B, Cc, Dd, A, None) == -1
    assert f(A, 32 * 48, 48, _img(), C.byref(p), B + 2, Cc, Dd, A, None) == -5
    assert f(A, 32 * 48, 47, _img(), C.byref(p), B, Cc, Dd, A, None) == -2        # row stride < W
    assert f(A, 32 * 48, 48, _img(), C.byref(_params(agg_radius=6)), B, Cc, Dd, A, None) == -3
    assert f(A, 32 * 3, 3, _img(w=3), C.byref(p), B, Cc, Dd, A, None) == -2      # W < 4
    assert f(A, 32 * 48, 48, _img(), C.byref(_params(lr_threshold=-1)), B, Cc, Dd, A, None) == -3
    assert f(A, 32 * 48, 48, _img(), C.byref(_params(gamma_r=0.0)), B, Cc, Dd, A, None) == -3


def test_aggregate_views_and_lr_check_validation(lib):
    """rsv_aggregate_views rejects bad arguments before launching: nulls, alignment,
    strides, guides of different sizes, a target guide that is not float32, a window
    radius out of range; rsv_lr_check: nulls, alignment, sizes and a negative
    tolerance."""
    p = _params()
    A, B, Cc, Dd, E = (FAKE + i * 4096 for i in range(5))
    f = lib.rsv_aggregate_views
    g8, gf = _img(), _img(dtype=1)
    ok = (A, 32 * 48, 48, B, 32 * 48 + 1, 48, g8, gf, C.byref(p), Cc, Dd, E, None)

    def call(**kw):
        args = list(ok)
        for i, v in kw.items():
            args[int(i[1:])] = v
        return f(*args)
    assert call(a0=None) == -1 and call(a3=None) == -1 and call(a9=None) == -1 and call(a11=None) == -1
    assert call(a3=B + 2) == -5 and call(a10=Dd + 2) == -5
    assert call(a2=47) == -2 and call(a5=47) == -2                 # row stride < W
    assert call(a4=0) == -2                                        # plane stride < 1
    assert call(a7=_img(h=31, dtype=1)) == -2                      # guides of different sizes
    assert call(a7=_img()) == -4                                   # target guide must be float32
    assert call(a8=C.byref(_params(lr_threshold=-1))) == -3
    assert call(a8=C.byref(_params(agg_radius=7))) == -3            # beyond RSV_MAX_AGG_RADIUS
    cv = lib.rsv_cost_argmax_views
    assert cv(None, 32 * 48, 48, B, 32 * 48 + 1, 48, 32, 48, 16, Cc, Dd, None) == -1
    assert cv(A, 32 * 48, 48, B, 32 * 48 + 1, 48, 32, 48, 16, Cc, None, None) == -1
    assert cv(A, 32 * 48, 48, B, 32 * 48 + 1, 47, 32, 48, 16, Cc, Dd, None) == -2   # row stride < W
    assert cv(A, 32 * 48, 48, B, 0, 48, 32, 48, 16, Cc, Dd, None) == -2             # plane stride < 1
    assert cv(A, 32 * 48, 48, B, 32 * 48 + 1, 48, 32, 48, 0, Cc, Dd, None) == -2    # D < 1
    assert cv(A, 32 * 48, 48, B + 2, 32 * 48 + 1, 48, 32, 48, 16, Cc, Dd, None) == -5
    rv = lib.rsv_aggregate_restricted_views
    args = list(ok[:9]) + [B, Cc, 2] + list(ok[9:])  # valid: never called, each case breaks one argument
    bad = list(args)
    bad[9] = None
    assert rv(*bad) == -1                                          # coarse_ref
    bad = list(args)
    bad[10] = Cc + 2
    assert rv(*bad) == -5                                          # coarse_tar misaligned
    bad = list(args)
    bad[11] = -1
    assert rv(*bad) == -3                                          # radius < 0
    bad = list(args)
    bad[7] = _img()
    assert rv(*bad) == -4                                          # target guide must be float32
    lr = lib.rsv_lr_check
    assert lr(None, B, 32, 48, 1, Cc, None) == -1
    assert lr(A, B, 32, 48, 1, None, None) == -1
    assert lr(A + 2, B, 32, 48, 1, Cc, None) == -5
    assert lr(A, B, 0, 48, 1, Cc, None) == -2
    assert lr(A, B, 32, 48, -1, Cc, None) == -3


def test_lds_probe_library_loads_and_rejects_bad_arguments():
    """libprobe.so (the LDS bandwidth probe bench.py uses) is built beside librsv.so,
    exports its entry point and rejects bad arguments before launching anything."""
    from paper_1807_07433_amd import build as B
    if not os.path.exists(B.PROBE_LIB):
        pytest.fail("libprobe.so is not built; run __graft_entry__.build()")
    probe = C.CDLL(B.PROBE_LIB)
    fn = probe.rsv_probe_lds_read
    fn.restype = C.c_int
    fn.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    assert fn(12, 1, 1, FAKE, None) == -1   # width must be 8 or 16
    assert fn(16, 0, 1, FAKE, None) == -1   # at least one block
    assert fn(16, 1, 0, FAKE, None) == -1   # at least one iteration
    assert fn(8, 1, 1, None, None) == -1    # output buffer required


def test_restricted_search_validation(lib):
    """rsv_cost_argmax and the restricted aggregations reject bad arguments before
    launching: nulls, alignment, shapes, a negative radius, radius 6 windows and W < 4."""
    p = _params()
    A, B, Cc, Dd, E = FAKE, FAKE + 4096, FAKE + 8192, FAKE + 12288, FAKE + 16384
    assert lib.rsv_cost_argmax(None, 32 * 48, 48, 32, 48, 32, A, None) == -1
    assert lib.rsv_cost_argmax(A, 32 * 48, 48, 32, 48, 32, None, None) == -1
    assert lib.rsv_cost_argmax(A, 32 * 48, 47, 32, 48, 32, B, None) == -2
    assert lib.rsv_cost_argmax(A, 32 * 48, 48, 32, 48, 0, B, None) == -2
    assert lib.rsv_cost_argmax(A, 32 * 48, 48, 32, 48, 513, B, None) == -2
    assert lib.rsv_cost_argmax(A + 2, 32 * 48, 48, 32, 48, 32, B, None) == -5
    f = lib.rsv_aggregate_restricted_argmax
    assert f(A, 32 * 48, 48, _img(), C.byref(p), None, 3, B, None) == -1
    assert f(A, 32 * 48, 48, _img(), C.byref(p), B, 3, None, None) == -1
    assert f(A, 32 * 48, 48, _img(), C.byref(p), B, -1, Cc, None) == -3
    assert f(A, 32 * 48, 48, _img(), C.byref(_params(agg_radius=6)), B, 3, Cc, None) == -3
    assert f(A, 32 * 3, 3, _img(w=3), C.byref(p), B, 3, Cc, None) == -2
    assert f(A, 32 * 48, 47, _img(), C.byref(p), B, 3, Cc, None) == -2
    assert f(A, 32 * 48, 48, _img(), C.byref(p), B + 2, 3, Cc, None) == -5
    g = lib.rsv_aggregate_restricted_select
    assert g(A, 32 * 48, 48, _img(), C.byref(p), B, 3, None, Cc, Dd, E, None) == -1
    assert g(A, 32 * 48, 48, _img(), C.byref(p), B, 3, Cc, Dd, None, E, None) == -1
    assert g(A, 32 * 48, 48, _img(), C.byref(_params(lr_threshold=-1)), B, 3, Cc, Dd, E, A, None) == -3
    assert g(A, 32 * 48, 48, _img(), C.byref(p), B, -2, Cc, Dd, E, A, None) == -3


def test_plane_ransac_validation(lib):
    """rsv_plane_ransac rejects bad arguments before launching: nulls, image and K
    ranges, a negative or NaN threshold, misalignment; the workspace size is 3K + 9
    doubles and 0 for K out of range."""
    A, B, Cc, Dd, E, F, G = (FAKE + i * 4096 for i in range(7))
    f = lib.rsv_plane_ransac
    assert lib.rsv_plane_ransac_workspace_bytes(16) == 8 * (3 * 16 + 9)
    assert lib.rsv_plane_ransac_workspace_bytes(0) == 0
    assert lib.rsv_plane_ransac_workspace_bytes(1025) == 0
    assert f(None, B, 32, 48, Cc, 16, 0.5, Dd, E, F, G, None) == -1
    assert f(A, B, 32, 48, Cc, 16, 0.5, Dd, E, F, None, None) == -1
    assert f(A, B, 0, 48, Cc, 16, 0.5, Dd, E, F, G, None) == -2
    assert f(A, B, 32, 48, Cc, 0, 0.5, Dd, E, F, G, None) == -2
    assert f(A, B, 32, 48, Cc, 1025, 0.5, Dd, E, F, G, None) == -2
    assert f(A, B, 32, 48, Cc, 16, -0.5, Dd, E, F, G, None) == -3
    assert f(A, B, 32, 48, Cc, 16, float("nan"), Dd, E, F, G, None) == -3
    assert f(A + 2, B, 32, 48, Cc, 16, 0.5, Dd, E, F, G, None) == -5
    assert f(A, B, 32, 48, Cc, 16, 0.5, Dd + 4, E, F, G, None) == -5


def test_batch_tuning_defaults_and_plan_validation(lib):
    """rsv_tuning_default fills the documented defaults; rsv_batch_plan_create rejects
    bad arguments before it allocates anything: nulls, an empty batch, tunings out of
    range (a negative volume budget among them), float images, mismatched pair sizes,
    D out of range."""
    from paper_1807_07433_amd.batch import PairDesc, Tuning
    t = Tuning()
    lib.rsv_tuning_default(C.byref(t))
    assert t.as_dict() == {"largest_first": 1, "cost_tiles_per_item": 2, "cost_blocks_per_cu": 0,
                           "agg_blocks_per_cu": 0, "per_pair_launches": 1, "volume_budget_mib": 2048}
    p = _params()

    def pair(**kw):
        d = PairDesc()
        d.left = kw.get("left", _img(h=32, w=48))
        d.right = kw.get("right", _img(h=32, w=48, data=FAKE + 8192))
        d.plane = _lib.Plane(1.0, 0.1, 0.0, 2.0)
        d.camera = _lib.Camera(1000.0, 0.3, 24.0, 16.0)
        d.D = kw.get("D", 16)
        d.disp_sub, d.valid = FAKE + 16384, FAKE + 20480
        return d

    def create(pairs, tuning=None, params=p):
        arr = (PairDesc * len(pairs))(*pairs)
        plan = C.c_void_p()
        return lib.rsv_batch_plan_create(arr, len(pairs), C.byref(params),
                                         C.byref(tuning) if tuning is not None else None, C.byref(plan))

    plan = C.c_void_p()
    assert lib.rsv_batch_plan_create(None, 1, C.byref(p), None, C.byref(plan)) == -1
    arr = (PairDesc * 1)(pair())
    assert lib.rsv_batch_plan_create(arr, 0, C.byref(p), None, C.byref(plan)) == -2
    for field, bad in (("cost_tiles_per_item", 0), ("cost_tiles_per_item", 17), ("cost_blocks_per_cu", -2),
                       ("agg_blocks_per_cu", -1), ("volume_budget_mib", -1)):
        tb = Tuning()
        lib.rsv_tuning_default(C.byref(tb))
        setattr(tb, field, bad)
        assert create([pair()], tb) == -3, field
    assert create([pair(left=_img(h=32, w=48, dtype=_lib.RSV_F32))]) == -4
    assert create([pair(right=_img(h=31, w=48, data=FAKE + 8192))]) == -2
    assert create([pair(D=0)]) == -2 and create([pair(D=_lib.RSV_MAX_D + 1)]) == -2
    assert create([pair()], params=_params(agg_radius=9)) == -3
