"""The C-ABI library on the CPU: it loads, exports every symbol its header
declares, and rejects bad arguments before touching the GPU (no compute
calls are made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "binarize.h")


@pytest.fixture(scope="module")
def L():
    import paper_1210_3165_amd as bz
    if not os.path.exists(bz.library_path()):
        from paper_1210_3165_amd import build
        build.build()
    return bz.lib()


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"defined"})


def test_header_declares_entry_points():
    names = declared_functions()
    for n in ("binarize", "binarize_async", "binarize_stats", "binarize_strerror",
              "binarize_version", "binarize_last_hip_error", "binarize_tuned",
              "binarize_default_tile"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in declared_functions():
        assert hasattr(L, name), f"libbinarize.so does not export {name}"


def test_version_and_strerror(L):
    assert L.binarize_version() == 1
    for code in range(0, -11, -1):
        s = L.binarize_strerror(code)
        assert isinstance(s, bytes) and len(s) > 0
    assert L.binarize_strerror(-999) == b"unknown error"


FAKE_IN = 0x10000000
FAKE_OUT = 0x20000000


@pytest.mark.parametrize("args,code", [
    ((None, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -1),           # null img
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, None), -1),            # null out
    ((FAKE_IN, 0, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -2),         # H < 1
    ((FAKE_IN, 16, -3, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -2),        # W < 1
    ((FAKE_IN, 65536, 32768, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -2),  # 2^31 pixels
    ((FAKE_IN, 16, 16, 4, 15, 0.5, 128.0, 0, FAKE_OUT), -3),        # RGBA
    ((FAKE_IN, 16, 16, 1, 0, 0.5, 128.0, 0, FAKE_OUT), -4),         # win 0
    ((FAKE_IN, 16, 16, 1, 256, 0.5, 128.0, 0, FAKE_OUT), -4),       # win 256
    ((FAKE_IN, 16, 16, 1, 15, float("nan"), 128.0, 0, FAKE_OUT), -5),
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 0.0, 0, FAKE_OUT), -5),          # R = 0
    ((FAKE_IN, 16, 16, 1, 15, 0.5, float("inf"), 0, FAKE_OUT), -5),
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 2, FAKE_OUT), -6),        # rule
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_IN + 100), -7),   # out inside img
    ((FAKE_IN, 16, 16, 3, 15, 0.5, 128.0, 0, FAKE_IN + 700), -7),   # RGB img is 768 B
])
def test_invalid_arguments_are_rejected_before_launch(L, args, code):
    vp = ctypes.c_void_p
    a = [vp(x) if i in (0, 8) else x for i, x in enumerate(args)]
    assert L.binarize(*a) == code
    assert L.binarize_async(*a, None) == code


@pytest.mark.parametrize("rule,k,R,code", [
    (0, 1.0001, 128.0, -5),    # |k| > 1
    (0, -1.5, 128.0, -5),
    (1, 2.0, 128.0, -5),
    (0, 0.5, 63.99, -5),       # Sauvola R < 64
    (0, 0.5, 1.0, -5),
    (1, -0.2, -1.0, -5),       # R must still be positive for Niblack
])
def test_parameter_range(L, rule, k, R, code):
    """Outside |k| <= 1 (and R >= 64 for Sauvola) the 1e-4 threshold bound
    does not hold, so the call is refused before any launch."""
    vp = ctypes.c_void_p
    assert L.binarize(vp(FAKE_IN), 16, 16, 1, 15, k, R, rule, vp(FAKE_OUT)) == code


@pytest.mark.parametrize("rule,k,R", [(0, 1.0, 64.0), (0, -1.0, 64.0), (1, -1.0, 1.0), (1, 1.0, 0.5)])
def test_parameter_range_limits_pass_validation(L, rule, k, R):
    """The limits themselves are accepted: validation passes and the call
    goes on to the launch (which needs a GPU, so here it may only fail in the
    HIP runtime, never with BZ_ERR_PARAM)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("would launch on the GPU with fake pointers")
    vp = ctypes.c_void_p
    assert L.binarize(vp(FAKE_IN), 16, 16, 1, 15, k, R, rule, vp(FAKE_OUT)) not in (-1, -2, -3, -4, -5, -6, -7)


def _pitched(L):
    vp, i, f, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_float, ctypes.c_int64
    L.binarize_pitched.argtypes = [vp, i, i, i, i64, i, f, f, i, vp, i64, vp]
    L.binarize_pitched.restype = i
    return L.binarize_pitched


@pytest.mark.parametrize("img,H,W,C,pin,out,pout,code", [
    (FAKE_IN, 16, 16, 1, 15, FAKE_OUT, 0, -2),            # input pitch below the row
    (FAKE_IN, 16, 16, 3, 47, FAKE_OUT, 0, -2),
    (FAKE_IN, 16, 16, 1, 0, FAKE_OUT, 15, -2),            # output pitch below the row
    (FAKE_IN, 16, 16, 1, -32, FAKE_OUT, 0, -2),           # negative pitch
    (FAKE_IN, 16, 16, 1, 64, FAKE_IN + 8, 64, -7),        # output rows straddle input rows
    (FAKE_IN, 16, 48, 1, 64, FAKE_IN + 40, 64, -7),       # output row i starts in input row i
    (FAKE_IN, 16, 16, 1, 64, FAKE_IN + 64 * 15 + 4, 64, -7),  # output row 0 inside the last input row
    (FAKE_IN, 16, 16, 1, 64, FAKE_IN - 64 * 15 + 12, 64, -7),  # last output row over input row 0
    (None, 16, 16, 1, 64, FAKE_OUT, 64, -1),
])
def test_pitched_invalid_arguments(L, img, H, W, C, pin, out, pout, code):
    fn = _pitched(L)
    vp = ctypes.c_void_p
    assert fn(vp(img) if img else None, H, W, C, pin, 15, 0.5, 128.0, 0, vp(out), pout, None) == code


def test_pitched_interleaved_rows_pass_alias_check(L):
    """Input and output rows interleaved in one buffer, never sharing a byte:
    the exact strided test accepts them (the call proceeds to the launch)."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("would launch on the GPU with fake pointers")
    fn = _pitched(L)
    vp = ctypes.c_void_p
    # input rows at [64 i, 64 i + 16), output rows at [64 i + 32, 64 i + 48)
    assert fn(vp(FAKE_IN), 16, 16, 1, 64, 15, 0.5, 128.0, 0, vp(FAKE_IN + 32), 64, None) not in (-2, -7)


def test_batch_one_call_arguments(L):
    import paper_1210_3165_amd as bz
    Lb = bz._batch_lib()
    assert Lb.binarize_batch(None, 1, None) == -1
    arr = (bz._Page * 1)()
    assert Lb.binarize_batch(arr, 0, None) == -2
    arr[0] = bz._Page(FAKE_IN, FAKE_IN + 8, 16, 16, 1, 15, 0.5, 128.0, 0, 0, 0, 0, 0)
    assert Lb.binarize_batch(arr, 1, None) in (-7, -8)  # alias, or the HIP runtime without a GPU


def test_stats_planes_must_not_alias(L):
    vp = ctypes.c_void_p
    base = [vp(FAKE_IN), 16, 16, 1, 15, 0.5, 128.0, 0, vp(FAKE_OUT)]
    planes = [vp(0x30000000), vp(0x30000000 + 16), None, None, None]  # gray overlaps s1
    assert L.binarize_stats(*base, *planes, None) == -7
    planes = [None, vp(FAKE_OUT + 8), None, None, None]  # s1 overlaps out
    assert L.binarize_stats(*base, *planes, None) == -7


@pytest.mark.parametrize("tile", [(64, 64), (256, 4), (256, 12), (128, 8192), (0, 64), (512, 64)])
def test_bad_tiles_are_rejected(L, tile):
    vp = ctypes.c_void_p
    rc = L.binarize_tuned(vp(FAKE_IN), 64, 64, 1, 15, 0.5, 128.0, 0, vp(FAKE_OUT),
                          tile[0], tile[1], None)
    assert rc == -9


def test_wide_window_needs_narrow_tile(L):
    vp = ctypes.c_void_p
    # a 255-wide window does not fit the 256-column tile's LDS budget
    rc = L.binarize_tuned(vp(FAKE_IN), 64, 64, 1, 255, 0.5, 128.0, 0, vp(FAKE_OUT), 256, 64, None)
    assert rc == -9


def test_default_tile_shapes(L):
    tw, th = ctypes.c_int(), ctypes.c_int()
    for win in (1, 15, 31, 61, 101, 151, 201, 255):
        assert L.binarize_default_tile(4096, 4096, 1, win, ctypes.byref(tw), ctypes.byref(th)) == 0
        assert tw.value in (128, 256)
        assert th.value % 8 == 0 and 8 <= th.value <= 4096
    assert L.binarize_default_tile(100, 100, 1, 255, ctypes.byref(tw), ctypes.byref(th)) == 0
    assert tw.value == 128
    assert L.binarize_default_tile(100, 100, 2, 15, ctypes.byref(tw), ctypes.byref(th)) == -3


def test_python_binding_refuses_cpu_tensors():
    import torch
    import paper_1210_3165_amd as bz
    with pytest.raises(ValueError):
        bz.binarize(torch.zeros((8, 8), dtype=torch.uint8), 3, 0.5)
    with pytest.raises(TypeError):
        bz.binarize(torch.zeros((8, 8), dtype=torch.float32), 3, 0.5)


FAKE_WS = 0x30000000
WS = 4096 + 512 * 1024  # BZ_OTSU_WS_BYTES


@pytest.mark.parametrize("args,code", [
    ((None, 16, 16, 1, FAKE_OUT, FAKE_WS, WS), -1),              # null img
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, None, WS), -10),             # null workspace
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, FAKE_WS, WS - 1), -10),      # workspace too small
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, FAKE_WS + 2, WS), -10),      # misaligned workspace
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, FAKE_WS + 4, WS), -10),      # not 16-byte aligned
    ((FAKE_IN, 0, 16, 1, FAKE_OUT, FAKE_WS, WS), -2),            # H < 1
    ((FAKE_IN, 65536, 32768, 1, FAKE_OUT, FAKE_WS, WS), -2),     # 2^31 pixels
    ((FAKE_IN, 16, 16, 2, FAKE_OUT, FAKE_WS, WS), -3),           # two channels
    ((FAKE_IN, 16, 16, 3, FAKE_IN + 700, FAKE_WS, WS), -7),      # out inside the RGB img
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, FAKE_IN + 208, WS), -7),     # workspace over img
    ((FAKE_IN, 16, 16, 1, FAKE_OUT, FAKE_OUT - 112, WS), -7),    # workspace over out
])
def test_otsu_invalid_arguments(L, args, code):
    vp = ctypes.c_void_p
    L.binarize_otsu.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp,
                                ctypes.c_size_t, vp]
    a = [vp(x) if i in (0, 4, 5) else x for i, x in enumerate(args)]
    assert L.binarize_otsu(*a, None) == code


def test_otsu_workspace_contract(L):
    vp = ctypes.c_void_p
    L.binarize_otsu_workspace_size.restype = ctypes.c_size_t
    assert L.binarize_otsu_workspace_size() == WS


@pytest.mark.parametrize("args,code", [
    ((None, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -1),           # null img
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, None), -1),            # null out
    ((FAKE_IN, 0, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT), -2),         # H < 1
    ((FAKE_IN, 16, 16, 4, 15, 0.5, 128.0, 0, FAKE_OUT), -3),        # RGBA
    ((FAKE_IN, 16, 16, 1, 14, 0.5, 128.0, 0, FAKE_OUT), -4),        # even window
    ((FAKE_IN, 16, 16, 1, 257, 0.5, 128.0, 0, FAKE_OUT), -4),       # too wide
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 3, FAKE_OUT), -5),        # unknown structure
    ((FAKE_IN, 16, 16, 1, 15, 0.5, -1.0, 0, FAKE_OUT), -5),         # R' <= 0
    ((FAKE_IN, 16, 16, 1, 15, float("inf"), 128.0, 0, FAKE_OUT), -5),
    ((FAKE_IN, 16, 16, 1, 15, 1.5, 128.0, 0, FAKE_OUT), -5),        # |k| > 1
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 32.0, 0, FAKE_OUT), -5),         # R' < 64
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 2, FAKE_IN + 10), -7),    # out inside img
])
def test_gs_invalid_arguments(L, args, code):
    vp = ctypes.c_void_p
    L.binarize_gs.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_float,
                              ctypes.c_float, ctypes.c_int, vp, vp, vp, vp, vp, vp]
    a = [vp(x) if i in (0, 8) else x for i, x in enumerate(args)]
    assert L.binarize_gs(*a, None, None, None, None, None) == code


def test_gs_stats_planes_must_not_alias(L):
    vp = ctypes.c_void_p
    base = [vp(FAKE_IN), 16, 16, 1, 15, 0.5, 128.0, 0, vp(FAKE_OUT)]
    assert L.binarize_gs(*base, vp(FAKE_OUT + 4), None, None, None, None) == -7   # s1 over out
    assert L.binarize_gs(*base, None, vp(0x30000000), vp(0x30000000 + 1020), None, None) == -7


@pytest.mark.parametrize("args,code", [
    ((None, FAKE_IN, 100, FAKE_WS), -1),
    ((FAKE_OUT, FAKE_IN, 100, None), -1),
    ((FAKE_OUT, FAKE_IN, 0, FAKE_WS), -2),
    ((FAKE_OUT, FAKE_IN, 1 << 31, FAKE_WS), -2),
    ((FAKE_OUT, FAKE_IN, 100, FAKE_WS + 4), -10),    # counts not 8-byte aligned
    ((FAKE_OUT, FAKE_IN, 100, FAKE_IN + 8), -7),     # counts over gt
])
def test_fmeasure_invalid_arguments(L, args, code):
    vp = ctypes.c_void_p
    L.binarize_fmeasure_counts.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    a = [vp(x) if i != 2 else x for i, x in enumerate(args)]
    assert L.binarize_fmeasure_counts(*a, None) == code


STAGED_WS = 8 * 16 * 16


@pytest.mark.parametrize("args,code", [
    ((None, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -1),            # null img
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, None, FAKE_WS, STAGED_WS), -1),             # null out
    ((FAKE_IN, 0, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -2),          # H < 1
    ((FAKE_IN, 16, 16, 2, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -3),         # two channels
    ((FAKE_IN, 16, 16, 1, 256, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -4),        # window too wide
    ((FAKE_IN, 16, 16, 1, 15, float("nan"), 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -5),
    ((FAKE_IN, 16, 16, 1, 15, -1.25, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -5),       # |k| > 1
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 16.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS), -5),          # Sauvola R < 64
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 2, FAKE_OUT, FAKE_WS, STAGED_WS), -6),         # unknown rule
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, None, STAGED_WS), -10),           # no workspace
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS, STAGED_WS - 1), -10),    # too small
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_WS + 2, STAGED_WS), -10),    # misaligned
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_IN + 8, FAKE_WS, STAGED_WS), -7),      # out over img
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_IN + 200, STAGED_WS), -7),   # ws over img
    ((FAKE_IN, 16, 16, 1, 15, 0.5, 128.0, 0, FAKE_OUT, FAKE_OUT - 100, STAGED_WS), -7),  # ws over out
])
def test_staged_invalid_arguments(L, args, code):
    vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    L.binarize_staged.argtypes = [vp, i, i, i, i, f, f, i, vp, vp, ctypes.c_size_t, vp]
    a = [vp(x) if j in (0, 8, 9) else x for j, x in enumerate(args)]
    assert L.binarize_staged(*a, None) == code


def test_staged_workspace_size(L):
    L.binarize_staged_workspace_size.restype = ctypes.c_size_t
    L.binarize_staged_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int]
    assert L.binarize_staged_workspace_size(4096, 4096) == 8 * 4096 * 4096
    assert L.binarize_staged_workspace_size(0, 5) == 0


def test_tile_lds_by_channels(L):
    """Gray tiles keep three 8-row blocks of input rows in LDS, so their
    footprint hardly grows with the window; colour tiles keep a ring of
    win + 8 rows."""
    g15, g151 = L.binarize_tile_lds(256, 15, 1), L.binarize_tile_lds(256, 151, 1)
    c15, c151 = L.binarize_tile_lds(256, 15, 3), L.binarize_tile_lds(256, 151, 3)
    assert 0 < g15 <= g151 <= 40896  # four workgroups per CU at any window a 256-column tile holds
    assert g151 - g15 < 8 * 1024
    assert c151 > 80 * 1024 and c15 > 0
    assert L.binarize_tile_lds(128, 255, 1) > 0
    assert L.binarize_tile_lds(256, 15, 2) == -3
    assert L.binarize_tile_lds(256, 0, 1) == -4
    assert L.binarize_tile_lds(192, 15, 1) == -9
