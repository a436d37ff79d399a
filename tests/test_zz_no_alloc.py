"""The allocation-free Otsu entry point (binarize_otsu_noalloc), called
through the C ABI, against binarize_otsu with a caller workspace: output
bytes, histogram, T and k* identical, on consecutive calls of decreasing size
(the library's scratch keeps the previous call's contents)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as bz
    return bz._otsu_lib()


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _reference(L, img, H, W, C):
    ws = torch.empty((4096 + 512 * 1024) // 4, dtype=torch.int32, device="cuda")
    out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.binarize_otsu(_p(img), H, W, C, _p(out), _p(ws), 4 * ws.numel(), s) == 0
    return out, ws[:258].clone()


def _noalloc(L, img, H, W, C, with_result=True):
    out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    res = torch.full((258,), -1, dtype=torch.int32, device="cuda") if with_result else None
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.binarize_otsu_noalloc(_p(img), H, W, C, _p(out), _p(res), s) == 0
    return out, res


def _page(H, W, C, seed):
    import pagegen
    return pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=seed, channels=C)


@pytest.mark.parametrize("shapes", [
    [(2048, 1536, 3), (333, 517, 1)],   # large RGB, then a smaller ragged gray page
    [(4096, 4096, 1), (1, 1, 1)],       # full-size gray, then a single pixel
])
def test_noalloc_equals_workspace_entry_point(L, oracle_mod, shapes):
    for i, (H, W, C) in enumerate(shapes):
        print(f"noalloc call {i}: {H}x{W}x{C}", flush=True)
        host = _page(H, W, C, seed=70 + i)
        img = torch.from_numpy(host).cuda()
        ref_out, ref_ws = _reference(L, img, H, W, C)
        out, res = _noalloc(L, img, H, W, C)
        torch.cuda.synchronize()
        assert torch.equal(out, ref_out), (H, W, C)
        assert torch.equal(res, ref_ws), (H, W, C)
        T, kstar, hist, oracle_out = oracle_mod.otsu(host)
        assert int(res[256]) == T and int(res[257]) == kstar
        assert np.array_equal(res[:256].cpu().numpy().astype(np.uint32), hist)
        assert np.array_equal(out.cpu().numpy(), oracle_out)


def test_noalloc_threshold_only_and_unaligned(L):
    """out NULL (threshold only) and an input at an odd byte offset."""
    H, W, C = 257, 301, 3
    host = _page(H, W, C, seed=5)
    buf = torch.zeros(host.size + 16, dtype=torch.uint8, device="cuda")
    img = buf[3:3 + host.size].view(H, W, C)
    img.copy_(torch.from_numpy(host))
    _, ref_ws = _reference(L, img, H, W, C)
    res = torch.full((258,), -1, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.binarize_otsu_noalloc(_p(img), H, W, C, None, _p(res), s) == 0
    torch.cuda.synchronize()
    assert torch.equal(res, ref_ws)


def test_noalloc_rejects_bad_arguments(L):
    img = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    out = torch.empty((16, 16), dtype=torch.uint8, device="cuda")
    res = torch.empty(300, dtype=torch.int32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.binarize_otsu_noalloc(None, 16, 16, 1, _p(out), None, s) == -1       # BZ_ERR_NULL
    assert L.binarize_otsu_noalloc(_p(img), 0, 16, 1, _p(out), None, s) == -2     # BZ_ERR_SHAPE
    assert L.binarize_otsu_noalloc(_p(img), 16, 16, 2, _p(out), None, s) == -3    # BZ_ERR_CHANNELS
    misaligned = ctypes.c_void_p(res.data_ptr() + 2)
    assert L.binarize_otsu_noalloc(_p(img), 16, 16, 1, _p(out), misaligned, s) == -10
    assert L.binarize_otsu_noalloc(_p(img), 16, 16, 1, _p(out), _p(img), s) == -7  # result over img
