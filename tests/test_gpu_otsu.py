"""GPU parity of the Otsu global threshold against the oracle (through the
C ABI): histogram, k*, T and the Eq. 2 output must all be bit-identical."""
import numpy as np
import pytest

import pagegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bz():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()
    return m


def _check(bz, oracle_mod, img_np, otsu=None, offset_in=0, offset_out=0):
    import torch
    dev = torch.device("cuda", 0)
    T, k, hist, ref = oracle_mod.otsu(img_np)
    # optionally place the input / output at an unaligned address
    flat = torch.empty(img_np.size + offset_in, dtype=torch.uint8, device=dev)
    img = flat[offset_in:].view(img_np.shape)
    img.copy_(torch.from_numpy(np.ascontiguousarray(img_np)))
    H, W = img_np.shape[:2]
    oflat = torch.empty(H * W + offset_out, dtype=torch.uint8, device=dev)
    out = oflat[offset_out:].view(H, W)
    o = otsu or bz.Otsu(dev)
    o.run(img, out)
    torch.cuda.synchronize()
    assert o.kstar == k and o.T == T, (o.kstar, k)
    assert np.array_equal(o.hist.cpu().numpy().astype(np.uint32), hist)
    got = out.cpu().numpy()
    assert np.array_equal(got, ref), f"{int((got != ref).sum())} pixels differ"
    return T


@pytest.mark.parametrize("H,W,C", [(256, 256, 1), (256, 256, 3), (1, 1, 1), (1, 17, 1), (3, 5, 3),
                                   (37, 1001, 1), (129, 77, 3), (1024, 768, 1), (1024, 768, 3)])
def test_otsu_pages(bz, oracle_mod, H, W, C):
    img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=H * 31 + W + C, channels=C)
    _check(bz, oracle_mod, img)


@pytest.mark.parametrize("off_in,off_out", [(1, 0), (0, 3), (5, 7)])
@pytest.mark.parametrize("C", [1, 3])
def test_otsu_unaligned_buffers(bz, oracle_mod, off_in, off_out, C):
    img = pagegen.page(301, 257, 120, seed=9 + C, channels=C)
    _check(bz, oracle_mod, img, offset_in=off_in, offset_out=off_out)


@pytest.mark.parametrize("v", [0, 1, 200, 255])
def test_otsu_constant(bz, oracle_mod, v):
    T = _check(bz, oracle_mod, np.full((50, 70), v, np.uint8))
    assert T == 1


def test_otsu_two_levels_and_random(bz, oracle_mod):
    img = np.where(np.random.default_rng(1).random((300, 300)) < 0.4, 17, 230).astype(np.uint8)
    assert _check(bz, oracle_mod, img) == 18
    _check(bz, oracle_mod, np.random.default_rng(2).integers(0, 256, (513, 511), dtype=np.uint8))
    rgb = np.random.default_rng(3).integers(0, 256, (200, 300, 3), dtype=np.uint8)
    _check(bz, oracle_mod, rgb)


def test_otsu_workspace_reused_across_calls(bz, oracle_mod):
    """One workspace, calls of different sizes in a row: the per-workgroup
    rows a larger call leaves behind do not leak into a smaller one."""
    import torch
    o = bz.Otsu(torch.device("cuda", 0))
    for i, (H, W, C) in enumerate([(2048, 2048, 1), (64, 64, 1), (1000, 1500, 3), (2048, 2048, 1)]):
        img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=70 + i, channels=C)
        _check(bz, oracle_mod, img, otsu=o)


def test_otsu_threshold_only(bz, oracle_mod):
    import torch
    img_np = pagegen.page(500, 400, 300, seed=4)
    T, k, hist, _ = oracle_mod.otsu(img_np)
    o = bz.Otsu(torch.device("cuda", 0))
    assert o.run(torch.from_numpy(img_np).cuda(), threshold_only=True) is None
    assert (o.T, o.kstar) == (T, k)
    assert np.array_equal(o.hist.cpu().numpy().astype(np.uint32), hist)


@pytest.mark.slow
@pytest.mark.parametrize("H,W,C", [(4096, 4096, 1), (3508, 2480, 3)])
def test_otsu_full_size(bz, oracle_mod, H, W, C):
    """The full-size pages of the benchmark (16.8 Mpx gray, A4 RGB)."""
    img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=11 + C, channels=C)
    _check(bz, oracle_mod, img)


def test_otsu_convenience_and_errors(bz, oracle_mod):
    import torch
    img_np = pagegen.page(100, 120, 40, seed=8)
    out, T = bz.otsu(torch.from_numpy(img_np).cuda())
    T0, _, _, ref = oracle_mod.otsu(img_np)
    assert T == T0 and np.array_equal(out.cpu().numpy(), ref)
    o = bz.Otsu(torch.device("cuda", 0))
    img = torch.zeros((16, 16), dtype=torch.uint8, device="cuda")
    with pytest.raises(bz.BinarizeError):
        o.run(img, out=img.view(16, 16))  # out is img
