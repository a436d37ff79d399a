"""The largest images the C ABI accepts (H * W_img * channels just below
2^31 bytes): the tile kernel and Otsu's threshold against the oracle.

The pages are a seeded 4096 x 4096 synthetic page repeated over the whole
area (generating 2 Gpx of strokes would take minutes); every window of the
result still mixes text, background ramp and noise."""
import numpy as np
import pytest

import pagegen
from conftest import f32

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()
    return m


def tiled(H, W, C):
    base = pagegen.page(4096, 4096, pagegen.strokes_for(4096, 4096), seed=77 + C, channels=C)
    reps = (-(-H // 4096), -(-W // 4096)) + ((1,) if C == 3 else ())
    return np.ascontiguousarray(np.tile(base, reps)[:H, :W])


def sample(H, W, n, seed):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n))
    xs = list(rng.integers(0, W, n))
    for y in (0, 1, 7, H // 2, H - 8, H - 2, H - 1):   # corners, borders, the far end
        for x in (0, 1, 255, 256, W // 2, W - 257, W - 2, W - 1):
            ys.append(y)
            xs.append(x)
    return np.array(ys, np.int32), np.array(xs, np.int32)


@pytest.mark.parametrize("H,W,C,rule,win,k", [(46340, 46340, 1, 0, 31, 0.34),
                                              (26754, 26754, 3, 1, 61, -0.2)])
def test_tile_kernel_at_max_size(bz, oracle_mod, H, W, C, rule, win, k):
    from oracle.compare import compare_out
    assert H * W * C < 2**31 and (H + 1) * (W + 1) * C >= 2**31
    img = tiled(H, W, C)
    k = f32(k)
    dimg = torch.from_numpy(img).cuda()
    out = bz.binarize(dimg, win, k, 128.0, rule)
    ys, xs = sample(H, W, 2000, seed=H)
    iy, ix = torch.from_numpy(ys.astype(np.int64)).cuda(), torch.from_numpy(xs.astype(np.int64)).cuda()
    got = out[iy, ix].cpu().numpy()
    torch.cuda.synchronize()
    assert bool(((out == 0) | (out == 255)).all())
    del out, dimg
    ref = oracle_mod.binarize_points(img, win, k, 128.0, rule, ys, xs)
    assert compare_out(got, ref.out, ref.gray, ref.t)["ok"]


def test_otsu_at_max_size(bz, oracle_mod):
    H = W = 46340
    img = tiled(H, W, 1)
    T, kstar, hist, _ = oracle_mod.otsu(img[:8, :8])  # warm the library
    T, kstar, hist, ref_out = oracle_mod.otsu(img)
    dimg = torch.from_numpy(img).cuda()
    o = bz.Otsu(dimg.device)
    out = o.run(dimg)
    torch.cuda.synchronize()
    assert (o.T, o.kstar) == (T, kstar)
    assert np.array_equal(o.hist.cpu().numpy().astype(np.uint32), hist)
    assert torch.equal(out, torch.from_numpy(ref_out).cuda())


def test_staged_equals_fused_at_max_size(bz):
    """The staged two-pass path on the largest gray page (a 17 GB plane
    workspace, 8.4 M row-pass workgroups): identical bytes to the fused
    kernel."""
    H = W = 46340
    img = torch.from_numpy(tiled(H, W, 1)).cuda()
    fused = bz.binarize(img, 31, f32(0.34), 128.0, 0)
    staged = bz.binarize_staged(img, 31, f32(0.34), 128.0, 0)
    torch.cuda.synchronize()
    assert torch.equal(fused, staged)
