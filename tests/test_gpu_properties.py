"""Whole-path properties of the HIP path that hold at any size (P8 symmetry,
P9 crop consistency), checked on pages large enough for many tiles and for
both input-row layouts of the tile kernel (the win + 8-row ring, and the
three-block layout that gray pages with wide windows take when they have
more tiles than the ring runs at once).  They need no oracle run at full
size: the stats planes S1, S2 and n must match exactly; output bytes may
differ only where f lies within 1e-4 of t (t from the GPU's own t plane,
itself checked against the oracle elsewhere), since flipping a page moves
pixels between the whole-window and per-pixel-n decision forms."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

T_TOL = 1e-4


def f32(x):
    return float(np.float32(x))


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()  # raises if the library is missing: no fallback
    return m


@pytest.fixture(scope="module")
def page():
    import pagegen
    return pagegen.config1()[0].img


def stats(bz, img, win, k, rule):
    res = bz.binarize_stats(torch.from_numpy(np.ascontiguousarray(img)).cuda(), win, k, 128.0, rule)
    torch.cuda.synchronize()
    return {n: v.cpu().numpy() for n, v in res.items()}


def outputs_agree(out_a, out_b, gray, t):
    """Bytes equal except where f is within T_TOL of t."""
    band = np.abs(gray.astype(np.float64) - t.astype(np.float64)) < T_TOL
    mism = out_a != out_b
    return int((mism & ~band).sum()) == 0


# (H, W, win, rule, k): 1024 x 768 pages (ring layout at every window) and a
# 4096 x 2051 page at win 101 (blocks layout; its transpose too)
CASES = [(1024, 768, 15, 0, 0.5), (1024, 768, 61, 1, -0.2), (1024, 768, 151, 0, 0.34),
         (4096, 2051, 101, 0, 0.5)]


@pytest.mark.parametrize("H,W,win,rule,k", CASES)
def test_symmetry_odd_window(bz, page, H, W, win, rule, k):
    """P8: for odd win the window is centred, so transposing or flipping the
    input transposes or flips S1, S2, n and the threshold plane."""
    k = f32(k)
    img = np.ascontiguousarray(page[:H, :W])
    print(f"P8 {H}x{W} win {win} rule {rule}", flush=True)
    base = stats(bz, img, win, k, rule)
    for name, op in (("transpose", np.transpose), ("fliplr", np.fliplr), ("flipud", np.flipud)):
        r = stats(bz, op(img), win, k, rule)
        for plane in ("gray", "s1", "s2", "n"):
            assert np.array_equal(r[plane], op(base[plane])), (name, plane)
        assert np.max(np.abs(r["t"].astype(np.float64) - op(base["t"]).astype(np.float64))) <= 2 * T_TOL, name
        assert outputs_agree(r["out"], op(base["out"]), r["gray"], r["t"]), name


@pytest.mark.parametrize("H,W,win,rule,k", CASES)
def test_crop_consistency(bz, page, H, W, win, rule, k):
    """P9: pixels further than win from a crop's edge see the same window in
    the crop as in the whole page (catches halo and tile-seam mistakes)."""
    k = f32(k)
    img = np.ascontiguousarray(page[:H, :W])
    full = stats(bz, img, win, k, rule)
    y0, x0 = 300, 200
    h, w = H - 2 * y0 // 3 - y0, W - 2 * x0 // 3 - x0
    print(f"P9 {H}x{W} crop {y0},{x0} {h}x{w} win {win}", flush=True)
    crop = stats(bz, img[y0:y0 + h, x0:x0 + w], win, k, rule)
    sl = (slice(win, h - win), slice(win, w - win))
    fsl = (slice(y0 + win, y0 + h - win), slice(x0 + win, x0 + w - win))
    for plane in ("s1", "s2", "n", "out"):
        assert np.array_equal(crop[plane][sl], full[plane][fsl]), plane
