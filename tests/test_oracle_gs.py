"""Pins for the oracle's sampled-window variant (Sec. 2, Eq. 5) and the
F-measure (Sec. 3, Eq. 6) (no GPU).

The structures (plus, x, star) are this library's own O(W) subsets of the
window; the checks below rebuild them as NumPy boolean masks over padded
images (a different construction from the oracle's offset list), and check
relations between them, symmetries and closed forms.
"""
import numpy as np
import pytest

import pagegen

PLUS, X, STAR = 0, 1, 2


def mask(structure, win):
    r = win // 2
    dy, dx = np.mgrid[-r:r + 1, -r:r + 1]
    plus = (dy == 0) | (dx == 0)
    x = (dy == dx) | (dy == -dx)
    return {PLUS: plus, X: x, STAR: plus | x}[structure]


def brute(f, win, k, Rp, structure):
    """Masked window statistics with NumPy, image padded with NaN."""
    H, W = f.shape
    r = win // 2
    pad = np.full((H + 2 * r, W + 2 * r), np.nan)
    pad[r:r + H, r:r + W] = f
    M = mask(structure, win)
    s1 = np.zeros((H, W)); s2 = np.zeros((H, W)); n = np.zeros((H, W)); t = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            vals = pad[y:y + win, x:x + win][M]
            vals = vals[~np.isnan(vals)]
            s1[y, x], s2[y, x], n[y, x] = vals.sum(), (vals ** 2).sum(), vals.size
            m, s = vals.mean(), vals.std()
            t[y, x] = m * (1 + k * (s / Rp - 1))
    return s1, s2, n, t


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
@pytest.mark.parametrize("win", [1, 3, 5, 9])
def test_gs_matches_masked_bruteforce(oracle_mod, structure, win):
    rng = np.random.default_rng(win * 3 + structure)
    for H, W in [(1, 1), (1, 7), (6, 1), (7, 9), (12, 5)]:
        f = rng.integers(0, 256, (H, W), dtype=np.uint8)
        r = oracle_mod.binarize_gs(f, win, 0.3, 100.0, structure)
        s1, s2, n, t = brute(f.astype(np.float64), win, 0.3, 100.0, structure)
        assert np.array_equal(r.s1, s1) and np.array_equal(r.s2, s2) and np.array_equal(r.n, n)
        assert np.allclose(r.t, t, rtol=0, atol=1e-9)
        assert np.array_equal(r.out, np.where(f < r.t, 0, 255))


def test_star_is_plus_and_x_sharing_the_centre(oracle_mod):
    img = pagegen.page(40, 56, 30, seed=3)
    f = img.astype(np.int64)
    for win in (3, 7, 15):
        p = oracle_mod.binarize_gs(img, win, 0.5, 128.0, PLUS)
        x = oracle_mod.binarize_gs(img, win, 0.5, 128.0, X)
        s = oracle_mod.binarize_gs(img, win, 0.5, 128.0, STAR)
        assert np.array_equal(s.s1.astype(np.int64), p.s1.astype(np.int64) + x.s1 - f)
        assert np.array_equal(s.s2.astype(np.int64), p.s2.astype(np.int64) + x.s2 - f * f)
        assert np.array_equal(s.n.astype(np.int64), p.n.astype(np.int64) + x.n - 1)


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
def test_interior_counts_and_border_counts(oracle_mod, structure):
    """Interior pixels see 2 win - 1 (plus, x) or 4 win - 3 (star) members;
    at the corner pixel a plus sees r + 1 per arm, an x only its diagonal."""
    win, r = 11, 5
    img = np.zeros((30, 30), np.uint8)
    n = oracle_mod.binarize_gs(img, win, 0.5, 128.0, structure).n
    full = {PLUS: 2 * win - 1, X: 2 * win - 1, STAR: 4 * win - 3}[structure]
    assert n[15, 15] == full
    corner = {PLUS: 2 * (r + 1) - 1, X: r + 1, STAR: 3 * (r + 1) - 2}[structure]
    assert n[0, 0] == corner


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
def test_transpose_and_flip_symmetry(oracle_mod, structure):
    img = pagegen.page(33, 47, 25, seed=9)
    a = oracle_mod.binarize_gs(img, 9, 0.4, 128.0, structure)
    b = oracle_mod.binarize_gs(np.ascontiguousarray(img.T), 9, 0.4, 128.0, structure)
    c = oracle_mod.binarize_gs(np.ascontiguousarray(img[:, ::-1]), 9, 0.4, 128.0, structure)
    for fld in ("s1", "s2", "n", "out"):
        assert np.array_equal(getattr(a, fld).T, getattr(b, fld))
        assert np.array_equal(getattr(a, fld)[:, ::-1], getattr(c, fld))


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
def test_constant_and_unit_window(oracle_mod, structure):
    """Constant image: s' = 0, t' = c (1 - k) <= c, so every pixel is 255.
    win = 1: S' is the pixel itself, t' = f (1 - k)."""
    c = 140
    r = oracle_mod.binarize_gs(np.full((9, 9), c, np.uint8), 5, 0.25, 128.0, structure)
    assert np.allclose(r.t, c * 0.75) and np.all(r.out == 255)
    img = pagegen.page(10, 12, 5, seed=1)
    r = oracle_mod.binarize_gs(img, 1, 0.5, 128.0, structure)
    assert np.all(r.n == 1) and np.allclose(r.t, img * 0.5)


def test_gs_rgb_uses_eq1(oracle_mod):
    img = pagegen.page(20, 24, 10, seed=2, channels=3)
    a = oracle_mod.binarize_gs(img, 7, 0.5, 128.0, STAR)
    b = oracle_mod.binarize_gs(oracle_mod.gray(img), 7, 0.5, 128.0, STAR)
    assert np.array_equal(a.s1, b.s1) and np.array_equal(a.out, b.out)


def test_gs_rejects_even_windows_and_bad_structures(oracle_mod):
    img = np.zeros((4, 4), np.uint8)
    with pytest.raises(ValueError):
        oracle_mod.binarize_gs(img, 4, 0.5, 128.0, PLUS)
    with pytest.raises(ValueError):
        oracle_mod.binarize_gs(img, 5, 0.5, 128.0, 3)
    with pytest.raises(ValueError):
        oracle_mod.binarize_gs(img, 5, 0.5, 0.0, PLUS)


# ------------------------------------------------------------------ Eq. 6

def test_fmeasure_hand_worked(oracle_mod):
    """TP 3, FP 1, FN 2: R = 3/5, P = 3/4, FM = 2 (9/20) / (27/20) = 2/3."""
    out = np.array([0, 0, 0, 0, 255, 255, 255], np.uint8)
    gt = np.array([1, 1, 1, 0, 1, 1, 0], np.uint8)
    tp, fp, fn = oracle_mod.fmeasure_counts(out, gt)
    assert (tp, fp, fn) == (3, 1, 2)
    assert oracle_mod.fmeasure(tp, fp, fn) == pytest.approx(2 / 3, abs=1e-15)


def test_fmeasure_extremes(oracle_mod):
    gt = np.array([[1, 0], [0, 1]], np.uint8)
    perfect = np.where(gt != 0, 0, 255).astype(np.uint8)
    assert oracle_mod.fmeasure(*oracle_mod.fmeasure_counts(perfect, gt)) == 1.0
    blank = np.full((2, 2), 255, np.uint8)
    assert oracle_mod.fmeasure_counts(blank, gt) == (0, 0, 2)
    assert oracle_mod.fmeasure(0, 0, 2) == 0.0
    inverted = 255 - perfect
    assert oracle_mod.fmeasure(*oracle_mod.fmeasure_counts(inverted, gt)) == 0.0
