"""Pins for the CPU oracle (no GPU).

Each check compares the oracle with something other than itself: exhaustive
enumeration, brute force with NumPy slicing, an int64 summed-area table (a
different algorithm), closed forms, NumPy's library statistics and values
worked out by hand.  Together they are meant to catch a dropped term, a wrong
sign, a wrong window anchor or a transposed operand anywhere in the oracle.
"""
import itertools

import numpy as np
import pytest

from conftest import f32

SAUVOLA, NIBLACK = 0, 1


def lohi(win):
    lo = win // 2
    return lo, win - 1 - lo


# ---------------------------------------------------------------- Eq. 1 gray

def test_gray_exhaustive_all_rgb_triples(oracle_mod):
    """Every (r, g, b) in 0..255^3: the oracle's gray level is the paper's
    weighted sum 0.299 r + 0.587 g + 0.114 b rounded to nearest, halves up."""
    v = np.arange(256, dtype=np.int64)
    r, g, b = np.meshgrid(v, v, v, indexing="ij")
    img = np.stack([r, g, b], axis=-1).astype(np.uint8).reshape(4096, 4096, 3)
    q = oracle_mod.gray(img).reshape(-1).astype(np.int64)
    r, g, b = r.reshape(-1), g.reshape(-1), b.reshape(-1)
    # exact rational value of the weighted sum, scaled by 1000
    num = 299 * r + 587 * g + 114 * b
    # round-half-up characterisation: 1000 q - 500 <= num < 1000 q + 500
    assert np.all(1000 * q - 500 <= num)
    assert np.all(num < 1000 * q + 500)
    # and against the real-valued weights evaluated in float64
    real = 0.299 * r + 0.587 * g + 0.114 * b
    assert np.max(np.abs(q - real)) <= 0.5 + 1e-9
    # weights sum to one: a neutral pixel keeps its level
    neutral = np.arange(256, dtype=np.uint8)[:, None, None].repeat(3, axis=2).reshape(16, 16, 3)
    assert np.array_equal(oracle_mod.gray(neutral).reshape(-1), np.arange(256))


def test_gray_channel_order(oracle_mod):
    """Byte 0 is red (weight .299), byte 2 is blue (weight .114)."""
    img = np.zeros((1, 3, 3), np.uint8)
    img[0, 0] = (255, 0, 0)
    img[0, 1] = (0, 255, 0)
    img[0, 2] = (0, 0, 255)
    assert oracle_mod.gray(img).tolist() == [[76, 150, 29]]  # 76.245, 149.685, 29.07


# ------------------------------------------------------------ window sums, n

def _brute(f, win):
    """Window sums by direct NumPy slicing of the clipped window."""
    H, W = f.shape
    lo, hi = lohi(win)
    s1 = np.zeros((H, W), np.int64)
    s2 = np.zeros((H, W), np.int64)
    n = np.zeros((H, W), np.int64)
    m = np.zeros((H, W))
    sd = np.zeros((H, W))
    f64 = f.astype(np.int64)
    for y in range(H):
        for x in range(W):
            w = f64[max(0, y - lo):y + hi + 1, max(0, x - lo):x + hi + 1]
            s1[y, x] = w.sum()
            s2[y, x] = (w * w).sum()
            n[y, x] = w.size
            m[y, x] = w.mean()
            sd[y, x] = w.std()
    return s1, s2, n, m, sd


def _sat(f, win):
    """Window sums from int64 summed-area tables (integral images)."""
    H, W = f.shape
    lo, hi = lohi(win)
    out = []
    for a in (f.astype(np.int64), f.astype(np.int64) ** 2, np.ones_like(f, dtype=np.int64)):
        I = np.zeros((H + 1, W + 1), np.int64)
        I[1:, 1:] = a.cumsum(0).cumsum(1)
        y = np.arange(H)[:, None]
        x = np.arange(W)[None, :]
        ya, yb = np.clip(y - lo, 0, H), np.clip(y + hi + 1, 0, H)
        xa, xb = np.clip(x - lo, 0, W), np.clip(x + hi + 1, 0, W)
        out.append(I[yb, xb] - I[ya, xb] - I[yb, xa] + I[ya, xa])
    return out


def test_sums_bruteforce_every_tiny_shape(oracle_mod):
    """P1: every H, W in 1..9 and win in 1..19, random bytes: S1, S2, n agree
    with brute-force slicing and with summed-area tables; m and s agree with
    NumPy's mean and std of the same window."""
    rng = np.random.default_rng(12345)
    for H, W in itertools.product(range(1, 10), range(1, 10)):
        f = rng.integers(0, 256, size=(H, W), dtype=np.uint8)
        for win in range(1, 20):
            r = oracle_mod.binarize(f, win, 0.3, 128.0, SAUVOLA)
            s1, s2, n, m, sd = _brute(f, win)
            a1, a2, an = _sat(f, win)
            assert np.array_equal(r.s1, s1) and np.array_equal(r.s1, a1), (H, W, win)
            assert np.array_equal(r.s2, s2) and np.array_equal(r.s2, a2), (H, W, win)
            assert np.array_equal(r.n, n) and np.array_equal(r.n, an), (H, W, win)
            assert np.allclose(r.m, m, rtol=0, atol=1e-9)
            assert np.allclose(r.s, sd, rtol=0, atol=1e-9)
            assert np.array_equal(r.gray, f)


def test_sums_rgb_match_gray_then_sums(oracle_mod):
    rng = np.random.default_rng(7)
    img = rng.integers(0, 256, size=(13, 17, 3), dtype=np.uint8)
    g = oracle_mod.gray(img)
    for win in (1, 4, 7, 30):
        r = oracle_mod.binarize(img, win, 0.2, 128.0, SAUVOLA)
        a1, a2, an = _sat(g, win)
        assert np.array_equal(r.gray, g)
        assert np.array_equal(r.s1, a1) and np.array_equal(r.s2, a2) and np.array_equal(r.n, an)


@pytest.mark.parametrize("win", [1, 2, 3, 14, 15, 16, 31, 101, 254, 255])
def test_clipped_border_count_closed_form(oracle_mod, win):
    """P4: n = nx * ny with nx = min(x+hi, W-1) - max(x-lo, 0) + 1; at the
    corner (0, 0) this is (hi + 1)^2 when the image is large enough."""
    H, W = 300, 280
    f = np.full((H, W), 9, np.uint8)
    r = oracle_mod.binarize(f, win, 0.5, 128.0, SAUVOLA)
    lo, hi = lohi(win)
    y = np.arange(H)[:, None]
    x = np.arange(W)[None, :]
    ny = np.minimum(y + hi, H - 1) - np.maximum(y - lo, 0) + 1
    nx = np.minimum(x + hi, W - 1) - np.maximum(x - lo, 0) + 1
    assert np.array_equal(r.n, (ny * nx).astype(np.uint32))
    assert r.n[0, 0] == (hi + 1) ** 2
    assert r.n[H - 1, W - 1] == (lo + 1) ** 2
    assert np.array_equal(r.s1, 9 * r.n)


def test_even_window_anchor(oracle_mod):
    """An even window puts the extra row/column above/left of the pixel:
    win 2 covers rows {y-1, y} and columns {x-1, x}."""
    f = np.array([[1, 2, 4, 8]], np.uint8)
    r = oracle_mod.binarize(f, 2, 0.0, 128.0, SAUVOLA)
    assert r.s1.tolist() == [[1, 3, 6, 12]]
    assert r.n.tolist() == [[1, 2, 2, 2]]
    r4 = oracle_mod.binarize(f, 4, 0.0, 128.0, SAUVOLA)  # lo 2, hi 1
    assert r4.s1.tolist() == [[3, 7, 15, 14]]


# --------------------------------------------------------- statistics, Eq. 4

def test_ramp_mean_and_variance(oracle_mod):
    """P5: f(x, y) = x; away from the left/right borders m = x exactly and
    s^2 = (win^2 - 1) / 12 (variance of win consecutive integers)."""
    H, W = 40, 256
    f = np.tile(np.arange(W, dtype=np.uint8), (H, 1))
    for win in (3, 15, 31, 61):
        r = oracle_mod.binarize(f, win, 0.5, 128.0, SAUVOLA)
        lo, hi = lohi(win)
        xs = slice(lo, W - hi)
        assert np.all(r.m[:, xs] == np.arange(W)[xs][None, :])
        assert np.allclose(r.s[:, xs] ** 2, (win * win - 1) / 12.0, atol=1e-9)


def test_two_level_edge_closed_form(oracle_mod):
    """P6: left half 0, right half 255.  A window that covers j bright columns
    out of win has p = j / win, m = 255 p and s = 255 sqrt(p (1 - p))."""
    H, W, win = 50, 120, 21
    f = np.zeros((H, W), np.uint8)
    f[:, W // 2:] = 255
    r = oracle_mod.binarize(f, win, 0.5, 128.0, SAUVOLA)
    lo, hi = lohi(win)
    y = H // 2
    for x in range(lo, W - hi):
        j = sum(1 for c in range(x - lo, x + hi + 1) if c >= W // 2)
        p = j / win
        assert r.m[y, x] == pytest.approx(255 * p, abs=1e-9)
        assert r.s[y, x] == pytest.approx(255 * np.sqrt(p * (1 - p)), abs=1e-9)


def test_checkerboard_hand_worked_thresholds(oracle_mod):
    """Values worked out by hand.  A 36/164 checkerboard with win 2 puts two
    36s and two 164s in every interior window: m = 100, s = 64 exactly.
    Sauvola k 0.5, R 128: t = 100 (1 + 0.5 (64/128 - 1)) = 75.
    Sauvola k 0.25, R 64: t = 100 (1 + 0.25 (1 - 1)) = 100.
    Niblack k -0.2: t = 100 - 12.8 = 87.2.  Niblack k 0.5: t = 132."""
    H = W = 8
    yy, xx = np.mgrid[0:H, 0:W]
    f = np.where((yy + xx) % 2 == 0, 36, 164).astype(np.uint8)
    inner = (slice(1, H), slice(1, W))
    cases = [(SAUVOLA, 0.5, 128.0, 75.0), (SAUVOLA, 0.25, 64.0, 100.0),
             (NIBLACK, -0.2, 128.0, 87.2), (NIBLACK, 0.5, 128.0, 132.0)]
    for rule, k, R, t in cases:
        r = oracle_mod.binarize(f, 2, k, R, rule)
        assert np.all(r.m[inner] == 100.0)
        assert np.all(r.s[inner] == 64.0)
        assert np.allclose(r.t[inner], t, atol=1e-12), (rule, k, R)
        expect = np.where(f[inner] < t, 0, 255)
        assert np.array_equal(r.out[inner], expect)


def test_window_covering_image_is_global_statistics(oracle_mod):
    """P7: with win >= 2 max(H, W) - 1 every window is the whole image, so m
    and s are NumPy's mean and population std; the result is a single global
    threshold (Eq. 2) applied everywhere."""
    rng = np.random.default_rng(3)
    f = rng.integers(0, 256, size=(37, 53), dtype=np.uint8)
    win = 2 * 53 - 1
    k, R = f32(0.34), 128.0
    r = oracle_mod.binarize(f, win, k, R, SAUVOLA)
    m, sd = f.astype(np.float64).mean(), f.astype(np.float64).std()
    assert np.allclose(r.m, m, atol=1e-9) and np.allclose(r.s, sd, atol=1e-9)
    T = r.t[0, 0]
    assert np.allclose(r.t, T, atol=1e-9)
    assert np.array_equal(r.out, np.where(f < T, 0, 255).astype(np.uint8))


# ---------------------------------------------------- Eq. 3 decision and ties

@pytest.mark.parametrize("c", [0, 1, 77, 128, 255])
def test_constant_image(oracle_mod, c):
    """P2: s = 0.  Sauvola t = c (1 - k), so f >= t for k >= 0 and every output
    is 255; Niblack t = c = f, an exact tie, which Eq. 3 sends to 255."""
    f = np.full((20, 30), c, np.uint8)
    for k in (0.0, 0.2, 0.5):
        r = oracle_mod.binarize(f, 7, k, 128.0, SAUVOLA)
        assert np.all(r.s == 0) and np.all(r.m == c)
        assert np.allclose(r.t, c * (1 - k), atol=1e-12)
        assert np.all(r.out == 255)
    r = oracle_mod.binarize(f, 7, -0.2, 128.0, NIBLACK)
    assert np.all(r.t == c) and np.all(r.out == 255)
    if c > 0:  # a negative Sauvola k lifts t above f: every pixel goes to 0
        r = oracle_mod.binarize(f, 7, -0.1, 128.0, SAUVOLA)
        assert np.all(r.out == 0)


def test_unit_window(oracle_mod):
    """P3: win 1 gives n = 1, m = f, s = 0 at every pixel."""
    rng = np.random.default_rng(11)
    f = rng.integers(0, 256, size=(9, 11), dtype=np.uint8)
    r = oracle_mod.binarize(f, 1, 0.5, 128.0, SAUVOLA)
    assert np.all(r.n == 1) and np.array_equal(r.m, f.astype(float)) and np.all(r.s == 0)
    assert np.allclose(r.t, 0.5 * f, atol=1e-12)
    assert np.all(r.out == 255)
    rn = oracle_mod.binarize(f, 1, 0.7, 128.0, NIBLACK)
    assert np.all(rn.out == 255)  # t == f everywhere


def test_decision_is_strict_less_than(oracle_mod):
    """Eq. 3 gives 0 only when f < t: a tie gives 255, one level below gives 0."""
    f = np.array([[10, 10, 10], [10, 9, 10], [10, 10, 10]], np.uint8)
    r = oracle_mod.binarize(f, 3, 0.0, 128.0, SAUVOLA)  # k = 0: t = m
    assert r.t[1, 1] == pytest.approx(89 / 9)
    assert r.out[1, 1] == 0          # 9 < 9.888...
    assert r.out[0, 0] == 255        # 10 >= t


# ------------------------------------------------------------ whole path

def test_symmetry_odd_window(oracle_mod):
    """P8: for odd win the window is centred, so transposing or flipping the
    input transposes or flips every output plane."""
    rng = np.random.default_rng(5)
    f = rng.integers(0, 256, size=(23, 31), dtype=np.uint8)
    k = f32(0.34)
    base = oracle_mod.binarize(f, 9, k, 128.0, SAUVOLA)
    for op in (np.transpose, np.fliplr, np.flipud):
        r = oracle_mod.binarize(np.ascontiguousarray(op(f)), 9, k, 128.0, SAUVOLA)
        assert np.array_equal(r.s1, op(base.s1)) and np.array_equal(r.s2, op(base.s2))
        assert np.array_equal(r.n, op(base.n))
        assert np.allclose(r.t, op(base.t), atol=1e-9)


def test_crop_consistency(oracle_mod):
    """P9: pixels further than win from a crop edge see the same window in
    the crop and in the full page."""
    import pagegen
    img = pagegen.page(96, 128, 60, seed=77)
    win = 11
    full = oracle_mod.binarize(img, win, 0.5, 128.0, SAUVOLA)
    y0, x0 = 20, 30
    crop = np.ascontiguousarray(img[y0:y0 + 50, x0:x0 + 70])
    r = oracle_mod.binarize(crop, win, 0.5, 128.0, SAUVOLA)
    sl = (slice(win, 50 - win), slice(win, 70 - win))
    fsl = (slice(y0 + win, y0 + 50 - win), slice(x0 + win, x0 + 70 - win))
    assert np.array_equal(r.s1[sl], full.s1[fsl])
    assert np.array_equal(r.out[sl], full.out[fsl])


def test_points_match_whole_image(oracle_mod):
    import pagegen
    img = pagegen.page(70, 90, 40, seed=8, channels=3)
    win, k = 13, f32(0.34)
    full = oracle_mod.binarize(img, win, k, 128.0, SAUVOLA)
    rng = np.random.default_rng(0)
    ys = rng.integers(0, 70, 300)
    xs = rng.integers(0, 90, 300)
    p = oracle_mod.binarize_points(img, win, k, 128.0, SAUVOLA, ys, xs)
    assert np.array_equal(p.gray, full.gray[ys, xs])
    assert np.array_equal(p.s1, full.s1[ys, xs]) and np.array_equal(p.n, full.n[ys, xs])
    assert np.array_equal(p.t, full.t[ys, xs]) and np.array_equal(p.out, full.out[ys, xs])


def test_max_window_sums_fit_u32(oracle_mod):
    """A saturated 255 page with the largest window: S1 = 255 win^2 and
    S2 = 255^2 win^2 stay below 2^32 up to win 255."""
    f = np.full((300, 300), 255, np.uint8)
    r = oracle_mod.binarize(f, 255, 0.5, 128.0, SAUVOLA)
    c = 150
    assert int(r.s1[c, c]) == 255 * 255 * 255
    assert int(r.s2[c, c]) == 255 * 255 * 255 * 255


def test_rejects_bad_arguments(oracle_mod):
    f = np.zeros((4, 4), np.uint8)
    with pytest.raises(ValueError):
        oracle_mod.binarize(f, 0, 0.5, 128.0, SAUVOLA)
    with pytest.raises(ValueError):
        oracle_mod.binarize(f, 256, 0.5, 128.0, SAUVOLA)
    with pytest.raises(ValueError):
        oracle_mod.binarize(f, 3, 0.5, 0.0, SAUVOLA)
    with pytest.raises(ValueError):
        oracle_mod.binarize(f, 3, 0.5, 128.0, 2)
