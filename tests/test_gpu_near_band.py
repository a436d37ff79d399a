"""Pixels just outside the tolerance band decide exactly as the oracle does.

The parity bar allows a binary mismatch only where |f - t_oracle| < 1e-4.
Ordinary pages have few pixels near their threshold (a handful per Mpx), so
these pages are built to put thousands of pixels at a chosen distance
delta (1.2e-4 .. 2.8e-4, either side) from it, with k at the ends of the
accepted range |k| <= 1 and Sauvola's R at its lower limit 64:

* a random two-level page {a, b} whose share of b makes one window count c
  of b-pixels frequent; every whole window with that count has the same
  m, s and t (Sec. 1, Eq. 4 / Niblack), and k is solved (in fp64, then
  rounded to the fp32 the GPU receives) so that f - t = delta for centre
  pixels f = a (or b);
* the same on pages shorter than half the window, so that every pixel takes
  the clipped-window form (n = rows x win in the interior columns).

Zero mismatches are allowed outside the band: a decision form whose rounding
exceeded 1e-4 at these parameters would flip all of them at once.  The fused
kernel, its stats variant (t plane within 1e-4) and the staged two-pass
path are all checked.
"""
import math

import numpy as np
import pytest

from conftest import f32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()
    return m


def solve_k(rule, n, a, b, R, centre_is_a, delta):
    """Window count c of b-pixels (nearest n/2 with |k| <= 1) and the fp32 k
    that puts the centre pixel at f - t = delta for windows of n pixels with
    c of them b; returns (c, k32, exact f - t for k32)."""
    best = None
    for c in range(1, n):
        S1 = c * b + (n - c) * a
        S2 = c * b * b + (n - c) * a * a
        m = S1 / n
        s = math.sqrt(n * S2 - S1 * S1) / n
        f = a if centre_is_a else b
        if rule == 0:
            k = (f - delta - m) / (m * (s / R - 1.0))
        else:
            k = (f - delta - m) / s
        if abs(k) > 0.999 or (best and abs(c - n / 2) >= abs(best[0] - n / 2)):
            continue
        best = (c, k, m, s, f)
    assert best, (rule, n, a, b, R)
    c, k, m, s, f = best
    k32 = f32(k)
    t = m * (1.0 + k32 * (s / R - 1.0)) if rule == 0 else m + k32 * s
    return c, k32, f - t


def two_level(H, W, a, b, p, C, seed):
    rng = np.random.default_rng(seed)
    g = np.where(rng.random((H, W)) < p, b, a).astype(np.uint8)
    if C == 1:
        return g
    # (v, v, v) has gray level v under Eq. 1: (1000 v + 500) / 1000 rounds down to v
    return np.repeat(g[:, :, None], 3, axis=2)


# (rule, win, R, a, b, centre is a, delta): k lands near +-1 for these levels
CASES = [
    (0, 15, 128.0, 60, 180, True, 2.0e-4),
    (0, 15, 128.0, 60, 180, False, -2.0e-4),
    (0, 31, 64.0, 100, 140, True, -1.2e-4),
    (0, 31, 64.0, 100, 140, False, 1.2e-4),
    (0, 101, 64.0, 90, 150, True, 2.8e-4),
    (0, 61, 64.0, 20, 74, True, 1.5e-4),      # k near +1 at R = 64
    (0, 15, 64.0, 20, 74, False, -1.5e-4),    # k near -1 at R = 64
    (1, 15, 128.0, 40, 200, True, 1.2e-4),
    (1, 31, 128.0, 40, 200, False, -2.0e-4),
    (1, 61, 128.0, 70, 110, True, -2.8e-4),
]


def _check(bz, oracle_mod, img, win, k, R, rule, min_near, label):
    from oracle.compare import compare_out, compare_stats
    ref = oracle_mod.binarize(img, win, k, R, rule)
    d = np.abs(ref.gray.astype(np.float64) - ref.t)
    near = (d >= 1e-4) & (d < 3e-4)
    dimg = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    st = {n_: v.cpu().numpy() for n_, v in bz.binarize_stats(dimg, win, k, R, rule).items()}
    out = bz.binarize(dimg, win, k, R, rule).cpu().numpy()
    staged = bz.binarize_staged(dimg, win, k, R, rule).cpu().numpy()
    rep = compare_stats(st, ref)
    print(label, "near-band pixels", int(near.sum()), rep, flush=True)
    assert int(near.sum()) >= min_near, (label, int(near.sum()))
    assert rep["ok"], (label, rep)
    assert compare_out(out, ref.out, ref.gray, ref.t)["ok"], label
    assert np.array_equal(out[near], ref.out[near]), label
    assert np.array_equal(staged, out), label
    assert np.array_equal(st["out"], out), label


@pytest.mark.parametrize("C", [1, 3])
@pytest.mark.parametrize("rule,win,R,a,b,centre_a,delta", CASES)
def test_near_band_whole_windows(bz, oracle_mod, rule, win, R, a, b, centre_a, delta, C):
    n = win * win
    c, k, ft = solve_k(rule, n, a, b, R, centre_a, delta)
    assert 1e-4 < abs(ft) < 3e-4 and abs(k) <= 1.0
    H, W = (520, 1040) if C == 1 else (400, 720)
    img = two_level(H, W, a, b, c / n, C, seed=win * 10 + C)
    _check(bz, oracle_mod, img, win, k, R, rule, 200, f"whole rule {rule} win {win} k {k:.6f} C {C}")


@pytest.mark.parametrize("C", [1, 3])
@pytest.mark.parametrize("rule,win,R,a,b,centre_a,delta", CASES)
def test_near_band_clipped_windows(bz, oracle_mod, rule, win, R, a, b, centre_a, delta, C):
    """Pages of win // 2 - 1 rows: every window is clipped vertically, so
    every pixel takes the per-pixel-n form (n = rows x win inside)."""
    rows = max(2, win // 2 - 1)
    n = rows * win
    c, k, ft = solve_k(rule, n, a, b, R, centre_a, delta)
    assert 1e-4 < abs(ft) < 3e-4 and abs(k) <= 1.0
    H, W = rows, max(1040, (400_000 if C == 1 else 240_000) // rows)
    img = two_level(H, W, a, b, c / n, C, seed=win * 10 + C + 5)
    _check(bz, oracle_mod, img, win, k, R, rule, 30, f"clipped rule {rule} win {win} rows {rows} k {k:.6f} C {C}")
