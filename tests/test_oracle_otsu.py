"""Pins for the oracle's Otsu global threshold (no GPU).

The paper's global baseline binarizes every pixel against one threshold T
(Sec. 1, Eq. 2) taken from Otsu's method.  The oracle maximizes the
between-class variance w0 w1 (mu0 - mu1)^2 over the split level k and sets
T = k* + 1.  These checks reach the same answer by other routes: Otsu's other
closed form (mu_T w - mu)^2 / (w (1 - w)) in exact rational arithmetic, the
equivalent minimum of the within-class variance with NumPy's var, closed
forms for two-level and constant images, and NumPy's bincount.
"""
from fractions import Fraction

import numpy as np
import pytest

import pagegen


def _exact_between(hist):
    """sigma_b^2(k) for every k, exact, from the normalized-histogram form
    (mu_T w(k) - mu(k))^2 / (w(k) (1 - w(k))), 0 where a class is empty."""
    N = int(hist.sum())
    p = [Fraction(int(h), N) for h in hist]
    muT = sum(i * p[i] for i in range(256))
    out, w, mu = [], Fraction(0), Fraction(0)
    for k in range(256):
        w += p[k]
        mu += k * p[k]
        if w == 0 or w == 1:
            out.append(Fraction(0))
        else:
            out.append((muT * w - mu) ** 2 / (w * (1 - w)))
    return out


@pytest.mark.parametrize("seed", range(6))
def test_otsu_exact_rational_argmax(oracle_mod, seed):
    """The oracle's k* is the first maximizer of the exact between-class
    variance (a different closed form, evaluated in rationals)."""
    rng = np.random.default_rng(seed)
    H, W = int(rng.integers(1, 40)), int(rng.integers(1, 40))
    if seed % 2:
        img = rng.integers(0, 256, (H, W), dtype=np.uint8)
    else:  # two noisy modes, like ink on paper
        ink = rng.random((H, W)) < 0.3
        img = np.where(ink, rng.normal(50, 12, (H, W)), rng.normal(190, 15, (H, W)))
        img = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    T, k, hist, out = oracle_mod.otsu(img)
    assert np.array_equal(hist, np.bincount(img.reshape(-1), minlength=256))
    sb = _exact_between(hist)
    best = max(sb)
    first = sb.index(best)
    assert k == first and T == first + 1
    assert np.array_equal(out, np.where(img < T, 0, 255).astype(np.uint8))


def test_otsu_within_class_minimum(oracle_mod):
    """Maximizing the between-class variance is minimizing the weighted
    within-class variance: brute force over every split with np.var."""
    img = pagegen.page(64, 80, 60, seed=17)
    T, k, _, _ = oracle_mod.otsu(img)
    f = img.reshape(-1).astype(np.float64)
    N = f.size
    best, arg = np.inf, None
    for kk in range(256):
        c0, c1 = f[f <= kk], f[f > kk]
        if c0.size == 0 or c1.size == 0:
            continue
        sw = c0.size / N * np.var(c0) + c1.size / N * np.var(c1)
        if sw < best - 1e-9:
            best, arg = sw, kk
    assert k == arg and T == arg + 1


@pytest.mark.parametrize("a,b,na,nb", [(10, 200, 2, 2), (0, 255, 1, 99), (100, 101, 50, 7)])
def test_otsu_two_levels(oracle_mod, a, b, na, nb):
    """Two gray levels a < b: every split a <= k < b separates them equally,
    the first is k* = a, so T = a + 1 and the a-pixels go to 0."""
    img = np.array([a] * na + [b] * nb, np.uint8).reshape(1, -1)
    T, k, hist, out = oracle_mod.otsu(img)
    assert (k, T) == (a, a + 1)
    assert out.tolist() == [[0] * na + [255] * nb]


@pytest.mark.parametrize("v", [0, 1, 128, 255])
def test_otsu_constant_image(oracle_mod, v):
    """No split separates anything (every sigma_b^2 is 0): k* = 0, T = 1."""
    img = np.full((5, 7), v, np.uint8)
    T, k, hist, out = oracle_mod.otsu(img)
    assert (k, T) == (0, 1)
    assert hist[v] == 35 and hist.sum() == 35
    assert np.all(out == (0 if v == 0 else 255))


def test_otsu_symmetric_modes_midpoint(oracle_mod):
    """Two equal, equally wide, overlapping Gaussian modes: the threshold sits
    midway.  (Modes with an empty gap between them make every split inside
    the gap score the same, and the first one wins.)"""
    rng = np.random.default_rng(3)
    vals = np.concatenate([rng.normal(60, 30, 20000), rng.normal(180, 30, 20000)])
    img = np.clip(np.rint(vals), 0, 255).astype(np.uint8).reshape(200, 200)
    T, _, _, _ = oracle_mod.otsu(img)
    assert abs(T - 120.5) <= 3


def test_otsu_rgb_goes_through_eq1_and_ignores_layout(oracle_mod):
    """An RGB page thresholds its Eq. 1 gray levels; shuffling the pixels
    (a global method) leaves T unchanged."""
    img = pagegen.page(48, 64, 40, seed=5, channels=3)
    T, k, hist, out = oracle_mod.otsu(img)
    g = oracle_mod.gray(img)
    T2, k2, hist2, _ = oracle_mod.otsu(g)
    assert (T, k) == (T2, k2) and np.array_equal(hist, hist2)
    assert np.array_equal(out, np.where(g < T, 0, 255).astype(np.uint8))
    perm = np.random.default_rng(0).permutation(g.size)
    T3, _, _, _ = oracle_mod.otsu(g.reshape(-1)[perm].reshape(g.shape[1], g.shape[0]))
    assert T3 == T
