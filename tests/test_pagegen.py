"""The synthetic page generator: determinism and the structure it promises."""
import hashlib
import json
import os

import numpy as np

import pagegen

HERE = os.path.dirname(os.path.abspath(__file__))


def test_pages_match_stored_digests():
    with open(os.path.join(HERE, "golden", "pages_sha256.json")) as fh:
        cases = json.load(fh)
    for c in cases:
        img = pagegen.page(c["H"], c["W"], c["strokes"], c["seed"], c["channels"])
        assert hashlib.sha256(img.tobytes()).hexdigest() == c["sha256"], c


def test_page_structure():
    img, mask = pagegen.page(512, 384, 300, seed=3, return_mask=True)
    assert img.dtype == np.uint8 and img.shape == (512, 384)
    bg = img[~mask].astype(float)
    fg = img[mask].astype(float)
    # strokes are dark (U[20,60] + noise), background bright (150..230 + noise)
    assert fg.mean() < 60 and bg.mean() > 170
    # noise sigma 8 about the background ramp in a flat stroke-free patch
    ys, xs = np.nonzero(~mask)
    ramp = 150 + 80 * (xs + ys) / (383 + 511)
    resid = img[ys, xs] - ramp
    assert 7.0 < resid.std() < 9.0
    assert abs(resid.mean()) < 0.5


def test_rgb_page_tint_and_layout():
    img = pagegen.page(64, 80, 10, seed=4, channels=3)
    assert img.shape == (64, 80, 3) and img.dtype == np.uint8
    px = img.reshape(-1, 3).astype(float)
    bright = px[px.min(1) > 100]
    # every channel is the same page scaled by its own tint in [0.8, 1.2]
    ratio = bright[:, 1:] / bright[:, :1]
    assert np.all(ratio.std(0) < 0.05)
    assert np.all((ratio.mean(0) > 0.8 / 1.2 - 0.02) & (ratio.mean(0) < 1.2 / 0.8 + 0.02))
    assert not np.array_equal(img[..., 0], img[..., 1])


def test_config3_specs_ranges():
    specs = pagegen.config3_specs(512)
    Hs = np.array([s[0] for s in specs])
    Ws = np.array([s[1] for s in specs])
    wins = {s[2] for s in specs}
    ks = np.array([s[3] for s in specs])
    assert Hs.min() >= 300 and Hs.max() <= 4000 and Ws.min() >= 300 and Ws.max() <= 4000
    assert wins <= set(pagegen.CONFIG3_WINDOWS)
    assert ks.min() >= 0.2 and ks.max() <= 0.5


def test_config4_request_ranges():
    rng = pagegen.rng_for(42)
    for _ in range(2000):
        H, W, C, win, k = pagegen.config4_request(rng)
        assert 0.9e5 <= H * W <= 1.7e7
        assert C in (1, 3) and win % 2 == 1 and 15 <= win <= 151
