"""Seeded synthetic document pages (inputs only; none of the method's arithmetic).

The paper evaluates on DIBCO 2009, H-DIBCO 2010 and its own CMATERdb-6 scans
(Sec. 3) and times 1024x768 pages (Sec. 3.2, Fig. 4).  None of those images is
available here, so every workload is a synthetic page with the structure of a
degraded document scan:

* background: uneven illumination, a linear ramp from 150 to 230 gray levels
  along the main diagonal;
* text: dark axis-aligned strokes (horizontal or vertical with probability 1/2),
  2..6 px thick, 10..60 px long, intensity U[20, 60], uniform positions clipped
  to the page, painted in order;
* sensor noise: additive Gaussian, sigma = 8, then rounded and clipped to
  [0, 255];
* colour pages: a per-page tint U[0.8, 1.2] per channel applied to the noisy
  float page before rounding (interleaved r, g, b).

The stroke mask is the page's ground truth (foreground = stroke pixels).
For accuracy studies ``degraded_page`` darkens the shading (background 60 to
230), lightens the ink (30..110) and raises the noise (sigma 12).

Both the HIP path and the CPU oracle consume these pages; this module holds
no part of the binarization method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# stroke density of the 4096 x 4096 reference page: 40,000 strokes
STROKES_PER_PIXEL = 40_000 / (4096 * 4096)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def page(H: int, W: int, n_strokes: int, seed: int, channels: int = 1,
         noise_sigma: float = 8.0, return_mask: bool = False,
         bg: tuple[float, float] = (150.0, 230.0), ink: tuple[float, float] = (20.0, 60.0)):
    """One synthetic page, uint8 HxW (channels=1) or HxWx3 (channels=3).
    bg: background levels at the top-left and bottom-right corners (linear
    ramp along the diagonal); ink: range of the stroke intensities."""
    if H < 1 or W < 1:
        raise ValueError("page must be at least 1x1")
    if channels not in (1, 3):
        raise ValueError("channels must be 1 or 3")
    rng = rng_for(seed)
    ys = np.arange(H, dtype=np.float32)[:, None]
    xs = np.arange(W, dtype=np.float32)[None, :]
    denom = float(max((W - 1) + (H - 1), 1))
    img = (float(bg[0]) + (float(bg[1]) - float(bg[0])) * (xs + ys) / denom).astype(np.float32)
    img = np.broadcast_to(img, (H, W)).copy()
    mask = np.zeros((H, W), dtype=bool) if return_mask else None

    n = int(n_strokes)
    horiz = rng.random(n) < 0.5
    thick = rng.integers(2, 7, size=n)
    length = rng.integers(10, 61, size=n)
    y0 = rng.integers(0, H, size=n)
    x0 = rng.integers(0, W, size=n)
    val = rng.uniform(float(ink[0]), float(ink[1]), size=n).astype(np.float32)
    for i in range(n):
        h, w = (thick[i], length[i]) if horiz[i] else (length[i], thick[i])
        ya, xa = y0[i], x0[i]
        img[ya:ya + h, xa:xa + w] = val[i]
        if mask is not None:
            mask[ya:ya + h, xa:xa + w] = True

    img += rng.standard_normal((H, W), dtype=np.float32) * np.float32(noise_sigma)
    if channels == 1:
        out = np.clip(np.rint(img), 0, 255).astype(np.uint8)
    else:
        tint = rng.uniform(0.8, 1.2, size=3).astype(np.float32)
        out = np.empty((H, W, 3), np.uint8)
        for c in range(3):
            out[:, :, c] = np.clip(np.rint(img * tint[c]), 0, 255).astype(np.uint8)
    if return_mask:
        return out, mask
    return out


DEGRADED = {"bg": (60.0, 230.0), "ink": (30.0, 110.0), "noise_sigma": 12.0}


def degraded_page(H: int, W: int, seed: int, channels: int = 1, return_mask: bool = True):
    """A harder page for accuracy studies: strong shading (background 60 to
    230 along the diagonal), fainter ink (30..110) and more noise (sigma 12),
    so that no single global threshold separates ink from paper everywhere."""
    return page(H, W, strokes_for(H, W), seed, channels, return_mask=return_mask, **DEGRADED)


def strokes_for(H: int, W: int) -> int:
    """Stroke count at the reference density for an HxW page."""
    return int(round(STROKES_PER_PIXEL * H * W))


# ---------------------------------------------------------------------------
# The five workloads (one synthetic stand-in per configuration)
# ---------------------------------------------------------------------------

@dataclass
class Job:
    """One page plus the parameters it is binarized with."""
    img: np.ndarray
    win: int
    k: float
    R: float = 128.0
    rule: int = 0  # 0 = Sauvola, 1 = Niblack
    mask: np.ndarray | None = field(default=None, repr=False)

    @property
    def H(self) -> int:
        return self.img.shape[0]

    @property
    def W(self) -> int:
        return self.img.shape[1]

    @property
    def channels(self) -> int:
        return 1 if self.img.ndim == 2 else self.img.shape[2]


def config0(seed_base: int = 0) -> list[Job]:
    """256x256 gray page, 200 strokes, Sauvola win 15, k 0.5, R 128."""
    img = page(256, 256, 200, seed=1000 * 0 + seed_base)
    return [Job(img, 15, 0.5, 128.0, 0)]


CONFIG1_CASES = [  # (rule, win, k)
    (0, 15, 0.5), (0, 31, 0.5), (0, 61, 0.5), (0, 101, 0.5), (1, 31, -0.2),
]


def config1(seed_base: int = 0, size: int = 4096) -> list[Job]:
    """4096x4096 gray page, 40k strokes; Sauvola k 0.5 at win 15/31/61/101 and
    Niblack k -0.2 at win 31 (one job per case, all on the same page)."""
    img = page(size, size, strokes_for(size, size), seed=1000 * 1 + seed_base)
    return [Job(img, w, k, 128.0, r) for (r, w, k) in CONFIG1_CASES]


def config2(n_pages: int = 64, seed_base: int = 0, H: int = 3508, W: int = 2480) -> list[Job]:
    """RGB pages 3508x2480 (A4 portrait at 300 dpi), tinted; Sauvola win 31,
    k 0.34, R 128."""
    return [Job(page(H, W, strokes_for(H, W), seed=1000 * 2 + seed_base + i, channels=3),
                31, 0.34, 128.0, 0) for i in range(n_pages)]


CONFIG3_WINDOWS = (15, 31, 61, 101, 151)


def config3_specs(n_pages: int = 512, seed_base: int = 0):
    """Shapes and parameters of the uneven batch: H, W ~ U{300..4000},
    win from {15, 31, 61, 101, 151}, k ~ U[0.2, 0.5], R 128."""
    rng = rng_for(1000 * 3 + 999_983 + seed_base)
    Hs = rng.integers(300, 4001, size=n_pages)
    Ws = rng.integers(300, 4001, size=n_pages)
    wins = rng.choice(np.array(CONFIG3_WINDOWS), size=n_pages)
    ks = rng.uniform(0.2, 0.5, size=n_pages)
    return [(int(Hs[i]), int(Ws[i]), int(wins[i]), float(np.float32(ks[i]))) for i in range(n_pages)]


def config3(n_pages: int = 512, seed_base: int = 0) -> list[Job]:
    out = []
    for i, (H, W, win, k) in enumerate(config3_specs(n_pages, seed_base)):
        img = page(H, W, strokes_for(H, W), seed=1000 * 3 + seed_base + i)
        out.append(Job(img, win, k, 128.0, 0))
    return out


def config4_request(rng: np.random.Generator):
    """Shape and parameters of one served request: pixel count log-uniform in
    [0.1, 16] Mpx, aspect U[0.5, 2], gray or RGB with p = 1/2, odd win in
    [15, 151], Sauvola k 0.5, R 128."""
    P = math.exp(rng.uniform(math.log(1e5), math.log(1.6e7)))
    a = rng.uniform(0.5, 2.0)
    H = max(1, int(round(math.sqrt(P * a))))
    W = max(1, int(round(P / H)))
    channels = 3 if rng.random() < 0.5 else 1
    win = int(rng.integers(7, 76)) * 2 + 1  # odd, 15..151
    return H, W, channels, win, 0.5


def config4_stream(rate: float, duration: float, seed: int, max_requests: int = 10_000):
    """Poisson arrivals at `rate` req/s for `duration` s (or max_requests):
    list of (arrival_s, H, W, channels, win, k) with the config4_request mix."""
    rng = rng_for(seed)
    t, out = 0.0, []
    while len(out) < max_requests:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        H, W, C, win, k = config4_request(rng)
        out.append((t, H, W, C, win, k))
    return out


def device_canvases(device):
    """One gray and one RGB 4096 x 4096 page as flat device tensors; served
    requests take contiguous H*W*C-byte views of them as their inputs."""
    import torch
    return {C: torch.from_numpy(page(4096, 4096, strokes_for(4096, 4096), seed=4000 + C,
                                     channels=C).reshape(-1)).to(device) for C in (1, 3)}


def pinned_canvases():
    """The same two canvases in pinned host memory (host-origin requests)."""
    import torch
    out = {}
    for C in (1, 3):
        src = torch.from_numpy(page(4096, 4096, strokes_for(4096, 4096), seed=4000 + C,
                                    channels=C).reshape(-1))
        dst = torch.empty(src.numel(), dtype=torch.uint8, pin_memory=True)
        dst.copy_(src)
        out[C] = dst
    return out


def canvas_view(canvases, H: int, W: int, C: int, rng: np.random.Generator):
    n = H * W * C
    base = canvases[C]
    off = int(rng.integers(0, base.numel() - n + 1))
    v = base[off:off + n]
    return v.view(H, W) if C == 1 else v.view(H, W, 3)
