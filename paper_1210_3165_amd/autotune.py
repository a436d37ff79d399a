"""Autotuner for the tile kernel's launch shape.

The binarized bytes never depend on the launch shape (every tile shape and
every batch configuration is bit-identical), only the speed does, so the
tuner is free to time candidates on random data of the real shapes.

* ``Tuner.single_tile(H, W, C, win)`` picks (tile_w, tile_h) for one-page
  launches: the tile count must fill 256 CUs, yet taller tiles amortize the
  win start-up rows each tile spends before its first output.
* ``Tuner.single(H, W, C, win)`` adds pass fusion to that choice: it times
  the unfused, two-pass form (``binarize_staged``: row window sums through two
  u32 planes in HBM, then the column pass) against the best fused tile, and
  ``Tuner.binarize`` runs whichever won.  All choices give identical bytes.
* ``Tuner.batch_config(specs)`` picks the persistent batch's LDS cap (2 or 4
  workgroups per CU) and tile height for a set of page shapes.

Results are cached as JSON, keyed by GPU architecture, channels, window
bucket and size bucket, in ``$BZ_TUNE_CACHE`` or
``~/.cache/paper_1210_3165_amd/tune.json``; tuning resumes from the cache.
"""
from __future__ import annotations

import json
import math
import os
import threading

import torch

from . import Batch, binarize, binarize_staged, tile_lds

WIN_BUCKETS = (15, 31, 61, 101, 151, 201, 255)
SINGLE_TILES = ((256, 32), (256, 64), (256, 128), (256, 256), (128, 64), (128, 128), (128, 256))
BATCH_TILE_H = (128, 256, 512)
BATCH_SAMPLE = 512  # pages the batch tuner times
LDS_4_PER_CU = 160 * 1024 // 4 - 64   # cap that lets 4 workgroups share a CU
LDS_2_PER_CU = 160 * 1024 // 2 - 64


def win_bucket(win: int) -> int:
    for b in WIN_BUCKETS:
        if win <= b:
            return b
    return WIN_BUCKETS[-1]


def size_bucket(n: float) -> int:
    """log2 bucket of a pixel count or a side length."""
    return max(0, int(round(math.log2(max(n, 1)))))


def tile_fits(tile_w: int, win: int, cap: int = 160 * 1024, channels: int = 1) -> bool:
    need = tile_lds(tile_w, win, channels)
    return need is not None and need <= cap


def default_cache_path() -> str:
    p = os.environ.get("BZ_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1210_3165_amd", "tune.json")


class Tuner:
    def __init__(self, path: str | None = None, reps: int = 8, device=None):
        self.path = path or default_cache_path()
        self.reps = reps
        self.device = torch.device(device) if device is not None else \
            torch.device("cuda", torch.cuda.current_device())
        self._lock = threading.Lock()
        self.cache = self._load()

    # ------------------------------------------------------------- cache
    def _load(self) -> dict:
        try:
            with open(self.path) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}

    def _save(self) -> None:
        """Merge this tuner's entries into the file on disk (entries other
        processes saved meanwhile are kept) and replace it atomically through
        a temporary file of this process and thread."""
        os.makedirs(os.path.dirname(os.path.abspath(self.path)), exist_ok=True)
        merged = self._load()
        merged.update(self.cache)
        self.cache = merged
        tmp = f"{self.path}.{os.getpid()}.{threading.get_ident()}.tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)

    def arch(self) -> str:
        return torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]

    # ------------------------------------------------------------- timing
    def _time(self, fn) -> float:
        stream = torch.cuda.current_stream(self.device)
        fn()
        torch.cuda.synchronize(self.device)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(self.reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize(self.device)
        return e0.elapsed_time(e1) / self.reps

    def _page(self, H: int, W: int, C: int) -> torch.Tensor:
        shape = (H, W) if C == 1 else (H, W, 3)
        return torch.randint(0, 256, shape, dtype=torch.uint8, device=self.device)

    # ------------------------------------------------------------- single page
    def single_tile(self, H: int, W: int, C: int, win: int, rule: int = 0) -> tuple[int, int]:
        key = f"{self.arch()}|single|C{C}|w{win_bucket(win)}|H{size_bucket(H)}|W{size_bucket(W)}"
        with self._lock:
            hit = self.cache.get(key)
        if hit:
            return tuple(hit["tile"])
        img = self._page(H, W, C)
        out = torch.empty((H, W), dtype=torch.uint8, device=self.device)
        best, best_ms = None, float("inf")
        results = {}
        for tw, th in SINGLE_TILES:
            if not tile_fits(tw, win, channels=C):
                continue
            ms = self._time(lambda: binarize(img, win, 0.5, 128.0, rule, out=out, tile=(tw, th)))
            results[f"{tw}x{th}"] = round(ms, 4)
            if ms < best_ms:
                best, best_ms = (tw, th), ms
        with self._lock:
            self.cache[key] = {"tile": list(best), "ms": round(best_ms, 4), "tried": results}
            self._save()
        return best

    def single(self, H: int, W: int, C: int, win: int, rule: int = 0) -> dict:
        """{"fused": bool, "tile": [tw, th], "fused_ms", "staged_ms"} for one
        page of this shape: the fused kernel at its best tile against the
        staged two-pass form."""
        tile = self.single_tile(H, W, C, win, rule)
        key = f"{self.arch()}|fusion|C{C}|w{win_bucket(win)}|H{size_bucket(H)}|W{size_bucket(W)}"
        with self._lock:
            hit = self.cache.get(key)
        if hit:
            return dict(hit)
        img = self._page(H, W, C)
        out = torch.empty((H, W), dtype=torch.uint8, device=self.device)
        ws = torch.empty(8 * H * W, dtype=torch.uint8, device=self.device)
        fused_ms = self._time(lambda: binarize(img, win, 0.5, 128.0, rule, out=out, tile=tile))
        staged_ms = self._time(lambda: binarize_staged(img, win, 0.5, 128.0, rule, out=out, workspace=ws))
        rec = {"fused": fused_ms <= staged_ms, "tile": list(tile), "fused_ms": round(fused_ms, 4),
               "staged_ms": round(staged_ms, 4)}
        with self._lock:
            self.cache[key] = rec
            self._save()
        return dict(rec)

    def binarize(self, img: torch.Tensor, win: int, k: float, R: float = 128.0, rule: int = 0,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        """Binarize one page with the tuned choice of fusion and tile."""
        H, W = img.shape[0], img.shape[1]
        C = 1 if img.dim() == 2 else img.shape[2]
        choice = self.single(H, W, C, win, rule)
        if choice["fused"]:
            return binarize(img, win, k, R, rule, out=out, tile=tuple(choice["tile"]))
        return binarize_staged(img, win, k, R, rule, out=out)

    # ------------------------------------------------------------- batch
    def batch_config(self, specs) -> dict:
        """specs: iterable of (H, W, C, win).  Returns {"lds_cap", "tile_h"}."""
        specs = list(specs)
        Cs = sorted({c for _, _, c, _ in specs})
        wmax = max(w for _, _, _, w in specs)
        mean_px = sum(h * w for h, w, _, _ in specs) / len(specs)
        key = (f"{self.arch()}|batch|C{'+'.join(map(str, Cs))}|w{win_bucket(wmax)}"
               f"|n{size_bucket(len(specs))}|px{size_bucket(mean_px)}")
        with self._lock:
            hit = self.cache.get(key)
        if hit:
            return dict(hit["config"])
        # time on the shapes themselves, up to 512 pages (an evenly spaced
        # subsample of larger sets): a batch run of that many pages takes
        # milliseconds, and smaller subsamples of uneven sets misjudged the
        # tile height
        step = max(1, -(-len(specs) // BATCH_SAMPLE))
        sample = specs[::step][:BATCH_SAMPLE]
        pages = [(self._page(h, w, c), torch.empty((h, w), dtype=torch.uint8, device=self.device), win)
                 for h, w, c, win in sample]
        caps = [LDS_2_PER_CU]
        if all(tile_fits(256 if tile_fits(256, win, LDS_4_PER_CU, c) else 128, win, LDS_4_PER_CU, c)
               for _, _, c, win in sample):
            caps.append(LDS_4_PER_CU)
        best, best_ms, results = None, float("inf"), {}
        for cap in caps:
            with Batch(len(pages), lds_cap=cap, device=self.device) as B:
                for th in BATCH_TILE_H:
                    jobs = [(img, out, win, 0.5, 128.0, 0, (0, th)) for img, out, win in pages]
                    ms = self._time(lambda: B.run(jobs, use_graph=True))
                    results[f"cap{cap}_h{th}"] = round(ms, 4)
                    if ms < best_ms:
                        best, best_ms = {"lds_cap": cap, "tile_h": th}, ms
        with self._lock:
            self.cache[key] = {"config": best, "ms": round(best_ms, 4), "tried": results,
                               "sampled_pages": len(sample)}
            self._save()
        return dict(best)
