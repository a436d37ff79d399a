"""F-measure study of the binarization methods on synthetic pages with known
ground truth (the accuracy comparison of Sec. 3, Tables 1-3, Eq. 6).

Methods: Otsu's global threshold (Eq. 2), Niblack, exact Sauvola (Eq. 4)
and the sampled-window Sauvola (Eq. 5) over this library's plus / x / star
structures.  As in the paper, every method is scored per page with its best
(window, k) combination, and the per-page best F-measures are averaged.

The page images are synthetic (``pagegen``): the paper's datasets (DIBCO
2009, H-DIBCO 2010, CMATERdb-6) are not available, and the generator's
stroke mask is the ground truth.  Binarization and the TP / FP / FN counts
run on the GPU; only Eq. 6 on the three counts is evaluated here.

    python -m paper_1210_3165_amd.evaluate [--pages 6] [--H 768 --W 1024] [--degraded]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import GS_PLUS, GS_STAR, GS_X, NIBLACK, SAUVOLA, Otsu, binarize, binarize_gs, fmeasure_counts

WINDOWS = (15, 31, 61)
SAUVOLA_K = (0.05, 0.1, 0.2, 0.3, 0.4, 0.5)
NIBLACK_K = (-0.8, -0.6, -0.4, -0.2, 0.0)
R = 128.0


def fmeasure(tp: int, fp: int, fn: int) -> float:
    """Eq. 6: 2 R P / (R + P) with R = TP / (TP + FN), P = TP / (TP + FP)."""
    if tp == 0:
        return 0.0
    rec = tp / (tp + fn)
    prec = tp / (tp + fp)
    return 2 * rec * prec / (rec + prec)


def methods(windows=WINDOWS, sauvola_k=SAUVOLA_K, niblack_k=NIBLACK_K):
    """(name, [(params, run(img, out))]) for every method and grid point."""
    yield "otsu", [({}, lambda img, out, o=None: Otsu(img.device).run(img, out))]
    yield "niblack", [({"win": w, "k": k}, lambda img, out, w=w, k=k: binarize(img, w, k, R, NIBLACK, out=out))
                      for w in windows for k in niblack_k]
    yield "sauvola", [({"win": w, "k": k}, lambda img, out, w=w, k=k: binarize(img, w, k, R, SAUVOLA, out=out))
                      for w in windows for k in sauvola_k]
    for name, st in (("gs-plus", GS_PLUS), ("gs-x", GS_X), ("gs-star", GS_STAR)):
        yield name, [({"win": w, "k": k},
                      lambda img, out, w=w, k=k, st=st: binarize_gs(img, w, k, R, st, out=out))
                     for w in windows for k in sauvola_k]


def evaluate(pages, windows=WINDOWS, sauvola_k=SAUVOLA_K, niblack_k=NIBLACK_K, device=None) -> dict:
    """pages: list of (img uint8 array, ground-truth mask).  Returns per-method
    mean of the per-page best F-measure and the chosen parameters."""
    dev = torch.device(device) if device is not None else torch.device("cuda", 0)
    res = {}
    grid = list(methods(windows, sauvola_k, niblack_k))
    for pi, (img_np, mask) in enumerate(pages):
        img = torch.from_numpy(np.ascontiguousarray(img_np)).to(dev)
        gt = torch.from_numpy(np.ascontiguousarray(mask, dtype=np.uint8)).to(dev)
        out = torch.empty(img_np.shape[:2], dtype=torch.uint8, device=dev)
        for name, points in grid:
            counts = []
            for params, run in points:
                run(img, out)
                counts.append((params, fmeasure_counts(out, gt).clone()))
            torch.cuda.synchronize(dev)
            scored = [(fmeasure(*(int(v) for v in c.cpu())), p) for p, c in counts]
            best_fm, best_p = max(scored, key=lambda s: s[0])
            r = res.setdefault(name, {"per_page": [], "params": []})
            r["per_page"].append(best_fm)
            r["params"].append(best_p)
    for r in res.values():
        r["mean_fm"] = float(np.mean(r["per_page"]))
    return res


def main(argv=None) -> int:
    import pagegen
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--pages", type=int, default=6)
    ap.add_argument("--H", type=int, default=768)
    ap.add_argument("--W", type=int, default=1024)
    ap.add_argument("--degraded", action="store_true", help="strong shading, faint ink, more noise")
    ap.add_argument("--seed", type=int, default=6000)
    args = ap.parse_args(argv)
    pages = []
    for i in range(args.pages):
        C = 3 if i % 2 else 1
        if args.degraded:
            pages.append(pagegen.degraded_page(args.H, args.W, args.seed + i, channels=C))
        else:
            pages.append(pagegen.page(args.H, args.W, pagegen.strokes_for(args.H, args.W), args.seed + i,
                                      channels=C, return_mask=True))
    res = evaluate(pages)
    rec = {"pages": args.pages, "H": args.H, "W": args.W, "degraded": args.degraded,
           "windows": list(WINDOWS), "sauvola_k": list(SAUVOLA_K), "niblack_k": list(NIBLACK_K),
           "methods": {k: {"mean_fm": v["mean_fm"], "per_page": v["per_page"], "params": v["params"]}
                       for k, v in res.items()}}
    for name, v in res.items():
        print(f"{name:10s} mean FM {100 * v['mean_fm']:6.2f}%", file=sys.stderr)
    print(json.dumps(rec))
    return 0


if __name__ == "__main__":
    sys.exit(main())
