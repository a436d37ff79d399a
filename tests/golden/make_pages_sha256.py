"""Writes pages_sha256.json: SHA-256 digests of small seeded synthetic pages.

Calls only the page generator (inputs, not expected results), so a change to
the generator that would silently change every workload fails a test.
Run from the repository root:  python tests/golden/make_pages_sha256.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import pagegen  # noqa: E402

CASES = [
    {"H": 256, "W": 256, "strokes": 200, "seed": 0, "channels": 1},
    {"H": 97, "W": 131, "strokes": 30, "seed": 5, "channels": 3},
    {"H": 1, "W": 1, "strokes": 1, "seed": 9, "channels": 1},
]


def digest(case):
    img = pagegen.page(case["H"], case["W"], case["strokes"], case["seed"], case["channels"])
    return hashlib.sha256(img.tobytes()).hexdigest()


if __name__ == "__main__":
    out = [dict(c, sha256=digest(c)) for c in CASES]
    with open(os.path.join(HERE, "pages_sha256.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
