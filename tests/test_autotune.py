"""The launch-shape autotuner: bucketing, cache round trip (CPU) and a real
tuning pass whose chosen shapes give identical bytes (GPU)."""
import json

import numpy as np
import pytest

from paper_1210_3165_amd import autotune


def test_buckets():
    assert [autotune.win_bucket(w) for w in (1, 15, 16, 31, 100, 101, 151, 200, 255)] == \
        [15, 15, 31, 31, 101, 101, 151, 201, 255]
    assert autotune.size_bucket(4096) == 12 and autotune.size_bucket(1) == 0
    assert autotune.size_bucket(3000 * 3000) == 23


def test_lds_caps_match_occupancy_targets():
    assert 4 * (autotune.LDS_4_PER_CU + 64) == 160 * 1024
    assert 2 * (autotune.LDS_2_PER_CU + 64) == 160 * 1024
    assert autotune.tile_fits(256, 31, autotune.LDS_4_PER_CU)
    assert not autotune.tile_fits(256, 255)
    assert autotune.tile_fits(128, 255)


def test_cache_round_trip(tmp_path):
    path = tmp_path / "tune.json"
    t = autotune.Tuner.__new__(autotune.Tuner)
    import threading
    t.path, t.reps, t._lock, t.cache = str(path), 1, threading.Lock(), {}
    t.cache["gfx950|single|C1|w15|H12|W12"] = {"tile": [256, 64], "ms": 0.04, "tried": {}}
    t._save()
    assert json.loads(path.read_text())["gfx950|single|C1|w15|H12|W12"]["tile"] == [256, 64]
    assert t._load() == t.cache


def test_cache_saves_merge_entries_of_other_tuners(tmp_path):
    """Two tuners on one cache file (say two processes): each save keeps the
    entries the other saved meanwhile, and no temporary file is left."""
    import threading
    path = str(tmp_path / "tune.json")
    a, b = (autotune.Tuner.__new__(autotune.Tuner) for _ in range(2))
    for t in (a, b):
        t.path, t.reps, t._lock = path, 1, threading.Lock()
        t.cache = t._load()
    a.cache["k_a"] = {"tile": [256, 64]}
    a._save()
    b.cache["k_b"] = {"tile": [128, 64]}  # b loaded before a saved
    b._save()
    on_disk = json.loads(open(path).read())
    assert set(on_disk) == {"k_a", "k_b"}
    a.cache["k_a2"] = {"tile": [256, 128]}
    a._save()
    assert set(json.loads(open(path).read())) == {"k_a", "k_b", "k_a2"}
    assert sorted(p.name for p in tmp_path.iterdir()) == ["tune.json"]


@pytest.mark.gpu
def test_tuned_shapes_are_bit_identical(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as bz
    import pagegen
    tuner = autotune.Tuner(path=str(tmp_path / "t.json"), reps=2)
    tw, th = tuner.single_tile(600, 900, 1, 31)
    assert (tw, th) in autotune.SINGLE_TILES
    img = torch.from_numpy(pagegen.page(600, 900, 300, seed=5)).cuda()
    assert torch.equal(bz.binarize(img, 31, 0.5, tile=(tw, th)), bz.binarize(img, 31, 0.5))
    cfg = tuner.batch_config([(300, 400, 1, 15), (500, 200, 3, 31), (700, 700, 1, 61)])
    assert cfg["tile_h"] in autotune.BATCH_TILE_H
    assert cfg["lds_cap"] in (autotune.LDS_2_PER_CU, autotune.LDS_4_PER_CU)
    # cached now: a second tuner reads the same answer without timing
    again = autotune.Tuner(path=str(tmp_path / "t.json"), reps=2)
    assert again.single_tile(600, 900, 1, 31) == (tw, th)
    jobs = [(pagegen.page(h, w, 50, seed=i, channels=c), win) for i, (h, w, c, win)
            in enumerate([(300, 400, 1, 15), (500, 200, 3, 31), (700, 700, 1, 61)])]
    dev = [(torch.from_numpy(im).cuda(), torch.empty(im.shape[:2], dtype=torch.uint8, device="cuda"), win,
            0.5, 128.0, 0, (0, cfg["tile_h"])) for im, win in jobs]
    with bz.Batch(4, lds_cap=cfg["lds_cap"]) as B:
        B.run(dev)
        torch.cuda.synchronize()
    for (im, win), d in zip(jobs, dev):
        assert np.array_equal(d[1].cpu().numpy(),
                              bz.binarize(torch.from_numpy(im).cuda(), win, 0.5).cpu().numpy())


@pytest.mark.gpu
def test_fusion_choice_is_measured_and_bit_identical(tmp_path):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as bz
    import pagegen
    tuner = autotune.Tuner(path=str(tmp_path / "t.json"), reps=2)
    choice = tuner.single(600, 900, 3, 31)
    assert choice["fused_ms"] > 0 and choice["staged_ms"] > 0
    assert choice["fused"] == (choice["fused_ms"] <= choice["staged_ms"])
    img = torch.from_numpy(pagegen.page(600, 900, 300, seed=6, channels=3)).cuda()
    ref = bz.binarize(img, 31, 0.5)
    assert torch.equal(tuner.binarize(img, 31, 0.5), ref)
    assert torch.equal(bz.binarize_staged(img, 31, 0.5), ref)
    again = autotune.Tuner(path=str(tmp_path / "t.json"), reps=2)
    assert again.single(600, 900, 3, 31) == choice
