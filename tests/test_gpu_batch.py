"""GPU: the batched persistent launch (and its graph replay) gives every page
exactly the bytes the single-page entry point gives it, and those agree
with the oracle."""
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


def mixed_jobs(seed, n, max_side=700):
    """Uneven pages: gray and RGB, Sauvola and Niblack (k = 0 included),
    windows 1..151 (odd and even), ragged sizes down to 1x1."""
    import pagegen
    rng = np.random.default_rng(seed)
    jobs = []
    for i in range(n):
        H, W = int(rng.integers(1, max_side)), int(rng.integers(1, max_side))
        if i == 0:
            H, W = 1, 1
        C = int(rng.choice([1, 3]))
        win = int(rng.choice([1, 2, 15, 16, 31, 61, 101, 151]))
        rule = int(rng.integers(0, 2))
        k = 0.0 if i % 7 == 3 else f32(float(rng.uniform(-0.3, 0.6)))
        img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=seed * 1000 + i, channels=C)
        jobs.append((img, win, k, 128.0, rule))
    return jobs


def run_batch(bz, B, jobs, use_graph):
    dev = []
    for img, win, k, R, rule in jobs:
        t = torch.from_numpy(img).cuda()
        o = torch.full(img.shape[:2], 7, dtype=torch.uint8, device="cuda")
        dev.append((t, o, win, k, R, rule))
    B.run(dev, use_graph=use_graph)
    torch.cuda.synchronize()
    return [d[1].cpu().numpy() for d in dev]


def single(bz, img, win, k, R, rule):
    out = bz.binarize(torch.from_numpy(img).cuda(), win, k, R, rule)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_single_pages(bz, oracle_mod, use_graph):
    from oracle.compare import compare_out
    jobs = mixed_jobs(11, 24)
    with bz.Batch(64) as B:
        outs = run_batch(bz, B, jobs, use_graph)
        info = B.info()
    assert info["grid"] > 0 and info["last_items"] > len(jobs) - 1
    for (img, win, k, R, rule), out in zip(jobs, outs):
        assert np.array_equal(out, single(bz, img, win, k, R, rule)), (img.shape, win, rule)
        if img.shape[0] * img.shape[1] * min(win, img.shape[0]) * min(win, img.shape[1]) < 3e8:
            ref = oracle_mod.binarize(img, win, k, R, rule)
            assert compare_out(out, ref.out, ref.gray, ref.t)["ok"]


@pytest.mark.parametrize("use_graph", [False, True])
def test_narrow_pages_of_every_row_end_overhang(bz, oracle_mod, use_graph):
    """One batch of narrow pages, widths 1..40 (below 16 pixels the edge row
    body, above it the wide body with every overhang 1..15 of a row's last
    chunk), gray and RGB, both rules: each equals the page run alone and the
    oracle."""
    import pagegen
    from oracle.compare import compare_out
    jobs = []
    for W in range(1, 41):
        C = 1 if W % 2 else 3
        win, rule, k = ((15, 0, f32(0.5)), (31, 1, f32(-0.2)), (61, 0, f32(0.34)))[W % 3]
        img = pagegen.page(20 + W % 7, W, 1, seed=5000 + W, channels=C)
        jobs.append((img, win, k, 128.0, rule))
    with bz.Batch(64) as B:
        outs = run_batch(bz, B, jobs, use_graph)
    for (img, win, k, R, rule), out in zip(jobs, outs):
        assert np.array_equal(out, single(bz, img, win, k, R, rule)), (img.shape, win, rule)
        ref = oracle_mod.binarize(img, win, k, R, rule)
        assert compare_out(out, ref.out, ref.gray, ref.t)["ok"], (img.shape, win, rule)


def test_graph_replays_with_changing_batches(bz):
    """One batch object, graph mode: batches with different page counts and
    kinds (forcing re-capture), each replayed several times with eager work
    and synchronisation in between; every replay is checked."""
    with bz.Batch(40) as B:
        for rep, seed in enumerate([21, 22, 21, 23, 23]):
            jobs = mixed_jobs(seed, 8 + 4 * (seed % 3), max_side=400)
            expect = [single(bz, *j) for j in jobs]
            for _ in range(2):
                outs = run_batch(bz, B, jobs, use_graph=True)
                for e, o in zip(expect, outs):
                    assert np.array_equal(e, o), (rep, seed)
                # eager work between replays
                x = torch.randn(1000, device="cuda").sum()
                torch.cuda.synchronize()
                assert torch.isfinite(x)


def test_config2_rgb_pages_batched(bz):
    """A4 RGB pages (3508 x 2480), Sauvola win 31, k 0.34, in one launch."""
    import pagegen
    pages = pagegen.config2(n_pages=2)
    jobs = [(p.img, p.win, f32(p.k), 128.0, 0) for p in pages] * 2
    with bz.Batch(8) as B:
        outs = run_batch(bz, B, jobs, use_graph=True)
    for (img, win, k, R, rule), out in zip(jobs, outs):
        assert np.array_equal(out, single(bz, img, win, k, R, rule))


def blocks_jobs(seed):
    """Pages for a batch whose LDS cap (40896 B, four workgroups per CU) is
    below the ring of the wider windows: gray pages at win 61-241 take the
    256-column blocks layout and win 255 the 128-column one (both rules, so
    every blocks group), gray win 15 / 31 and RGB pages the ring; ragged sizes
    of one to several tiles."""
    import pagegen
    rng = np.random.default_rng(seed)
    spec = [(1, 61, 0), (1, 101, 1), (1, 151, 0), (1, 241, 1), (1, 255, 0), (1, 255, 1), (1, 15, 0),
            (3, 31, 1), (3, 61, 0), (1, 31, 1), (1, 101, 0)]
    jobs = []
    for i, (C, win, rule) in enumerate(spec):
        H, W = int(rng.integers(40, 700)), int(rng.integers(40, 900))
        k = f32(float(rng.uniform(-0.3, 0.6)))
        img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=seed * 100 + i, channels=C)
        jobs.append((img, win, k, 128.0, rule))
    return jobs


@pytest.mark.parametrize("use_graph", [False, True])
def test_blocks_layout_pages_in_a_small_cap_batch(bz, oracle_mod, use_graph):
    """With an LDS cap of a quarter CU, gray pages whose ring does not fit run
    in the blocks layout (one kernel per blocks tile variant, after the ring
    kernel): every page's bytes equal the single-page entry point's, and the
    oracle's where it finishes quickly."""
    from oracle.compare import compare_out
    jobs = blocks_jobs(31)
    with bz.Batch(16, lds_cap=40896) as B:
        outs = run_batch(bz, B, jobs, use_graph)
        # four workgroups per CU at this cap
        assert B.info()["grid"] == 4 * torch.cuda.get_device_properties(0).multi_processor_count
    for (img, win, k, R, rule), out in zip(jobs, outs):
        assert np.array_equal(out, single(bz, img, win, k, R, rule)), (img.shape, win, rule)
        if img.shape[0] * img.shape[1] * min(win, img.shape[0]) * min(win, img.shape[1]) < 3e8:
            ref = oracle_mod.binarize(img, win, k, R, rule)
            assert compare_out(out, ref.out, ref.gray, ref.t)["ok"], (img.shape, win, rule)


@pytest.mark.parametrize("use_graph", [False, True])
def test_every_occupancy_class_in_one_batch(bz, oracle_mod, use_graph):
    """With the largest LDS cap, RGB pages at win 15, 61, 101 and 151-201 need
    the LDS share of 4, 3, 2 and 1 workgroups per CU: one batch makes a
    launch per class (plus the blocks launches of the wide gray pages and a
    128-column ring page), one after another.  Every page equals its
    single-page run, and the oracle where it finishes quickly."""
    import pagegen
    from oracle.compare import compare_out
    rng = np.random.default_rng(77)
    spec = [(3, 15, 0, None), (3, 61, 1, None), (3, 101, 0, None), (3, 151, 1, None), (3, 201, 0, None),
            (1, 101, 0, None), (1, 151, 1, None), (3, 101, 1, (128, 64)), (1, 31, 0, None)]
    jobs, dev = [], []
    for i, (C, win, rule, tile) in enumerate(spec):
        H, W = int(rng.integers(60, 420)), int(rng.integers(60, 600))
        k = f32(float(rng.uniform(-0.3, 0.6)))
        img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=7700 + i, channels=C)
        jobs.append((img, win, k, 128.0, rule))
        t = torch.from_numpy(img).cuda()
        dev.append((t, torch.full(img.shape[:2], 7, dtype=torch.uint8, device="cuda"), win, k, 128.0, rule, tile))
    with bz.Batch(16, lds_cap=163776) as B:
        B.run(dev, use_graph=use_graph)
        torch.cuda.synchronize()
    for (img, win, k, R, rule), d in zip(jobs, dev):
        out = d[1].cpu().numpy()
        assert np.array_equal(out, single(bz, img, win, k, R, rule)), (img.shape, win, rule)
        if img.shape[0] * img.shape[1] * min(win, img.shape[0]) * min(win, img.shape[1]) < 3e8:
            ref = oracle_mod.binarize(img, win, k, R, rule)
            assert compare_out(out, ref.out, ref.gray, ref.t)["ok"], (img.shape, win, rule)


def test_graph_recaptures_when_the_kernel_groups_change(bz):
    """Graph mode on one batch object: a batch with blocks pages, then one
    with ring pages only (fewer kernels in the graph), then the first again;
    each replayed twice and checked."""
    a = blocks_jobs(41)
    b = [j for j in blocks_jobs(42) if j[1] <= 31 or j[0].ndim == 3]
    expect = {id(j): single(bz, *j) for j in a + b}
    with bz.Batch(16, lds_cap=40896) as B:
        for jobs in (a, b, a):
            for _ in range(2):
                outs = run_batch(bz, B, jobs, use_graph=True)
                for j, o in zip(jobs, outs):
                    assert np.array_equal(expect[id(j)], o), (j[0].shape, j[1])


@pytest.mark.parametrize("use_graph", [False, True])
def test_back_to_back_runs_on_two_streams(bz, use_graph):
    """One batch object, five runs enqueued without waiting, alternating
    between two streams: each run uses the object's other set of run
    buffers, and the third waits for the first before reusing its set; every
    run's pages must come out as when binarized alone."""
    sets = [mixed_jobs(50 + i, 6, max_side=500) for i in range(5)]
    expect = [[single(bz, *j) for j in jobs] for jobs in sets]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    dev = []
    for jobs in sets:
        d = []
        for img, win, k, R, rule in jobs:
            t = torch.from_numpy(img).cuda()
            d.append((t, torch.full(img.shape[:2], 7, dtype=torch.uint8, device="cuda"), win, k, R, rule))
        dev.append(d)
    torch.cuda.synchronize()
    with bz.Batch(16) as B:
        for i, d in enumerate(dev):
            B.run(d, use_graph=use_graph, stream=streams[i % 2])
        torch.cuda.synchronize()
    for i, (d, e) in enumerate(zip(dev, expect)):
        for j, (job, ref) in enumerate(zip(d, e)):
            assert np.array_equal(job[1].cpu().numpy(), ref), (i, j)


def test_batch_rejects_bad_pages(bz):
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    out = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    rgb = torch.zeros((64, 64, 3), dtype=torch.uint8, device="cuda")
    with bz.Batch(2, lds_cap=48 * 1024) as B:
        with pytest.raises(bz.BinarizeError) as ei:
            B.run([(rgb, out, 255, 0.5, 128.0, 0)])  # an RGB ring that needs more LDS than the cap
        assert ei.value.code == -9
        B.run([(img, out, 255, 0.5, 128.0, 0)])  # a gray page of that window fits in the blocks layout
        with pytest.raises(bz.BinarizeError) as ei:
            B.run([(img, out, 0, 0.5, 128.0, 0)])
        assert ei.value.code == -4
        with pytest.raises(bz.BinarizeError) as ei:
            B.run([(img, out, 15, 0.5, 128.0, 0)] * 3)  # more pages than max_pages
        assert ei.value.code == -2
        B.run([(img, out, 15, 0.5, 128.0, 0)])  # still usable after errors
        torch.cuda.synchronize()
        assert torch.all(out == 255)


def test_batch_rejects_pages_that_write_over_each_other(bz):
    """Pages of a batch run concurrently: an output shared by two pages, or
    one page's output inside another page's input, is refused before any
    launch; shared inputs and outputs packed back to back are fine."""
    import pagegen
    a = torch.from_numpy(pagegen.page(40, 50, 30, seed=11)).cuda()
    b = torch.from_numpy(pagegen.page(40, 50, 30, seed=12)).cuda()
    buf = torch.zeros(3 * 40 * 50, dtype=torch.uint8, device="cuda")
    o0, o1 = buf[:2000].view(40, 50), buf[2000:4000].view(40, 50)
    rgb = torch.from_numpy(pagegen.page(40, 50, 30, seed=13, channels=3)).cuda()  # 6000 bytes
    with bz.Batch(4) as B:
        cases = [
            [(a, o0, 15, 0.5, 128.0, 0), (b, o0, 15, 0.5, 128.0, 0)],                    # same output
            [(a, o0, 15, 0.5, 128.0, 0), (b, buf[1999:3999].view(40, 50), 15, 0.5, 128.0, 0)],  # one byte shared
            [(rgb, o0, 15, 0.5, 128.0, 0),
             (a, rgb.view(-1)[1000:3000].view(40, 50), 15, 0.5, 128.0, 0)],              # output inside an RGB input
        ]
        for jobs in cases:
            with pytest.raises(bz.BinarizeError) as ei:
                B.run(jobs)
            assert ei.value.code == -7
        # a shared input and outputs packed back to back
        B.run([(a, o0, 15, 0.5, 128.0, 0), (a, o1, 31, -0.2, 128.0, 1), (b, buf[4000:].view(40, 50), 61, 0.3, 128.0, 0)])
        torch.cuda.synchronize()
        assert torch.equal(o0, bz.binarize(a, 15, 0.5, 128.0, 0))
        assert torch.equal(o1, bz.binarize(a, 31, -0.2, 128.0, 1))
        assert torch.equal(buf[4000:].view(40, 50), bz.binarize(b, 61, 0.3, 128.0, 0))
