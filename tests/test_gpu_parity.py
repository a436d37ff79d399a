"""GPU parity: the HIP path, called through the C ABI, against the CPU oracle
on the same seeded inputs, element by element.

Bar (see oracle/compare.py): gray, S1, S2, n bit-identical; |t - t_oracle| <=
1e-4; binary output identical except where |f - t_oracle| < 1e-4.
"""
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
    m.lib()  # raises if the library is missing: no fallback
    return m


def gpu_stats(bz, img, win, k, R, rule):
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    res = bz.binarize_stats(t, win, k, R, rule)
    torch.cuda.synchronize()
    return {name: v.cpu().numpy() for name, v in res.items()}


def gpu_out(bz, img, win, k, R, rule, tile=None):
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    out = bz.binarize(t, win, k, R, rule, tile=tile)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def full_check(bz, oracle_mod, img, win, k, R, rule, label=""):
    from oracle.compare import compare_out, compare_stats
    k = f32(k)
    R = f32(R)
    ref = oracle_mod.binarize(img, win, k, R, rule)
    g = gpu_stats(bz, img, win, k, R, rule)
    rep = compare_stats(g, ref)
    assert rep["ok"], (label, rep)
    # the product entry point (no stats planes) decides identically
    out = gpu_out(bz, img, win, k, R, rule)
    assert np.array_equal(out, g["out"]), label
    assert compare_out(out, ref.out, ref.gray, ref.t)["ok"]
    return rep


def oracle_cost(H, W, win):
    return 2.0 * H * W * min(win, H) * min(win, W)


# ------------------------------------------------------------ workloads

def test_config0_full_page(bz, oracle_mod):
    import pagegen
    job = pagegen.config0()[0]
    rep = full_check(bz, oracle_mod, job.img, job.win, job.k, job.R, job.rule, "config0")
    print("config0", rep)


@pytest.mark.parametrize("rule,win,k", [(0, 15, 0.5), (0, 31, 0.5), (0, 61, 0.5), (0, 101, 0.5),
                                        (1, 31, -0.2)])
def test_config1_cases_reduced_page(bz, oracle_mod, rule, win, k):
    """The 4096^2 workload's generator and parameters on a 384 x 440 page:
    several tiles in both directions plus ragged right and bottom tails."""
    import pagegen
    img = pagegen.page(384, 440, pagegen.strokes_for(384, 440), seed=1001)
    full_check(bz, oracle_mod, img, win, k, 128.0, rule, f"cfg1 {rule} {win}")


def test_config2_rgb_reduced_page(bz, oracle_mod):
    import pagegen
    img = pagegen.page(300, 212, pagegen.strokes_for(300, 212), seed=2000, channels=3)
    full_check(bz, oracle_mod, img, 31, 0.34, 128.0, 0, "cfg2 rgb")


def test_config3_mixed_windows_reduced(bz, oracle_mod):
    import pagegen
    rng = np.random.default_rng(3)
    for i, win in enumerate((15, 31, 61, 101, 151)):
        H, W = int(rng.integers(300, 420)), int(rng.integers(300, 420))
        if oracle_cost(H, W, win) > 4e9:
            H = W = 300
        img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=3000 + i)
        full_check(bz, oracle_mod, img, win, float(rng.uniform(0.2, 0.5)), 128.0, 0, f"cfg3 {win}")


# ------------------------------------------------------------ fuzz

def test_seeded_fuzz(bz, oracle_mod):
    """Random shapes 1..300, windows 1..255 (odd and even), k in [-1, 1],
    R in {64, 128, 255}, gray and RGB, both rules; oracle cost bounded."""
    import pagegen
    rng = np.random.default_rng(2024)
    done = 0
    while done < 40:
        H, W = int(rng.integers(1, 301)), int(rng.integers(1, 301))
        win = int(rng.integers(1, 256))
        if oracle_cost(H, W, win) > 6e8:
            continue
        C = int(rng.choice([1, 3]))
        rule = int(rng.integers(0, 2))
        k = float(rng.uniform(-1, 1))
        R = float(rng.choice([64.0, 128.0, 255.0]))
        if rng.random() < 0.5:
            img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=int(rng.integers(1 << 30)),
                               channels=C)
        else:
            shape = (H, W) if C == 1 else (H, W, 3)
            img = rng.integers(0, 256, size=shape, dtype=np.uint8)
        full_check(bz, oracle_mod, img, win, k, R, rule, f"fuzz {H}x{W}x{C} win {win} rule {rule}")
        done += 1


# ------------------------------------------------------------ edge cases

@pytest.mark.parametrize("H,W,win", [(1, 1, 1), (1, 1, 255), (1, 300, 15), (300, 1, 15),
                                     (2, 2, 2), (7, 5, 255), (17, 33, 64), (40, 40, 79),
                                     (16, 256, 240), (33, 257, 241), (20, 520, 255),
                                     (130, 90, 1), (64, 64, 128)])
def test_edge_shapes(bz, oracle_mod, H, W, win):
    rng = np.random.default_rng(H * 1000 + W + win)
    for C in (1, 3):
        shape = (H, W) if C == 1 else (H, W, 3)
        img = rng.integers(0, 256, size=shape, dtype=np.uint8)
        for rule, k in ((0, 0.5), (1, -0.2)):
            full_check(bz, oracle_mod, img, win, k, 128.0, rule, f"edge {H}x{W}x{C} {win}")


@pytest.mark.parametrize("c", [0, 1, 128, 255])
def test_constant_page_no_mismatch_even_in_band(bz, c):
    """s = 0: Sauvola t = c(1-k) and Niblack t = c = f (an exact tie, 255).
    Every pixel must match, including those inside the tolerance band."""
    img = np.full((70, 300), c, np.uint8)
    for rule, k in ((0, 0.5), (0, 0.0), (1, -0.2), (1, 0.7)):
        out = gpu_out(bz, img, 15, k, 128.0, rule)
        assert np.all(out == 255), (c, rule, k)
    if c > 0:
        assert np.all(gpu_out(bz, img, 15, -0.1, 128.0, 0) == 0)


def test_unit_window_is_pointwise(bz):
    rng = np.random.default_rng(1)
    img = rng.integers(0, 256, size=(50, 77), dtype=np.uint8)
    assert np.all(gpu_out(bz, img, 1, 0.5, 128.0, 0) == 255)
    assert np.all(gpu_out(bz, img, 1, 0.9, 128.0, 1) == 255)


def test_ramp_and_two_level(bz, oracle_mod):
    ramp = np.tile(np.arange(256, dtype=np.uint8), (64, 1))
    full_check(bz, oracle_mod, ramp, 31, 0.5, 128.0, 0, "ramp")
    full_check(bz, oracle_mod, ramp, 31, 0.3, 128.0, 1, "ramp niblack")
    edge = np.zeros((64, 300), np.uint8)
    edge[:, 150:] = 255
    full_check(bz, oracle_mod, edge, 21, 0.5, 128.0, 0, "edge")


def test_gray_conversion_exhaustive(bz, oracle_mod):
    """Eq. 1 on the GPU for all 2^24 RGB triples, bit-exact."""
    v = np.arange(256, dtype=np.uint8)
    r, g, b = np.meshgrid(v, v, v, indexing="ij")
    img = np.stack([r, g, b], axis=-1).reshape(4096, 4096, 3)
    s = gpu_stats(bz, img, 1, 0.5, 128.0, 0)
    assert np.array_equal(s["gray"], oracle_mod.gray(img))


# ------------------------------------------------------------ layout

@pytest.mark.parametrize("tile", [(256, 16), (256, 48), (256, 256), (128, 16), (128, 96), (128, 512)])
def test_tile_shapes_bit_identical(bz, oracle_mod, tile):
    import pagegen
    from oracle.compare import compare_out
    img = pagegen.page(333, 517, pagegen.strokes_for(333, 517), seed=44)
    k = f32(0.5)
    ref = oracle_mod.binarize(img, 31, k, 128.0, 0)
    base = gpu_out(bz, img, 31, k, 128.0, 0)
    out = gpu_out(bz, img, 31, k, 128.0, 0, tile=tile)
    assert np.array_equal(out, base)
    assert compare_out(out, ref.out, ref.gray, ref.t)["ok"]


@pytest.mark.parametrize("C", [1, 3])
def test_tile_shapes_identical_full_page(bz, C):
    """A 4096-square page at four windows: 128- and 256-column tiles of
    several heights give the same bytes.  The decision form is chosen per
    256-column block of the page and per 8-row step, never per tile."""
    import pagegen
    img = torch.from_numpy(pagegen.page(4096, 4096, pagegen.strokes_for(4096, 4096), seed=11 + C,
                                        channels=C)).cuda()
    for win, k in ((15, 0.5), (31, 0.34), (61, 0.2), (101, 0.5)):
        k = f32(k)
        base = bz.binarize(img, win, k, 128.0, 0, tile=(256, 64))
        for tile in ((128, 64), (256, 128), (128, 32), (256, 8)):
            out = bz.binarize(img, win, k, 128.0, 0, tile=tile)
            torch.cuda.synchronize()
            assert torch.equal(out, base), (C, win, tile, int((out != base).sum()))


@pytest.mark.parametrize("offset", [1, 2, 3, 5, 13])
def test_unaligned_buffers(bz, oracle_mod, offset):
    """Image and output starting at odd byte offsets, widths not a multiple
    of 4 or 16."""
    from oracle.compare import compare_out
    rng = np.random.default_rng(offset)
    for C, (H, W) in ((1, (97, 301)), (3, (61, 203))):
        shape = (H, W) if C == 1 else (H, W, 3)
        img = rng.integers(0, 256, size=shape, dtype=np.uint8)
        n = img.size
        buf = torch.zeros(n + 64, dtype=torch.uint8, device="cuda")
        view = buf[offset:offset + n].view(*shape)
        view.copy_(torch.from_numpy(img))
        obuf = torch.zeros(H * W + 64, dtype=torch.uint8, device="cuda")
        out = obuf[offset + 3:offset + 3 + H * W].view(H, W)
        bz.binarize(view, 25, 0.4, 128.0, 0, out=out)
        torch.cuda.synchronize()
        ref = oracle_mod.binarize(img, 25, f32(0.4), 128.0, 0)
        assert compare_out(out.cpu().numpy(), ref.out, ref.gray, ref.t)["ok"], (C, offset)
        # bytes around the output are untouched
        assert int(obuf[:offset + 3].sum()) == 0 and int(obuf[offset + 3 + H * W:].sum()) == 0


@pytest.mark.parametrize("C", [1, 3])
def test_aligned_input_any_output_offset(bz, oracle_mod, C):
    """Input rows 16-byte aligned, output buffer at byte offsets 1..16: the
    aligned body needs 8-byte-aligned output rows and otherwise the general
    body runs; every offset gives the same bytes, matching the oracle, and
    the bytes around the output stay untouched."""
    from oracle.compare import compare_out
    import pagegen
    H, W = 150, 528  # W * C a multiple of 16
    img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=31 + C, channels=C)
    dimg = torch.from_numpy(img).cuda()
    assert dimg.data_ptr() % 16 == 0
    ref = oracle_mod.binarize(img, 31, f32(0.34), 128.0, 0)
    first = None
    for off in (16, 1, 2, 4, 8, 12):
        obuf = torch.zeros(H * W + 64, dtype=torch.uint8, device="cuda")
        out = obuf[off:off + H * W].view(H, W)
        bz.binarize(dimg, 31, f32(0.34), 128.0, 0, out=out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert compare_out(got, ref.out, ref.gray, ref.t)["ok"], (C, off)
        if first is None:
            first = got
        assert np.array_equal(got, first), (C, off)
        assert int(obuf[:off].sum()) == 0 and int(obuf[off + H * W:].sum()) == 0, (C, off)


@pytest.mark.parametrize("C,rule,win,k", [(1, 0, 15, 0.5), (1, 0, 31, 0.34), (1, 1, 31, -0.2), (1, 0, 61, 0.5),
                                          (3, 0, 31, 0.34), (3, 1, 15, -0.2), (1, 0, 101, 0.5)])
def test_interior_tiles_full_compare(bz, oracle_mod, C, rule, win, k):
    """A page large enough for interior tiles (whole windows, no clamping,
    16-byte aligned rows: the specialised tile body), compared pixel by pixel
    with the oracle; the same page one byte off alignment (general body only)
    gives identical bytes."""
    import pagegen
    from oracle.compare import compare_stats
    H, W = 700, 1104  # W * C is a multiple of 16
    img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=900 + win + C, channels=C)
    k = f32(k)
    ref = oracle_mod.binarize(img, win, k, 128.0, rule)
    g = gpu_stats(bz, img, win, k, 128.0, rule)
    rep = compare_stats(g, ref)
    assert rep["ok"], rep
    aligned = gpu_out(bz, img, win, k, 128.0, rule)
    assert np.array_equal(aligned, g["out"])
    buf = torch.zeros(img.size + 16, dtype=torch.uint8, device="cuda")
    shifted = buf[1:1 + img.size].view(*img.shape)
    shifted.copy_(torch.from_numpy(img))
    out = bz.binarize(shifted, win, k, 128.0, rule)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), aligned)


@pytest.mark.parametrize("C", [1, 3])
def test_every_row_end_overhang(bz, oracle_mod, C):
    """Widths 14..33: every position of the row's last column inside its
    16-pixel chunk (the chunk that reaches past the row end loads the row's
    last 16 pixels and shifts them; overhangs 1..15), the narrowest pages
    (below 16 pixels) and whole chunks; compared with the oracle pixel by
    pixel, and at a one-byte input and output offset byte for byte."""
    import pagegen
    H = 24
    for W in range(14, 34):
        img = pagegen.page(H, W, 1, seed=4000 + 10 * W + C, channels=C)
        for win, rule, k in ((15, 0, 0.5), (61, 0, 0.34), (31, 1, -0.2)):
            full_check(bz, oracle_mod, img, win, k, 128.0, rule, f"overhang {H}x{W}x{C} win {win}")
            base = gpu_out(bz, img, win, f32(k), 128.0, rule)
            ibuf = torch.zeros(img.size + 16, dtype=torch.uint8, device="cuda")
            shifted = ibuf[1:1 + img.size].view(*img.shape)
            shifted.copy_(torch.from_numpy(img))
            obuf = torch.zeros(H * W + 16, dtype=torch.uint8, device="cuda")
            out = obuf[1:1 + H * W].view(H, W)
            bz.binarize(shifted, win, f32(k), 128.0, rule, out=out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), base), (W, C, win)
            assert int(obuf[:1].sum()) == 0 and int(obuf[1 + H * W:].sum()) == 0


@pytest.mark.parametrize("H,W,win", [(33, 16, 15), (40, 16, 101), (70, 48, 61), (129, 272, 31),
                                     (40, 272, 255), (60, 528, 101), (64, 1040, 15)])
def test_aligned_pages_outside_chunks(bz, oracle_mod, H, W, win):
    """Pages whose rows are 16-byte aligned take the aligned-staging body on
    every tile, including tiles whose staged columns reach whole 16-pixel
    chunks past the left or right edge (staged as zeros) and pages narrower
    than one tile: compared with the oracle pixel by pixel, and with the same
    page one byte off alignment (general body), byte for byte."""
    import pagegen
    assert W % 16 == 0 and oracle_cost(H, W, win) < 6e8
    for C in (1, 3):
        img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=H + W + win + C, channels=C)
        for rule, k in ((0, 0.5), (1, -0.2)):
            full_check(bz, oracle_mod, img, win, k, 128.0, rule, f"aligned {H}x{W}x{C} win {win}")
            aligned = gpu_out(bz, img, win, f32(k), 128.0, rule)
            buf = torch.zeros(img.size + 16, dtype=torch.uint8, device="cuda")
            shifted = buf[1:1 + img.size].view(*img.shape)
            shifted.copy_(torch.from_numpy(img))
            out = bz.binarize(shifted, win, f32(k), 128.0, rule)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), aligned), (H, W, C, win, rule)


# ------------------------------------------------------------ full size

def sample_points(H, W, win, n, seed):
    rng = np.random.default_rng(seed)
    ys = list(rng.integers(0, H, n))
    xs = list(rng.integers(0, W, n))
    # corners, borders and tile seams
    for y in (0, 1, win // 2, H - 1 - win // 2, H - 2, H - 1):
        for x in (0, 1, win // 2, 127, 128, 255, 256, 257, W - 1 - win // 2, W - 2, W - 1):
            if 0 <= y < H and 0 <= x < W:
                ys.append(y)
                xs.append(x)
    return np.array(ys, np.int32), np.array(xs, np.int32)


@pytest.fixture(scope="module")
def page4096():
    import pagegen
    return pagegen.config1()[0].img


@pytest.mark.parametrize("rule,win,k", [(0, 15, 0.5), (0, 31, 0.5), (0, 61, 0.5), (0, 101, 0.5),
                                        (1, 31, -0.2)])
def test_full_size_4096_full_page(bz, oracle_mod, page4096, rule, win, k):
    """The whole 4096 x 4096 page in the default launch configuration (the
    one the benchmark times) against the oracle at every pixel: gray, S1,
    S2 and n bit-identical, t within 1e-4, the output band-aware; the product
    entry point gives the stats run's bytes; corners, borders and tile seams
    are asserted again on their own."""
    from oracle.compare import as_u32, compare_out, compare_stats
    img = page4096
    k = f32(k)
    print(f"4096 full page: rule {rule} win {win}", flush=True)
    timg = torch.from_numpy(img).cuda()
    out = bz.binarize(timg, win, k, 128.0, rule).cpu().numpy()
    st = {n: v.cpu().numpy() for n, v in bz.binarize_stats(timg, win, k, 128.0, rule).items()}
    ref = oracle_mod.binarize(img, win, k, 128.0, rule)
    rep = compare_stats(st, ref)
    print("4096", rule, win, rep, flush=True)
    assert rep["ok"], rep
    assert compare_out(out, ref.out, ref.gray, ref.t)["ok"]
    assert np.array_equal(out, st["out"])
    ys, xs = sample_points(4096, 4096, win, 0, seed=win)
    assert np.array_equal(as_u32(st["s1"][ys, xs]), ref.s1[ys, xs])
    assert np.array_equal(as_u32(st["n"][ys, xs]), ref.n[ys, xs])
    assert compare_out(out[ys, xs], ref.out[ys, xs], ref.gray[ys, xs], ref.t[ys, xs])["ok"]


@pytest.mark.parametrize("H,W,win,rule,k", [(2048, 2051, 151, 0, 0.5), (4096, 2051, 101, 1, -0.2),
                                            (2304, 2048, 151, 0, -0.7), (4096, 3100, 61, 0, 1.0)])
def test_blocks_layout_pages(bz, oracle_mod, page4096, H, W, win, rule, k):
    """Gray pages with wide windows and more tiles than the win + 8-row ring
    runs at once take the three-block layout of the input rows (aligned and
    unaligned bodies: W = 2051 is not a multiple of 16).  Every pixel against
    the oracle; bit-identical to the ring layout (forced by one 4096-row tile
    per tile column: fewer tiles than the ring runs at once), to the batched
    launch (its blocks-layout kernel, 128-row tiles) and to a row-strided
    view."""
    from oracle.compare import compare_out
    k = f32(k)
    img = np.ascontiguousarray(page4096[:H, :W])
    print(f"blocks layout: {H}x{W} win {win} rule {rule} k {k}", flush=True)
    timg = torch.from_numpy(img).cuda()
    out = bz.binarize(timg, win, k, 128.0, rule)
    ring = bz.binarize(timg, win, k, 128.0, rule, tile=(256, 4096))
    batched = torch.empty_like(out)
    bz.batch([(timg, batched, win, k, 128.0, rule)])
    torch.cuda.synchronize()
    # the same page as a row-strided view of the whole 4096-wide page
    full = torch.from_numpy(page4096).cuda()
    strided = bz.binarize(full[:H, :W], win, k, 128.0, rule)
    torch.cuda.synchronize()
    out, ring, batched, strided = (t.cpu().numpy() for t in (out, ring, batched, strided))
    assert np.array_equal(out, ring)
    assert np.array_equal(out, batched)
    assert np.array_equal(out, strided)
    ref = oracle_mod.binarize(img, win, k, 128.0, rule)
    rep = compare_out(out, ref.out, ref.gray, ref.t)
    print("blocks", H, W, win, rep, flush=True)
    assert rep["ok"], rep


def test_rgb_a4_page_full(bz, oracle_mod):
    """One A4 RGB page of the batch workload (3508 x 2480, win 31, k 0.34),
    every pixel against the oracle."""
    import pagegen
    from oracle.compare import compare_out
    job = pagegen.config2(n_pages=1)[0]
    k = f32(job.k)
    out = bz.binarize(torch.from_numpy(job.img).cuda(), job.win, k, 128.0, 0).cpu().numpy()
    ref = oracle_mod.binarize(job.img, job.win, k, 128.0, 0)
    rep = compare_out(out, ref.out, ref.gray, ref.t)
    print("a4 rgb", rep, flush=True)
    assert rep["ok"], rep


# ------------------------------------------------------------ errors

def test_errors_raise(bz):
    img = torch.zeros((32, 32), dtype=torch.uint8, device="cuda")
    with pytest.raises(bz.BinarizeError):
        bz.binarize(img, 0, 0.5)
    with pytest.raises(bz.BinarizeError):
        bz.binarize(img, 15, 0.5, R=-1.0)
    with pytest.raises(bz.BinarizeError):
        bz.binarize(img, 15, 0.5, tile=(64, 64))
    big = torch.zeros(64 * 64, dtype=torch.uint8, device="cuda")
    with pytest.raises(bz.BinarizeError):
        bz.binarize(big[:1024].view(32, 32), 15, 0.5, out=big[512:1536].view(32, 32))


def test_repeated_runs_deterministic(bz):
    import pagegen
    img = torch.from_numpy(pagegen.page(512, 512, 500, seed=9)).cuda()
    first = bz.binarize(img, 61, 0.5).clone()
    for _ in range(5):
        assert torch.equal(bz.binarize(img, 61, 0.5), first)
