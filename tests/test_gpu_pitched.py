"""Row-pitched pages through the C ABI: crops and padded-row layouts of a
larger buffer (the M x N image matrix of Sec. 1 as a window into memory).

binarize_pitched, the one-call binarize_batch and a batch object's graph
replay are compared with the oracle on each crop (made contiguous on the
host), and the bytes of the output buffer outside the crop's rows -- between
rows included -- must stay untouched.
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
    m.lib()
    return m


def big_page(H, W, C, seed):
    import pagegen
    return pagegen.page(H, W, pagegen.strokes_for(H, W), seed=seed, channels=C)


# (y0, x0, h, w): aligned and odd offsets, ragged widths, one row, one column
CROPS = [(0, 0, 300, 512), (17, 33, 250, 301), (5, 16, 200, 256), (1, 3, 1, 777), (40, 901, 333, 1),
         (100, 480, 257, 528)]


@pytest.mark.parametrize("C", [1, 3])
def test_pitched_crops_against_oracle(bz, oracle_mod, C):
    from oracle.compare import compare_out
    H, W = 640, 1408  # W * C a multiple of 16: crops at x0 % 16 == 0 keep 16-byte aligned rows
    host = big_page(H, W, C, seed=60 + C)
    dev = torch.from_numpy(host).cuda()
    for (y0, x0, h, w) in CROPS:
        for rule, k, win in ((0, 0.5, 31), (1, -0.2, 15), (0, 0.34, 101)):
            print(f"crop {y0},{x0} {h}x{w} C {C} rule {rule} win {win}", flush=True)
            crop = dev[y0:y0 + h, x0:x0 + w]
            obuf = torch.zeros((h + 6, w + 40), dtype=torch.uint8, device="cuda")
            out = obuf[3:3 + h, 17:17 + w]
            bz.binarize(crop, win, f32(k), 128.0, rule, out=out)
            torch.cuda.synchronize()
            ref = oracle_mod.binarize(np.ascontiguousarray(host[y0:y0 + h, x0:x0 + w]), win, f32(k), 128.0, rule)
            got = out.cpu().numpy()
            rep = compare_out(got, ref.out, ref.gray, ref.t)
            assert rep["ok"], (y0, x0, h, w, rule, win, rep)
            mask = torch.ones_like(obuf, dtype=torch.bool)
            mask[3:3 + h, 17:17 + w] = False
            assert int(obuf[mask].sum()) == 0, "bytes outside the output rows were written"
            # contiguous copies give the same bytes as the strided views
            ref_dev = bz.binarize(crop.contiguous(), win, f32(k), 128.0, rule)
            assert torch.equal(ref_dev, out)


def test_interleaved_rows_one_buffer(bz, oracle_mod):
    """Input rows and output rows alternate inside one buffer (pitch 2 W):
    they share no byte, so the call is accepted and each output row lands
    between two input rows."""
    from oracle.compare import compare_out
    H, W = 300, 500
    host = big_page(H, W, 1, seed=3)
    buf = torch.zeros((H, 2 * W), dtype=torch.uint8, device="cuda")
    buf[:, :W].copy_(torch.from_numpy(host))
    img, out = buf[:, :W], buf[:, W:]
    bz.binarize(img, 25, f32(0.4), 128.0, 0, out=out)
    torch.cuda.synchronize()
    ref = oracle_mod.binarize(host, 25, f32(0.4), 128.0, 0)
    assert compare_out(out.cpu().numpy(), ref.out, ref.gray, ref.t)["ok"]
    assert np.array_equal(buf[:, :W].cpu().numpy(), host)  # input untouched


def test_pitched_output_overlapping_input_is_refused(bz):
    buf = torch.zeros((64, 128), dtype=torch.uint8, device="cuda")
    with pytest.raises(bz.BinarizeError):
        bz.binarize(buf[:, :64], 15, 0.5, out=buf[:, 32:96])


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_of_crops_equals_single_calls(bz, use_graph):
    """Crops of two big pages (gray and RGB) batched into one persistent
    launch, through the one-call binarize_batch and through a batch object
    (direct or graph replay), give each crop's single-call bytes."""
    pages = {1: torch.from_numpy(big_page(640, 1408, 1, seed=8)).cuda(),
             3: torch.from_numpy(big_page(480, 704, 3, seed=9)).cuda()}
    jobs, singles = [], []
    rng = np.random.default_rng(5)
    for i in range(24):
        C = 1 if i % 3 else 3
        src = pages[C]
        h = int(rng.integers(1, src.shape[0] // 2))
        w = int(rng.integers(1, src.shape[1] // 2))
        y0 = int(rng.integers(0, src.shape[0] - h))
        x0 = int(rng.integers(0, src.shape[1] - w))
        win = int(rng.choice([15, 31, 61, 101, 151]))
        k = f32(float(rng.uniform(0.2, 0.5)))
        crop = src[y0:y0 + h, x0:x0 + w]
        obuf = torch.zeros((h, w + 7), dtype=torch.uint8, device="cuda")
        jobs.append((crop, obuf[:, 3:3 + w], win, k, 128.0, 0))
        singles.append(bz.binarize(crop, win, k, 128.0, 0))
    bz.batch(jobs)
    torch.cuda.synchronize()
    for (crop, out, *_), ref in zip(jobs, singles):
        assert torch.equal(out, ref)
        out.zero_()
    with bz.Batch(max_pages=32) as b:
        b.run(jobs, use_graph=use_graph)
        torch.cuda.synchronize()
        for (crop, out, *_), ref in zip(jobs, singles):
            assert torch.equal(out, ref)


@pytest.mark.parametrize("pitch_in,pitch_out", [((1 << 28) - 16, (1 << 28) - 8), (1 << 28, 4096), (4096, 1 << 28)])
def test_pitches_near_the_aligned_body_limit(bz, oracle_mod, pitch_in, pitch_out):
    """Rows 2^28 - 16 bytes apart still take the aligned body, whose staging
    loads and output stores use 32-bit offsets from a step's first row (up to
    7 pitches plus a row); a pitch of 2^28 on either side takes the general
    body.  18 rows (two full 8-row blocks and a ragged one), against the
    oracle, with the bytes between output rows untouched."""
    from oracle.compare import compare_out
    H, W = 18, 272
    host = big_page(H, W, 1, seed=71)
    print(f"pitch_in {pitch_in} pitch_out {pitch_out}", flush=True)
    src = torch.zeros((H - 1) * pitch_in + W, dtype=torch.uint8, device="cuda")
    img = torch.as_strided(src, (H, W), (pitch_in, 1))
    img.copy_(torch.from_numpy(host).cuda())
    dst = torch.zeros((H - 1) * pitch_out + W, dtype=torch.uint8, device="cuda")
    out = torch.as_strided(dst, (H, W), (pitch_out, 1))
    for rule, k, win in ((0, 0.5, 15), (1, -0.2, 31)):
        dst.zero_()
        bz.binarize(img, win, f32(k), 128.0, rule, out=out)
        torch.cuda.synchronize()
        ref = oracle_mod.binarize(host, win, f32(k), 128.0, rule)
        rep = compare_out(out.cpu().numpy(), ref.out, ref.gray, ref.t)
        assert rep["ok"], (pitch_in, pitch_out, rule, win, rep)
        # nothing written between the output rows: the whole buffer sums to the rows' sum
        assert int(dst.sum(dtype=torch.int64)) == int(out.sum(dtype=torch.int64))
    del src, dst
    torch.cuda.empty_cache()
