"""GPU parity of the sampled-window variant (Sec. 2, Eq. 5) and of the
F-measure counts (Sec. 3) against the oracle, through the C ABI.

Bar: S1', S2', n' bit-identical; |t' - t'_oracle| <= 1e-4; output identical
except where |f - t'_oracle| < 1e-4; TP/FP/FN counts exact."""
import numpy as np
import pytest

import pagegen
from conftest import f32

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PLUS, X, STAR = 0, 1, 2


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()
    return m


def check(bz, oracle_mod, img, win, k, Rp, structure, label=""):
    from oracle.compare import T_TOL, as_u32, compare_out
    k, Rp = f32(k), f32(Rp)
    ref = oracle_mod.binarize_gs(img, win, k, Rp, structure)
    f = oracle_mod.gray(img)
    t_img = torch.from_numpy(np.ascontiguousarray(img)).cuda()
    g = bz.binarize_gs(t_img, win, k, Rp, structure, stats=True)
    out_only = bz.binarize_gs(t_img, win, k, Rp, structure)
    torch.cuda.synchronize()
    g = {name: v.cpu().numpy() for name, v in g.items()}
    assert np.array_equal(as_u32(g["s1"]), ref.s1), label
    assert np.array_equal(as_u32(g["s2"]), ref.s2), label
    assert np.array_equal(as_u32(g["n"]), ref.n), label
    terr = float(np.abs(g["t"].astype(np.float64) - ref.t).max())
    assert terr <= T_TOL, (label, terr)
    rep = compare_out(g["out"], ref.out, f, ref.t)
    assert rep["ok"], (label, rep)
    assert np.array_equal(out_only.cpu().numpy(), g["out"]), label
    return rep


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
@pytest.mark.parametrize("C", [1, 3])
@pytest.mark.parametrize("win", [1, 3, 15, 31])
def test_gs_pages(bz, oracle_mod, structure, C, win):
    img = pagegen.page(200, 300, 150, seed=win * 7 + C + 10 * structure, channels=C)
    check(bz, oracle_mod, img, win, 0.34, 128.0, structure, f"s{structure} C{C} w{win}")


@pytest.mark.parametrize("structure", [PLUS, X, STAR])
@pytest.mark.parametrize("win", [101, 255])
def test_gs_wide_windows(bz, oracle_mod, structure, win):
    img = pagegen.page(300, 410, 250, seed=win + structure)
    check(bz, oracle_mod, img, win, 0.5, 128.0, structure, f"s{structure} w{win}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (150, 1), (5, 5), (33, 129), (31, 127)])
@pytest.mark.parametrize("structure", [PLUS, X, STAR])
def test_gs_small_and_ragged(bz, oracle_mod, shape, structure):
    H, W = shape
    img = pagegen.page(H, W, max(1, H * W // 200), seed=H * 1000 + W)
    check(bz, oracle_mod, img, 31, 0.2, 128.0, structure, f"{shape} s{structure}")


@pytest.mark.parametrize("k,Rp", [(0.0, 128.0), (-0.2, 128.0), (0.5, 64.0), (0.9, 200.0)])
def test_gs_parameters(bz, oracle_mod, k, Rp):
    img = pagegen.page(128, 256, 100, seed=77)
    for structure in (PLUS, X, STAR):
        check(bz, oracle_mod, img, 15, k, Rp, structure, f"k{k} R{Rp} s{structure}")


def test_gs_constant_page(bz, oracle_mod):
    img = np.full((64, 130), 90, np.uint8)
    for structure in (PLUS, X, STAR):
        check(bz, oracle_mod, img, 9, 0.5, 128.0, structure)


@pytest.mark.parametrize("offset", [1, 2, 3, 5, 13])
def test_gs_unaligned_input(bz, oracle_mod, offset):
    """Input at odd byte offsets and widths that are not a multiple of 4:
    the staging fetches 16-pixel chunks with word loads clamped to each row,
    so every alignment of the rows against the words must give the same
    sums as the oracle."""
    from oracle.compare import as_u32, compare_out
    for C, (H, W) in ((1, (70, 301)), (3, (45, 203))):
        img = pagegen.page(H, W, 60, seed=offset * 10 + C, channels=C)
        buf = torch.zeros(img.size + 32, dtype=torch.uint8, device="cuda")
        view = buf[offset:offset + img.size].view(*img.shape)
        view.copy_(torch.from_numpy(img))
        for structure in (PLUS, X, STAR):
            ref = oracle_mod.binarize_gs(img, 15, f32(0.34), f32(128.0), structure)
            g = bz.binarize_gs(view, 15, f32(0.34), f32(128.0), structure, stats=True)
            torch.cuda.synchronize()
            assert np.array_equal(as_u32(g["s1"].cpu().numpy()), ref.s1), (offset, C, structure)
            assert np.array_equal(as_u32(g["s2"].cpu().numpy()), ref.s2), (offset, C, structure)
            rep = compare_out(g["out"].cpu().numpy(), ref.out, oracle_mod.gray(img), ref.t)
            assert rep["ok"], (offset, C, structure, rep)


@pytest.mark.slow
@pytest.mark.parametrize("H,W,C,structure", [(4096, 4096, 1, STAR), (3508, 2480, 3, PLUS)])
def test_gs_full_size(bz, oracle_mod, H, W, C, structure):
    img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=H + C, channels=C)
    check(bz, oracle_mod, img, 31, 0.34, 128.0, structure, f"{H}x{W}x{C}")


@pytest.mark.parametrize("n,off_out,off_gt", [(1, 0, 0), (17, 0, 0), (1000, 1, 0), (4096 * 33 + 5, 0, 3),
                                              (1 << 20, 0, 0)])
def test_fmeasure_counts(bz, oracle_mod, n, off_out, off_gt):
    rng = np.random.default_rng(n)
    out = np.where(rng.random(n) < 0.3, 0, 255).astype(np.uint8)
    gt = (rng.random(n) < 0.25).astype(np.uint8) * rng.integers(1, 256, n).astype(np.uint8)
    ref = oracle_mod.fmeasure_counts(out, gt)
    dev = torch.device("cuda", 0)
    ob = torch.empty(n + off_out, dtype=torch.uint8, device=dev)
    gb = torch.empty(n + off_gt, dtype=torch.uint8, device=dev)
    ob[off_out:].copy_(torch.from_numpy(out))
    gb[off_gt:].copy_(torch.from_numpy(gt))
    c = bz.fmeasure_counts(ob[off_out:], gb[off_gt:])
    torch.cuda.synchronize()
    assert tuple(int(v) for v in c.cpu()) == ref


def test_fmeasure_of_a_binarized_page(bz, oracle_mod):
    """End to end: a page with its stroke mask, binarized on the GPU, counted
    on the GPU; counts equal the oracle's on the oracle's own output up to
    the pixels in the tie band."""
    img, mask = pagegen.page(512, 512, 600, seed=5, return_mask=True)
    t_img = torch.from_numpy(img).cuda()
    out = bz.binarize(t_img, 31, 0.34, 128.0)
    c = bz.fmeasure_counts(out, torch.from_numpy(mask.astype(np.uint8)).cuda())
    torch.cuda.synchronize()
    got = tuple(int(v) for v in c.cpu())
    assert got == oracle_mod.fmeasure_counts(out.cpu().numpy(), mask)
    ref = oracle_mod.binarize(img, 31, f32(0.34), 128.0)
    band = int((np.abs(ref.gray - ref.t) < 1e-4).sum())
    want = oracle_mod.fmeasure_counts(ref.out, mask)
    assert sum(abs(a - b) for a, b in zip(got, want)) <= 2 * band
    assert oracle_mod.fmeasure(*got) > 0.5
