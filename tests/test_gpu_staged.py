"""The staged (unfused) path: row window sums through two HBM planes, then
the column pass and the decision.  Its output must equal the fused tile
kernel's byte for byte (same exact sums, same choice of decision form), and
therefore match the oracle to the same bar."""
import numpy as np
import pytest

import pagegen
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


def both(bz, img, win, k, rule, R=128.0):
    t = torch.from_numpy(np.ascontiguousarray(img)).cuda() if isinstance(img, np.ndarray) else img
    fused = bz.binarize(t, win, f32(k), R, rule)
    staged = bz.binarize_staged(t, win, f32(k), R, rule)
    torch.cuda.synchronize()
    return fused, staged


@pytest.mark.parametrize("C", [1, 3])
@pytest.mark.parametrize("rule,k", [(0, 0.5), (1, -0.2)])
def test_staged_equals_fused_full_page(bz, C, rule, k):
    img = torch.from_numpy(pagegen.page(4096, 4096, pagegen.strokes_for(4096, 4096), seed=70 + C,
                                        channels=C)).cuda()
    for win in (15, 31, 61, 101):
        fused, staged = both(bz, img, win, k, rule)
        assert torch.equal(fused, staged), (C, rule, win, int((fused != staged).sum()))


@pytest.mark.parametrize("H,W", [(1, 1), (1, 300), (300, 1), (7, 5), (33, 257), (130, 529), (700, 1104)])
@pytest.mark.parametrize("win", [1, 2, 15, 64, 101, 255])
def test_staged_equals_fused_shapes(bz, H, W, win):
    rng = np.random.default_rng(H * 7 + W + win)
    for C in (1, 3):
        img = pagegen.page(H, W, max(1, pagegen.strokes_for(H, W)), seed=int(rng.integers(1 << 30)),
                           channels=C)
        for rule, k in ((0, 0.5), (0, 0.0), (0, -0.3), (1, -0.2)):
            fused, staged = both(bz, img, win, k, rule)
            assert torch.equal(fused, staged), (H, W, C, win, rule, k)


def test_staged_matches_oracle(bz, oracle_mod):
    from oracle.compare import compare_out
    for C, (H, W) in ((1, (96, 333)), (3, (70, 200))):
        img = pagegen.page(H, W, pagegen.strokes_for(H, W), seed=5 + C, channels=C)
        for win, rule, k in ((15, 0, 0.5), (31, 1, -0.2), (61, 0, 0.34)):
            ref = oracle_mod.binarize(img, win, f32(k), 128.0, rule)
            out = bz.binarize_staged(torch.from_numpy(img).cuda(), win, f32(k), 128.0, rule)
            torch.cuda.synchronize()
            assert compare_out(out.cpu().numpy(), ref.out, ref.gray, ref.t)["ok"], (C, win, rule)


def test_staged_unaligned_input_and_reused_workspace(bz):
    ws = torch.empty(8 * 300 * 520, dtype=torch.uint8, device="cuda")
    for off, (H, W) in ((1, (97, 301)), (3, (300, 520)), (0, (20, 33))):
        img = pagegen.page(H, W, 50, seed=off + H)
        buf = torch.zeros(img.size + 16, dtype=torch.uint8, device="cuda")
        view = buf[off:off + img.size].view(H, W)
        view.copy_(torch.from_numpy(img))
        fused = bz.binarize(view, 25, 0.4, 128.0, 0)
        staged = bz.binarize_staged(view, 25, 0.4, 128.0, 0, workspace=ws)
        torch.cuda.synchronize()
        assert torch.equal(fused, staged), (off, H, W)


def test_staged_workspace_too_small_raises(bz):
    img = torch.zeros((64, 64), dtype=torch.uint8, device="cuda")
    with pytest.raises(bz.BinarizeError):
        bz.binarize_staged(img, 15, 0.5, 128.0, 0, workspace=torch.empty(100, dtype=torch.uint8, device="cuda"))
