"""The single-page entry points enqueue only kernel launches (no memsets, no
allocation, no host synchronisation), so a caller can capture them in a HIP
graph.  Each test captures once, then replays several times with new inputs
copied in between and eager work and synchronisations interleaved, and checks
every replay against the eager result of the same input."""
import numpy as np
import pytest

import pagegen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bz():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1210_3165_amd as m
    m.lib()
    return m


def pages(n, H, W, C=1):
    return [torch.from_numpy(pagegen.page(H, W, pagegen.strokes_for(H, W), seed=500 + i, channels=C)).cuda()
            for i in range(n)]


def replay_check(capture, eager, inputs, static_in):
    """capture(): enqueue the work on the current stream reading static_in;
    eager(x): the same work on x, returning tensors to compare."""
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    capture()  # eager warm-up (first-call attribute setup happens here)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        outs = capture()
    for x in inputs:
        static_in.copy_(x)
        g.replay()
        torch.cuda.synchronize()
        want = eager(x)
        torch.cuda.synchronize()
        got = outs if isinstance(outs, (list, tuple)) else [outs]
        for a, b in zip(got, want):
            assert torch.equal(a, b)
        _ = torch.zeros(1024, device="cuda").sum()  # unrelated eager work between replays


@pytest.mark.parametrize("C,win,rule,k", [(1, 15, 0, 0.5), (3, 61, 0, 0.34), (1, 31, 1, -0.2)])
def test_binarize_in_graph(bz, C, win, rule, k):
    xs = pages(3, 700, 1104, C)
    static_in = torch.empty_like(xs[0])
    static_out = torch.empty(xs[0].shape[:2], dtype=torch.uint8, device="cuda")
    replay_check(lambda: [bz.binarize(static_in, win, k, 128.0, rule, out=static_out)],
                 lambda x: [bz.binarize(x, win, k, 128.0, rule)], xs, static_in)


def test_otsu_in_graph(bz):
    xs = pages(3, 900, 1300)
    static_in = torch.empty_like(xs[0])
    static_out = torch.empty_like(xs[0])
    o = bz.Otsu(static_in.device)

    def capture():
        o.run(static_in, static_out)
        return [static_out, o.hist]

    def eager(x):
        e = bz.Otsu(x.device)
        out = e.run(x)
        return [out, e.hist.clone()]

    replay_check(capture, eager, xs, static_in)


def test_gs_and_fmeasure_in_graph(bz):
    H, W = 600, 800
    data = [pagegen.page(H, W, pagegen.strokes_for(H, W), seed=600 + i, return_mask=True) for i in range(3)]
    xs = [torch.from_numpy(d[0]).cuda() for d in data]
    gt = torch.from_numpy(data[0][1].astype(np.uint8)).cuda()
    static_in = torch.empty_like(xs[0])
    static_out = torch.empty_like(xs[0])
    counts = torch.empty(3, dtype=torch.int64, device="cuda")

    def capture():
        bz.binarize_gs(static_in, 31, 0.34, 128.0, "star", out=static_out)
        bz.fmeasure_counts(static_out, gt, counts=counts)
        return [static_out, counts]

    def eager(x):
        out = bz.binarize_gs(x, 31, 0.34, 128.0, "star")
        return [out, bz.fmeasure_counts(out, gt)]

    replay_check(capture, eager, xs, static_in)
