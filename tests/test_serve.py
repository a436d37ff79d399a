"""Serving loop: the scheduler on a simulated device (CPU: admission,
continuous batching, out-of-order completion, timeouts, cancellation, the
completion watchdog, the pool's cap) and real mixes on the GPU whose every
result equals the page binarized alone and agrees with the oracle at sampled
pixels."""
import math

import numpy as np
import pytest

from paper_1210_3165_amd.serve import FakeExecutor, Request, Server, SimClock


def reqs(specs):
    return [Request(i, t, H, W, C, win) for i, (t, H, W, C, win) in enumerate(specs)]


def test_every_request_completes_once_and_latency_is_consistent():
    rng = np.random.default_rng(0)
    specs = [(float(t), int(rng.integers(100, 2000)), int(rng.integers(100, 2000)), int(rng.choice([1, 3])), 31)
             for t in np.cumsum(rng.exponential(1e-3, 500))]
    rs = reqs(specs)
    st = Server(FakeExecutor(slots=4, rate_px_s=5e9), hbm_budget=1 << 30).run(rs, SimClock())
    assert len(st.completed) == 500 and not st.refused
    assert sorted(r.rid for r in st.completed) == list(range(500))
    for r in st.completed:
        assert r.arrival <= r.admitted <= r.dispatched <= r.done
    s = st.summary()
    assert 0 < s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]


def test_admission_respects_the_footprint_budget_and_refuses_oversize():
    budget = 40_000_000
    big = Request(0, 0.0, 5000, 5000, 3, 15)          # 100 MB > budget: refused
    rs = [big] + [Request(i, 0.0, 2000, 2000, 1, 15) for i in range(1, 30)]  # 8 MB each
    st = Server(FakeExecutor(slots=8, rate_px_s=1e8), hbm_budget=budget).run(rs, SimClock())
    assert [r.rid for r in st.refused] == [0]
    assert len(st.completed) == 29
    assert st.max_admitted_bytes <= budget
    # at most 5 requests (40 MB) fit at once: some had to wait for admission
    assert any(r.admitted > r.arrival for r in st.completed)


def test_slot_exhaustion_forms_bigger_batches():
    """One slot and a burst: the first batch holds the first arrival, every
    request that arrives meanwhile joins the next batch (continuous batching)."""
    rs = [Request(i, i * 1e-5, 1000, 1000, 1, 15) for i in range(40)]
    ex = FakeExecutor(slots=1, rate_px_s=1e9)  # 1 ms per page
    st = Server(ex, hbm_budget=1 << 30, max_batch_pages=64).run(rs, SimClock())
    assert len(st.completed) == 40
    assert st.batches < 10 and max(st.batch_sizes) > 10
    slots_busy = [s for s, _, _ in ex.submitted]
    assert set(slots_busy) == {0}


def test_out_of_order_completion():
    """Later batches finishing first must not confuse the bookkeeping."""
    order = {0: 50.0, 1: 1.0, 2: 0.2, 3: 1.0}
    rs = [Request(i, i * 1e-4, 500, 500, 1, 15) for i in range(60)]
    ex = FakeExecutor(slots=4, rate_px_s=1e9, jitter=lambda n: order.get(n % 4, 1.0))
    st = Server(ex, hbm_budget=1 << 30, max_batch_pages=4).run(rs, SimClock())
    assert sorted(r.rid for r in st.completed) == list(range(60))
    done_order = [r.rid for r in st.completed]
    assert done_order != sorted(done_order)  # completions really were reordered
    for r in st.completed:
        assert r.done >= r.dispatched


def test_timeouts_drop_waiting_requests_and_free_their_footprint():
    """One slot, 1 ms per page, 30 simultaneous arrivals with a 5 ms timeout:
    the first few are dispatched in time, the rest time out while queued;
    nothing dispatched is dropped and the footprint returns to zero."""
    rs = [Request(i, 0.0, 1000, 1000, 1, 15, timeout=5e-3) for i in range(30)]
    ex = FakeExecutor(slots=1, rate_px_s=1e9, latency_s=0.0)
    st = Server(ex, hbm_budget=1 << 30, max_batch_pages=2).run(rs, SimClock())
    assert len(st.completed) + len(st.timed_out) == 30
    assert 0 < len(st.completed) < 30 and st.timed_out
    for r in st.completed:
        assert r.status == "done" and r.dispatched <= r.arrival + r.timeout
    for r in st.timed_out:
        assert r.status == "timed_out" and r.done > r.arrival + r.timeout and math.isnan(r.dispatched)
    assert st.summary()["timed_out"] == len(st.timed_out)


def test_cancel_removes_queued_requests_only():
    """Requests cancelled while queued are dropped; a request already on the
    device still completes even when cancelled afterwards."""
    rs = [Request(i, 0.0, 1000, 1000, 1, 15) for i in range(20)]
    ex = FakeExecutor(slots=1, rate_px_s=1e9, latency_s=0.0)
    srv = Server(ex, hbm_budget=1 << 30, max_batch_pages=1)

    def on_done(r):
        if r.rid == 0:
            for q in (0, 5, 6, 7):  # 0 has finished already, 5..7 are still queued
                srv.cancel(q)

    st = srv.run(rs, SimClock(), on_done=on_done)
    assert sorted(r.rid for r in st.cancelled) == [5, 6, 7]
    assert sorted(r.rid for r in st.completed) == [i for i in range(20) if i not in (5, 6, 7)]


def test_watchdog_fails_a_stuck_batch_and_retires_its_slot():
    """The second batch never completes (simulated hang): after the watchdog
    interval its requests are failed, its slot is never used again, and every
    other request completes on the remaining slot."""
    rs = [Request(i, i * 1e-4, 500, 500, 1, 15) for i in range(40)]
    ex = FakeExecutor(slots=2, rate_px_s=1e9, jitter=lambda n: math.inf if n == 1 else 1.0)
    st = Server(ex, hbm_budget=1 << 30, max_batch_pages=4, watchdog_s=0.05).run(rs, SimClock())
    stuck = ex.submitted[1]
    assert sorted(r.rid for r in st.failed) == sorted(stuck[1])
    assert all(r.status == "failed" for r in st.failed)
    assert ex.abandoned == [stuck[0]]
    assert all(s != stuck[0] for s, _, t in ex.submitted[2:])
    assert len(st.completed) + len(st.failed) == 40


def test_all_slots_stuck_fails_the_rest():
    rs = [Request(i, i * 1e-3, 500, 500, 1, 15) for i in range(10)]
    ex = FakeExecutor(slots=1, rate_px_s=1e9, jitter=lambda n: math.inf)
    st = Server(ex, hbm_budget=1 << 30, max_batch_pages=2, watchdog_s=0.01).run(rs, SimClock())
    assert not st.completed and len(st.failed) == 10


def test_buffer_pool_stays_within_its_cap():
    """Idle pooled buffers are freed, largest first, when a new size class
    would push the pool past its cap (CPU tensors stand in for device ones)."""
    from paper_1210_3165_amd.serve import _BufferPool
    pool = _BufferPool("cpu", cap=3 << 20)
    a = pool.get(1 << 20)            # 1 MiB class
    b = pool.get((1 << 20) + 1)      # 2 MiB class
    assert pool.bytes == 3 << 20
    pool.put(a)
    pool.put(b)
    c = pool.get(3 << 19)            # 2 MiB class again: reused, nothing new
    assert c is b and pool.bytes == 3 << 20
    pool.put(c)
    d = pool.get(3 << 20)            # 4 MiB class: both idle buffers are freed first
    assert d.numel() == 4 << 20 and pool.bytes == 4 << 20


def _oracle_sample_check(oracle_mod, page, out, win, k, R, rule, seed, n=300):
    """The served result at n random pixels plus the corners, against the
    oracle at the same pixels (band-aware: mismatches only where
    |f - t_oracle| < 1e-4)."""
    from conftest import f32
    from oracle.compare import compare_out
    H, W = out.shape
    rng = np.random.default_rng(seed)
    ys = np.concatenate([rng.integers(0, H, n), [0, 0, H - 1, H - 1]]).astype(np.int32)
    xs = np.concatenate([rng.integers(0, W, n), [0, W - 1, 0, W - 1]]).astype(np.int32)
    ref = oracle_mod.binarize_points(page, win, f32(k), f32(R), rule, ys, xs)
    rep = compare_out(out[ys, xs], ref.out, ref.gray, ref.t)
    assert rep["ok"], rep


@pytest.mark.gpu
def test_gpu_served_mix_equals_pages_alone(oracle_mod):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import pagegen
    import paper_1210_3165_amd as bz
    from paper_1210_3165_amd.serve import GpuBatchExecutor, WallClock
    dev = torch.device("cuda:0")
    canv = pagegen.device_canvases(dev)
    rng = np.random.default_rng(3)
    stream = pagegen.config4_stream(2000.0, 0.05, seed=4)
    rs = []
    for i, (t, H, W, C, win, k) in enumerate(stream):
        H, W = min(H, 1500), min(W, 1500)  # keep the test light
        t = (i // 6) * 2e-3  # bursts of 6 simultaneous arrivals force mixed batches
        r = Request(i, t, H, W, C, win, k, rule=i % 2)
        r.img = pagegen.canvas_view(canv, H, W, C, rng)
        rs.append(r)
    assert len(rs) > 40
    ex = GpuBatchExecutor(slots=2, max_pages=16, min_persistent=2)  # every mix through the batch kernel
    clock = WallClock()
    ex.start(clock)
    outs = {}

    def keep(r):  # consume the result before its buffer is recycled
        outs[r.rid] = r.out.clone()
        torch.cuda.current_stream().synchronize()

    st = Server(ex, hbm_budget=256 << 20, max_batch_pages=16).run(rs, clock, on_done=keep)
    torch.cuda.synchronize()
    assert len(st.completed) == len(rs) and not st.refused
    assert max(st.batch_sizes) > 1  # requests really were served in mixes
    for r in rs:
        alone = bz.binarize(r.img, r.win, r.k, r.R, r.rule)
        assert torch.equal(alone, outs[r.rid]), r.rid
        _oracle_sample_check(oracle_mod, r.img.cpu().numpy(), outs[r.rid].cpu().numpy(), r.win, r.k, r.R,
                             r.rule, seed=r.rid)
    ex.close()


@pytest.mark.gpu
def test_gpu_host_payloads_equal_pages_alone(oracle_mod):
    """Host-origin requests (pinned host in, pinned host out) in bursty mixes:
    every result equals the page binarized alone on the device."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import pagegen
    import paper_1210_3165_amd as bz
    from paper_1210_3165_amd.serve import GpuHostBatchExecutor, WallClock
    canv = pagegen.pinned_canvases()
    rng = np.random.default_rng(5)
    rs = []
    for i, (t, H, W, C, win, k) in enumerate(pagegen.config4_stream(2000.0, 0.04, seed=6)):
        H, W = min(H, 1200), min(W, 1200)
        r = Request(i, (i // 5) * 2e-3, H, W, C, win, k, rule=i % 2)
        r.img = pagegen.canvas_view(canv, H, W, C, rng)
        assert r.img.is_pinned()
        rs.append(r)
    assert len(rs) > 30
    ex = GpuHostBatchExecutor(slots=3, max_pages=8, min_persistent=2)
    clock = WallClock()
    ex.start(clock)
    outs = {}

    def keep(r):
        assert r.out.device.type == "cpu"
        outs[r.rid] = r.out.clone()

    st = Server(ex, hbm_budget=256 << 20, max_batch_pages=8).run(rs, clock, on_done=keep)
    torch.cuda.synchronize()
    assert len(st.completed) == len(rs) and not st.refused
    assert max(st.batch_sizes) > 1
    for r in rs:
        alone = bz.binarize(r.img.cuda(), r.win, r.k, r.R, r.rule).cpu()
        assert torch.equal(alone, outs[r.rid]), r.rid
        _oracle_sample_check(oracle_mod, r.img.numpy(), outs[r.rid].numpy(), r.win, r.k, r.R, r.rule,
                             seed=1000 + r.rid)
    ex.close()
