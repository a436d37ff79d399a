"""Benchmark of exact Sauvola / Niblack binarization on one MI355X.

Default workload: the 4096 x 4096 gray synthetic page, binarized with Sauvola
(k 0.5, R 128) at windows 15, 31, 61 and 101 and with Niblack (k -0.2) at
window 31.  One step = those five binarizations, each on its own input/output
buffer pair from a rotating pool larger than the 256 MB Infinity Cache, so the
bytes come from HBM.  Inputs are resident in HBM before timing starts.

Prints ONE JSON line (rank 0):
  value      Gpixel/s over the timed steps (pixels binarized / time), the
             launches of each window taken in turn by --streams streams (the
             pages are independent, so one launch's last tiles overlap the
             next one's first)
  value_one_stream  the same K steps with every launch on one stream
  hbm_frac   the timed steps' algorithmic bytes (2 per pixel) per second
             against the 8 TB/s MI355X peak
  roofline   achieved algorithmic HBM GB/s of the dominant kernel (Sauvola,
             gray, 256-column tiles: 2 bytes per pixel) from HIP events
             around each window's run of back-to-back launches on one stream
             (the kernel's own duration), against the 8 TB/s MI355X peak
  cpu_baseline  the CPU oracle timed on this host on a bounded pixel sample

    python bench.py [--steps K] [--warmup W] [--streams S] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpixel/s + % HBM peak, Sauvola W=15–101; served p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
CASES = [  # (rule, win, k) of the 4096^2 workload
    (0, 15, 0.5), (0, 31, 0.5), (0, 61, 0.5), (0, 101, 0.5), (1, 31, -0.2),
]
RULE_NAME = {0: "sauvola", 1: "niblack"}
# Tiles of the three-stream pass, by window.  The library's default sizes a
# launch to fill the GPU alone in one round of 64-row tiles; with launches
# overlapping on several streams that balance matters less and taller tiles
# spend fewer rows on each tile's window start-up.  At win 101 a 128-row tile
# count no longer exceeds what the ring layout runs at once, so the page
# falls back to the ring at two workgroups per CU: 96 rows keep the blocks
# layout there.  Every tile shape gives the same bytes.
STREAM_TILES = {15: (256, 128), 31: (256, 128), 61: (256, 128), 101: (256, 96)}
DOMINANT = "bz_page_kernel<256, gray, sauvola>"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_bz_page_kernel_sauvola_gray_4096.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_bz_page_kernel_sauvola_gray_4096.json")
# one VALU wave instruction per quad-cycle: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_PEAK_LANE_OPS = 256 * 4 * 16 * 2.4e9


from paper_1210_3165_amd.build import kernel_source_sha  # noqa: E402


def _current_record(path):
    """A committed counter record, if it was taken on the current kernel
    source; else None."""
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    return rec if rec.get("source_sha") == kernel_source_sha() else None


def measured_traffic():
    """HBM bytes per launch from committed rocprofv3 counter runs."""
    rec = _current_record(TRAFFIC_FILE)
    return rec.get("bytes_per_launch") if rec else None


def measured_valu(pixels: int, avg_launch_ms: float):
    """VALU lane instructions per pixel from a committed SQ counter run, and
    the issue rate they imply at the measured launch time, against one VALU
    wave instruction per quad-cycle on every SIMD."""
    rec = _current_record(VALU_FILE)
    if not rec or not rec.get("valu_lane_ops_per_px"):
        return None
    ops = float(rec["valu_lane_ops_per_px"])
    rate = ops * pixels / (avg_launch_ms * 1e-3)
    return {"lane_ops_per_px": ops, "achieved_T_lane_ops_s": rate / 1e12,
            "peak_T_lane_ops_s": VALU_PEAK_LANE_OPS / 1e12, "frac": rate / VALU_PEAK_LANE_OPS}


def _f32(x: float) -> float:
    return float(np.float32(x))


def run_cpu_baseline(img: np.ndarray, budget_s: float) -> dict:
    """The oracle (unchanged, all host threads) on a random pixel sample of
    the same five cases, scaled to Gpixel/s."""
    import oracle
    oracle.build(force=False)
    H, W = img.shape[:2]
    rng = np.random.default_rng(12345)
    def timed(n):
        ys = rng.integers(0, H, n).astype(np.int32)
        xs = rng.integers(0, W, n).astype(np.int32)
        t0 = time.perf_counter()
        for rule, win, k in CASES:
            oracle.binarize_points(img, win, _f32(k), 128.0, rule, ys, xs)
        return time.perf_counter() - t0

    # grow a probe sample until it takes a measurable time, then size the
    # final sample to the budget
    n = 256
    while n < 16_000_000:
        dt = timed(n)
        if dt > 0.1 * budget_s:
            break
        n *= 4
    n = int(min(16_000_000, max(256, n * budget_s / max(dt, 1e-6))))
    ys = rng.integers(0, H, n).astype(np.int32)
    xs = rng.integers(0, W, n).astype(np.int32)
    t0 = time.perf_counter()
    for rule, win, k in CASES:
        oracle.binarize_points(img, win, _f32(k), 128.0, rule, ys, xs)
    dt = time.perf_counter() - t0
    px = n * len(CASES)
    return {
        "value": px / dt / 1e9,
        "unit": "Gpixel/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{n} random pixels of the 4096x4096 page for each of the 5 cases "
                  f"({px} window evaluations, {dt:.1f} s); direct window loop, fp64",
    }


def batch_jobs(name: str, dev):
    """Device-resident pages of the batched workloads.

    batch-rgb:   64 RGB A4 pages (3508 x 2480), Sauvola win 31, k 0.34, R 128;
                 4 distinct generated pages, each placed in 16 buffers.
    batch-mixed: 512 gray pages, H, W ~ U{300..4000}, win from
                 {15, 31, 61, 101, 151}, k ~ U[0.2, 0.5], R 128; page contents
                 are crops of one generated 4000 x 4000 page.
    """
    import torch

    import pagegen
    jobs = []
    if name == "batch-rgb":
        pages = pagegen.config2(n_pages=4)
        for i in range(64):
            p = pages[i % 4]
            img = torch.from_numpy(p.img).to(dev)
            jobs.append((img, torch.empty(p.img.shape[:2], dtype=torch.uint8, device=dev), p.win,
                         _f32(p.k), 128.0, 0))
    elif name == "batch-mixed":
        big = pagegen.page(4000, 4000, pagegen.strokes_for(4000, 4000), seed=3000)
        rng = np.random.default_rng(7)
        for (H, W, win, k) in pagegen.config3_specs(512):
            y0 = int(rng.integers(0, 4001 - H))
            x0 = int(rng.integers(0, 4001 - W))
            img = torch.from_numpy(np.ascontiguousarray(big[y0:y0 + H, x0:x0 + W])).to(dev)
            jobs.append((img, torch.empty((H, W), dtype=torch.uint8, device=dev), win, k, 128.0, 0))
    else:
        raise ValueError(name)
    return jobs


def run_batch_workload(name: str, reps: int, lds_cap: int = 0, tile_h: int = 0) -> dict:
    """Per-image launches vs the batched launch (direct and graph replay)
    on the same device-resident pages; outputs checked identical."""
    import torch

    import paper_1210_3165_amd as bz
    dev = torch.device("cuda:0")
    jobs = batch_jobs(name, dev)
    px = sum(j[1].numel() for j in jobs)
    stream = torch.cuda.current_stream(dev)

    def timed(fn):
        # back-to-back calls: each call's host work (marshalling and
        # planning the pages) overlaps the GPU's work on the previous one;
        # only the first call's host work falls inside the timed span
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def per_image():
        for img, out, win, k, R, rule in jobs:
            bz.binarize(img, win, k, R, rule, out=out)

    ms_single = timed(per_image)
    ref = [j[1].clone() for j in jobs]
    res = {"workload": name, "pages": len(jobs), "pixels": px,
           "per_image": {"ms": ms_single, "gpix_s": px / ms_single / 1e6}}
    tuned = None
    if lds_cap < 0:  # autotune cap and tile height for these shapes
        from paper_1210_3165_amd.autotune import Tuner
        specs = [(j[1].shape[0], j[1].shape[1], 1 if j[0].dim() == 2 else 3, j[2]) for j in jobs]
        tuned = Tuner().batch_config(specs)
        lds_cap, tile_h = tuned["lds_cap"], tuned["tile_h"]
    if tile_h:
        jobs = [j[:6] + ((0, tile_h),) for j in jobs]
    with bz.Batch(len(jobs), lds_cap=lds_cap) as B:
        for mode, graph in (("batch_direct", False), ("batch_graph", True)):
            ms = timed(lambda: B.run(jobs, use_graph=graph))
            same = all(torch.equal(r, j[1]) for r, j in zip(ref, jobs))
            res[mode] = {"ms": ms, "gpix_s": px / ms / 1e6, "identical_to_per_image": same}
        res["batch_grid"] = B.info()["grid"]
        res["lds_cap"] = B.info()["lds_cap"]
        res["batch_tile_h"] = tile_h or 128
        res["autotuned"] = tuned is not None
    return res


def run_serve_workload(rates, duration: float, slots: int, max_pages: int, payload: str = "device",
                       sizes: str = "config4", warm: bool = True) -> dict:
    """Poisson request streams served on the same inputs in several modes:
    device-resident payloads with continuous batching (persistent batched
    launches on `slots` streams) and in the plain form (one launch per
    request); host-origin payloads (pinned host in and out, copies on the
    slots' streams) batched and one request per batch.  sizes: "config4"
    (the served mix: 0.1-16 Mpx, gray or RGB, odd win 15-151), "page4096"
    (every request a 4096^2 gray page, Sauvola win 31: tens of thousands of
    requests per second reach the GPU's capacity) or "page512" (512^2 gray
    pages, Sauvola win 31: per-request launch and host costs dominate)."""
    import torch

    import pagegen
    from paper_1210_3165_amd.serve import (GpuBatchExecutor, GpuHostBatchExecutor, GpuSingleExecutor,
                                           Request, Server, WallClock)
    dev = torch.device("cuda:0")
    canv = {"device": pagegen.device_canvases(dev)}
    if payload in ("host", "both"):
        canv["host"] = pagegen.pinned_canvases()
    free, _ = torch.cuda.mem_get_info(dev)
    budget = int(min(free * 0.5, 32 << 30))
    modes = {"device": ["batched", "single"], "host": ["host-batched", "host-single"],
             "both": ["batched", "single", "host-batched", "host-single"]}[payload]

    def stream(rate, seed):
        if sizes == "config4":
            return pagegen.config4_stream(rate, duration, seed)
        side = 4096 if sizes == "page4096" else 512
        rng = np.random.default_rng(seed)
        t, out = 0.0, []
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration or len(out) >= 10_000:
                return out
            out.append((t, side, side, 1, 31, 0.5))

    def requests(rate, seed, where):
        rng = np.random.default_rng(seed)
        out = []
        for i, (t, H, W, C, win, k) in enumerate(stream(rate, seed)):
            r = Request(i, t, H, W, C, win, k)
            r.img = pagegen.canvas_view(canv[where], H, W, C, rng)
            out.append(r)
        return out

    def serve(mode, reqs):
        if mode == "batched":
            ex, mp = GpuBatchExecutor(slots, max_pages, pool_cap=budget), max_pages
        elif mode == "single":
            ex, mp = GpuSingleExecutor(slots, pool_cap=budget), 1
        else:
            ex, mp = (GpuHostBatchExecutor(slots, max_pages, pool_cap=budget),
                      (max_pages if mode == "host-batched" else 1))
        clock = WallClock()
        ex.start(clock)
        st = Server(ex, budget, max_batch_pages=mp).run(reqs, clock)
        torch.cuda.synchronize()
        ex.close()
        s = st.summary()
        span = max(r.done for r in st.completed) - min(r.arrival for r in st.completed)
        s["payload_GBps"] = sum(r.footprint for r in st.completed) / span / 1e9 if span > 0 else 0.0
        return s

    if warm:
        for mode in modes:  # warm-up (kernels loaded, pools filled)
            serve(mode, requests(1000.0, 1, "host" if mode.startswith("host") else "device")[:100])
    res = {"workload": "serve", "sizes": sizes, "duration_s": duration, "slots": slots,
           "max_batch_pages": max_pages, "hbm_budget_GB": budget / 1e9, "payload": payload, "runs": []}
    for rate in rates:
        for mode in modes:
            s = serve(mode, requests(rate, 5000 + int(rate), "host" if mode.startswith("host") else "device"))
            res["runs"].append({"rate": rate, "mode": mode, **s})
    return res


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def run_oracle_single_thread_cfg0() -> dict:
    """The oracle on the 256^2 page (Sauvola win 15, k 0.5) with one OpenMP
    thread, in a child process (OMP_NUM_THREADS is read when the runtime
    starts)."""
    import subprocess
    code = ("import sys, time; sys.path.insert(0, %r)\n"
            "import oracle, pagegen\n"
            "oracle.build(force=False)\n"
            "job = pagegen.config0()[0]\n"
            "oracle.binarize(job.img, job.win, job.k, job.R, job.rule)\n"
            "t = []\n"
            "for _ in range(5):\n"
            "    t0 = time.perf_counter(); oracle.binarize(job.img, job.win, job.k, job.R, job.rule)\n"
            "    t.append(time.perf_counter() - t0)\n"
            "print(min(t), oracle.num_threads())\n") % ROOT
    env = dict(os.environ, OMP_NUM_THREADS="1")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=300)
    sec, threads = out.stdout.split()[-2:]
    return {"ms": float(sec) * 1e3, "threads": int(threads), "pixels": 256 * 256,
            "gpix_s": 256 * 256 / float(sec) / 1e9}


def run_latency_cfg0(reps: int = 50) -> dict:
    """Isolated single-launch latency on the 256^2 page (Sauvola win 15): each
    launch alone on an idle GPU, bracketed by events (device time) and by host
    time from the call to the end of its synchronisation."""
    import torch

    import pagegen
    import paper_1210_3165_amd as bz
    job = pagegen.config0()[0]
    img = torch.from_numpy(job.img).cuda()
    out = torch.empty_like(img)
    k = _f32(job.k)
    dev_us, host_us = [], []
    for _ in range(reps + 5):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        bz.binarize(img, job.win, k, job.R, job.rule, out=out)
        e1.record()
        e1.synchronize()
        host_us.append((time.perf_counter() - t0) * 1e6)
        dev_us.append(e0.elapsed_time(e1) * 1e3)
    dev_us, host_us = np.array(dev_us[5:]), np.array(host_us[5:])
    return {"page": "256x256 gray, Sauvola win 15", "reps": reps,
            "device_us_p50": float(np.percentile(dev_us, 50)), "device_us_p90": float(np.percentile(dev_us, 90)),
            "host_us_p50": float(np.percentile(host_us, 50)), "host_us_p90": float(np.percentile(host_us, 90))}


def run_copy_stream(dev, mib: int = 1024, reps: int = 5) -> float:
    """Achievable streaming bandwidth: one copy kernel over a buffer of `mib`
    MiB (read + write bytes per second), no per-buffer launches."""
    import torch
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device=dev)
    b = torch.empty(n, dtype=torch.uint8, device=dev)
    a.fill_(1)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    return gbps


def sample_sclk(step, min_samples: int = 2, seconds: float = 2.0, limit_s: float = 10.0, sync=None):
    """Shader clock under the bench's own load: `step` (steps of the five
    cases, launched as for `value`) runs back to back, untimed, while a
    helper thread reads the GFX clock of every XCD with `amd-smi metric
    --clock` (each reading takes a tool start-up, longer than the whole timed
    region, so the readings are taken over this run of the same steps right
    after it; the first comes after 0.3 s of load).
    None where the tool is missing or prints no GFX clocks.  `sync` waits
    for the launched steps (torch.cuda.synchronize by default)."""
    import re
    import shutil
    import subprocess
    import threading
    if sync is None:
        import torch
        sync = torch.cuda.synchronize
    exe = shutil.which("amd-smi")
    if not exe:
        return None
    readings, stop = [], threading.Event()

    def sampler():
        while not stop.is_set():
            try:
                r = subprocess.run([exe, "metric", "--clock"], capture_output=True, text=True, timeout=20)
            except (OSError, subprocess.SubprocessError):
                return
            clk = [int(v) for v in re.findall(r"GFX_\d+:\s*\n\s*CLK:\s*(\d+)\s*MHz", r.stdout)]
            if not clk:
                return
            readings.append(clk)

    th = threading.Thread(target=sampler, daemon=True)
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < 0.3:  # under load before the first reading
        for _ in range(20):
            step()
        sync()
    t0 = time.perf_counter()
    th.start()
    while th.is_alive() and time.perf_counter() - t0 < limit_s and \
            (len(readings) < min_samples or time.perf_counter() - t0 < seconds):
        for _ in range(20):
            step()
        sync()
    stop.set()
    t_stop = time.perf_counter()
    while th.is_alive() and time.perf_counter() - t_stop < 25:  # busy until the reading in flight ends
        for _ in range(20):
            step()
        sync()
    th.join(timeout=5)
    if not readings:
        return None
    flat = sorted(v for clk in readings for v in clk)
    return {"median": flat[len(flat) // 2], "p10": flat[len(flat) // 10], "p90": flat[(9 * len(flat)) // 10],
            "min": flat[0], "max": flat[-1], "share_below_2000": sum(v < 2000 for v in flat) / len(flat),
            "readings": len(readings),
            "xcds": len(readings[0]), "max_clk": 2400,
            "source": "amd-smi metric --clock (GFX clock of every XCD) during an untimed run of the "
                      "same steps right after the timed region"}


def compact_serve(res: dict) -> list:
    return [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
             if k in ("rate", "mode", "requests", "mean_batch", "p50_ms", "p99_ms", "gpix_s", "req_s")}
            for r in res["runs"]]


def compact_batch(res: dict) -> dict:
    out = {"pages": res["pages"], "pixels": res["pixels"]}
    for mode in ("per_image", "batch_direct", "batch_graph"):
        out[mode + "_gpix_s"] = round(res[mode]["gpix_s"], 2)
    out["identical"] = res["batch_direct"]["identical_to_per_image"] and res["batch_graph"]["identical_to_per_image"]
    return out


def run_otsu_workload(reps: int, pool_mb: int) -> dict:
    """Otsu's global threshold (histogram, selection, Eq. 2 decision) on the
    4096^2 gray page and on A4 RGB pages, from a rotating buffer pool."""
    import torch

    import pagegen
    import paper_1210_3165_amd as bz
    dev = torch.device("cuda:0")
    runs = []
    for (H, W, C) in [(4096, 4096, 1), (3508, 2480, 3)]:
        img = torch.from_numpy(pagegen.page(H, W, pagegen.strokes_for(H, W), seed=4000 + C,
                                            channels=C)).to(dev)
        n = max(2, math.ceil(pool_mb * 2**20 / (H * W * (C + 1))))
        ins = [img.clone() for _ in range(n)]
        outs = [torch.empty((H, W), dtype=torch.uint8, device=dev) for _ in range(n)]
        o = bz.Otsu(dev)
        for i in range(n):
            o.run(ins[i], outs[i])
        torch.cuda.synchronize()
        res = {"H": H, "W": W, "channels": C, "T": o.T}
        for mode in ("threshold+decision", "threshold only"):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for r in range(reps):
                o.run(ins[r % n], outs[r % n], threshold_only=(mode == "threshold only"))
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            nbytes = H * W * ((2 * C + 1) if mode == "threshold+decision" else C)
            res[mode] = {"us": ms * 1e3, "gpix_s": H * W / (ms * 1e-3) / 1e9,
                         "alg_GBps": nbytes / (ms * 1e-3) / 1e9,
                         "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
        runs.append(res)
    return {"workload": "otsu", "runs": runs}


def run_gs_workload(reps: int) -> dict:
    """Exact Sauvola against the sampled-window variant (plus, x, star) on the
    4096^2 gray page, per window: microseconds per launch from HIP events."""
    import torch

    import pagegen
    import paper_1210_3165_amd as bz
    dev = torch.device("cuda:0")
    S = 4096
    img = torch.from_numpy(pagegen.config1(size=S)[0].img).to(dev)
    out = torch.empty((S, S), dtype=torch.uint8, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    rows = []
    for win in (15, 31, 61, 101):
        row = {"win": win, "exact_us": timed(lambda: bz.binarize(img, win, 0.5, 128.0, out=out))}
        for name in ("plus", "x", "star"):
            row[f"{name}_us"] = timed(lambda: bz.binarize_gs(img, win, 0.5, 128.0, name, out=out))
        rows.append(row)
    return {"workload": "gs", "H": S, "W": S, "reps": reps, "runs": rows}


def run_fusion_workload(reps: int) -> dict:
    """Pass fusion on 4096^2 pages, gray and RGB: the fused tile kernel (one
    pass) against the staged form (row window sums to two u32 planes, then the
    column pass), Sauvola k=0.5 per window; microseconds per page from HIP
    events, and whether the two outputs are identical."""
    import torch

    import pagegen
    import paper_1210_3165_amd as bz
    dev = torch.device("cuda:0")
    S = 4096
    pages = {1: pagegen.config1(size=S)[0].img,
             3: pagegen.page(S, S, pagegen.strokes_for(S, S), seed=3000, channels=3)}
    ws = torch.empty(8 * S * S, dtype=torch.uint8, device=dev)
    o1 = torch.empty((S, S), dtype=torch.uint8, device=dev)
    o2 = torch.empty((S, S), dtype=torch.uint8, device=dev)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    rows = []
    for C, host in pages.items():
        img = torch.from_numpy(host).to(dev)
        for win in (15, 31, 61, 101):
            fused = timed(lambda: bz.binarize(img, win, 0.5, 128.0, out=o1))
            staged = timed(lambda: bz.binarize_staged(img, win, 0.5, 128.0, out=o2, workspace=ws))
            rows.append({"channels": C, "win": win, "fused_us": fused, "staged_us": staged,
                         "identical": bool(torch.equal(o1, o2))})
    return {"workload": "fusion", "H": S, "W": S, "reps": reps, "runs": rows}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--pool-mb", type=int, default=1024, help="rotating buffer pool size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="page4096: skip the batch, serve, latency and copy figures added to the line")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work")
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--streams", type=int, default=3,
                    help="page4096: streams the timed launches take in turn for `value` (the launch "
                         "stream and S - 1 more; 1: one stream)")
    ap.add_argument("--lds-cap", type=int, default=0,
                    help="batch: LDS bytes per workgroup (0: default, -1: autotune cap and tile height)")
    ap.add_argument("--batch-tile-h", type=int, default=0, help="batch: tile height (0: default)")
    ap.add_argument("--workload", default="page4096",
                    choices=["page4096", "batch-rgb", "batch-mixed", "serve", "otsu", "gs", "fusion"],
                    help="page4096: the metric line; batch-*: per-image vs persistent batch; "
                         "serve: continuous batching vs one launch per request; "
                         "otsu: the global-threshold baseline; gs: exact vs sampled window")
    ap.add_argument("--rates", default="200,1000,5000", help="serve: Poisson rates, req/s")
    ap.add_argument("--duration", type=float, default=2.0, help="serve: seconds per rate and mode")
    ap.add_argument("--slots", type=int, default=4, help="serve: concurrent batches (streams)")
    ap.add_argument("--max-batch", type=int, default=32, help="serve: pages per micro-batch")
    ap.add_argument("--payload", default="device", choices=["device", "host", "both"],
                    help="serve: device-resident inputs, pinned host inputs/outputs, or both")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the binarizer has no multi-GPU path "
              "(pages are independent and need no collective)", file=sys.stderr)
        return 2

    import torch

    import pagegen
    import paper_1210_3165_amd as bz

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    bz.lib()
    if args.workload == "serve":
        rates = [float(x) for x in args.rates.split(",")]
        print(json.dumps(run_serve_workload(rates, args.duration, args.slots, args.max_batch, args.payload)),
              flush=True)
        return 0
    if args.workload == "gs":
        print(json.dumps(run_gs_workload(max(5, args.steps // 20))), flush=True)
        return 0
    if args.workload == "fusion":
        print(json.dumps(run_fusion_workload(max(5, args.steps // 20))), flush=True)
        return 0
    if args.workload == "otsu":
        print(json.dumps(run_otsu_workload(max(10, args.steps), args.pool_mb)), flush=True)
        return 0
    if args.workload != "page4096":
        print(json.dumps(run_batch_workload(args.workload, max(12, args.steps // 20), args.lds_cap,
                                            args.batch_tile_h)), flush=True)
        return 0

    S = args.size
    page = pagegen.config1(size=S)[0].img
    px = S * S
    pair_bytes = 2 * px
    n_pairs = max(2, math.ceil(args.pool_mb * 2**20 / pair_bytes))
    src = torch.from_numpy(page).to(dev)
    ins = [src.clone() for _ in range(n_pairs)]
    outs = [torch.empty((S, S), dtype=torch.uint8, device=dev) for _ in range(n_pairs)]
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)
    idx = 0

    def launch(case, tile=None):
        nonlocal idx
        rule, win, k = case
        b = idx % n_pairs
        idx += 1
        bz.binarize(ins[b], win, k, 128.0, rule, out=outs[b], tile=tile)

    # the launch stream and S - 1 more, all at the default priority
    streams = [stream] + [torch.cuda.Stream(dev) for _ in range(max(0, args.streams - 1))]

    def run_overlapped(k_steps):
        """k_steps steps grouped by case, launch j of a case on streams[j % S]:
        the other streams start after an event on the launch stream, which
        waits for their last launches before the case's end event.  Tiles:
        STREAM_TILES on more than one stream, else the library's default."""
        evs = []
        for c in CASES:
            tile = STREAM_TILES[c[1]] if len(streams) > 1 else None
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for st in streams[1:]:
                st.wait_event(e0)
            for j in range(k_steps):
                st = streams[j % len(streams)]
                if st is stream:
                    launch(c, tile)
                else:
                    with torch.cuda.stream(st):
                        launch(c, tile)
            for st in streams[1:]:
                e = torch.cuda.Event()
                e.record(st)
                stream.wait_event(e)
            e1.record(stream)
            evs.append((e0, e1))
        return evs

    for _ in range(args.warmup):
        for c in CASES:
            launch(c)
    run_overlapped(args.warmup)
    torch.cuda.synchronize()

    # kernel durations (the roofline and value_one_stream): K steps, grouped
    # by case.  The K launches of one case run back to back on the launch
    # stream (each on the next buffer pair of the pool), bracketed by one
    # pair of HIP events: no event marker sits between two launches.  The
    # five cases follow each other on the same stream, so the first start and
    # the last end bracket all K steps.
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in CASES]
    torch.cuda.synchronize()
    for i, c in enumerate(CASES):
        ev[i][0].record(stream)
        for _ in range(args.steps):
            launch(c)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    total_ms_one = ev[0][0].elapsed_time(ev[-1][1])
    case_ms = [e0.elapsed_time(e1) / args.steps for e0, e1 in ev]

    # timed region of `value`: the same K steps, grouped by case, with the
    # launches of each case taken in turn by the streams; the first case's
    # start event and the last case's end event, both on the launch stream,
    # bracket all K steps
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    evo = run_overlapped(args.steps)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = evo[0][0].elapsed_time(evo[-1][1])
    case_ms_overlapped = [e0.elapsed_time(e1) / args.steps for e0, e1 in evo]

    cases = []
    for i, (rule, win, k) in enumerate(CASES):
        ms = case_ms[i]
        cases.append({"rule": RULE_NAME[rule], "win": win, "k": k, "ms": ms,
                      "gpix_s": px / (ms * 1e-3) / 1e9,
                      "hbm_frac": 2 * px / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                      "gpix_s_streams": px / (case_ms_overlapped[i] * 1e-3) / 1e9})
    # dominant kernel: the Sauvola gray launches (4 of the 5 per step)
    avg_ms = float(np.mean([case_ms[i] for i, c in enumerate(CASES) if c[0] == 0]))
    achieved = 2 * px / (avg_ms * 1e-3) / 1e9

    # achievable copy bandwidth over the same pool (plain copy kernel)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 4 * n_pairs
    e0.record(stream)
    for r in range(reps):
        outs[r % n_pairs].copy_(ins[(r + 1) % n_pairs])
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 2 * px * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    copy_stream_gbps = run_copy_stream(dev)

    traffic = measured_traffic()
    step_ms = total_ms / args.steps
    rec = {
        "metric": METRIC,
        "value": px * len(CASES) / (step_ms * 1e-3) / 1e9,
        "value_one_stream": px * len(CASES) / (total_ms_one / args.steps * 1e-3) / 1e9,
        # the whole timed job's algorithmic bytes (2 per pixel) over its time,
        # as a share of the HBM peak; roofline.frac is the same for one kernel
        # from its own launch duration
        "hbm_frac": 2 * px * len(CASES) / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "unit": "Gpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/f32",
        "data": "synthetic",
        "config": {
            "workload": f"{S}x{S} u8 gray synthetic page; one step = Sauvola k=0.5 R=128 at "
                        "win 15, 31, 61, 101 + Niblack k=-0.2 at win 31",
            "H": S, "W": S, "channels": 1,
            "tiles": {str(w): list(bz.default_tile(S, S, 1, w)) for _, w, _ in CASES},
            "pool_pairs": n_pairs,
            "streams": len(streams),
            "tiles_streams": ({str(w): list(STREAM_TILES[w]) for _, w, _ in CASES} if len(streams) > 1
                              else None),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "kernel": DOMINANT,
            "bytes_per_launch": 2 * px,
            "avg_launch_ms": avg_ms,
            "valu": measured_valu(px, avg_ms),
        },
        "cases": cases,
        "copy_GBps": copy_gbps,
        "copy_stream_GBps": copy_stream_gbps,
        "wall_s": t_wall,
    }
    # which roof limits the dominant kernel: the instruction-issue (VALU)
    # fraction against the HBM fraction, from the measured figures
    valu = rec["roofline"]["valu"]
    hbm_frac = rec["roofline"]["frac"]
    rec["roofline"]["limited_by"] = ("valu-issue/latency" if valu and valu["frac"] > hbm_frac else "hbm")
    rec["roofline"]["frac_of_copy_stream"] = achieved / copy_stream_gbps
    if not args.no_extras:
        rec["sclk_mhz"] = sample_sclk(lambda: run_overlapped(4))  # the load of `value`
        del ins, outs
        torch.cuda.empty_cache()
        extras = {}
        extras["latency_cfg0"] = run_latency_cfg0()
        # batches at the default LDS cap (each launch of a batch takes the
        # occupancy its pages' tiles allow) and 256-row tiles
        extras["batch_a4_rgb_64"] = compact_batch(run_batch_workload("batch-rgb", 12, 0, 256))
        extras["batch_uneven_512"] = compact_batch(run_batch_workload("batch-mixed", 12, 0, 256))
        torch.cuda.empty_cache()
        extras["serve"] = compact_serve(run_serve_workload([200.0, 1000.0, 5000.0], 1.0, 4, 32, "both"))
        torch.cuda.empty_cache()
        # offered loads above what the GPU can finish: completed requests
        # per second is the capacity of each mode
        extras["serve_saturation"] = {
            "pages": "4096x4096 gray, Sauvola win 31 (16.8 Mpx per request), offered 60000 req/s",
            "runs": compact_serve(run_serve_workload([60000.0], 0.15, 4, 32, "device", sizes="page4096",
                                                     warm=False))}
        torch.cuda.empty_cache()
        extras["serve_small"] = {
            "pages": "512x512 gray, Sauvola win 31 (0.26 Mpx per request)",
            "runs": compact_serve(run_serve_workload([20000.0, 200000.0], 0.05, 4, 32, "device",
                                                     sizes="page512", warm=True))}
        rec["extras"] = extras
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = run_cpu_baseline(page, args.cpu_budget)
        rec["cpu_baseline"]["cpu_model"] = cpu_model()
        rec["cpu_baseline"]["single_thread_cfg0"] = run_oracle_single_thread_cfg0()
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
