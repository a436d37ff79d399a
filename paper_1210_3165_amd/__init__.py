"""Exact locally adaptive (Sauvola / Niblack) binarization on AMD MI355X.

Thin Python binding over ``libbinarize.so`` (C ABI in ``include/binarize.h``):
argument marshalling only.  Every step of the computation -- Eq. 1 gray
conversion, exact window sums, the Eq. 4 / Niblack threshold and the Eq. 3
decision of Mollah, Basu and Nasipuri (arXiv:1210.3165) -- runs in the HIP
kernels, and so does the global baseline the paper compares against
(Otsu's threshold with the Eq. 2 decision).  PyTorch supplies device memory
and streams; there is no CPU fallback: without the built library every call
raises.
"""
from __future__ import annotations

import ctypes
import os

import torch

__all__ = [
    "SAUVOLA", "NIBLACK", "BinarizeError", "binarize", "binarize_stats", "binarize_staged",
    "default_tile", "tile_lds", "library_path", "lib", "Batch", "batch", "Otsu", "otsu", "otsu_noalloc",
    "binarize_gs", "fmeasure_counts", "GS_PLUS", "GS_X", "GS_STAR",
]

SAUVOLA = 0
NIBLACK = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libbinarize.so")
_lib = None


class BinarizeError(RuntimeError):
    """A libbinarize entry point returned a negative status."""

    def __init__(self, code: int, where: str):
        msg = lib().binarize_strerror(code).decode()
        if code == -8:
            msg += f" (hipError {lib().binarize_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{code}]")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


def lib() -> ctypes.CDLL:
    """The loaded libbinarize.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_1210_3165_amd.build` (or __graft_entry__.build())")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    L.binarize.argtypes = [vp, i, i, i, i, f, f, i, vp]
    L.binarize_async.argtypes = [vp, i, i, i, i, f, f, i, vp, vp]
    L.binarize_tuned.argtypes = [vp, i, i, i, i, f, f, i, vp, i, i, vp]
    L.binarize_stats.argtypes = [vp, i, i, i, i, f, f, i, vp, vp, vp, vp, vp, vp, vp]
    L.binarize_default_tile.argtypes = [i, i, i, i, ctypes.POINTER(i), ctypes.POINTER(i)]
    L.binarize_tile_lds.argtypes = [i, i, i]
    L.binarize_staged.argtypes = [vp, i, i, i, i, f, f, i, vp, vp, ctypes.c_size_t, vp]
    L.binarize_pitched.argtypes = [vp, i, i, i, ctypes.c_int64, i, f, f, i, vp, ctypes.c_int64, vp]
    L.binarize_staged_workspace_size.argtypes = [i, i]
    L.binarize_staged_workspace_size.restype = ctypes.c_size_t
    for name in ("binarize", "binarize_async", "binarize_tuned", "binarize_stats",
                 "binarize_default_tile", "binarize_version", "binarize_last_hip_error",
                 "binarize_tile_lds", "binarize_staged", "binarize_pitched"):
        getattr(L, name).restype = ctypes.c_int
    L.binarize_strerror.argtypes = [i]
    L.binarize_strerror.restype = ctypes.c_char_p
    _lib = L
    return L


def _rule(rule) -> int:
    if isinstance(rule, str):
        r = {"sauvola": SAUVOLA, "niblack": NIBLACK}.get(rule.lower())
        if r is None:
            raise ValueError(f"unknown rule {rule!r}")
        return r
    return int(rule)


def _check_image(img: torch.Tensor) -> tuple[int, int, int]:
    if not isinstance(img, torch.Tensor):
        raise TypeError("img must be a torch.Tensor")
    if img.dtype != torch.uint8:
        raise TypeError(f"img must be uint8, got {img.dtype}")
    if img.device.type != "cuda":
        raise ValueError("img must live on a GPU (device 'cuda'); there is no CPU path")
    if not img.is_contiguous():
        raise ValueError("img must be contiguous (rows of W*channels bytes)")
    if img.dim() == 2:
        return img.shape[0], img.shape[1], 1
    if img.dim() == 3 and img.shape[2] in (1, 3):
        return img.shape[0], img.shape[1], img.shape[2]
    raise ValueError(f"img must be HxW or HxWx3, got {tuple(img.shape)}")


def _row_view(t: torch.Tensor, what: str) -> tuple[int, int, int, int]:
    """(H, W, C, pitch) of an HxW or HxWx3 uint8 CUDA tensor whose rows are
    each contiguous (a crop of a larger image, or padded rows); pitch is the
    byte distance between rows."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8:
        raise TypeError(f"{what} must be a uint8 torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must live on a GPU (device 'cuda'); there is no CPU path")
    if t.dim() == 2:
        H, W, C = t.shape[0], t.shape[1], 1
        rows_ok = W == 1 or t.stride(1) == 1
    elif t.dim() == 3 and t.shape[2] in (1, 3):
        H, W, C = t.shape
        rows_ok = (W == 1 or t.stride(1) == C) and (C == 1 or t.stride(2) == 1)
    else:
        raise ValueError(f"{what} must be HxW or HxWx3, got {tuple(t.shape)}")
    if not rows_ok:
        raise ValueError(f"{what}: each row must be contiguous (W*channels bytes)")
    pitch = t.stride(0) if H > 1 else W * C
    if pitch < W * C:
        raise ValueError(f"{what}: rows overlap (row stride {pitch} < {W * C})")
    return H, W, C, pitch


def _stream_ptr(stream, device) -> int:
    if stream is None:  # the raw handle of the device's current stream, no Stream object
        idx = torch.device(device).index
        return torch._C._cuda_getCurrentRawStream(torch.cuda.current_device() if idx is None else idx)
    return stream.cuda_stream


class _NoSwitch:
    def __enter__(self):
        return None

    def __exit__(self, *exc):
        return False


_NO_SWITCH = _NoSwitch()


def _on_device(device):
    """Context that makes `device` current for the library's calls; free when
    it already is (the common single-GPU case)."""
    idx = torch.device(device).index
    if idx is None or idx == torch.cuda.current_device():
        return _NO_SWITCH
    return torch.cuda.device(idx)


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _keep_for(stream, device, *tensors) -> None:
    """Tensors allocated here come from the current stream's pool; when the
    work runs on another stream, tell the allocator so that it does not hand
    their memory out again before that stream has finished with it."""
    if stream is None or stream == torch.cuda.current_stream(device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(stream)


def binarize(img: torch.Tensor, win: int, k: float, R: float = 128.0, rule=SAUVOLA,
             out: torch.Tensor | None = None, tile: tuple[int, int] | None = None,
             stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """Binarize an HxW (gray) or HxWx3 (interleaved RGB) uint8 CUDA tensor.

    Returns (or fills) an HxW uint8 tensor of {0, 255} on the same device,
    enqueued on ``stream`` (default: the current stream).  ``img`` and
    ``out`` may be row-strided views (a crop, padded rows): each row must be
    contiguous; such calls go through ``binarize_pitched``.  ``tile`` forces
    the (tile_w, tile_h) workgroup tile; the result does not depend on it.
    """
    H, W, C, pitch_in = _row_view(img, "img")
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=img.device)
        _keep_for(stream, img.device, out)
    elif out.dim() != 2 or tuple(out.shape) != (H, W) or out.device != img.device:
        raise ValueError("out must be an HxW uint8 tensor on the image's device")
    pitch_out = _row_view(out, "out")[3]
    L = lib()
    with _on_device(img.device):
        s = ctypes.c_void_p(_stream_ptr(stream, img.device))
        if pitch_in != W * C or pitch_out != W:
            if tile is not None:
                raise ValueError("tile is only supported for contiguous images")
            rc = L.binarize_pitched(_ptr(img), H, W, C, pitch_in, int(win), float(k), float(R), _rule(rule),
                                    _ptr(out), pitch_out, s)
        elif tile is None:
            rc = L.binarize_async(_ptr(img), H, W, C, int(win), float(k), float(R), _rule(rule),
                                  _ptr(out), s)
        else:
            rc = L.binarize_tuned(_ptr(img), H, W, C, int(win), float(k), float(R), _rule(rule),
                                  _ptr(out), int(tile[0]), int(tile[1]), s)
    if rc:
        raise BinarizeError(rc, "binarize")
    return out


def binarize_staged(img: torch.Tensor, win: int, k: float, R: float = 128.0, rule=SAUVOLA,
                    out: torch.Tensor | None = None, workspace: torch.Tensor | None = None,
                    stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """As ``binarize``, computed in two passes through HBM (row window sums
    to two u32 planes, then the column pass and the decision).  Identical
    bytes; slower.  ``workspace`` (optional) is a uint8 CUDA tensor of at
    least 8*H*W bytes, allocated here when not given."""
    H, W, C = _check_image(img)
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=img.device)
        _keep_for(stream, img.device, out)
    elif out.shape != (H, W) or out.dtype != torch.uint8 or out.device != img.device \
            or not out.is_contiguous():
        raise ValueError("out must be a contiguous HxW uint8 tensor on the image's device")
    L = lib()
    need = int(L.binarize_staged_workspace_size(H, W))
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=img.device)
        _keep_for(stream, img.device, workspace)
    elif workspace.device != img.device or not workspace.is_contiguous():
        raise ValueError("workspace must be a contiguous tensor on the image's device")
    with _on_device(img.device):
        s = ctypes.c_void_p(_stream_ptr(stream, img.device))
        rc = L.binarize_staged(_ptr(img), H, W, C, int(win), float(k), float(R), _rule(rule), _ptr(out),
                               _ptr(workspace), workspace.numel() * workspace.element_size(), s)
    if rc:
        raise BinarizeError(rc, "binarize_staged")
    return out


def binarize_stats(img: torch.Tensor, win: int, k: float, R: float = 128.0, rule=SAUVOLA,
                   stream: torch.cuda.Stream | None = None) -> dict[str, torch.Tensor]:
    """Binarize and also return every intermediate plane: gray (u8), s1, s2, n
    (int32 views of the u32 planes), t (f32) and out (u8)."""
    H, W, C = _check_image(img)
    dev = img.device
    res = {
        "out": torch.empty((H, W), dtype=torch.uint8, device=dev),
        "gray": torch.empty((H, W), dtype=torch.uint8, device=dev),
        "s1": torch.empty((H, W), dtype=torch.int32, device=dev),
        "s2": torch.empty((H, W), dtype=torch.int32, device=dev),
        "n": torch.empty((H, W), dtype=torch.int32, device=dev),
        "t": torch.empty((H, W), dtype=torch.float32, device=dev),
    }
    _keep_for(stream, dev, *res.values())
    L = lib()
    with _on_device(dev):
        s = ctypes.c_void_p(_stream_ptr(stream, dev))
        rc = L.binarize_stats(_ptr(img), H, W, C, int(win), float(k), float(R), _rule(rule),
                              _ptr(res["out"]), _ptr(res["gray"]), _ptr(res["s1"]),
                              _ptr(res["s2"]), _ptr(res["n"]), _ptr(res["t"]), s)
    if rc:
        raise BinarizeError(rc, "binarize_stats")
    return res


def tile_lds(tile_w: int, win: int, channels: int = 1) -> int | None:
    """LDS bytes a workgroup of this tile width needs for the window and
    channel count, or None if the tile cannot hold it."""
    rc = lib().binarize_tile_lds(int(tile_w), int(win), int(channels))
    return None if rc < 0 else rc


def default_tile(H: int, W: int, channels: int, win: int) -> tuple[int, int]:
    """(tile_w, tile_h) the library picks for a problem on the current device."""
    tw, th = ctypes.c_int(), ctypes.c_int()
    rc = lib().binarize_default_tile(int(H), int(W), int(channels), int(win),
                                     ctypes.byref(tw), ctypes.byref(th))
    if rc:
        raise BinarizeError(rc, "binarize_default_tile")
    return tw.value, th.value


# ---------------------------------------------------------------------------
# Batched persistent launch
# ---------------------------------------------------------------------------

class _Page(ctypes.Structure):
    _fields_ = [("img", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("H", ctypes.c_int), ("W_img", ctypes.c_int), ("channels", ctypes.c_int),
                ("win", ctypes.c_int), ("k", ctypes.c_float), ("R", ctypes.c_float),
                ("rule", ctypes.c_int), ("tile_w", ctypes.c_int), ("tile_h", ctypes.c_int),
                ("pitch_in", ctypes.c_int64), ("pitch_out", ctypes.c_int64)]


def _batch_lib() -> ctypes.CDLL:
    L = lib()
    if not getattr(L, "_batch_ready", False):
        L.binarize_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
        L.binarize_batch_create.restype = ctypes.c_int
        L.binarize_batch_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Page), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_void_p]
        L.binarize_batch_run.restype = ctypes.c_int
        L.binarize_batch_info.argtypes = [ctypes.c_void_p] + [ctypes.POINTER(ctypes.c_int)] * 3
        L.binarize_batch_info.restype = ctypes.c_int
        L.binarize_batch_destroy.argtypes = [ctypes.c_void_p]
        L.binarize_batch_destroy.restype = None
        L.binarize_batch.argtypes = [ctypes.POINTER(_Page), ctypes.c_int, ctypes.c_void_p]
        L.binarize_batch.restype = ctypes.c_int
        L._batch_ready = True
    return L


def _page_struct(job, i: int) -> _Page:
    """bz_page of one job (img, out, win, k, R, rule[, (tile_w, tile_h)]);
    img and out may be row-strided views."""
    img, out, win, k, R, rule = job[:6]
    tile = job[6] if len(job) > 6 and job[6] is not None else (0, 0)
    H, W, C, pin = _row_view(img, f"page {i} img")
    if out.dim() != 2 or tuple(out.shape) != (H, W) or out.device != img.device:
        raise ValueError(f"page {i}: out must be an HxW uint8 tensor on the image's device")
    pout = _row_view(out, f"page {i} out")[3]
    return _Page(img.data_ptr(), out.data_ptr(), H, W, C, int(win), float(k), float(R),
                 _rule(rule), int(tile[0]), int(tile[1]), pin, pout)


def batch(jobs, stream: torch.cuda.Stream | None = None) -> None:
    """Binarize many pages in a few persistent launches through the one-call
    ``binarize_batch`` (library-managed batch objects).  ``jobs`` as for
    ``Batch.run``; the tensors must stay alive until the stream has
    finished the batch."""
    if not jobs:
        return
    dev = jobs[0][0].device
    arr = (_Page * len(jobs))()
    for i, job in enumerate(jobs):
        arr[i] = _page_struct(job, i)
    with _on_device(dev):
        s = ctypes.c_void_p(_stream_ptr(stream, dev))
        rc = _batch_lib().binarize_batch(arr, len(jobs), s)
    if rc:
        raise BinarizeError(rc, "binarize_batch")


class Batch:
    """Many pages in a few persistent launches (``binarize_batch_*`` in the C ABI:
    one per tile group and occupancy class, one after another).

    ``run(jobs)`` takes a list of ``(img, out, win, k, R, rule)`` or
    ``(img, out, win, k, R, rule, (tile_w, tile_h))`` tuples of CUDA tensors
    and enqueues the whole batch on the current stream; with
    ``use_graph=True`` the launch sequence is a replayed HIP graph.  The
    tensors must stay alive until the stream has finished the batch.
    """

    def __init__(self, max_pages: int, lds_cap: int = 0, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        L = _batch_lib()
        h = ctypes.c_void_p()
        with _on_device(self.device):
            rc = L.binarize_batch_create(int(max_pages), int(lds_cap), ctypes.byref(h))
        if rc:
            raise BinarizeError(rc, "binarize_batch_create")
        self._h = h
        self.max_pages = int(max_pages)
        self._keep = None

    def run(self, jobs, use_graph: bool = True, stream: torch.cuda.Stream | None = None) -> None:
        if self._h is None:
            raise RuntimeError("batch is closed")
        n = len(jobs)
        arr = (_Page * max(n, 1))()
        for i, job in enumerate(jobs):
            arr[i] = _page_struct(job, i)
        with _on_device(self.device):
            s = ctypes.c_void_p(_stream_ptr(stream, self.device))
            rc = _batch_lib().binarize_batch_run(self._h, arr, n, 1 if use_graph else 0, s)
        if rc:
            raise BinarizeError(rc, "binarize_batch_run")
        self._keep = jobs  # the tensors must outlive the enqueued work

    def info(self) -> dict:
        g, l, it = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = _batch_lib().binarize_batch_info(self._h, ctypes.byref(g), ctypes.byref(l), ctypes.byref(it))
        if rc:
            raise BinarizeError(rc, "binarize_batch_info")
        return {"grid": g.value, "lds_cap": l.value, "last_items": it.value}

    def close(self) -> None:
        if self._h is not None:
            _batch_lib().binarize_batch_destroy(self._h)
            self._h = None
            self._keep = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Otsu global threshold (the paper's global baseline)
# ---------------------------------------------------------------------------

OTSU_WS_WORDS = (4096 + 512 * 1024) // 4  # BZ_OTSU_WS_BYTES / 4
OTSU_WS_HIST, OTSU_WS_T, OTSU_WS_KSTAR = 0, 256, 257


def _otsu_lib() -> ctypes.CDLL:
    L = lib()
    if not getattr(L, "_otsu_ready", False):
        vp, i = ctypes.c_void_p, ctypes.c_int
        L.binarize_otsu.argtypes = [vp, i, i, i, vp, vp, ctypes.c_size_t, vp]
        L.binarize_otsu.restype = i
        L.binarize_otsu_workspace_size.argtypes = []
        L.binarize_otsu_workspace_size.restype = ctypes.c_size_t
        L.binarize_otsu_noalloc.argtypes = [vp, i, i, i, vp, vp, vp]
        L.binarize_otsu_noalloc.restype = i
        if L.binarize_otsu_workspace_size() != 4 * OTSU_WS_WORDS:
            raise ImportError("libbinarize.so has a different Otsu workspace size; rebuild it")
        L._otsu_ready = True
    return L


class Otsu:
    """Otsu's global threshold (``binarize_otsu`` in the C ABI) with its own
    device workspace.  ``run`` enqueues the histogram, the selection of T and
    (unless ``threshold_only``) the Eq. 2 decision on the stream; afterwards
    ``hist``, ``T`` and ``kstar`` read the workspace (``T``/``kstar`` sync;
    all three first order the current stream after the last run's stream).
    Calls on one object must be ordered (one stream, or synchronised)."""

    def __init__(self, device=None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        _otsu_lib()
        self.ws = torch.empty(OTSU_WS_WORDS, dtype=torch.int32, device=self.device)
        self._last_stream = None

    def _ws_view(self, lo: int, hi: int) -> torch.Tensor:
        cur = torch.cuda.current_stream(self.device)
        if self._last_stream is not None and self._last_stream != cur:
            cur.wait_stream(self._last_stream)
        return self.ws[lo:hi]

    def run(self, img: torch.Tensor, out: torch.Tensor | None = None, threshold_only: bool = False,
            stream: torch.cuda.Stream | None = None) -> torch.Tensor | None:
        H, W, C = _check_image(img)
        if img.device != self.device:
            raise ValueError("img is on another device than the workspace")
        if threshold_only:
            out = None
        elif out is None:
            out = torch.empty((H, W), dtype=torch.uint8, device=img.device)
            _keep_for(stream, img.device, out)
        elif out.shape != (H, W) or out.dtype != torch.uint8 or out.device != img.device \
                or not out.is_contiguous():
            raise ValueError("out must be a contiguous HxW uint8 tensor on the image's device")
        _keep_for(stream, self.device, self.ws)
        with _on_device(self.device):
            s = ctypes.c_void_p(_stream_ptr(stream, self.device))
            rc = _otsu_lib().binarize_otsu(_ptr(img), H, W, C, _ptr(out), _ptr(self.ws),
                                           4 * OTSU_WS_WORDS, s)
        if rc:
            raise BinarizeError(rc, "binarize_otsu")
        self._last_stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        return out

    @property
    def hist(self) -> torch.Tensor:
        """Histogram of the last run's gray levels (256 counts, device)."""
        return self._ws_view(OTSU_WS_HIST, OTSU_WS_HIST + 256)

    @property
    def T(self) -> int:
        return int(self._ws_view(OTSU_WS_T, OTSU_WS_T + 1).item())

    @property
    def kstar(self) -> int:
        return int(self._ws_view(OTSU_WS_KSTAR, OTSU_WS_KSTAR + 1).item())


def otsu(img: torch.Tensor, out: torch.Tensor | None = None,
         stream: torch.cuda.Stream | None = None) -> tuple[torch.Tensor, int]:
    """Binarize with Otsu's global threshold; returns (out, T).  Synchronises
    to read T; use ``Otsu`` to keep everything on the stream."""
    o = Otsu(img.device)
    out = o.run(img, out, stream=stream)
    return out, o.T


def otsu_noalloc(img: torch.Tensor, out: torch.Tensor | None = None, result: torch.Tensor | None = None,
                 stream: torch.cuda.Stream | None = None) -> torch.Tensor | None:
    """Otsu's threshold and decision through ``binarize_otsu_noalloc``: the
    library's own scratch replaces the workspace, so the call allocates no
    device memory when ``out`` (and ``result``, an int32 CUDA tensor of at
    least 258 words receiving histogram, T and k*) are given.  Calls on one
    device share that scratch and must be ordered."""
    H, W, C = _check_image(img)
    if out is not None and (out.shape != (H, W) or out.dtype != torch.uint8 or out.device != img.device
                            or not out.is_contiguous()):
        raise ValueError("out must be a contiguous HxW uint8 tensor on the image's device")
    if result is not None and (result.dtype != torch.int32 or result.numel() < OTSU_WS_KSTAR + 1
                               or result.device != img.device or not result.is_contiguous()):
        raise ValueError("result must be a contiguous int32 tensor of >= 258 words on the image's device")
    with _on_device(img.device):
        s = ctypes.c_void_p(_stream_ptr(stream, img.device))
        rc = _otsu_lib().binarize_otsu_noalloc(_ptr(img), H, W, C, _ptr(out), _ptr(result), s)
    if rc:
        raise BinarizeError(rc, "binarize_otsu_noalloc")
    return out


# ---------------------------------------------------------------------------
# Sampled-window variant (Sec. 2, Eq. 5) and F-measure counts (Sec. 3)
# ---------------------------------------------------------------------------

GS_PLUS, GS_X, GS_STAR = 0, 1, 2
_GS_NAMES = {"plus": GS_PLUS, "x": GS_X, "star": GS_STAR}


def _gs_lib() -> ctypes.CDLL:
    L = lib()
    if not getattr(L, "_gs_ready", False):
        vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.binarize_gs.argtypes = [vp, i, i, i, i, f, f, i, vp, vp, vp, vp, vp, vp]
        L.binarize_gs.restype = i
        L.binarize_fmeasure_counts.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
        L.binarize_fmeasure_counts.restype = i
        L._gs_ready = True
    return L


def _structure(s) -> int:
    if isinstance(s, str):
        if s.lower() not in _GS_NAMES:
            raise ValueError(f"unknown structure {s!r} (plus, x, star)")
        return _GS_NAMES[s.lower()]
    return int(s)


def binarize_gs(img: torch.Tensor, win: int, k: float, Rp: float = 128.0, structure="plus",
                out: torch.Tensor | None = None, stats: bool = False,
                stream: torch.cuda.Stream | None = None):
    """Sampled-window Sauvola over an odd win x win window's plus / x / star
    structure (this library's structures; Eq. 5 with R' = Rp).  Returns out,
    or with stats=True a dict with out, s1, s2, n (int32 views of u32) and
    t (f32)."""
    H, W, C = _check_image(img)
    dev = img.device
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=dev)
        _keep_for(stream, dev, out)
    elif out.shape != (H, W) or out.dtype != torch.uint8 or out.device != dev or not out.is_contiguous():
        raise ValueError("out must be a contiguous HxW uint8 tensor on the image's device")
    planes = {}
    if stats:
        for name, dt in (("s1", torch.int32), ("s2", torch.int32), ("n", torch.int32), ("t", torch.float32)):
            planes[name] = torch.empty((H, W), dtype=dt, device=dev)
        _keep_for(stream, dev, *planes.values())
    with _on_device(dev):
        s = ctypes.c_void_p(_stream_ptr(stream, dev))
        rc = _gs_lib().binarize_gs(_ptr(img), H, W, C, int(win), float(k), float(Rp), _structure(structure),
                                   _ptr(out), _ptr(planes.get("s1")), _ptr(planes.get("s2")),
                                   _ptr(planes.get("n")), _ptr(planes.get("t")), s)
    if rc:
        raise BinarizeError(rc, "binarize_gs")
    if stats:
        planes["out"] = out
        return planes
    return out


def fmeasure_counts(out: torch.Tensor, gt: torch.Tensor, counts: torch.Tensor | None = None,
                    stream: torch.cuda.Stream | None = None) -> torch.Tensor:
    """TP, FP, FN of a binarized page (0 = text) against a ground-truth mask
    (nonzero = text), counted on the GPU into a 3-element int64 device
    tensor (enqueued on the stream)."""
    for name, t in (("out", out), ("gt", gt)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or t.device.type != "cuda" \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous uint8 CUDA tensor")
    if out.numel() != gt.numel() or out.device != gt.device:
        raise ValueError("out and gt must have the same size and device")
    if counts is None:
        counts = torch.empty(3, dtype=torch.int64, device=out.device)
        _keep_for(stream, out.device, counts)
    with _on_device(out.device):
        s = ctypes.c_void_p(_stream_ptr(stream, out.device))
        rc = _gs_lib().binarize_fmeasure_counts(_ptr(out), _ptr(gt), out.numel(), _ptr(counts), s)
    if rc:
        raise BinarizeError(rc, "binarize_fmeasure_counts")
    return counts
