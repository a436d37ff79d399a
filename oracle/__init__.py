"""CPU oracle for exact locally adaptive binarization (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never touches it, and the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, double precision, a direct
window loop per pixel); this module only builds it with gcc and marshals NumPy
arrays through ctypes.  See ``oracle.c`` for the definitions it follows
(Sec. 1 Eq. 1, 2, 3, 4, Sec. 2 Eq. 5 and Sec. 3 Eq. 6 of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SAUVOLA = 0
NIBLACK = 1

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP over rows)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", "-std=c99",
               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    f64p = ctypes.POINTER(ctypes.c_double)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_gray.argtypes = [u8p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, u8p]
    lib.oracle_gray.restype = ctypes.c_int
    lib.oracle_binarize.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    u8p, u32p, u32p, u32p, f64p, f64p, f64p, u8p]
    lib.oracle_binarize.restype = ctypes.c_int
    lib.oracle_binarize_points.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                           i32p, i32p, ctypes.c_int64,
                                           u8p, u32p, u32p, u32p, f64p, f64p, f64p, u8p]
    lib.oracle_binarize_points.restype = ctypes.c_int
    lib.oracle_num_threads.restype = ctypes.c_int
    lib.oracle_otsu.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, u32p,
                                ctypes.POINTER(ctypes.c_int), u8p]
    lib.oracle_otsu.restype = ctypes.c_int
    lib.oracle_binarize_gs.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       u32p, u32p, u32p, f64p, u8p]
    lib.oracle_binarize_gs.restype = ctypes.c_int
    lib.oracle_version.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None, ctype):
    if a is None:
        return ctypes.POINTER(ctype)()
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_image(img: np.ndarray) -> tuple[np.ndarray, int, int, int]:
    img = np.ascontiguousarray(img, dtype=np.uint8)
    if img.ndim == 2:
        return img, img.shape[0], img.shape[1], 1
    if img.ndim == 3 and img.shape[2] in (1, 3):
        return img, img.shape[0], img.shape[1], img.shape[2]
    raise ValueError(f"image must be HxW or HxWx{{1,3}}, got {img.shape}")


@dataclass
class OracleResult:
    gray: np.ndarray
    s1: np.ndarray
    s2: np.ndarray
    n: np.ndarray
    m: np.ndarray
    s: np.ndarray
    t: np.ndarray
    out: np.ndarray


def gray(img: np.ndarray) -> np.ndarray:
    """Eq. 1 gray levels of an HxW or HxWx3 uint8 image."""
    img, H, W, C = _as_image(img)
    g = np.empty((H, W), np.uint8)
    rc = _load().oracle_gray(_ptr(img, ctypes.c_uint8), H, W, C, _ptr(g, ctypes.c_uint8))
    if rc:
        raise ValueError(f"oracle_gray failed ({rc})")
    return g


def binarize(img: np.ndarray, win: int, k: float, R: float = 128.0,
             rule: int = SAUVOLA) -> OracleResult:
    """Whole-image reference: gray, window sums, n, m, s, t and the binary output."""
    img, H, W, C = _as_image(img)
    npx = (H, W)
    g = np.empty(npx, np.uint8)
    s1 = np.empty(npx, np.uint32)
    s2 = np.empty(npx, np.uint32)
    n = np.empty(npx, np.uint32)
    m = np.empty(npx, np.float64)
    s = np.empty(npx, np.float64)
    t = np.empty(npx, np.float64)
    out = np.empty(npx, np.uint8)
    rc = _load().oracle_binarize(_ptr(img, ctypes.c_uint8), H, W, C, int(win), float(k), float(R),
                                 int(rule), _ptr(g, ctypes.c_uint8), _ptr(s1, ctypes.c_uint32),
                                 _ptr(s2, ctypes.c_uint32), _ptr(n, ctypes.c_uint32),
                                 _ptr(m, ctypes.c_double), _ptr(s, ctypes.c_double),
                                 _ptr(t, ctypes.c_double), _ptr(out, ctypes.c_uint8))
    if rc:
        raise ValueError(f"oracle_binarize failed ({rc})")
    return OracleResult(g, s1, s2, n, m, s, t, out)


def binarize_points(img: np.ndarray, win: int, k: float, R: float, rule: int,
                    ys: np.ndarray, xs: np.ndarray) -> OracleResult:
    """The same quantities at chosen pixels only (for full-size images)."""
    img, H, W, C = _as_image(img)
    ys = np.ascontiguousarray(ys, dtype=np.int32)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    if ys.shape != xs.shape or ys.ndim != 1:
        raise ValueError("ys and xs must be 1-D arrays of equal length")
    p = ys.shape[0]
    f = np.empty(p, np.uint8)
    s1 = np.empty(p, np.uint32)
    s2 = np.empty(p, np.uint32)
    n = np.empty(p, np.uint32)
    m = np.empty(p, np.float64)
    s = np.empty(p, np.float64)
    t = np.empty(p, np.float64)
    out = np.empty(p, np.uint8)
    rc = _load().oracle_binarize_points(_ptr(img, ctypes.c_uint8), H, W, C, int(win), float(k),
                                        float(R), int(rule), _ptr(ys, ctypes.c_int32),
                                        _ptr(xs, ctypes.c_int32), p, _ptr(f, ctypes.c_uint8),
                                        _ptr(s1, ctypes.c_uint32), _ptr(s2, ctypes.c_uint32),
                                        _ptr(n, ctypes.c_uint32), _ptr(m, ctypes.c_double),
                                        _ptr(s, ctypes.c_double), _ptr(t, ctypes.c_double),
                                        _ptr(out, ctypes.c_uint8))
    if rc:
        raise ValueError(f"oracle_binarize_points failed ({rc})")
    return OracleResult(f, s1, s2, n, m, s, t, out)


def num_threads() -> int:
    """OpenMP threads the oracle uses on this host."""
    return int(_load().oracle_num_threads())


def otsu(img: np.ndarray):
    """Otsu's global threshold (Sec. 1, Eq. 2 baseline): returns (T, k*, hist,
    out) with out = 0 where f < T = k* + 1."""
    img, H, W, C = _as_image(img)
    hist = np.empty(256, np.uint32)
    out = np.empty((H, W), np.uint8)
    k = ctypes.c_int()
    T = _load().oracle_otsu(_ptr(img, ctypes.c_uint8), H, W, C, _ptr(hist, ctypes.c_uint32),
                            ctypes.byref(k), _ptr(out, ctypes.c_uint8))
    if T < 0:
        raise ValueError(f"oracle_otsu failed ({T})")
    return T, k.value, hist, out


GS_PLUS, GS_X, GS_STAR = 0, 1, 2


def binarize_gs(img: np.ndarray, win: int, k: float, Rp: float, structure: int) -> OracleResult:
    """Sampled-window Sauvola (Sec. 2, Eq. 5) over the structure's members of
    the odd win x win window: s1, s2, n, t and out (gray, m, s are None)."""
    img, H, W, C = _as_image(img)
    s1 = np.empty((H, W), np.uint32)
    s2 = np.empty((H, W), np.uint32)
    n = np.empty((H, W), np.uint32)
    t = np.empty((H, W), np.float64)
    out = np.empty((H, W), np.uint8)
    rc = _load().oracle_binarize_gs(_ptr(img, ctypes.c_uint8), H, W, C, int(win), float(k), float(Rp),
                                    int(structure), _ptr(s1, ctypes.c_uint32), _ptr(s2, ctypes.c_uint32),
                                    _ptr(n, ctypes.c_uint32), _ptr(t, ctypes.c_double),
                                    _ptr(out, ctypes.c_uint8))
    if rc:
        raise ValueError(f"oracle_binarize_gs failed ({rc})")
    return OracleResult(None, s1, s2, n, None, None, t, out)


def fmeasure_counts(out: np.ndarray, gt: np.ndarray) -> tuple[int, int, int]:
    """(TP, FP, FN) of a binarized page against its ground truth (Sec. 3).
    Foreground is text: output 0 (f < t, Eq. 3) and gt != 0."""
    fg = np.asarray(out) == 0
    truth = np.asarray(gt) != 0
    tp = int(np.count_nonzero(fg & truth))
    fp = int(np.count_nonzero(fg & ~truth))
    fn = int(np.count_nonzero(~fg & truth))
    return tp, fp, fn


def fmeasure(tp: int, fp: int, fn: int) -> float:
    """Eq. 6: FM = 2 R P / (R + P), R = TP / (TP + FN), P = TP / (TP + FP);
    0 when there is no true positive."""
    if tp == 0:
        return 0.0
    R = tp / (tp + fn)
    P = tp / (tp + fp)
    return 2 * R * P / (R + P)
