"""Element-by-element comparison of a GPU result with the oracle (test
infrastructure; works on NumPy arrays only and imports nothing of the HIP path).

The parity bar:
  * gray levels, window sums S1, S2 and counts n: bit-identical;
  * threshold t: |t_gpu - t_oracle| <= T_TOL at every pixel;
  * binary output: identical except at pixels whose gray level lies within
    T_TOL of the oracle's threshold (|f - t_oracle| < T_TOL), where fp32 and
    fp64 may legitimately round to opposite sides; those are counted.
"""
from __future__ import annotations

import numpy as np

T_TOL = 1e-4


def as_u32(a) -> np.ndarray:
    a = np.asarray(a)
    if a.dtype in (np.int32, np.uint32):
        return a.view(np.uint32)
    return a.astype(np.uint32)


def compare_out(out_gpu, ref_out, ref_f, ref_t, tol: float = T_TOL) -> dict:
    """Compare binary outputs only (the product path)."""
    out_gpu = np.asarray(out_gpu)
    band = np.abs(np.asarray(ref_f, np.float64) - np.asarray(ref_t, np.float64)) < tol
    mism = out_gpu != np.asarray(ref_out)
    rep = {
        "pixels": int(out_gpu.size),
        "n_band": int(band.sum()),
        "n_mismatch_in_band": int((mism & band).sum()),
        "n_mismatch_out_of_band": int((mism & ~band).sum()),
        "alphabet_ok": bool(np.all((out_gpu == 0) | (out_gpu == 255))),
    }
    rep["ok"] = rep["n_mismatch_out_of_band"] == 0 and rep["alphabet_ok"]
    return rep


def compare_stats(gpu: dict, ref, tol: float = T_TOL) -> dict:
    """Compare every plane of a stats run (dict of NumPy arrays: gray, s1, s2,
    n, t, out) with an OracleResult."""
    rep = compare_out(gpu["out"], ref.out, ref.gray, ref.t, tol)
    rep["gray_equal"] = bool(np.array_equal(np.asarray(gpu["gray"]), ref.gray))
    rep["s1_equal"] = bool(np.array_equal(as_u32(gpu["s1"]), ref.s1))
    rep["s2_equal"] = bool(np.array_equal(as_u32(gpu["s2"]), ref.s2))
    rep["n_equal"] = bool(np.array_equal(as_u32(gpu["n"]), ref.n))
    terr = np.abs(np.asarray(gpu["t"], np.float64) - ref.t)
    rep["max_abs_t_err"] = float(terr.max()) if terr.size else 0.0
    rep["ok"] = (rep["ok"] and rep["gray_equal"] and rep["s1_equal"] and rep["s2_equal"]
                 and rep["n_equal"] and rep["max_abs_t_err"] <= tol)
    return rep
