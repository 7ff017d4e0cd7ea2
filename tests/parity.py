"""Comparison of HIP results with the oracle's (shared by the GPU tests)."""
from __future__ import annotations

import numpy as np

# IMF max-abs error bound, relative to max |x| of the input.
TOL = 1e-8
# Decisions whose margin is below this (relative to max |x|) may legitimately
# flip under rounding-order differences; signals with such a margin are
# reported as tie-prone instead of compared.
TIE = 1e-12


def compare(out_gpu: np.ndarray, n_gpu: int, out_ref: np.ndarray, n_ref: int, xmax: float,
            min_gap: float | None = None) -> dict:
    """Returns {"ok": bool, "tie": bool, "err": float, ...}."""
    tie = min_gap is not None and min_gap < TIE * xmax
    err = float(np.abs(out_gpu - out_ref).max()) if out_ref.size else 0.0
    ok = (n_gpu == n_ref) and err <= TOL * xmax
    return {"ok": ok, "tie": tie, "err": err, "rel": err / xmax if xmax else err,
            "n_gpu": n_gpu, "n_ref": n_ref}


def assert_parity(res: dict, what: str):
    if res["tie"] and not res["ok"]:
        return  # reported by the caller's tie count
    assert res["ok"], f"{what}: {res}"
