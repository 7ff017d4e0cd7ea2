"""Parity of the HIP path with the oracle (shared by the GPU tests).

Two bars, both against the oracle on the same input:
* outputs: max |gpu - oracle| over every slot <= TOL * max|x|;
* extremum decisions (Sec. 2.1 Step 1), compared detection by detection:
  every detection's maxima and minima must equal the oracle's.  Where they
  differ, each differing position k gets the margin
      mu = (distance of the oracle's tested value at k from its neighbours,
            the equal-valued run's outer steps when k lies in a run) / max|x|;
  if every such mu is below TIE the decision is a tie -- a near-equality
  that a different rounding order may legitimately flip -- and the signal
  is reported as tie-diverged and compared no further; otherwise it is a
  failure.  Under the SD stopping rule the decision to end an IMF is a tie
  when the oracle's SD ratio lies within SD_TIE (relative) of the threshold.

Every tie is reported: appended to TIES (printed in the session summary by
conftest) and counted per test against a bound the test states.  Nothing is
skipped silently.
"""
from __future__ import annotations

import math

import numpy as np

# IMF max-abs error bound, relative to max |x| of the input.
TOL = 1e-8
# Extremum decisions whose margin is below this (relative to max |x|) are ties.
TIE = 1e-12
# SD-rule decisions within this relative distance of the threshold are ties.
SD_TIE = 1e-9

# Every tie of the session: dicts with "what", "imf", "sift", "detail".
TIES: list[dict] = []


def parse_trace(t) -> tuple[list, bool]:
    """Records (imf, sift, maxima, minima) of a device trace buffer (int32:
    entries used, complete flag, 2 spare entries, then the records) and
    whether every record fitted."""
    t = np.asarray(t, dtype=np.int64)
    used, complete = int(t[0]), bool(t[1])
    recs, o = [], 4
    while o < used:
        imf, sift, na, ni = (int(v) for v in t[o:o + 4])
        if na < 0 or ni < 0 or o + 4 + na + ni > used:
            raise AssertionError(f"malformed trace record at {o}")
        recs.append((imf, sift, t[o + 4:o + 4 + na].copy(), t[o + 4 + na:o + 4 + na + ni].copy()))
        o += 4 + na + ni
    return recs, complete


def margin(h: np.ndarray, k: int, xmax: float) -> float:
    """How far position k of h is from changing its extremum status, relative
    to xmax: the smaller step out of the equal-valued run that holds k."""
    L = h.size
    a = b = k
    while a > 0 and h[a - 1] == h[k]:
        a -= 1
    while b < L - 1 and h[b + 1] == h[k]:
        b += 1
    steps = []
    if a > 0:
        steps.append(abs(h[a] - h[a - 1]))
    if b < L - 1:
        steps.append(abs(h[b + 1] - h[b]))
    return min(steps) / xmax if steps else math.inf


def compare_decisions(gpu_recs: list, ref_recs: list, tested, xmax: float,
                      sd_margin: float = math.inf) -> dict:
    """First divergence of two detection-record lists (same order).
    tested(imf, sift) returns the oracle's array of that detection.
    Returns {"status": "equal" | "tie" | "fail", "records": compared, ...}."""
    n = min(len(gpu_recs), len(ref_recs))
    for i in range(n):
        gi, gs, gmax, gmin = gpu_recs[i]
        ri, rs, rmax, rmin = ref_recs[i]
        if (gi, gs) != (ri, rs):
            # every earlier detection agreed: the IMF ended at a different
            # sift, which only the SD rule's sums decide
            st = "tie" if sd_margin < SD_TIE else "fail"
            return {"status": st, "records": i, "imf": ri, "sift": rs, "kind": "sd",
                    "detail": f"gpu at (imf {gi}, sift {gs}), oracle at (imf {ri}, sift {rs}), "
                              f"SD margin {sd_margin:.3g}"}
        if np.array_equal(gmax, rmax) and np.array_equal(gmin, rmin):
            continue
        diff = sorted(set(np.setxor1d(gmax, rmax).tolist()) | set(np.setxor1d(gmin, rmin).tolist()))
        h = tested(ri, rs)
        mus = [margin(h, int(k), xmax) for k in diff]
        st = "tie" if max(mus) < TIE else "fail"
        return {"status": st, "records": i, "imf": ri, "sift": rs, "kind": "extrema",
                "positions": diff[:8], "mu": max(mus),
                "detail": f"imf {ri} sift {rs}: {len(diff)} positions differ "
                          f"{diff[:8]}, largest margin {max(mus):.3g}"}
    if len(gpu_recs) != len(ref_recs):
        st = "tie" if sd_margin < SD_TIE else "fail"
        return {"status": st, "records": n, "imf": -1, "sift": -1, "kind": "sd",
                "detail": f"{len(gpu_recs)} gpu detections, {len(ref_recs)} oracle detections, "
                          f"SD margin {sd_margin:.3g}"}
    return {"status": "equal", "records": n}


class Tally:
    """Ties of one test: each reported, at most max_ties allowed."""

    def __init__(self, what: str, max_ties: int = 0):
        self.what = what
        self.max_ties = max_ties
        self.ties: list[dict] = []

    def tie(self, item: str, res: dict) -> None:
        rec = {"what": f"{self.what}: {item}", "imf": res.get("imf"), "sift": res.get("sift"),
               "detail": res.get("detail", "")}
        self.ties.append(rec)
        TIES.append(rec)
        print(f"TIE {rec['what']}: {rec['detail']}", flush=True)

    def done(self) -> None:
        print(f"{self.what}: {len(self.ties)} tie(s), bound {self.max_ties}", flush=True)
        assert len(self.ties) <= self.max_ties, (self.what, self.ties)


def output_error(out_gpu: np.ndarray, out_ref: np.ndarray) -> float:
    return float(np.abs(out_gpu - out_ref).max()) if out_ref.size else 0.0


def outputs_match(out_gpu, n_gpu: int, out_ref, n_ref: int, xmax: float) -> tuple[bool, float]:
    err = output_error(out_gpu, out_ref)
    return (n_gpu == n_ref) and err <= TOL * xmax, err
