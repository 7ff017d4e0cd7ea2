"""The oracle's pins catch plausible mistakes (no GPU needed).

Each case plants one slip in a copy of the oracle's C source -- a dropped
factor, a wrong sign, an off-by-one index, a transposed operand, a misread
step -- compiles that copy with the oracle's own flags, binds it in place of
the oracle in a child process, and runs every pin of ``test_oracle_pins``
against it.  At least one pin must fail for every slip; the pins that do are
listed in the case's message when one does not.  The real oracle stays
untouched, and the child never loads the HIP library.
"""
import json
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")
SRC = os.path.join(ROOT, "oracle", "semd_oracle.c")

# (name, passage, original text, planted text)
MUTANTS = [
    # Sec. 3.2: the crossfade weights
    ("serialize_weight_not_flipped", "Sec. 3.2, E = X_A^f a + X_B^f a^f",
     "double q = xb_f * af[j];", "double q = xb_f * a[j];"),
    ("serialize_head_not_flipped", "Sec. 3.2, flip of X_A",
     "double xa_f = X[(c + 1) * M + (D - 1 - j)];", "double xa_f = X[(c + 1) * M + j];"),
    ("serialize_weights_include_end", "Sec. 3.2, a_i = i/(D+1)",
     "a[i - 1] = (double)i / (double)(D + 1);", "a[i - 1] = (double)i / (double)D;"),
    ("deserialize_wrong_stride", "Sec. 3.3, reshape to (M+D) x N",
     "out[c * M + m] = T[c * R + m];", "out[c * M + m] = T[c * M + m];"),
    # Sec. 2.1 Step 1: extrema
    ("plateau_ceiling_middle", "Sec. 2.1 Step 1, plateau reading",
     "int64_t mid = (k + b) / 2;", "int64_t mid = (k + b + 1) / 2;"),
    ("end_run_off_by_one", "Sec. 2.1 Step 1, end-sample reading",
     "if (k >= 1 && b <= L - 2) {", "if (k >= 1 && b <= L - 3) {"),
    ("plateau_start", "Sec. 2.1 Step 1, plateau reading",
     "if (h[k - 1] < h[k] && h[b + 1] < h[b]) imax[na++] = mid;",
     "if (h[k - 1] < h[k] && h[b + 1] < h[b]) imax[na++] = k;"),
    ("siftable_two_extrema", "IMF loop stopping reading",
     "return nmax >= 1 && nmin >= 1 && nmax + nmin >= 3;",
     "return nmax >= 1 && nmin >= 1 && nmax + nmin >= 2;"),
    # Sec. 2.1 Step 2: natural cubic spline
    ("spline_diag_factor_dropped", "Sec. 2.1 Step 2, spline equations",
     "double diag = 2.0 * (g0 + g1);", "double diag = 2.0 * g0 + g1;"),
    ("spline_rhs_sign", "Sec. 2.1 Step 2, spline equations",
     "double rhs = 6.0 * (s1 - s0);", "double rhs = 6.0 * (s0 - s1);"),
    ("spline_offdiag_transposed", "Sec. 2.1 Step 2, spline equations",
     "double sub = g0, sup = g1;", "double sub = g1, sup = g0;"),
    ("spline_eval_wrong_index", "Sec. 2.1 Step 2, cubic pieces",
     "(y[j + 1] - Mpp[j + 1] * g2 / 6.0) * B / g", "(y[j + 1] - Mpp[j] * g2 / 6.0) * B / g"),
    ("spline_eval_cubic_scale", "Sec. 2.1 Step 2, cubic pieces",
     "double cub = (Mpp[j] * A3 + Mpp[j + 1] * B3) / (6.0 * g);",
     "double cub = (Mpp[j] * A3 + Mpp[j + 1] * B3) / (6.0 * g2);"),
    ("mirror_about_length", "Sec. 2.1 Step 2, mirror boundary reading",
     "t[q] = (double)(2 * (L - 1) - idx[p]);", "t[q] = (double)(2 * L - idx[p]);"),
    ("mirror_one_knot", "Sec. 2.1 Step 2, mirror boundary reading",
     "const int64_t P = n < 2 ? n : 2;", "const int64_t P = n < 1 ? n : 1;"),
    # Sec. 2.1 Steps 3-5: mean, candidate, residue, stopping
    ("mean_difference", "Sec. 2.1 Step 3, local mean",
     "double m = 0.5 * (up[k] + lo[k]);", "double m = 0.5 * (up[k] - lo[k]);"),
    ("residue_added", "Sec. 2.1 Step 5, residue update",
     "r[k] = r[k] - h[k];", "r[k] = r[k] + h[k];"),
    ("sd_against_new_candidate", "SD rule reading (change over the old candidate)",
     "den += h[k] * h[k];", "den += (h[k] - m) * (h[k] - m);"),
    ("sift_count_short", "S sifts per IMF",
     "for (int s = 0; s < S; ++s) {", "for (int s = 0; s < S - 1; ++s) {"),
    ("sd_margin_over_den", "SD rule, distance of the closest decision",
     "const double margin = fabs(num - lim) / lim;",
     "const double margin = fabs(num - lim) / den;"),
    # Sec. 4 opening: standard (slice-wise) EMD
    ("slices_column_offset", "standard EMD, one column per signal",
     "(size_t)(c * M), R + (size_t)k * (size_t)M,", "(size_t)c, R + (size_t)k * (size_t)M,"),
    # Sec. 2.2: EEMD and CEEMDAN
    ("splitmix_shift", "SplitMix64 definition",
     "z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;", "z = (z ^ (z >> 28)) * 0x94D049BB133111EBull;"),
    ("noise_not_centred", "noise stream reading",
     "int64_t c = (int64_t)acc - (int64_t)(6ull << 53);",
     "int64_t c = (int64_t)acc - (int64_t)(5ull << 53);"),
    ("noise_stream_key", "noise stream reading",
     "uint64_t s1 = semd_ref_splitmix64(seed, item + 1);",
     "uint64_t s1 = semd_ref_splitmix64(seed, item);"),
    ("eemd_noise_subtracted", "Sec. 2.2 EEMD Step 1, x_m = x + beta w_m",
     "xm[k] = x[k] + bw;", "xm[k] = x[k] - bw;"),
    ("ceemdan_sample_std", "Sec. 2.2 CEEMDAN, std of the residue",
     "return sqrt(q / (double)L);", "return sqrt(q / (double)(L - 1));"),
    ("eemd_mean_off_by_one", "Sec. 2.2 EEMD Step 3, ensemble mean",
     "acc[i] = acc[i] / (double)NR;", "acc[i] = acc[i] / (double)(NR + 1);"),
    ("ceemdan_noise_mode_index", "Sec. 2.2 CEEMDAN Step 3, E_{i-1}(w_m)",
     "(size_t)(i - 2)) * (size_t)L;", "(size_t)(i - 1)) * (size_t)L;"),
    ("ceemdan_beta_from_input", "Sec. 2.2 CEEMDAN, beta_{i-1} from r_{i-1}",
     "const double beta = eps * pop_std(r, L);", "const double beta = eps;"),
    ("ceemdan_residue_kept", "Sec. 2.2 CEEMDAN Step 3, r_i = r_{i-1} - c_i",
     "r[k] = r[k] - c[k];         /* r_i = r_{i-1} - c_i */",
     "r[k] = r[k] - 0.5 * c[k];"),
]

CHILD = r"""
import ctypes, json, sys
sys.path[:0] = [sys.argv[2], sys.argv[3]]
import oracle
oracle._lib = oracle.bind(ctypes.CDLL(sys.argv[1]))
import test_oracle_pins as P

def cases(fn):
    out = [{}]
    for mark in getattr(fn, "pytestmark", []):
        if mark.name != "parametrize":
            continue
        names = mark.args[0]
        names = [n.strip() for n in names.split(",")] if isinstance(names, str) else list(names)
        nxt = []
        for c in out:
            for v in mark.args[1]:
                if hasattr(v, "values"):  # pytest.param
                    v = v.values[0] if len(names) == 1 else v.values
                vals = [v] if len(names) == 1 else list(v)
                nxt.append(dict(c, **dict(zip(names, vals))))
        out = nxt
    return out

failed, ran = [], 0
for name in sorted(vars(P)):
    fn = getattr(P, name)
    if not name.startswith("test_") or not callable(fn):
        continue
    for kw in cases(fn):
        ran += 1
        try:
            fn(**kw)
        except Exception:
            failed.append(name)
            break
print(json.dumps({"ran": ran, "failed": failed}))
"""


@pytest.mark.parametrize("name,passage,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, passage, orig, planted, tmp_path):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation site for {name} not unique in the oracle"
    mutant = tmp_path / "semd_oracle_mutant.c"
    mutant.write_text(src.replace(orig, planted))
    so = oracle.compile_source(str(mutant), str(tmp_path / "libmutant.so"))
    p = subprocess.run([sys.executable, "-c", CHILD, so, ROOT, TESTS], capture_output=True,
                       text=True, timeout=300)
    if p.returncode != 0:
        pytest.fail(f"{name}: child ended with {p.returncode} (a slip should fail a pin, "
                    f"not crash)\n{p.stderr[-2000:]}")
    res = json.loads(p.stdout.strip().splitlines()[-1])
    assert res["ran"] >= 40
    assert res["failed"], f"no pin catches {name} ({passage})"
