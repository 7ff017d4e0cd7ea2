"""Pins of the CPU oracle to facts outside itself (no GPU needed).

Each test ties one oracle function to something it does not compute by itself:
the hand-derived worked example of Sec. 3.2, closed forms (lengths, the
continuity of the transition of Sec. 3.1), an independent library routine
(scipy's peak finder and natural cubic spline, numpy's dense solver), brute
force over every small input, exact invariants of the arithmetic (sign and
power-of-two scaling), and published SplitMix64 test vectors.  A plausible
slip in the oracle -- a dropped flip, a swapped weight, an off-by-one in the
plateau rule, a wrong mirror, a transposed Thomas coefficient -- fails one of
them.
"""
import itertools
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.signal import find_peaks

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Sec. 3.2 / 3.3 -- serialization and deserialization
# --------------------------------------------------------------------------

def _read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, rest = line.split(":", 1)
            vals[key.strip()] = rest.split()
    return vals


def test_serialize_worked_example():
    g = _read_golden("serialize_worked_example.txt")
    M, N, D = (int(v) for v in g["M N D"])
    X = np.array([float(v) for v in g["X"]])
    want = [Fraction(v) for v in g["x"]]
    x = oracle.serialize(X, M, N, D)
    assert x.size == len(want) == M * N + D * N - D
    for got, w in zip(x, want):
        # each transition sample is a*A + af*B with three roundings
        assert abs(Fraction(got) - w) <= Fraction(3, 2**52) * abs(w)


@pytest.mark.parametrize("M,N,D", [(1, 1, 0), (1, 5, 1), (7, 1, 3), (5, 4, 0), (5, 4, 5),
                                   (17, 6, 3), (100, 3, 50), (128, 128, 26)])
def test_serial_length_closed_form(M, N, D):
    assert oracle.serial_length(M, N, D) == M * N + D * N - D == (M + D) * N - D


def test_serialize_d0_is_vec():
    rng = np.random.default_rng(1)
    X = rng.standard_normal(37 * 5)
    assert np.array_equal(oracle.serialize(X, 37, 5, 0), X)


@pytest.mark.parametrize("D", [0, 1, 2, 9])
def test_round_trip_bit_exact(D):
    rng = np.random.default_rng(2 + D)
    M, N = 9, 6
    X = rng.standard_normal(M * N) * 10.0 ** rng.integers(-300, 300, M * N)
    X[0] = -0.0
    X[1] = 5e-324  # subnormal
    X[2] = 1.7e308
    y = oracle.serialize(X, M, N, D)
    back = oracle.deserialize(y, M, N, D)
    assert back.tobytes() == X.tobytes()


def test_round_trip_d_equals_m():
    rng = np.random.default_rng(7)
    M, N = 6, 4
    X = rng.standard_normal(M * N)
    assert oracle.deserialize(oracle.serialize(X, M, N, M), M, N, M).tobytes() == X.tobytes()


def test_constant_columns_give_linear_crossfade():
    # Sec. 3.1: h(t) = (1 - t/D) f(T - t) + (t/D) g(D - t) blends the end of one
    # signal into the start of the next; with constant columns the discrete
    # transition is a straight ramp strictly between the two levels.
    M, N, D = 8, 3, 5
    levels = [2.0, -6.0, 10.0]
    X = np.concatenate([np.full(M, v) for v in levels])
    x = oracle.serialize(X, M, N, D)
    for i in range(N - 1):
        seg = x[i * (M + D) + M: i * (M + D) + M + D]
        lo, hi = sorted((levels[i], levels[i + 1]))
        assert np.all(seg > lo) and np.all(seg < hi)
        d = np.diff(np.concatenate([[levels[i]], seg, [levels[i + 1]]]))
        assert np.allclose(d, (levels[i + 1] - levels[i]) / (D + 1), rtol=0, atol=1e-13)


def test_transition_ends_approach_neighbours():
    # Continuity: h(0) = f(T) and h(D) = g(0).  The first transition sample
    # leans on the LAST sample of column i, the last one on the FIRST sample of
    # column i+1 (the flips of X_B and X_A), with weight D/(D+1).
    rng = np.random.default_rng(3)
    M, N, D = 50, 2, 40
    X = rng.standard_normal(M * N)
    x = oracle.serialize(X, M, N, D)
    e = x[M: M + D]
    f_T, g_0 = X[M - 1], X[M]
    assert abs(e[0] - f_T) <= (abs(X[M + D - 1]) + abs(f_T)) / (D + 1) + 1e-15
    assert abs(e[-1] - g_0) <= (abs(X[M - D]) + abs(g_0)) / (D + 1) + 1e-15
    # and exactly a convex combination of those two flipped partners
    j = 1
    want = (j / (D + 1)) * X[M + D - j] + ((D + 1 - j) / (D + 1)) * X[M - j]
    assert e[0] == want


# --------------------------------------------------------------------------
# Sec. 2.1 Step 1 -- extrema
# --------------------------------------------------------------------------

def _brute_extrema(h):
    """Direct definition, written independently: a sample is a maximum if it
    sits in a run of equal values, strictly above both samples bounding the
    run, the run touching neither end; the extremum is the run's floor-middle."""
    L = len(h)
    mx, mn = [], []
    for k in range(1, L - 1):
        a = k
        while a - 1 >= 0 and h[a - 1] == h[k]:
            a -= 1
        b = k
        while b + 1 < L and h[b + 1] == h[k]:
            b += 1
        if a == 0 or b == L - 1 or k != (a + b) // 2:
            continue
        if h[a - 1] < h[k] and h[b + 1] < h[k]:
            mx.append(k)
        if h[a - 1] > h[k] and h[b + 1] > h[k]:
            mn.append(k)
    return mx, mn


def test_extrema_brute_force_and_scipy_all_small_inputs():
    n = 0
    for L in range(3, 9):
        for seq in itertools.product((0.0, 1.0, 2.0), repeat=L):
            h = np.array(seq)
            imax, imin = oracle.extrema(h)
            bmx, bmn = _brute_extrema(seq)
            assert list(imax) == bmx and list(imin) == bmn, seq
            assert list(imax) == list(find_peaks(h)[0]), seq
            assert list(imin) == list(find_peaks(-h)[0]), seq
            n += 1
    assert n == sum(3 ** L for L in range(3, 9))


def test_extrema_sign_symmetry_and_scipy_random():
    rng = np.random.default_rng(11)
    for _ in range(20):
        h = np.round(rng.standard_normal(500) * 3)  # many exact plateaus
        imax, imin = oracle.extrema(h)
        nmax, nmin = oracle.extrema(-h)
        assert np.array_equal(imax, nmin) and np.array_equal(imin, nmax)
        assert np.array_equal(imax, find_peaks(h)[0])
        assert np.array_equal(imin, find_peaks(-h)[0])


def test_extrema_alternate():
    rng = np.random.default_rng(12)
    h = rng.standard_normal(2001)
    imax, imin = oracle.extrema(h)
    both = np.sort(np.concatenate([imax, imin]))
    kinds = np.isin(both, imax)
    assert np.all(kinds[1:] != kinds[:-1])  # maxima and minima alternate


# --------------------------------------------------------------------------
# Sec. 2.1 Step 2 -- natural cubic spline and envelopes
# --------------------------------------------------------------------------

def _mirrored_knots(h, idx):
    L = len(h)
    P = min(2, len(idx))
    t = ([-idx[p] for p in range(P - 1, -1, -1)] + list(idx)
         + [2 * (L - 1) - idx[len(idx) - 1 - p] for p in range(P)])
    y = [h[i] for i in idx[:P][::-1]] + [h[i] for i in idx] + [h[i] for i in idx[::-1][:P]]
    return np.array(t, float), np.array(y, float)


def test_spline_matches_scipy_natural():
    rng = np.random.default_rng(21)
    for n in (3, 4, 7, 40, 300):
        t = np.cumsum(rng.integers(1, 30, n)).astype(float) - 40
        y = rng.standard_normal(n) * 5
        L = int(t[-1])
        t[0] = min(t[0], -1.0)
        Mpp = oracle.spline_solve(t, y)
        got = oracle.spline_eval(t, y, Mpp, L)
        want = CubicSpline(t, y, bc_type="natural")(np.arange(L, dtype=float))
        scale = np.abs(y).max()
        assert np.abs(got - want).max() <= 1e-12 * scale
        sp = CubicSpline(t, y, bc_type="natural")
        assert np.allclose(Mpp, sp(t, 2), rtol=1e-11, atol=1e-12 * scale)


def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(22)
    for n in (3, 5, 17, 50):
        t = np.cumsum(rng.integers(1, 9, n)).astype(float) - 3
        y = rng.standard_normal(n)
        g = np.diff(t)
        A = np.zeros((n - 2, n - 2))
        r = np.zeros(n - 2)
        for j in range(1, n - 1):
            i = j - 1
            A[i, i] = 2 * (g[j - 1] + g[j])
            if i > 0:
                A[i, i - 1] = g[j - 1]
            if i < n - 3:
                A[i, i + 1] = g[j]
            r[i] = 6 * ((y[j + 1] - y[j]) / g[j] - (y[j] - y[j - 1]) / g[j - 1])
        want = np.concatenate([[0.0], np.linalg.solve(A, r), [0.0]])
        assert np.allclose(oracle.spline_solve(t, y), want, rtol=1e-12, atol=1e-13)


def test_spline_constant_and_linear_exactness():
    t = np.array([-7.0, -2, 2, 7, 11, 30, 40])
    c = oracle.spline_eval(t, np.full(7, 3.25), oracle.spline_solve(t, np.full(7, 3.25)), 38)
    assert np.all(c == 3.25)
    y = 0.5 * t - 1.0
    lin = oracle.spline_eval(t, y, oracle.spline_solve(t, y), 38)
    assert np.abs(lin - (0.5 * np.arange(38) - 1.0)).max() <= 1e-13


def test_envelope_interpolates_extrema_and_uses_mirror_knots():
    rng = np.random.default_rng(23)
    h = np.cumsum(rng.standard_normal(700))
    imax, imin = oracle.extrema(h)
    for idx in (imax, imin):
        env = oracle.envelope(h, idx)
        assert np.abs(env[idx] - h[idx]).max() <= 1e-12 * np.abs(h).max()
        t, y = _mirrored_knots(h, list(idx))
        want = CubicSpline(t, y, bc_type="natural")(np.arange(h.size, dtype=float))
        assert np.abs(env - want).max() <= 1e-12 * np.abs(h).max()


def test_envelope_single_extremum():
    h = np.array([0.0, 1, 3, 2, 1, 0.5, 0.25, 0.1])
    env = oracle.envelope(h, np.array([2]))
    # knots -2, 2, 12 all at 3.0: a natural spline through equal values is flat
    assert np.all(env == 3.0)


# --------------------------------------------------------------------------
# Sec. 2.1 Steps 1-5 -- EMD
# --------------------------------------------------------------------------

def _on_grid_cosine(L):
    s = math.sqrt(0.5)
    table = np.array([1.0, s, 0.0, -s, -1.0, -s, 0.0, s])
    return table[np.arange(L) % 8]


@pytest.mark.parametrize("L", [41, 81, 8 * 125 + 1])
def test_on_grid_cosine_is_one_imf_exactly(L):
    # Every maximum is 1, every minimum -1 and all knot gaps are 8 or 16, so
    # both envelopes are exactly flat, the mean is exactly 0 and the sinusoid
    # comes back unchanged as a single IMF with an exactly zero residue.
    x = _on_grid_cosine(L)
    out, n = oracle.emd(x, 6, 10)
    assert n == 1
    assert np.array_equal(out[0], x)
    assert np.all(out[1:6] == 0.0)
    assert np.all(out[6] == 0.0)


def test_off_grid_sinusoid_energy_in_first_imf():
    k = np.arange(4096)
    x = np.sin(2 * math.pi * k / 37.3 + 0.4)
    out, n = oracle.emd(x, 6, 10)
    assert n >= 1
    assert np.sum(out[0] ** 2) >= 0.999 * np.sum(x ** 2)


def test_monotone_input_has_no_imf():
    x = np.linspace(-3.0, 5.0, 300) ** 3
    out, n = oracle.emd(x, 6, 10)
    assert n == 0
    assert np.array_equal(out[6], x)
    assert np.all(out[:6] == 0.0)


def test_reconstruction():
    rng = np.random.default_rng(31)
    for L in (50, 777, 3000):
        x = np.cumsum(rng.standard_normal(L)) + rng.standard_normal(L)
        out, n = oracle.emd(x, 8, 10)
        assert 1 <= n <= 8
        assert np.abs(out.sum(0) - x).max() <= 1e-12 * np.abs(x).max()


def test_sign_and_power_of_two_scale_are_exact():
    rng = np.random.default_rng(32)
    x = rng.standard_normal(1500) + np.sin(np.arange(1500) / 9.0)
    out, n = oracle.emd(x, 6, 10)
    neg, nn = oracle.emd(-x, 6, 10)
    two, n2 = oracle.emd(4.0 * x, 6, 10)
    assert n == nn == n2
    assert np.array_equal(neg, -out)
    assert np.array_equal(two, 4.0 * out)


def test_time_reversal_symmetry():
    rng = np.random.default_rng(33)
    x = rng.standard_normal(1200) + 2 * np.sin(np.arange(1200) / 31.0)
    out, n = oracle.emd(x, 6, 10)
    rev, nr = oracle.emd(x[::-1].copy(), 6, 10)
    assert n == nr
    assert np.abs(rev[:, ::-1] - out).max() <= 1e-10 * np.abs(x).max()


def test_serial_decompose_reconstructs_input_samples():
    rng = np.random.default_rng(34)
    M, N, D = 200, 4, 40
    X = rng.standard_normal(M * N).cumsum()
    out, n = oracle.decompose(X, M, N, D, 6, 10)
    assert np.abs(out.sum(0) - X).max() <= 1e-12 * np.abs(X).max()


def test_slices_match_single_column_serial():
    rng = np.random.default_rng(35)
    M, N = 300, 3
    X = rng.standard_normal(M * N)
    out, n = oracle.decompose_slices(X, M, N, 6, 10)
    for c in range(N):
        one, n1 = oracle.decompose(X[c * M:(c + 1) * M], M, 1, 0, 6, 10)
        assert n1 == n[c]
        assert np.array_equal(one, out[:, c * M:(c + 1) * M])


# --------------------------------------------------------------------------
# Sec. 2.2 -- EEMD noise and ensemble
# --------------------------------------------------------------------------

def test_splitmix64_published_vectors():
    # Reference outputs of SplitMix64 for state 0 and state 1234567.
    assert oracle.splitmix64(0, 1) == 0xE220A8397B1DCDAF
    assert oracle.splitmix64(0, 2) == 0x6E789E6AA1B965F4
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [oracle.splitmix64(1234567, n) for n in range(1, 6)] == want


def test_noise_moments_and_determinism():
    w = oracle.noise(99, 3, 5, 200_000)
    assert abs(w.mean()) < 3 / math.sqrt(w.size)
    assert abs(w.var() - 1.0) < 3 * math.sqrt(2.0 / w.size) * 1.2
    assert np.abs(w).max() <= 6.0
    assert np.array_equal(w, oracle.noise(99, 3, 5, 200_000))
    assert not np.array_equal(w[:100], oracle.noise(99, 3, 6, 100))
    assert not np.array_equal(w[:100], oracle.noise(99, 4, 5, 100))


def test_eemd_identity():
    rng = np.random.default_rng(41)
    M, N, D, K, NR = 150, 3, 10, 6, 8
    X = rng.standard_normal(M * N).cumsum()
    x = oracle.serialize(X, M, N, D)
    beta = 0.2 * x.std()
    out = oracle.eemd(X, M, N, D, K, 10, NR, beta, 7, 2)
    L = x.size
    wbar = np.zeros(L)
    for m in range(NR):
        wbar += beta * oracle.noise(7, 2, m, L)
    wbar /= NR
    lhs = out.sum(0) - X
    rhs = oracle.deserialize(wbar, M, N, D)
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(X).max()


def test_eemd_single_noiseless_realization_is_emd():
    rng = np.random.default_rng(42)
    M, N, D = 120, 2, 20
    X = rng.standard_normal(M * N)
    e = oracle.eemd(X, M, N, D, 5, 10, 1, 0.0, 1, 0)
    d, _ = oracle.decompose(X, M, N, D, 5, 10)
    assert np.array_equal(e, d)


def test_two_extrema_residue_is_not_sifted():
    # IMF-loop stop reading: a residue with one maximum and one minimum (fewer
    # than 3 extrema) is left as the residue, untouched.
    L = 400
    x = np.sin(2 * math.pi * np.arange(L) / (L - 1)) + 0.001 * np.arange(L)
    imax, imin = oracle.extrema(x)
    assert len(imax) == 1 and len(imin) == 1
    out, n = oracle.emd(x, 6, 10)
    assert n == 0 and np.array_equal(out[6], x)
    # three extrema are enough to be sifted
    x3 = np.sin(2 * math.pi * np.arange(L) / (L - 1) * 1.3)
    imax, imin = oracle.extrema(x3)
    assert len(imax) + len(imin) == 3
    assert oracle.emd(x3, 6, 10)[1] >= 1


def test_noise_stream_definition():
    # Stream layout of this library (a convention, not the paper's): stream key
    # s2 = SM(SM(seed, item+1), m+1); sample k sums the 12 outputs
    # SM(s2, 12k+1..12k+12) >> 11 as integers, subtracts 6*2^53, converts to
    # double once and scales by 2^-53.  SM(s, n) is the n-th SplitMix64 output.
    MASK = 2**64 - 1

    def sm(s, n):
        z = (s + n * 0x9E3779B97F4A7C15) & MASK
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    seed, item, m = 12345, 6, 7
    s2 = sm(sm(seed, item + 1), m + 1)
    want = []
    for k in range(4):
        acc = sum(sm(s2, 12 * k + j + 1) >> 11 for j in range(12))
        want.append(float(acc - 6 * 2**53) * 2.0**-53)
    assert list(oracle.noise(seed, item, m, 4)) == want


# ---------------------------------------------------------------------------
# SD stopping rule (Step 5 criterion left open by Sec. 2.1; Huang et al. 1998)
# ---------------------------------------------------------------------------

def _one_sift(h):
    """One sift by the pinned envelope routine: (new candidate, m)."""
    imax, imin = oracle.extrema(h)
    m = 0.5 * (oracle.envelope(h, imax) + oracle.envelope(h, imin))
    return h - m, m


def test_sd_rule_limits_reduce_to_fixed_counts():
    x = workloads.config0().X[:1000]
    fixed, nf = oracle.emd(x, 6, 10)
    tiny, nt = oracle.emd(x, 6, 10, sd=1e-300)   # never below: all S sifts
    assert nt == nf and tiny.tobytes() == fixed.tobytes()
    one, n1 = oracle.emd(x, 6, 1)
    huge, nh = oracle.emd(x, 6, 10, sd=1e300)    # always below: one sift per IMF
    assert nh == n1 and huge.tobytes() == one.tobytes()


def test_sd_rule_stops_at_the_first_sift_below_the_threshold():
    # SD of each sift of the first IMF computed here with numpy; thresholds
    # placed between consecutive SD values stop the IMF after that sift
    x = workloads.config0().X[:1000]
    h = x.copy()
    sds, hs = [], []
    for _ in range(6):
        h_new, m = _one_sift(h)
        sds.append(float(np.sum(m * m) / np.sum(h * h)))
        h = h_new
        hs.append(h.copy())
    assert all(sds[i] > sds[i + 1] for i in range(5))  # this signal converges monotonically
    for stop in range(1, 5):
        thr = 0.5 * (sds[stop - 1] + sds[stop])       # sift stop+1 is the first below
        out, n = oracle.emd(x, 1, 10, sd=thr)
        assert n == 1
        np.testing.assert_allclose(out[0], hs[stop], rtol=0, atol=1e-12 * np.abs(x).max())


def test_sd_margin_reports_the_closest_decision():
    # the margin of the stopping tests: infinite without the SD rule; with a
    # threshold placed between two consecutive SD values, the distance of
    # the nearer one relative to the threshold
    x = workloads.config0().X[:1000]
    _, _, st = oracle.emd(x, 1, 10, with_stats=True)
    assert st["sd_margin"] == float("inf")
    h = x.copy()
    sds = []
    for _ in range(3):
        h_new, m = _one_sift(h)
        sds.append(float(np.sum(m * m) / np.sum(h * h)))
        h = h_new
    thr = 0.5 * (sds[1] + sds[2])  # the IMF ends after its third sift
    _, n, st = oracle.emd(x, 1, 10, with_stats=True, sd=thr)
    assert n == 1 and st["n_sifts"] == 3
    want = min(abs(s - thr) / thr for s in sds)
    assert abs(st["sd_margin"] - want) <= 1e-9 * want


def test_sd_rule_in_slices_and_ensemble():
    # slice-wise EMD with the SD rule is the SD-rule EMD of each column; an
    # ensemble of one noiseless realization is the plain SD-rule decomposition
    it = workloads.config0()
    M, N, K, S, thr = it.M, it.N, 6, 10, 0.2
    out, n = oracle.decompose_slices(it.X, M, N, K, S, sd=thr)
    for c in range(N):
        col, nc = oracle.emd(it.X[c * M:(c + 1) * M], K, S, sd=thr)
        assert n[c] == nc
        assert out[:, c * M:(c + 1) * M].tobytes() == col.tobytes()
    ens = oracle.eemd(it.X, M, N, 20, K, S, 1, 0.0, 7, sd=thr)
    plain, _ = oracle.decompose(it.X, M, N, 20, K, S, sd=thr)
    assert ens.tobytes() == plain.tobytes()
    fixed, _ = oracle.decompose(it.X, M, N, 20, K, S)
    assert plain.tobytes() != fixed.tobytes()  # the rule does stop early here


# --------------------------------------------------------------------------
# CEEMDAN (Sec. 2.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("sd", [0.0, 0.2])
def test_ceemdan_without_noise_is_emd(sd):
    # eps = 0, NR = 1: every stage takes the first mode of the residue
    # itself, which is exactly how EMD peels its modes off
    it = workloads.config0()
    ref, nr = oracle.decompose(it.X, it.M, it.N, 50, 6, 10, sd=sd)
    out, n = oracle.ceemdan(it.X, it.M, it.N, 50, 6, 10, 1, 0.0, 3, 0, sd=sd)
    assert n == nr
    assert out.tobytes() == ref.tobytes()


def test_ceemdan_is_complete_and_scale_equivariant():
    it = workloads.config0()
    M, N = it.M, it.N
    out, n = oracle.ceemdan(it.X, M, N, 20, 6, 10, 6, 0.2, 11, 2)
    assert 2 <= n <= 6
    assert np.all(out[n:6] == 0.0)
    assert np.abs(out.sum(0) - it.X).max() <= 1e-12 * np.abs(it.X).max()
    # the noise amplitude follows the residue's spread, so scaling the input
    # by a power of two scales every mode exactly
    big, nb = oracle.ceemdan(it.X * 8.0, M, N, 20, 6, 10, 6, 0.2, 11, 2)
    assert nb == n and big.tobytes() == (out * 8.0).tobytes()


def test_ceemdan_monotone_input_has_no_mode():
    x = np.linspace(-2.0, 3.0, 500) ** 3
    out, n = oracle.ceemdan(x, 500, 1, 0, 4, 10, 4, 0.2, 1, 0)
    assert n == 0
    assert np.array_equal(out[4], x) and np.all(out[:4] == 0.0)


def test_ceemdan_first_stage_is_the_ensemble_first_mode():
    # stage 1 is the EEMD first mode with beta = eps * std(x)
    it = workloads.config0()
    M, N, D, eps = it.M, it.N, 50, 0.2
    x = oracle.serialize(it.X, M, N, D)
    beta = eps * float(np.sqrt(np.mean((x - np.mean(x)) ** 2)))
    out, n = oracle.ceemdan(it.X, M, N, D, 1, 10, 5, eps, 9, 4)
    ee = oracle.eemd(it.X, M, N, D, 1, 10, 5, beta, 9, 4)
    assert n == 1
    assert np.abs(out[0] - ee[0]).max() <= 1e-12 * np.abs(it.X).max()


def test_ceemdan_second_stage_uses_the_first_noise_mode():
    # Sec. 2.2 CEEMDAN Step 3 for i = 2: c_2 is the ensemble mean of the first
    # mode of r_1 + beta_1 E_1(w_m), where r_1 = x - c_1, beta_1 = eps std(r_1)
    # and E_1(w_m) is the first mode of the EMD of noise realization m.
    L, S, NR, eps, seed, item = 600, 10, 4, 0.2, 5, 1
    k = np.arange(L)
    x = (np.sin(2 * np.pi * k / 9.5) + 0.6 * np.sin(2 * np.pi * k / 47.0)
         + 0.3 * np.cos(2 * np.pi * k / 173.0))
    out, n = oracle.ceemdan(x, L, 1, 0, 2, S, NR, eps, seed, item)
    assert n == 2
    r1 = x - out[0]
    beta1 = eps * float(np.sqrt(np.mean((r1 - np.mean(r1)) ** 2)))
    acc = np.zeros(L)
    for m in range(NR):
        e1 = oracle.emd(oracle.noise(seed, item, m, L), 1, S)[0][0]
        acc += oracle.emd(r1 + beta1 * e1, 1, S)[0][0]
    assert np.abs(out[1] - acc / NR).max() <= 1e-12 * np.abs(x).max()
    assert np.abs(out[2] - (r1 - out[1])).max() <= 1e-13 * np.abs(x).max()


def test_trace_records_every_detection_of_the_sifting_loop():
    """The oracle's decision trace replays Sec. 2.1 Steps 1-5 as assembled
    here from its pinned primitives (extrema, envelope): one record per
    detection -- the residue's before each IMF, the candidate's before each
    later sift -- with the same index sets, and the tested arrays bit-equal."""
    rng = np.random.default_rng(8)
    x = np.cumsum(rng.standard_normal(700)) + 2.0 * np.sin(np.arange(700) / 5.0)
    K, S = 4, 3
    slots, n, recs, complete = oracle.emd_trace(x, K, S)
    ref, nr = oracle.emd(x, K, S)
    assert complete and n == nr and np.array_equal(slots, ref)
    want, tested = [], {}
    r = x.copy()
    for i in range(K):
        mx, mn = oracle.extrema(r)
        want.append((i, 0, mx, mn))
        tested[(i, 0)] = r.copy()
        if not (len(mx) >= 1 and len(mn) >= 1 and len(mx) + len(mn) >= 3):
            break
        h = r.copy()
        for s in range(S):
            if s > 0:
                mx, mn = oracle.extrema(h)
                want.append((i, s, mx, mn))
                tested[(i, s)] = h.copy()
                if not (len(mx) >= 1 and len(mn) >= 1 and len(mx) + len(mn) >= 3):
                    break
            up, lo = oracle.envelope(h, mx), oracle.envelope(h, mn)
            h = h - 0.5 * (up + lo)
        r = r - h
    assert len(recs) == len(want)
    for (i, s, a, b), (wi, ws, wa, wb) in zip(recs, want):
        assert (i, s) == (wi, ws)
        assert np.array_equal(a, wa) and np.array_equal(b, wb)
        assert np.array_equal(oracle.emd_tested(x, K, S, i, s), tested[(i, s)])
    assert oracle.emd_tested(x, K, S, K + 1, 0) is None
    # a buffer too small for the second record keeps only the first
    first = 4 + len(recs[0][2]) + len(recs[0][3])
    _, _, part, complete = oracle.emd_trace(x, K, S, cap=first + 3)
    assert not complete and len(part) == 1


def test_decision_comparator_classifies_ties_and_failures():
    """The parity comparator: equal records pass; a differing position whose
    tested value is within 1e-12 * max|x| of a neighbour is a tie; a clear
    difference, or an IMF ending elsewhere without an SD tie, fails."""
    import parity
    h = np.array([0.0, 1.0, 0.5, 2.0, 2.0 + 1e-15, 1.0, 3.0, 0.0])
    rec = [(0, 0, np.array([1, 4]), np.array([2, 5]))]
    tested = lambda i, s: h  # noqa: E731
    assert parity.compare_decisions(rec, rec, tested, 3.0)["status"] == "equal"
    # GPU saw the maximum at 3 instead of 4: positions 3 and 4 sit in a near-equal pair
    g = [(0, 0, np.array([1, 3]), np.array([2, 5]))]
    res = parity.compare_decisions(g, rec, tested, 3.0)
    assert res["status"] == "tie" and res["positions"] == [3, 4]
    # GPU missed the maximum at 1, whose steps are 1.0 and 0.5: a failure
    g = [(0, 0, np.array([4]), np.array([2, 5]))]
    assert parity.compare_decisions(g, rec, tested, 3.0)["status"] == "fail"
    # equal-valued run: the margin is taken at the run's outer steps
    hp = np.array([0.0, 1.0, 1.0, 1.0, 0.0])
    assert parity.margin(hp, 2, 1.0) == 1.0
    # an IMF ending at another sift is a tie only at an SD tie
    a = [(0, 0, np.array([1]), np.array([2])), (0, 1, np.array([1]), np.array([2]))]
    b = [(0, 0, np.array([1]), np.array([2])), (1, 0, np.array([1]), np.array([2]))]
    assert parity.compare_decisions(a, b, tested, 3.0, sd_margin=1e-12)["status"] == "tie"
    assert parity.compare_decisions(a, b, tested, 3.0, sd_margin=1e-3)["status"] == "fail"
    assert parity.compare_decisions(a, a[:1], tested, 3.0)["status"] == "fail"
    # the device trace layout: used, complete, 2 spare, then records
    buf = np.array([4 + 6, 1, 0, 0, 0, 0, 1, 1, 7, 9], dtype=np.int32)
    recs, complete = parity.parse_trace(buf)
    assert complete and len(recs) == 1 and list(recs[0][2]) == [7] and list(recs[0][3]) == [9]
