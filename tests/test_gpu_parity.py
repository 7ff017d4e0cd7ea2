"""HIP path against the CPU oracle, element by element, through the C ABI.

Sizes span several thread blocks and ragged tails; the tolerance for every
floating-point output is 1e-8 * max|x| (integer and index outputs, the
serialization, deserialization and noise must be bit-exact)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2106_15319_amd as semd
import workloads
import parity
from parity import SD_TIE, TOL, Tally

pytestmark = pytest.mark.gpu

DEV = "cuda"
ONCHIP_ = semd.SEMD_PATH_ONCHIP
STREAM_ = semd.SEMD_PATH_STREAM


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def assert_same(a, b, what=""):
    """Bit-identical arrays (reported by their largest difference)."""
    a, b = np.asarray(a), np.asarray(b)
    assert a.shape == b.shape, (what, a.shape, b.shape)
    if a.tobytes() != b.tobytes():
        d = np.abs(a.astype(np.float64) - b.astype(np.float64))
        raise AssertionError(f"{what}: not bit-identical, max |diff| = {np.nanmax(d):.3e}, "
                             f"{int(np.count_nonzero(d))} of {d.size} differ")


# --------------------------------------------------------------------------
# single steps
# --------------------------------------------------------------------------

@pytest.mark.parametrize("M,N,D", [(4, 2, 2), (1000, 3, 0), (1000, 3, 50), (112, 92, 20),
                                   (128, 128, 26), (7, 5, 7), (1, 9, 1), (33, 1, 0)])
def test_serialize_deserialize_bit_exact(M, N, D):
    rng = np.random.default_rng(M * 7 + N + D)
    X = rng.standard_normal(M * N) * 10.0 ** rng.integers(-5, 5, M * N)
    x = host(semd.semd_serialize(dev(X), [M, N], D))
    want = oracle.serialize(X, M, N, D)
    assert_same(x, want, "serialize")
    y = rng.standard_normal(want.size)
    back = host(semd.semd_deserialize(dev(y), [M, N], D))
    assert_same(back, oracle.deserialize(y, M, N, D), "deserialize")


def test_noise_bit_exact_million_draws():
    for (seed, item, m) in [(0, 0, 0), (2106_15319, 17, 63)]:
        w = host(semd.semd_noise(seed, item, m, 1_000_000))
        assert_same(w, oracle.noise(seed, item, m, 1_000_000), "noise")


def _plateau_signal(rng, L):
    h = np.round(rng.standard_normal(L) * 2.0)
    # long flat runs across many 16-sample blocks, touching and not touching ends
    for _ in range(4):
        a = int(rng.integers(0, L))
        b = min(L, a + int(rng.integers(1, 400)))
        h[a:b] = h[a]
    return h


@pytest.mark.parametrize("L", [3, 4, 5, 17, 31, 1000, 4095, 4096, 4097, 10304, 16383, 16384])
def test_extrema_identical_index_sets(L):
    rng = np.random.default_rng(L)
    for h in (rng.standard_normal(L), _plateau_signal(rng, L), np.zeros(L),
              np.arange(L, dtype=float), np.cos(np.arange(L) * 2.1)):
        imax, imin = semd.semd_extrema(dev(h))
        rmax, rmin = oracle.extrema(h)
        assert np.array_equal(imax.cpu().numpy(), rmax)
        assert np.array_equal(imin.cpu().numpy(), rmin)


def test_extrema_constant_blocks_across_threads():
    # runs that cover whole 16-sample blocks and start inside another block
    L = 8000
    h = np.zeros(L)
    h[1000:1700] = 5.0   # max plateau spanning ~44 blocks
    h[3000:3333] = -2.0  # min plateau
    h[5000:] = 1.0       # run touching the end: not an extremum
    h[0:37] = 3.0        # run touching the start: not an extremum
    imax, imin = semd.semd_extrema(dev(h))
    rmax, rmin = oracle.extrema(h)
    assert np.array_equal(imax.cpu().numpy(), rmax) and np.array_equal(imin.cpu().numpy(), rmin)
    # the zero run 37..999 between 3 and 5 is a minimum plateau too
    assert list(rmax) == [1349] and list(rmin) == [518, 3166]


@pytest.mark.parametrize("L", [50, 1001, 4096, 9999, 16384])
def test_single_sift(L):
    rng = np.random.default_rng(100 + L)
    x = np.cumsum(rng.standard_normal(L)) + 3 * np.sin(np.arange(L) / 7.0)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 1, 1)
    tally = Tally(f"single sift L={L}")
    _check_item(x, L, 1, 0, 1, 1, host(out), int(host(n)[0]), tally)
    tally.done()


# --------------------------------------------------------------------------
# whole decompositions
# --------------------------------------------------------------------------

def _decision_cases():
    """(name, X, M, N, D, K, S, sd) inputs for the per-detection comparison:
    the configured workloads' shapes, uint8 plateaus, plateaus across tiles,
    white noise (the densest knot sets), the SD rule."""
    c0 = workloads.config0()
    face = workloads.config2(1)[0]
    tex = workloads.config1(1)[0]
    L = 20000
    plat = np.zeros(L)
    plat[3000:9000] = 5.0
    plat[9500:15000] = -3.0
    plat += 0.25 * np.sin(np.arange(L) / 900.0) * (np.arange(L) % 4096 < 100)
    noise = np.random.default_rng(91).standard_normal(12000)
    long_it = workloads.config3_item(2, (30000, 3))
    return [("config0 D=0", c0.X, 1000, 3, 0, 6, 10, 0.0),
            ("config0 D=50", c0.X, 1000, 3, 50, 6, 10, 0.0),
            ("face D=0", face.X, 112, 92, 0, 8, 10, 0.0),
            ("face D=20", face.X, 112, 92, 20, 8, 10, 0.0),
            ("texture 128 D=0", tex.X, 128, 128, 0, 8, 10, 0.0),
            ("plateaus", plat, L, 1, 0, 4, 4, 0.0),
            ("white noise", noise, 12000, 1, 0, 3, 4, 0.0),
            ("series 30000x3", long_it.X, 30000, 3, 0, 6, 10, 0.0),
            ("config0 SD 0.05", c0.X, 1000, 3, 50, 8, 30, 0.05)]


# every case on the streaming path, and on chip where the serialized length fits
_DECISION_RUNS = [(c, STREAM_) for c in range(9)] + \
    [(c, ONCHIP_) for c in (0, 1, 2, 3, 4, 6, 8)]


@pytest.mark.parametrize("case,path", _DECISION_RUNS)
def test_extremum_decisions_equal_oracle_every_detection(case, path):
    """Every extremum detection of the decomposition (the residue's before
    each IMF and the candidate's before each sift) has the oracle's maxima
    and minima, position for position, on both paths; a difference is
    accepted only as a reported tie.  The recorded run is the compared one:
    its outputs equal semd_decompose_ex's (bit for bit on the streaming
    path; on chip the recording shape may associate differently, so to
    rounding) and the oracle's within the output bound."""
    name, X, M, N, D, K, S, sd = _decision_cases()[case]
    L = M * N + D * N - D
    assert path == STREAM_ or L <= semd.semd_resident_max_length()
    print(f"case {name} path {path} L {L}", flush=True)
    out_t, n_t, tr = semd.semd_decompose_trace(dev(X), [M, N], D, K, S, path=path, sd=sd)
    recs, complete = parity.parse_trace(host(tr))
    assert complete
    out, n = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path, sd=sd)
    assert int(host(n_t)[0]) == int(host(n)[0])
    if path == STREAM_:
        assert_same(host(out_t), host(out), "recorded run vs plain run")
    else:
        assert np.abs(host(out_t) - host(out)).max() <= 1e-12 * np.abs(X).max()
    x = oracle.serialize(X, M, N, D)
    _, nr, ref_recs, ok = oracle.emd_trace(x, K, S, sd=sd)
    assert ok
    st = oracle.emd(x, K, S, with_stats=True, sd=sd)[2]
    res = parity.compare_decisions(recs, ref_recs,
                                   lambda i, s: oracle.emd_tested(x, K, S, i, s, sd=sd),
                                   float(np.abs(X).max()),
                                   st["sd_margin"] if sd > 0 else float("inf"))
    tally = Tally(f"decisions {name} path={path}")
    if res["status"] == "tie":
        tally.tie(name, res)
    else:
        assert res["status"] == "equal", res
        assert len(recs) == len(ref_recs)
        print(f"{name}: {len(recs)} detections, "
              f"{sum(len(r[2]) + len(r[3]) for r in recs)} extrema, all equal", flush=True)
        _check_item(X, M, N, D, K, S, host(out_t), int(host(n_t)[0]), tally, path=path, sd=sd)
    tally.done()

def _gpu_trace(x, K, S, path=semd.SEMD_PATH_AUTO, sd=0.0):
    """Detection records of the GPU's decomposition of the serialized 1D x."""
    L = x.size
    _, _, tr = semd.semd_decompose_trace(dev(x), [L, 1], 0, K, S, path=path, sd=sd)
    recs, complete = parity.parse_trace(host(tr))
    assert complete, "trace buffer too small"
    return recs


def _diagnose(x, K, S, path, sd, xmax):
    """Where the GPU's and the oracle's extremum decisions on the serialized
    x first part, and whether that is a tie (parity.compare_decisions)."""
    recs = _gpu_trace(x, K, S, path, sd)
    _, _, ref_recs, complete = oracle.emd_trace(x, K, S, sd=sd)
    assert complete
    st = oracle.emd(x, K, S, with_stats=True, sd=sd)[2]
    return parity.compare_decisions(
        recs, ref_recs, lambda i, s: oracle.emd_tested(x, K, S, i, s, sd=sd), xmax,
        st["sd_margin"] if sd > 0 else float("inf"))


def _check_item(X, M, N, D, K, S, out, n, tally, path=semd.SEMD_PATH_AUTO, sd=0.0, what="",
                stats=None):
    """One decomposition against the oracle's: outputs within TOL * max|x|
    and equal IMF counts, else the extremum decisions are compared detection
    by detection and the first difference must be a tie (reported)."""
    ref, nr, st = oracle.decompose(X, M, N, D, K, S, with_stats=True, sd=sd)
    xmax = float(np.abs(X).max()) if X.size else 0.0
    ok, err = parity.outputs_match(out, n, ref, nr, xmax)
    label = what or f"M={M} N={N} D={D} K={K} S={S} sd={sd}"
    if ok:
        if stats is not None:
            assert int(stats[0]) == st["n_sifts"], (label, int(stats[0]), st["n_sifts"])
        return {"ok": True, "tie": False, "err": err, "n": nr, "stats": st}
    res = _diagnose(oracle.serialize(X, M, N, D), K, S, path, sd, xmax)
    if res["status"] == "tie":
        tally.tie(label, res)
        return {"ok": False, "tie": True, "err": err, "n": nr, "stats": st}
    raise AssertionError(f"{label}: outputs differ (max err {err:.3g} vs bound "
                         f"{TOL * xmax:.3g}, n_imfs {n} vs {nr}); decisions: {res}")


@pytest.mark.parametrize("D", [0, 50])
def test_config0_series(D):
    it = workloads.config0()
    out, n = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], D, 6, 10)
    tally = Tally(f"config 0 series D={D}")
    _check_item(it.X, it.M, it.N, D, 6, 10, host(out), int(host(n)[0]), tally)
    tally.done()
    assert int(host(n)[0]) >= 3


@pytest.mark.parametrize("D", [0, 20])
def test_config2_faces_batch_subset(D):
    items = workloads.config2(12)
    Xs = [dev(i.X) for i in items]
    outs, counts = semd.decompose_batch(Xs, [(i.M, i.N) for i in items], D, 8, 10)
    counts = host(counts)
    tally = Tally(f"config 2 faces D={D}", max_ties=1)
    for k, i in enumerate(items):
        _check_item(i.X, i.M, i.N, D, 8, 10, host(outs[k]), int(counts[k]), tally,
                    what=f"face {k} D={D}")
    tally.done()


def test_config2_full_face_batch_sampled():
    """The face batch at its full size in the launch configuration the bench
    times (1,024 images of 112x92, D = 0, K = 8, S = 10, one batched launch
    through prepared descriptors): 16 images spread over the batch against
    the oracle element by element, and for every image the IMF count in
    range, the unused slots zero and the slots summing back to the input."""
    K, S = 8, 10
    items = workloads.config2(1024)
    M, N = items[0].M, items[0].N
    n = len(items)
    X = torch.from_numpy(np.stack([it.X for it in items])).to(DEV)
    out = torch.empty((n, K + 1, M * N), dtype=torch.float64, device=DEV)
    counts = torch.zeros(n, dtype=torch.int32, device=DEV)
    semd.PreparedBatch([X[i] for i in range(n)], [[M, N]] * n, [out[i] for i in range(n)],
                       counts, 0, K, S).run()
    cnt = host(counts)
    assert cnt.min() >= 1 and cnt.max() <= K
    # slots n_imfs .. K-1 zero, all slots summing back to the input
    slot = torch.arange(K, device=DEV).view(1, K, 1)
    unused = slot >= counts.view(n, 1, 1).long()
    assert float((out[:, :K] * unused).abs().max()) == 0.0
    xmax = X.abs().amax(dim=1)
    recon = (out.sum(dim=1) - X).abs().amax(dim=1)
    assert bool((recon <= 1e-12 * xmax).all()), float((recon / xmax).max())
    rng = np.random.default_rng(2106)
    pick = sorted(set([0, 1, 255, 256, 511, 512, 767, n - 1] +
                      rng.choice(n, 8, replace=False).tolist()))
    tally = Tally("config 2 full batch", max_ties=1)
    o = host(out[pick])
    for j, i in enumerate(pick):
        _check_item(items[i].X, M, N, 0, K, S, o[j], int(cnt[i]), tally, what=f"face {i}")
    tally.done()


@pytest.mark.parametrize("D", [0, 26])
def test_config1_textures_subset(D):
    """Config 1 textures (128 x 128), at D = 0 and at the paper's 20 % of
    the side (D = 26, L = 19,686: streaming path)."""
    items = workloads.config1(4)
    tally = Tally(f"config 1 textures D={D}", max_ties=1)
    for k, i in enumerate(items):
        out, n = semd.semd_decompose_ex(dev(i.X), [i.M, i.N], D, 8, 10)
        _check_item(i.X, i.M, i.N, D, 8, 10, host(out), int(host(n)[0]), tally,
                    what=f"texture {k} D={D}")
    tally.done()


def test_batch_equals_plain_bit_exact():
    items = workloads.config2(3) + workloads.config1(1, size=64)
    shapes = [(i.M, i.N) for i in items]
    Xs = [dev(i.X) for i in items]
    outs, counts = semd.decompose_batch(Xs, shapes, 10, 8, 10)
    for k, i in enumerate(items):
        o, n = semd.semd_decompose_ex(Xs[k], [i.M, i.N], 10, 8, 10)
        assert_same(host(o), host(outs[k]), "batch vs plain")
        assert int(host(n)[0]) == int(host(counts)[k])


def test_uneven_batch_mixed_lengths():
    rng = np.random.default_rng(5)
    shapes = [(int(m), int(c)) for m, c in zip(rng.integers(3, 2000, 9), rng.integers(1, 8, 9))]
    shapes = [(M, N) for (M, N) in shapes if M * N <= 16384] + [(16384, 1), (5, 1), (2, 1)]
    Xs = [workloads.series(workloads.rng_for(9, k), N, M) for k, (M, N) in enumerate(shapes)]
    outs, counts = semd.decompose_batch([dev(x) for x in Xs], shapes, 0, 6, 10)
    counts = host(counts)
    tally = Tally("uneven batch", max_ties=1)
    for k, (M, N) in enumerate(shapes):
        _check_item(Xs[k], M, N, 0, 6, 10, host(outs[k]), int(counts[k]), tally)
    tally.done()


@pytest.mark.parametrize("path,M,N,D", [(semd.SEMD_PATH_ONCHIP, 1000, 3, 50),
                                         (semd.SEMD_PATH_STREAM, 1000, 3, 50),
                                         (semd.SEMD_PATH_AUTO, 20000, 2, 0),
                                         (semd.SEMD_PATH_AUTO, 16384, 1, 0)])
def test_caller_workspace_matches_library_workspace(path, M, N, D):
    """semd_decompose_ex with a caller's workspace (filled with garbage
    first, then reused dirty) gives bit-identical outputs to the
    library-allocated one, and both match the oracle; an undersized
    workspace is refused."""
    K, S = 6, 10
    X = workloads.series(workloads.rng_for(21, M + N), N, M)
    need = semd.semd_workspace_bytes([M, N], D, K, S, path=path)
    ws = torch.full((need,), 0xA5, dtype=torch.uint8, device=DEV)
    assert ws.data_ptr() % 256 == 0
    a, na = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path)
    b, nb = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path, workspace=ws)
    c, nc = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path, workspace=ws)
    assert_same(host(a), host(b), "caller workspace")
    assert_same(host(a), host(c), "reused workspace")
    assert int(host(na)[0]) == int(host(nb)[0]) == int(host(nc)[0])
    tally = Tally(f"caller workspace path={path} M={M} N={N}")
    _check_item(X, M, N, D, K, S, host(b), int(host(nb)[0]), tally, path=path)
    tally.done()
    with pytest.raises(semd.SemdError) as ei:
        semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path, workspace=ws[:need - 256])
    assert ei.value.code == semd.SEMD_EINVAL


def test_determinism():
    it = workloads.config2(1)[0]
    a, _ = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], 20, 8, 10)
    b, _ = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], 20, 8, 10)
    assert_same(host(a), host(b), "determinism")


# --------------------------------------------------------------------------
# edge cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [1, 2, 3])
def test_tiny_signals(L):
    x = np.array([1.0, -2.0, 0.5][:L])
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 4, 10)
    ref, nr = oracle.emd(x, 4, 10)
    assert int(host(n)[0]) == nr == 0
    assert np.array_equal(host(out), ref)


def test_monotone_and_on_grid_cosine():
    x = np.linspace(-3.0, 5.0, 300) ** 3
    out, n = semd.semd_decompose_ex(dev(x), [300, 1], 0, 6, 10)
    assert int(host(n)[0]) == 0 and np.array_equal(host(out)[6], x)
    s = math.sqrt(0.5)
    L = 8 * 700 + 1
    c = np.array([1.0, s, 0.0, -s, -1.0, -s, 0.0, s])[np.arange(L) % 8]
    out, n = semd.semd_decompose_ex(dev(c), [L, 1], 0, 6, 10)
    o = host(out)
    assert int(host(n)[0]) == 1
    assert np.abs(o[0] - c).max() <= 1e-12 and np.abs(o[6]).max() <= 1e-12


def test_non_finite_input_reported():
    x = np.ones(500)
    x[123] = np.nan
    out, n = semd.semd_decompose_ex(dev(x), [500, 1], 0, 3, 10)
    assert int(host(n)[0]) == -semd.SEMD_ENONFINITE
    assert np.all(host(out) == 0.0)


def test_largest_resident_signal():
    L = semd.semd_resident_max_length()
    rng = np.random.default_rng(77)
    x = rng.standard_normal(L)  # white noise: the densest knot sets
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 3, 4)
    tally = Tally("white noise at the largest resident length")
    _check_item(x, L, 1, 0, 3, 4, host(out), int(host(n)[0]), tally)
    tally.done()


def test_alternating_signal_worst_case_knots():
    L = 16384
    k = np.arange(L)
    x = np.where(k % 2 == 0, 1.0, -1.0) * (1.0 + 0.001 * np.sin(k / 50.0))
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 2, 2)
    tally = Tally("alternating signal")
    _check_item(x, L, 1, 0, 2, 2, host(out), int(host(n)[0]), tally)
    tally.done()


# --------------------------------------------------------------------------
# EEMD
# --------------------------------------------------------------------------

def _realization(X, M, N, D, beta, seed, item, m):
    """Serialized input of EEMD realization m, x + beta * w_m (Sec. 2.2 Step 1)."""
    x = oracle.serialize(X, M, N, D)
    return x + beta * oracle.noise(seed, item, m, x.size)


def _check_eemd(out, X, M, N, D, K, S, NR, beta, seed, item, tally, path=semd.SEMD_PATH_AUTO,
                sd=0.0, ref=None, what=""):
    """An ensemble mean against the oracle's; on a mismatch, the realization
    whose extremum decisions first part from the oracle's must be a tie."""
    if ref is None:
        ref = oracle.eemd(X, M, N, D, K, S, NR, beta, seed, item, sd=sd)
    xmax = float(np.abs(X).max())
    err = parity.output_error(out, ref)
    if err <= TOL * xmax:
        return err
    for m in range(NR):
        res = _diagnose(_realization(X, M, N, D, beta, seed, item, m), K, S, path, sd, xmax)
        if res["status"] == "equal":
            continue
        if res["status"] == "tie":
            tally.tie(f"{what} realization {m}", res)
            return err
        raise AssertionError(f"{what} realization {m}: {res}")
    raise AssertionError(f"{what}: ensemble mean differs by {err:.3g} although every "
                         "realization's extremum decisions equal the oracle's")


def test_eemd_matches_oracle():
    it = workloads.config0()
    M, N, D, K, S, NR, seed = it.M, it.N, 50, 6, 10, 8, 1234
    x = oracle.serialize(it.X, M, N, D)
    beta = 0.2 * float(x.std())
    out = torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV)
    cnt = torch.empty(1, dtype=torch.int32, device=DEV)
    semd.semd_eemd_batch([dev(it.X)], [[M, N]], [out], cnt, D, K, S, NR, seed, [beta], [5])
    tally = Tally("EEMD config 0")
    _check_eemd(host(out), it.X, M, N, D, K, S, NR, beta, seed, 5, tally, what="config 0")
    tally.done()
    assert 1 <= int(host(cnt)[0]) <= K


def _oracle_eemd_threads(items, D, K, S, NR, betas, seed, ids, threads=16):
    """The oracle's EEMD of many series with the realizations spread over host
    threads: each realization is the oracle's EMD of x + beta w_m, and the
    mean is accumulated in m order and divided by NR, as the oracle's own
    EEMD does (its realizations are independent)."""
    from concurrent.futures import ThreadPoolExecutor

    def one(job):
        i, m = job
        it = items[i]
        x = _realization(it.X, it.M, it.N, D, betas[i], seed, ids[i], m)
        slots, _ = oracle.emd(x, K, S)
        return i, m, slots

    jobs = [(i, m) for i in range(len(items)) for m in range(NR)]
    # longest first, so the pool's tail holds the short ones
    jobs.sort(key=lambda j: -items[j[0]].M * items[j[0]].N)
    res = {}
    with ThreadPoolExecutor(threads) as pool:
        for i, m, slots in pool.map(one, jobs):
            res[(i, m)] = slots
    out = []
    for i, it in enumerate(items):
        acc = np.zeros_like(res[(i, 0)])
        for m in range(NR):
            acc = acc + res[(i, m)]
        acc = acc / float(NR)
        out.append(np.stack([oracle.deserialize(acc[k], it.M, it.N, D) for k in range(K + 1)]))
    return out


@pytest.mark.timeout(1200)
def test_eemd_uneven_wave_full_size():
    """The uneven-series EEMD workload at its full size, in the launch
    configuration the bench times: wave 0 of the 4,096-series batch (256
    series of 2-16 channels x 1e3-6.5e4 samples) in one semd_eemd_batch
    call with 64 realizations each, K = 6, S = 10, D = 0.  Its first 32
    series are compared with the oracle element by element (all 64
    realizations, the oracle on 16 host threads); every series of the wave
    has its IMF count in range, finite outputs, and slots that sum to the
    input plus the realizations' mean noise (beta times the mean of the
    noise streams, Sec. 2.2) within 1e-11 * max|x|."""
    K, S, D, NR, seed = 6, 10, 0, 64, 2106
    shapes = workloads.config3_shapes(workloads.CONFIG3_SERIES)
    idx = list(workloads.config3_wave(0))
    items = [workloads.config3_item(i, shapes[i]) for i in idx]
    print(f"wave 0: {len(items)} series, {sum(it.M * it.N for it in items)} samples", flush=True)
    Xs = [dev(it.X) for it in items]
    outs = [torch.empty((K + 1, it.M * it.N), dtype=torch.float64, device=DEV) for it in items]
    cnt = torch.empty(len(items), dtype=torch.int32, device=DEV)
    sig = [0.2 * float(np.std(it.X)) for it in items]
    semd.PreparedBatch(Xs, [[it.M, it.N] for it in items], outs, cnt, D, K, S, ensemble=NR,
                       seed=seed, noise_sigmas=sig, item_ids=idx).run()
    c = host(cnt)
    assert c.min() >= 1 and c.max() <= K
    for j, it in enumerate(items):
        o = outs[j]
        assert bool(torch.isfinite(o).all())
        wsum = torch.zeros(it.M * it.N, dtype=torch.float64, device=DEV)
        for m in range(NR):
            wsum = wsum + semd.semd_noise(seed, idx[j], m, it.M * it.N)
        resid = (o.sum(dim=0) - Xs[j] - sig[j] * (wsum / NR)).abs().max()
        assert float(resid) <= 1e-11 * float(np.abs(it.X).max()), (j, float(resid))
    n_ref = 32
    refs = _oracle_eemd_threads(items[:n_ref], D, K, S, NR, sig[:n_ref], seed, idx[:n_ref])
    tally = Tally("EEMD uneven wave 0", max_ties=1)
    for j in range(n_ref):
        it = items[j]
        _check_eemd(host(outs[j]), it.X, it.M, it.N, D, K, S, NR, sig[j], seed, idx[j], tally,
                    ref=refs[j], what=f"series {idx[j]}")
    tally.done()


def test_eemd_zero_noise_single_realization_is_emd():
    it = workloads.config2(1)[0]
    out = torch.empty((9, it.M * it.N), dtype=torch.float64, device=DEV)
    semd.semd_eemd_batch([dev(it.X)], [[it.M, it.N]], [out], None, 20, 8, 10, 1, 0, [0.0])
    plain, _ = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], 20, 8, 10)
    assert np.array_equal(host(out), host(plain))


# --------------------------------------------------------------------------
# streaming path (many workgroups per signal)
# --------------------------------------------------------------------------

STREAM = semd.SEMD_PATH_STREAM
ONCHIP = semd.SEMD_PATH_ONCHIP


def _series(cfg, k, M, N):
    return workloads.series(workloads.rng_for(cfg, k), N, M)


@pytest.mark.parametrize("M,N,D", [(3, 1, 0), (5, 1, 0), (100, 1, 0), (2047, 1, 0), (2048, 1, 0),
                                   (2049, 1, 0), (1000, 3, 0), (1000, 3, 50), (1000, 5, 200)])
def test_stream_small_matches_oracle(M, N, D):
    X = _series(11, M * 10 + N, M, N)
    out, n = semd.semd_decompose_ex(dev(X), [M, N], D, 6, 10, path=STREAM)
    tally = Tally(f"streaming M={M} N={N} D={D}")
    _check_item(X, M, N, D, 6, 10, host(out), int(host(n)[0]), tally, path=STREAM)
    tally.done()


_WALK_KINDS = ["chirp", "noise", "burst"]
_WALK_LENGTHS = [4097, 6143, 16385, 18433]


def _walk_inputs(L: int, kind: str) -> np.ndarray:
    """Inputs for the two forms of the streaming evaluation's walk: a wave
    whose 512 samples fall in at most 64 segments of each envelope shares
    its segments across lanes; denser waves walk per lane."""
    t = np.arange(L, dtype=np.float64)
    rng = workloads.rng_for(12, _WALK_LENGTHS.index(L) * 3 + _WALK_KINDS.index(kind))
    if kind == "chirp":
        # extremum spacing from ~L/8 down to 3 samples along the signal, so
        # the per-wave segment count crosses 64 inside it
        f = 1.0 / 2000.0 + (1.0 / 6.0 - 1.0 / 2000.0) * (t / L) ** 2
        return np.sin(2.0 * np.pi * np.cumsum(f)) + 0.3 * np.sin(t / 97.0)
    if kind == "noise":
        return rng.standard_normal(L)
    # smooth, with a white-noise burst inside one wave of the second tile
    x = np.sin(t / 131.0) + 0.5 * np.sin(t / 17.0)
    b0 = min(L - 1, 2048 + 700)
    x[b0:b0 + 300] += rng.standard_normal(len(x[b0:b0 + 300]))
    return x


@pytest.mark.parametrize("L", _WALK_LENGTHS)
@pytest.mark.parametrize("kind", _WALK_KINDS)
def test_stream_walk_forms_match_oracle(L, kind):
    x = _walk_inputs(L, kind)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 6, 10, path=STREAM)
    tally = Tally(f"streaming walk L={L} {kind}")
    _check_item(x, L, 1, 0, 6, 10, host(out), int(host(n)[0]), tally, path=STREAM)
    tally.done()


def _random_stream_case(i: int) -> np.ndarray:
    """Seeded streaming inputs of random length and kind (noise, chirp,
    stepped plateaus, sinusoid mixes, and sums of them)."""
    rng = workloads.rng_for(13, i)
    L = int(rng.integers(16385, 70000))
    t = np.arange(L, dtype=np.float64)
    kind = i % 4
    if kind == 0:
        x = rng.standard_normal(L)
    elif kind == 1:
        f = rng.uniform(1e-4, 1e-3) + rng.uniform(0.05, 0.2) * (t / L) ** rng.uniform(1, 3)
        x = np.sin(2.0 * np.pi * np.cumsum(f))
    elif kind == 2:
        edges = np.sort(rng.integers(0, L, size=int(rng.integers(20, 200))))
        x = np.zeros(L)
        for e in edges:
            x[e:] += rng.normal()
        x += 0.1 * np.sin(t / rng.uniform(20, 400))
    else:
        x = sum(rng.uniform(0.3, 2.0) * np.sin(2 * np.pi * t * rng.uniform(1e-4, 0.2) +
                                               rng.uniform(0, 2 * np.pi)) for _ in range(4))
        x += 0.05 * rng.standard_normal(L)
    return x


@pytest.mark.parametrize("i", range(12))
def test_stream_random_lengths_match_oracle(i):
    x = _random_stream_case(i)
    L = x.size
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 5, 6, path=STREAM)
    tally = Tally(f"streaming random case {i} L={L}")
    _check_item(x, L, 1, 0, 5, 6, host(out), int(host(n)[0]), tally, path=STREAM)
    tally.done()


@pytest.mark.parametrize("K,S,noisy", [(12, 1, False), (12, 1, True), (12, 2, True),
                                        (24, 3, False), (4, 1, True)])
def test_stream_short_imfs_to_final_residue(K, S, noisy):
    """IMFs of one to three sifts on the streaming path, most of them ended
    by the residue running out of extrema before K: every IMF-ending sift
    detects the new residue's extrema itself and the next step takes its
    candidate from r, including a final step right after an IMF end."""
    L = 20000
    t = np.arange(L, dtype=np.float64)
    x = (np.sin(2 * np.pi * t / 37.0) + 0.6 * np.sin(2 * np.pi * t / 523.0) +
         0.3 * np.sin(2 * np.pi * t / 4111.0) + 2e-4 * t)
    if noisy:
        x = x + 0.2 * np.random.default_rng(31).standard_normal(L)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, K, S, path=STREAM)
    tally = Tally(f"streaming short IMFs K={K} S={S} noisy={noisy}")
    res = _check_item(x, L, 1, 0, K, S, host(out), int(host(n)[0]), tally, path=STREAM)
    tally.done()
    assert res["n"] >= 3


def test_stream_faces_and_textures():
    items = workloads.config2(4) + workloads.config1(2)
    shapes = [(i.M, i.N) for i in items]
    outs, counts = semd.decompose_batch([dev(i.X) for i in items], shapes, 0, 8, 10, path=STREAM)
    counts = host(counts)
    tally = Tally("streaming faces and textures", max_ties=1)
    for k, i in enumerate(items):
        _check_item(i.X, i.M, i.N, 0, 8, 10, host(outs[k]), int(counts[k]), tally, path=STREAM)
    tally.done()


def test_stream_equals_onchip():
    items = workloads.config2(2) + [workloads.config0()]
    for i in items:
        a, na = semd.semd_decompose_ex(dev(i.X), [i.M, i.N], 7, 8, 10, path=ONCHIP)
        b, nb = semd.semd_decompose_ex(dev(i.X), [i.M, i.N], 7, 8, 10, path=STREAM)
        assert int(host(na)[0]) == int(host(nb)[0])
        assert np.abs(host(a) - host(b)).max() <= TOL * np.abs(i.X).max()


def test_stream_plateaus_across_tiles():
    # equal-valued runs longer than a tile (2048 samples), entered and left
    # in every direction, plus runs touching both ends
    L = 20000
    x = np.zeros(L)
    x[:3000] = 2.0
    x[3000:9000] = 5.0     # maximum plateau over ~3 tiles
    x[9000:9500] = 1.0
    x[9500:15000] = -3.0   # minimum plateau over ~3 tiles
    x[15000:15100] = 0.5   # shoulder
    x[15100:17000] = 0.7
    x[17000:] = -1.0
    x += 0.25 * np.sin(np.arange(L) / 900.0) * (np.arange(L) % 4096 < 100)
    imax, imin = oracle.extrema(x)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 4, 3, path=STREAM)
    tally = Tally("plateaus across tiles")
    _check_item(x, L, 1, 0, 4, 3, host(out), int(host(n)[0]), tally, path=STREAM)
    tally.done()
    assert len(imax) >= 1 and len(imin) >= 1


@pytest.mark.parametrize("M,N,K,S", [(20000, 3, 6, 10), (500, 500, 6, 10), (1024, 1024, 8, 10)])
def test_stream_long_signals(M, N, K, S):
    """Long signals on the streaming path, the 1024 x 1024 texture (the
    serving mix's large request) at its served K = 8, S = 10."""
    if M == N:
        X = workloads.texture(workloads.rng_for(12, M), M, N)
    else:
        X = _series(12, M, M, N)
    out, n = semd.semd_decompose_ex(dev(X), [M, N], 0, K, S)  # auto: streaming by length
    tally = Tally(f"long signal M={M} N={N}")
    _check_item(X, M, N, 0, K, S, host(out), int(host(n)[0]), tally)
    tally.done()


@pytest.mark.timeout(900)
def test_stream_longest_signal():
    """The longest serialized signal the library takes, 2^28 samples of
    white noise (the densest knot sets, about L/3 knots per envelope): two
    IMFs of one sift each, element by element against the oracle."""
    L, K, S = 1 << 28, 2, 1
    x = np.random.default_rng(2828).standard_normal(L)
    print(f"longest signal: L={L} K={K} S={S}", flush=True)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, K, S)
    o = host(out)
    del out
    torch.cuda.empty_cache()
    tally = Tally("white noise at the longest length")
    _check_item(x, L, 1, 0, K, S, o, int(host(n)[0]), tally)
    tally.done()


def test_auto_routes_mixed_batch():
    shapes = [(100, 3), (30000, 2), (5000, 2), (11, 1), (40000, 1)]
    Xs = [_series(13, k, M, N) for k, (M, N) in enumerate(shapes)]
    outs, counts = semd.decompose_batch([dev(x) for x in Xs], shapes, 10, 6, 10)
    counts = host(counts)
    tally = Tally("auto-routed mixed batch", max_ties=1)
    for k, (M, N) in enumerate(shapes):
        _check_item(Xs[k], M, N, 10, 6, 10, host(outs[k]), int(counts[k]), tally)
    tally.done()


@pytest.mark.parametrize("L", [1, 2, 3])
def test_stream_tiny_signals(L):
    x = np.array([1.0, -2.0, 0.5][:L])
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 4, 10, path=STREAM)
    ref, nr = oracle.emd(x, 4, 10)
    assert int(host(n)[0]) == nr == 0
    assert np.array_equal(host(out), ref)


def test_stream_non_finite_and_monotone():
    x = np.ones(5000)
    x[4000] = np.inf
    out, n = semd.semd_decompose_ex(dev(x), [5000, 1], 0, 3, 10, path=STREAM)
    assert int(host(n)[0]) == -semd.SEMD_ENONFINITE
    assert np.all(host(out) == 0.0)
    m = np.linspace(0.0, 1.0, 9000) ** 2
    out, n = semd.semd_decompose_ex(dev(m), [9000, 1], 0, 3, 10, path=STREAM)
    assert int(host(n)[0]) == 0 and np.array_equal(host(out)[3], m)


def test_stream_graph_replays_repeat():
    # every streaming decomposition replays one captured step graph K*S
    # times; repeated calls, with unrelated eager work and synchronizations
    # in between, give bit-identical results that match the oracle
    it = workloads.config3_item(5, (6000, 3))
    x = dev(it.X)
    runs = []
    for r in range(3):
        out, n = semd.semd_decompose_ex(x, [it.M, it.N], 0, 6, 10, path=STREAM)
        junk = torch.randn(1 << 20, dtype=torch.float64, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        runs.append((host(out), int(host(n)[0]), float(junk[-1])))
    for o, nn, _ in runs[1:]:
        assert nn == runs[0][1]
        assert_same(o, runs[0][0], "graph replay")
    tally = Tally("repeated streaming runs")
    _check_item(it.X, it.M, it.N, 0, 6, 10, runs[0][0], runs[0][1], tally, path=STREAM)
    tally.done()


def test_stream_eemd_long_signal():
    M, N, D, K, S, NR, seed = 15000, 2, 50, 6, 10, 4, 99
    X = _series(14, 0, M, N)
    x = oracle.serialize(X, M, N, D)
    beta = 0.2 * float(x.std())
    out = torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV)
    semd.semd_eemd_batch([dev(X)], [[M, N]], [out], None, D, K, S, NR, seed, [beta], [3])
    tally = Tally("EEMD long streaming signal")
    _check_eemd(host(out), X, M, N, D, K, S, NR, beta, seed, 3, tally, what="long signal")
    tally.done()


# --------------------------------------------------------------------------
# serving engine
# --------------------------------------------------------------------------

def _engine_run(eng, reqs, K, S, D, sd=0.0, path=semd.SEMD_PATH_AUTO):
    outs, tickets = [], {}
    for k, (X, M, N) in enumerate(reqs):
        out = torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV)
        cnt = torch.empty(1, dtype=torch.int32, device=DEV)
        t = eng.admit(dev(X), (M, N), out, cnt, D, K, S, sd=sd, path=path)
        assert t is not None
        tickets[t] = k
        outs.append((out, cnt))
    done = set()
    for _ in range(K * S + 4):
        eng.step()
        done.update(eng.poll())
        if len(done) == len(reqs):
            break
    torch.cuda.synchronize()
    done.update(eng.poll())
    assert done == set(tickets)
    return outs


@pytest.mark.parametrize("path", [semd.SEMD_PATH_AUTO, STREAM])
def test_engine_matches_plain_path_and_mix(path):
    """Each request's outputs are the same bits alone in the engine, in a mix
    with others, and from semd_decompose_ex on the same path (AUTO: the short
    requests run whole on chip, the long one streams), and match the oracle."""
    K, S, D = 6, 10, 10
    reqs = [(_series(15, k, M, N), M, N) for k, (M, N) in
            enumerate([(3000, 2), (500, 3), (12000, 4), (40, 1), (2049, 1)])]
    eng = semd.Engine(1 << 30, 64)
    mixed = _engine_run(eng, reqs, K, S, D, path=path)
    for k, (X, M, N) in enumerate(reqs):
        alone_eng = _engine_run(eng, [(X, M, N)], K, S, D, path=path)[0]
        ref, nref = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=path)
        # same arithmetic alone, in the mix and on the plain path: bit-identical
        assert_same(host(mixed[k][0]), host(alone_eng[0]), "engine mix vs alone")
        assert_same(host(mixed[k][0]), host(ref), "engine vs plain path")
        assert int(host(mixed[k][1])[0]) == int(host(nref)[0])
        tally = Tally(f"engine request {k} path={path}")
        _check_item(X, M, N, D, K, S, host(mixed[k][0]), int(host(mixed[k][1])[0]), tally,
                    path=path)
        tally.done()
    eng.close()


def test_engine_short_requests_finish_within_two_steps():
    """A short request routed on chip completes with the step that launches
    it (reported by the poll after the next step), whatever streaming work
    is resident."""
    K, S, D = 6, 10, 0
    eng = semd.Engine(1 << 30, 16)
    long_x = _series(17, 0, 20000, 2)
    lo = torch.empty((K + 1, 40000), dtype=torch.float64, device=DEV)
    tl = eng.admit(dev(long_x), (20000, 2), lo, None, D, K, S)
    eng.step()
    short_x = _series(17, 1, 1000, 3)
    so = torch.empty((K + 1, 3000), dtype=torch.float64, device=DEV)
    sc = torch.empty(1, dtype=torch.int32, device=DEV)
    ts = eng.admit(dev(short_x), (1000, 3), so, sc, D, K, S)
    done = set()
    for _ in range(2):
        eng.step()
        done.update(eng.poll())
    torch.cuda.synchronize()
    done.update(eng.poll())
    assert ts in done and tl not in done
    ref, nref = semd.semd_decompose_ex(dev(short_x), [1000, 3], D, K, S)
    assert_same(host(so), host(ref), "on-chip engine request")
    for _ in range(K * S + 4):
        if tl in done:
            break
        eng.step()
        done.update(eng.poll())
    torch.cuda.synchronize()
    done.update(eng.poll())
    assert tl in done
    eng.close()


def test_engine_multi_step_calls_match_single_steps():
    """semd_engine_step_n: several steps per call give each request the same
    bits as semd_decompose_ex, with a request admitted between bursts and
    bursts that run past a request's end; n_steps outside [1, 64] is
    rejected."""
    K, S, D = 5, 8, 4
    shapes = [(9000, 3), (1500, 2), (30000, 1), (700, 4)]
    Xs = [_series(19, k, M, N) for k, (M, N) in enumerate(shapes)]
    outs = [torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV) for M, N in shapes]
    cnts = [torch.empty(1, dtype=torch.int32, device=DEV) for _ in shapes]
    eng = semd.Engine(1 << 30, 16)
    with pytest.raises(RuntimeError):
        eng.step_n(0)
    with pytest.raises(RuntimeError):
        eng.step_n(semd.SEMD_ENGINE_MAX_STEPS + 1)
    owner = {}
    for k in (0, 1, 2):
        M, N = shapes[k]
        owner[eng.admit(dev(Xs[k]), (M, N), outs[k], cnts[k], D, K, S)] = k
    eng.step_n(7)
    M, N = shapes[3]
    owner[eng.admit(dev(Xs[3]), (M, N), outs[3], cnts[3], D, K, S)] = 3
    done = set()
    for _ in range(K * S):
        eng.step_n(13)
        done.update(eng.poll())
        if len(done) == len(shapes):
            break
    torch.cuda.synchronize()
    done.update(eng.poll())
    assert done == set(owner)
    eng.close()
    for k, (M, N) in enumerate(shapes):
        ref, nref = semd.semd_decompose_ex(dev(Xs[k]), [M, N], D, K, S)
        assert_same(host(outs[k]), host(ref), f"engine burst request {k}")
        assert int(host(cnts[k])[0]) == int(host(nref)[0])


def test_engine_admission_budget_and_staggered_arrivals():
    K, S, D = 4, 6, 0
    M, N = 6000, 3  # 18,000 samples: streaming
    fp = semd.Engine.footprint([M, N], D, K, S)
    eng = semd.Engine(int(fp * 2.5), 8)  # room for two requests at a time
    Xs = [_series(16, k, M, N) for k in range(5)]
    outs = [torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV) for _ in Xs]
    cnts = [torch.empty(1, dtype=torch.int32, device=DEV) for _ in Xs]
    t0 = eng.admit(dev(Xs[0]), (M, N), outs[0], cnts[0], D, K, S)
    for _ in range(3):
        eng.step()  # the first request is already sifting when the next arrive
    t1 = eng.admit(dev(Xs[1]), (M, N), outs[1], cnts[1], D, K, S)
    assert t0 is not None and t1 is not None
    assert eng.admit(dev(Xs[2]), (M, N), outs[2], cnts[2], D, K, S) is None  # over budget
    pending = [2, 3, 4]
    done = set()
    owner = {t0: 0, t1: 1}
    for _ in range(10 * K * S):
        while pending:
            t = eng.admit(dev(Xs[pending[0]]), (M, N), outs[pending[0]], cnts[pending[0]], D, K,
                          S)
            if t is None:
                break
            owner[t] = pending.pop(0)
        eng.step()
        done.update(eng.poll())
        if len(done) == 5:
            break
    assert len(done) == 5 and not pending
    tally = Tally("engine staggered arrivals")
    for t, k in owner.items():
        _check_item(Xs[k], M, N, D, K, S, host(outs[k]), int(host(cnts[k])[0]), tally,
                    path=STREAM)
    tally.done()
    eng.close()


# --------------------------------------------------------------------------
# launch-shape tuning
# --------------------------------------------------------------------------

def test_every_launch_shape_gives_identical_results():
    # the shape table changes speed, not the decomposition: a face image
    # (bucket 12288) and a 3000-sample series (bucket 3072) under every
    # compiled shape that fits.  Shapes with the same thread count give the
    # same bits; across thread counts the spline solve may associate its
    # scans differently (when a sift has more knots than threads), so those
    # agree to rounding.
    arch = semd.semd_tune_get().splitlines()[0]
    cases = [(workloads.config2(1)[0], 12288, 8), (workloads.config0(), 3072, 6)]
    shapes = [(256, 4), (256, 8), (256, 12), (256, 16), (512, 8), (512, 12), (512, 16),
              (1024, 4), (1024, 8), (1024, 12), (1024, 16)]
    try:
        for it, bound, K in cases:
            x = dev(it.X)
            ref, by_nt = None, {}
            for nt, c in shapes:
                if nt * c < bound:
                    continue
                semd.semd_tune_set(f"{arch}\nlatency {bound} {nt} {c}\n")
                out, n = semd.semd_decompose_ex(x, [it.M, it.N], 0, K, 10, path=ONCHIP)
                got = (host(out), int(host(n)[0]))
                if nt in by_nt:
                    assert got[1] == by_nt[nt][1]
                    assert_same(got[0], by_nt[nt][0], f"shape {nt}x{c}")
                else:
                    by_nt[nt] = got
                if ref is None:
                    ref = got
                else:
                    assert got[1] == ref[1]
                    assert np.abs(got[0] - ref[0]).max() <= 1e-12 * np.abs(it.X).max()
    finally:
        semd.semd_tune_reset()


@pytest.mark.parametrize("target", [1, 1024, 65536])
def test_stream_solve_target_gives_identical_results(target):
    """The tuned streaming solve target changes how solve blocks map to
    workgroups (the launch's fold), not the decomposition: a streaming batch
    gives the same bits under it as under the built-in value."""
    rng = np.random.default_rng(31)
    shapes = [(30000, 2), (17000, 1), (9000, 4), (120000, 1)]
    items = [(rng.standard_normal(M * N) + np.sin(np.arange(M * N) / 7.0), M, N)
             for M, N in shapes]
    Xs = [dev(x) for x, _, _ in items]
    try:
        semd.semd_tune_reset()
        ref, rc = semd.decompose_batch(Xs, [(M, N) for _, M, N in items], 0, 5, 6)
        header = semd.semd_tune_get().splitlines()[0]
        semd.semd_tune_set(f"{header}\nstream-solve {target}\n")
        assert semd.semd_tune_get().splitlines()[1:] == [f"stream-solve {target}"]
        got, gc = semd.decompose_batch(Xs, [(M, N) for _, M, N in items], 0, 5, 6)
    finally:
        semd.semd_tune_reset()
    for k in range(len(items)):
        assert_same(host(got[k]), host(ref[k]), f"solve target {target}, item {k}")
    assert np.array_equal(host(gc), host(rc))


def test_autotune_round_trip():
    try:
        semd.semd_autotune(4096, 256)
        text = semd.semd_tune_get()
        lines = text.splitlines()
        assert lines[0].startswith(f"semd-tune {semd.semd_abi_version()} gfx")
        entries = [l.split() for l in lines[1:] if not l.startswith("stream-solve")]
        assert {e[0] for e in entries} == {"latency", "throughput"}
        assert {int(e[1]) for e in entries} == {1024, 2048, 3072, 4096}
        for e in entries:
            assert int(e[2]) * int(e[3]) >= int(e[1])
        solve = [l.split() for l in lines[1:] if l.startswith("stream-solve")]
        assert len(solve) == 1 and int(solve[0][1]) in (1024, 2048, 4096, 8192, 16384)
        semd.semd_tune_reset()
        assert semd.semd_tune_get().splitlines()[1:] == []
        semd.semd_tune_set(text)
        assert semd.semd_tune_get() == text
        with pytest.raises(semd.SemdError):
            semd.semd_tune_set(text.replace("gfx", "gfy", 1))
        with pytest.raises(semd.SemdError):
            semd.semd_tune_set(lines[0] + "\nlatency 4096 256 4\n")  # too small a shape
        with pytest.raises(semd.SemdError):
            semd.semd_tune_set(lines[0] + "\nstream-solve 0\n")
        with pytest.raises(semd.SemdError):
            semd.semd_tune_set(lines[0] + "\nstream-solve\n")
        assert semd.semd_tune_get() == text  # unchanged by the rejected tables
        # decompositions under the tuned table still match the oracle
        it = workloads.config0()
        out, n = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], 0, 6, 10)
        tally = Tally("tuned table")
        _check_item(it.X, it.M, it.N, 0, 6, 10, host(out), int(host(n)[0]), tally)
        tally.done()
    finally:
        semd.semd_tune_reset()


# --------------------------------------------------------------------------
# standard (slice-wise) EMD
# --------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["series", "texture", "long"])
def test_slices_match_oracle(kind):
    if kind == "series":
        it = workloads.config0()
    elif kind == "texture":
        it = workloads.config1(1, 64)[0]
    else:  # columns longer than the on-chip limit: streaming path
        it = workloads.config3_item(7, (20000, 2))
    K, S = 6, 10
    out, n = semd.semd_decompose_slices(dev(it.X), [it.M, it.N], K, S)
    out, n = host(out), host(n)
    # each column is a decomposition of its own: compared column by column
    tally = Tally(f"slices {kind}", max_ties=1)
    M = it.M
    for i in range(it.N):
        col = it.X[i * M:(i + 1) * M]
        _check_item(col, M, 1, 0, K, S, out[:, i * M:(i + 1) * M], int(n[i]), tally,
                    what=f"column {i}")
    tally.done()


def test_slices_equal_single_column_serial():
    # one column: slice-wise and serial decompositions are the same EMD
    it = workloads.config3_item(3, (3000, 1))
    a, na = semd.semd_decompose_slices(dev(it.X), [it.M, 1], 6, 10)
    b, nb = semd.semd_decompose_ex(dev(it.X), [it.M, 1], 0, 6, 10)
    assert int(host(na)[0]) == int(host(nb)[0])
    assert_same(host(a), host(b), "slices vs serial")


# --------------------------------------------------------------------------
# SD stopping rule
# --------------------------------------------------------------------------

def _check_sd(X, M, N, D, K, S, thr, out, n, tally, stats=None, path=semd.SEMD_PATH_AUTO):
    r = _check_item(X, M, N, D, K, S, out, n, tally, path=path, sd=thr, stats=stats)
    return r, r["stats"]


@pytest.mark.parametrize("path", [ONCHIP, STREAM])
@pytest.mark.parametrize("thr", [0.3, 0.05, 1e-3])
def test_sd_rule_matches_oracle(path, thr):
    items = [workloads.config0()] + workloads.config2(3) + workloads.config1(1, size=64)
    K, S, D = 8, 30, 20
    shapes = [(i.M, i.N) for i in items]
    outs = [torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV) for M, N in shapes]
    counts = torch.empty(len(items), dtype=torch.int32, device=DEV)
    stats = torch.empty((len(items), 3), dtype=torch.int64, device=DEV)
    semd.semd_decompose_batch([dev(i.X) for i in items], [list(s) for s in shapes], outs, counts,
                              D, K, S, stats=stats, path=path, sd=thr)
    counts, stats = host(counts), host(stats)
    tally, early = Tally(f"SD rule {thr} path={path}", max_ties=1), 0
    for k, i in enumerate(items):
        r, st = _check_sd(i.X, i.M, i.N, D, K, S, thr, host(outs[k]), int(counts[k]), tally,
                          stats[k], path=path)
        early += st["n_sifts"] < r["n"] * S
    tally.done()
    assert early >= 1  # the rule ended IMFs before the sift limit


def test_sd_rule_stream_equals_onchip_and_engine():
    K, S, D, thr = 8, 30, 10, 0.05
    reqs = [(workloads.config2(1)[0].X, 112, 92), (_series(21, 0, 3000, 2), 3000, 2)]
    eng = semd.Engine(1 << 30, 16)
    served = _engine_run(eng, reqs, K, S, D, sd=thr, path=STREAM)
    eng.close()
    for k, (X, M, N) in enumerate(reqs):
        a, na = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=ONCHIP, sd=thr)
        b, nb = semd.semd_decompose_ex(dev(X), [M, N], D, K, S, path=STREAM, sd=thr)
        # the engine runs the streaming kernels: the same sums, the same bits
        assert_same(host(served[k][0]), host(b), "engine vs streaming path")
        tally = Tally(f"SD rule request {k}")
        _, st = _check_sd(X, M, N, D, K, S, thr, host(a), int(host(na)[0]), tally, path=ONCHIP)
        tally.done()
        if st["sd_margin"] >= SD_TIE:
            # the two paths solve in different chunkings: equal within rounding
            assert int(host(na)[0]) == int(host(nb)[0])
            assert np.abs(host(a) - host(b)).max() <= TOL * np.abs(X).max()


@pytest.mark.parametrize("kind", ["white", "alternating"])
def test_sd_rule_dense_knot_stores(kind):
    # the densest knot sets: the sift runs from the global knot store
    L = semd.semd_resident_max_length()
    k = np.arange(L)
    if kind == "white":
        x = np.random.default_rng(78).standard_normal(L)
    else:
        x = np.where(k % 2 == 0, 1.0, -1.0) * (1.0 + 0.001 * np.sin(k / 50.0))
    thr = 0.1
    for path in (ONCHIP, STREAM):
        out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 3, 8, path=path, sd=thr)
        tally = Tally(f"SD rule {kind} path={path}")
        _check_sd(x, L, 1, 0, 3, 8, thr, host(out), int(host(n)[0]), tally, path=path)
        tally.done()


def test_sd_rule_long_signal_stream():
    it = workloads.config3_item(5, (20000, 3))
    K, S, D, thr = 6, 20, 40, 0.2
    out, n = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], D, K, S, sd=thr)
    tally = Tally("SD rule long signal")
    _check_sd(it.X, it.M, it.N, D, K, S, thr, host(out), int(host(n)[0]), tally)
    tally.done()


def test_sd_rule_slices_and_eemd():
    it = workloads.config0()
    M, N, K, S, thr = it.M, it.N, 6, 20, 0.2
    out, n = semd.semd_decompose_slices(dev(it.X), [M, N], K, S, sd=thr)
    out, n = host(out), host(n)
    tally = Tally("SD rule slices and EEMD", max_ties=1)
    for i in range(N):
        col = it.X[i * M:(i + 1) * M]
        _check_item(col, M, 1, 0, K, S, out[:, i * M:(i + 1) * M], int(n[i]), tally, sd=thr,
                    what=f"column {i}")
    D, NR, seed = 50, 4, 99
    beta = 0.2 * float(oracle.serialize(it.X, M, N, D).std())
    eo = torch.empty((K + 1, M * N), dtype=torch.float64, device=DEV)
    semd.semd_eemd_batch([dev(it.X)], [[M, N]], [eo], None, D, K, S, NR, seed, [beta], [3],
                         sd=thr)
    _check_eemd(host(eo), it.X, M, N, D, K, S, NR, beta, seed, 3, tally, sd=thr, what="EEMD")
    tally.done()


# --------------------------------------------------------------------------
# transition-length sweep input (Sec. 4.1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("D", [1, 2, 50, 200, 500, 1000])
@pytest.mark.parametrize("rule", ["fixed", "sd"])
def test_mask_series_sweep_matches_oracle(D, rule):
    it = workloads.config5()
    K, S, sd = (8, 10, 0.0) if rule == "fixed" else (8, 100, 0.05)
    out, n = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], D, K, S, sd=sd)
    tally = Tally(f"mask series D={D} {rule}")
    _check_sd(it.X, it.M, it.N, D, K, S, sd, host(out), int(host(n)[0]), tally)
    tally.done()


# --------------------------------------------------------------------------
# CEEMDAN
# --------------------------------------------------------------------------

def _ceemdan(items, D, K, S, NR, seed, eps, path=semd.SEMD_PATH_AUTO, sd=0.0, ids=None):
    outs = [torch.empty((K + 1, i.M * i.N), dtype=torch.float64, device=DEV) for i in items]
    cnt = torch.empty(len(items), dtype=torch.int32, device=DEV)
    semd.semd_ceemdan_batch([dev(i.X) for i in items], [[i.M, i.N] for i in items], outs, cnt, D,
                            K, S, NR, seed, eps, ids, path=path, sd=sd)
    return [host(o) for o in outs], [int(c) for c in host(cnt)]


@pytest.mark.parametrize("path", [semd.SEMD_PATH_AUTO, STREAM])
@pytest.mark.parametrize("sd", [0.0, 0.2])
def test_ceemdan_matches_oracle(path, sd):
    items = [workloads.config0(), workloads.config5()]
    K, S, NR, seed, D = 6, 10, 6, 31, 50
    outs, ns = _ceemdan(items, D, K, S, NR, seed, [0.2, 0.1], path=path, sd=sd, ids=[4, 9])
    for k, (it, eps, iid) in enumerate(zip(items, [0.2, 0.1], [4, 9])):
        ref, nr = oracle.ceemdan(it.X, it.M, it.N, D, K, S, NR, eps, seed, iid, sd=sd)
        assert ns[k] == nr
        err = np.abs(outs[k] - ref).max()
        assert err <= TOL * np.abs(it.X).max(), (k, err)


def test_ceemdan_without_noise_is_the_plain_decomposition():
    it = workloads.config2(1)[0]
    K, S, D = 8, 10, 20
    outs, ns = _ceemdan([it], D, K, S, 1, 5, [0.0])
    plain, n = semd.semd_decompose_ex(dev(it.X), [it.M, it.N], D, K, S)
    assert ns[0] == int(host(n)[0])
    assert_same(outs[0], host(plain), "CEEMDAN(eps=0, NR=1) vs EMD")


def test_ceemdan_long_signal_and_edge_cases():
    long_it = workloads.config3_item(11, (20000, 2))  # streaming path
    mono = workloads.Item(np.linspace(-2.0, 3.0, 700) ** 3, 700, 1)
    bad = workloads.Item(np.ones(300), 300, 1)
    bad.X[17] = np.inf
    K, S, NR, seed = 3, 8, 2, 77
    outs, ns = _ceemdan([long_it, mono, bad], 0, K, S, NR, seed, [0.2, 0.2, 0.2])
    ref, nr = oracle.ceemdan(long_it.X, long_it.M, long_it.N, 0, K, S, NR, 0.2, seed, 0)
    assert ns[0] == nr
    assert np.abs(outs[0] - ref).max() <= TOL * np.abs(long_it.X).max()
    assert ns[1] == 0 and np.array_equal(outs[1][K], mono.X) and np.all(outs[1][:K] == 0.0)
    assert ns[2] == -semd.SEMD_ENONFINITE and np.all(outs[2] == 0.0)


@pytest.mark.parametrize("L", [6000, 8192, 12000])
def test_knot_store_modes_over_several_sifts(L):
    # white noise puts about 2L/3 knots into a sift: around these lengths the
    # on-chip kernel moves between both envelopes in LDS, one at a time in
    # LDS (the upper one parked in global memory), and the global knot store
    x = np.random.default_rng(4000 + L).standard_normal(L)
    out, n = semd.semd_decompose_ex(dev(x), [L, 1], 0, 3, 4, path=ONCHIP)
    tally = Tally(f"knot store modes L={L}")
    _check_item(x, L, 1, 0, 3, 4, host(out), int(host(n)[0]), tally, path=ONCHIP)
    tally.done()
