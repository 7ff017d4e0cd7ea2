"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no Serial-EMD arithmetic: it only draws signals.  Both the
HIP path (benchmark, smoke check) and the oracle side (tests) take their inputs
from here, so the two see identical bytes.

Every signal is returned as a column-major M x N float64 matrix (the columns
are the signals to be serialized, Sec. 3.2), flattened with ``order="F"``,
together with (M, N).

Recipes (stand-ins; the paper's own data are not available):
  * series    -- per channel, the sum of 3 sinusoids with frequency
                 U[0.002, 0.2] cycles/sample, amplitude U[0.5, 2], phase
                 U[0, 2pi), plus N(0, 0.05^2) noise (multivariate signals of
                 Sec. 4.1; channel count and length vary by workload).
  * texture   -- sum of 3 oriented unit-amplitude gratings with periods 4, 16
                 and 64 px, orientation U[0, pi), phase U[0, 2pi), plus
                 N(0, 0.05^2) (artificial texture images of Sec. 4.2).
  * mask      -- the six-variate signal of Sec. 4.1: four unit sinusoids
                 (32, 16, 8, 2 Hz at 1 kHz, zero phase) picked per variate by
                 the paper's pick-up mask; no noise (the D sweep's input).
  * face-like -- 112 x 92 grey image: 4..8 Gaussian blobs (sigma U[8, 30] px,
                 amplitude U[40, 200]) plus gratings of period 6 and 24 px at
                 12 grey levels each, clipped to [0, 255] and rounded to uint8
                 (stand-in for the face images of Sec. 4.3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 2106_15319


def rng_for(config: int, item: int | None = None) -> np.random.Generator:
    ss = np.random.SeedSequence(BASE_SEED + config)
    if item is None:
        return np.random.default_rng(ss)
    return np.random.default_rng(ss.spawn(item + 1)[item])


def series(rng: np.random.Generator, channels: int, M: int) -> np.ndarray:
    """M x channels matrix (column = channel), column-major flat."""
    k = np.arange(M, dtype=np.float64)
    X = np.empty((M, channels), dtype=np.float64, order="F")
    for c in range(channels):
        f = rng.uniform(0.002, 0.2, size=3)
        A = rng.uniform(0.5, 2.0, size=3)
        ph = rng.uniform(0.0, 2 * math.pi, size=3)
        col = np.zeros(M)
        for s in range(3):
            col += A[s] * np.sin(2 * math.pi * f[s] * k + ph[s])
        col += rng.normal(0.0, 0.05, size=M)
        X[:, c] = col
    return X.ravel(order="F")


def texture(rng: np.random.Generator, H: int, W: int) -> np.ndarray:
    """H x W image; its columns are the signals.  Column-major flat."""
    r = np.arange(H, dtype=np.float64)[:, None]
    c = np.arange(W, dtype=np.float64)[None, :]
    img = np.zeros((H, W))
    for P in (4.0, 16.0, 64.0):
        th = rng.uniform(0.0, math.pi)
        ph = rng.uniform(0.0, 2 * math.pi)
        img += np.sin(2 * math.pi * (r * math.cos(th) + c * math.sin(th)) / P + ph)
    img += rng.normal(0.0, 0.05, size=(H, W))
    return np.asfortranarray(img).ravel(order="F")


def face_like(rng: np.random.Generator, H: int = 112, W: int = 92) -> np.ndarray:
    """H x W uint8-valued image as float64, column-major flat."""
    r = np.arange(H, dtype=np.float64)[:, None]
    c = np.arange(W, dtype=np.float64)[None, :]
    img = np.zeros((H, W))
    for _ in range(int(rng.integers(4, 9))):
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        sg = rng.uniform(8.0, 30.0)
        amp = rng.uniform(40.0, 200.0)
        img += amp * np.exp(-((r - cy) ** 2 + (c - cx) ** 2) / (2 * sg * sg))
    for P in (6.0, 24.0):
        th = rng.uniform(0.0, math.pi)
        ph = rng.uniform(0.0, 2 * math.pi)
        img += 12.0 * np.sin(2 * math.pi * (r * math.cos(th) + c * math.sin(th)) / P + ph)
    img = np.rint(np.clip(img, 0.0, 255.0)).astype(np.uint8).astype(np.float64)
    return np.asfortranarray(img).ravel(order="F")


# Which of the four sinusoids (rows: 32, 16, 8, 2 Hz) each of the six variates
# U..Z holds: the pick-up mask of Sec. 4.1 (8 Hz is common to all).
PICKUP_MASK = np.array([[1, 1, 0, 1, 0, 0],
                        [1, 1, 1, 0, 1, 0],
                        [1, 1, 1, 1, 1, 1],
                        [1, 0, 1, 1, 0, 1]])
PICKUP_FREQS_HZ = (32.0, 16.0, 8.0, 2.0)


def mask_series(M: int = 1000, fs: float = 1000.0) -> np.ndarray:
    """The six-variate signal of Sec. 4.1: variate j is the sum of the unit
    sinusoids sin(2 pi f_i k / fs), k = 0..M-1, over the rows i of column j of
    the pick-up mask.  M x 6, column-major flat.  (The sampling rate, the
    amplitudes and the phases are not given in the paper: 1 s at 1 kHz, unit
    amplitude and zero phase are this recipe's choice.)"""
    k = np.arange(M, dtype=np.float64)
    X = np.zeros((M, PICKUP_MASK.shape[1]), dtype=np.float64, order="F")
    for i, f in enumerate(PICKUP_FREQS_HZ):
        wave = np.sin(2 * math.pi * f * k / fs)
        for j in range(PICKUP_MASK.shape[1]):
            if PICKUP_MASK[i, j]:
                X[:, j] += wave
    return X.ravel(order="F")


@dataclass
class Item:
    X: np.ndarray  # column-major flat M*N float64
    M: int
    N: int


def config0() -> Item:
    """One 3-channel series, 1000 samples per channel."""
    return Item(series(rng_for(0), 3, 1000), 1000, 3)


def config5() -> Item:
    """The six-variate pick-up-mask series of Sec. 4.1 (1000 samples each),
    the input of the transition-length sweep."""
    return Item(mask_series(1000), 1000, 6)


def config1(n: int = 64, size: int = 128) -> list[Item]:
    """n texture images of size x size (columns are the signals)."""
    return [Item(texture(rng_for(1, i), size, size), size, size) for i in range(n)]


def config2(n: int = 1024) -> list[Item]:
    """n face-like 112 x 92 images (M = 112 rows, N = 92 columns)."""
    return [Item(face_like(rng_for(2, i)), 112, 92) for i in range(n)]


def config3_shapes(n: int = 4096) -> list[tuple[int, int]]:
    """(M, channels) of the uneven series batch: channels U{2..16}, M
    log-uniform in [1e3, 6.5e4]."""
    rng = rng_for(3)
    out = []
    for _ in range(n):
        ch = int(rng.integers(2, 17))
        M = int(round(math.exp(rng.uniform(math.log(1e3), math.log(6.5e4)))))
        out.append((M, ch))
    return out


def config3_item(i: int, shape: tuple[int, int]) -> Item:
    M, ch = shape
    return Item(series(rng_for(3, i), ch, M), M, ch)


def config3_items(indices, shapes, threads: int = 16) -> list[Item]:
    """config3_item(i, shapes[i]) for every i in indices (the same arrays),
    with the seed children spawned once and the series generated on host
    threads."""
    from concurrent.futures import ThreadPoolExecutor

    indices = list(indices)
    if not indices:
        return []
    kids = np.random.SeedSequence(BASE_SEED + 3).spawn(max(indices) + 1)

    def one(i):
        M, ch = shapes[i]
        return Item(series(np.random.default_rng(kids[i]), ch, M), M, ch)

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        return list(ex.map(one, indices))


# The uneven batch is processed in waves of consecutive series, each wave one
# batched EEMD call whose realization buffers fit device memory comfortably.
CONFIG3_SERIES = 4096
CONFIG3_WAVES = 16


def config3_wave(w: int, n: int = CONFIG3_SERIES, waves: int = CONFIG3_WAVES) -> range:
    """Indices of the series in wave w (of `waves` equal consecutive groups)."""
    per = (n + waves - 1) // waves
    return range(w * per, min(n, (w + 1) * per))


def serving_request(i: int) -> tuple[str, Item]:
    """Request i of the serving mix: 60% textures 64..512 px, 30% series
    (2..16 channels x 1e3..65536 samples), 10% 1024 x 1024 textures."""
    rng = rng_for(4, i)
    u = rng.uniform()
    if u < 0.6:
        s = int(round(math.exp(rng.uniform(math.log(64), math.log(512)))))
        return "texture", Item(texture(rng, s, s), s, s)
    if u < 0.9:
        ch = int(rng.integers(2, 17))
        M = int(round(math.exp(rng.uniform(math.log(1e3), math.log(65536)))))
        return "series", Item(series(rng, ch, M), M, ch)
    return "large", Item(texture(rng, 1024, 1024), 1024, 1024)
