"""Seeded synthetic push-broom hyperspectral inputs.

The paper's flight and bench data are not available, so every workload here
is drawn from a seeded generator shaped like the paper's sensor (900-sample
lines of 300 bands at 12 bits, Section "System Implementation / Data
Acquisition") and like the measured configurations (270 bands x 640 samples,
300 bands x 1024 samples, mixed-endmember scenes, implanted anomalies).

This module is shared by the tests, the benchmark and the oracle's fixtures.
It holds no part of the detector's arithmetic (no mean, covariance, inverse
or score): it only draws cubes.  Cubes are band-interleaved-by-line (BIL),
i.e. arrays of shape [lines][bands][samples]; pixel index p = line*S + sample.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FULL_SCALE_12BIT = 4095


def _haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of R's diagonal folded into Q (Mezzadri's construction)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    return q * np.sign(np.diag(r))[None, :]


def pixels_to_bil(px: np.ndarray, lines: int, samples: int) -> np.ndarray:
    """[lines*samples, bands] pixel rows -> BIL [lines][bands][samples]."""
    b = px.shape[1]
    return np.ascontiguousarray(px.reshape(lines, samples, b).transpose(0, 2, 1))


def bil_to_pixels(cube: np.ndarray) -> np.ndarray:
    """BIL [lines][bands][samples] -> [lines*samples, bands] pixel rows."""
    l, b, s = cube.shape
    return np.ascontiguousarray(cube.transpose(0, 2, 1).reshape(l * s, b))


# --------------------------------------------------------------------------
# Gaussian background with implanted anomalies (small float64 cube)
# --------------------------------------------------------------------------
@dataclass
class GaussCube:
    cube: np.ndarray          # BIL float64 [L][B][S]
    anomalies: np.ndarray     # sorted pixel indices of the implanted anomalies
    mean: np.ndarray          # population mean [B]
    cov: np.ndarray           # population covariance [B][B]


def gauss_cube(seed: int = 0, lines: int = 64, samples: int = 128, bands: int = 32,
               n_anomalies: int = 5, shift_sigmas: float = 6.0,
               log10_eig=(-4.0, -1.0)) -> GaussCube:
    """Background ~ N(mu, Q diag(D) Q^T), mu_k ~ U[0.1, 0.9], Q Haar,
    D_k = 10^U[lo, hi].  Each anomaly pixel is moved by shift_sigmas times the
    background standard deviation along its own random unit direction u,
    sigma_u = sqrt(u^T Sigma u)."""
    rng = np.random.default_rng(seed)
    n = lines * samples
    mu = rng.uniform(0.1, 0.9, bands)
    q = _haar_orthogonal(rng, bands)
    d = 10.0 ** rng.uniform(log10_eig[0], log10_eig[1], bands)
    z = rng.standard_normal((n, bands))
    px = mu[None, :] + (z * np.sqrt(d)[None, :]) @ q.T
    anom = np.sort(rng.choice(n, size=n_anomalies, replace=False))
    for p in anom:
        u = rng.standard_normal(bands)
        u /= np.linalg.norm(u)
        sigma_u = np.linalg.norm(np.sqrt(d) * (q.T @ u))
        px[p] += shift_sigmas * sigma_u * u
    cov = (q * d[None, :]) @ q.T
    return GaussCube(pixels_to_bil(px, lines, samples), anom, mu, cov)


# --------------------------------------------------------------------------
# Mixed-endmember 12-bit sensor cube (uint16)
# --------------------------------------------------------------------------
def smooth_endmembers(rng: np.random.Generator, bands: int, count: int,
                      full_scale: int = FULL_SCALE_12BIT) -> np.ndarray:
    """count smooth random spectra: full_scale * clip(c0 + sum of three
    Gaussian bumps, 0.05, 0.95), c0 ~ U[0.2, 0.5], heights ~ U[-0.2, 0.3],
    centres ~ U[0, B), widths ~ U[B/20, B/5]."""
    b = np.arange(bands, dtype=np.float64)
    out = np.empty((count, bands))
    for e in range(count):
        c0 = rng.uniform(0.2, 0.5)
        h = rng.uniform(-0.2, 0.3, 3)
        p = rng.uniform(0.0, bands, 3)
        w = rng.uniform(bands / 20.0, bands / 5.0, 3)
        s = c0 + sum(h[m] * np.exp(-((b - p[m]) ** 2) / (2.0 * w[m] ** 2)) for m in range(3))
        out[e] = full_scale * np.clip(s, 0.05, 0.95)
    return out


@dataclass
class SensorCube:
    cube: np.ndarray          # BIL uint16 [L][B][S]
    anomalies: np.ndarray     # sorted pixel indices carrying the unseen endmember
    endmembers: np.ndarray    # [5][B]


def sensor_cube(seed: int = 0, lines: int = 2000, samples: int = 640, bands: int = 270,
                anomaly_fraction: float = 5e-4, noise_frac: float = 0.01,
                full_scale: int = FULL_SCALE_12BIT, chunk_lines: int = 50) -> SensorCube:
    """Each pixel is a Dirichlet(1,1,1,1) mix of four smooth endmembers plus
    i.i.d. Gaussian noise (sd = noise_frac * full scale), rounded and clipped
    to [0, full_scale], stored as uint16.  round(anomaly_fraction * N) pixels
    chosen uniformly are mixed with a fifth, unseen endmember at abundance
    alpha ~ U[0.3, 1.0].  Generated in line chunks with per-chunk child
    generators so memory stays bounded at sensor scale."""
    rng = np.random.default_rng(seed)
    n = lines * samples
    em = smooth_endmembers(rng, bands, 5, full_scale)
    n_anom = int(round(anomaly_fraction * n))
    anom = np.sort(rng.choice(n, size=n_anom, replace=False)) if n_anom else np.zeros(0, np.int64)
    alpha_all = rng.uniform(0.3, 1.0, n_anom)
    cube = np.empty((lines, bands, samples), dtype=np.uint16)
    sd = noise_frac * full_scale
    for c0 in range(0, lines, chunk_lines):
        c1 = min(lines, c0 + chunk_lines)
        crng = np.random.default_rng([seed, 7, c0])
        m = (c1 - c0) * samples
        a = crng.dirichlet(np.ones(4), size=m)
        px = a @ em[:4]
        p0, p1 = c0 * samples, c1 * samples
        lo, hi = np.searchsorted(anom, p0), np.searchsorted(anom, p1)
        if hi > lo:
            idx = anom[lo:hi] - p0
            al = alpha_all[lo:hi][:, None]
            px[idx] = (1.0 - al) * px[idx] + al * em[4][None, :]
        px += crng.normal(0.0, sd, size=px.shape)
        np.rint(px, out=px)
        np.clip(px, 0, full_scale, out=px)
        cube[c0:c1] = px.astype(np.uint16).reshape(c1 - c0, samples, bands).transpose(0, 2, 1)
    return SensorCube(cube, anom, em)


# --------------------------------------------------------------------------
# Ill-conditioned float32 cube with a wide per-band dynamic range
# --------------------------------------------------------------------------
@dataclass
class StressCube:
    cube: np.ndarray          # BIL float32 [L][B][S]
    gains: np.ndarray         # per-band scale g_k, range exactly 1e3
    core_eigs: np.ndarray     # eigenvalues of the core covariance, range exactly 1e6


def stress_cube(seed: int = 0, lines: int = 5000, samples: int = 1024, bands: int = 300,
                log10_cond: float = 6.0, log10_range: float = 3.0,
                chunk_lines: int = 50) -> StressCube:
    """x = g * (mu + Q diag(sqrt(D)) z): core covariance Q diag(D) Q^T with
    D = 10^U[-log10_cond, 0] and two entries pinned to the ends (condition
    number exactly 10^log10_cond); per-band gains g_k = 10^(log10_range*v_k),
    v_k ~ U[0, 1] with two entries pinned to 0 and 1 (range exactly
    10^log10_range); mu_k ~ U[0.1, 0.9].  float32 output."""
    rng = np.random.default_rng(seed)
    q = _haar_orthogonal(rng, bands)
    u = rng.uniform(-log10_cond, 0.0, bands)
    u[0], u[-1] = -log10_cond, 0.0
    d = 10.0 ** u
    v = rng.uniform(0.0, 1.0, bands)
    v[1], v[-2] = 0.0, 1.0
    g = 10.0 ** (log10_range * v)
    mu = rng.uniform(0.1, 0.9, bands)
    a = q * np.sqrt(d)[None, :]
    cube = np.empty((lines, bands, samples), dtype=np.float32)
    for c0 in range(0, lines, chunk_lines):
        c1 = min(lines, c0 + chunk_lines)
        crng = np.random.default_rng([seed, 11, c0])
        z = crng.standard_normal(((c1 - c0) * samples, bands))
        px = (mu[None, :] + z @ a.T) * g[None, :]
        cube[c0:c1] = px.astype(np.float32).reshape(c1 - c0, samples, bands).transpose(0, 2, 1)
    return StressCube(cube, g, d)


# --------------------------------------------------------------------------
# Served streams: shapes, rates and Poisson block arrivals
# --------------------------------------------------------------------------
@dataclass
class StreamSpec:
    stream_id: int
    seed: int
    samples: int
    bands: int
    rate_lines_per_s: float
    arrivals: np.ndarray = field(repr=False)     # arrival time of each block [s]
    block_lines: np.ndarray = field(repr=False)  # lines in each block


def served_streams(seed: int = 0, n_streams: int = 16, duration_s: float = 30.0,
                   widths=(320, 640, 1024), band_counts=(120, 200, 270, 300),
                   rate_range=(100.0, 400.0), block_range=(16, 128)) -> list:
    """n_streams specs: the first len(widths)*len(band_counts) cover every
    (S, B) combination, the rest are seeded random picks.  Block sizes are
    uniform integers in block_range; block arrivals are a Poisson process of
    mean gap E[block]/rate over duration_s."""
    rng = np.random.default_rng([seed, 5])
    combos = [(s, b) for s in widths for b in band_counts]
    specs = []
    mean_block = 0.5 * (block_range[0] + block_range[1])
    for i in range(n_streams):
        if i < len(combos):
            s, b = combos[i]
        else:
            s = int(rng.choice(widths))
            b = int(rng.choice(band_counts))
        r = rng.uniform(*rate_range)
        gap = mean_block / r
        t, ts, ls = 0.0, [], []
        while True:
            t += rng.exponential(gap)
            if t > duration_s:
                break
            ts.append(t)
            ls.append(int(rng.integers(block_range[0], block_range[1] + 1)))
        specs.append(StreamSpec(i, seed * 1000 + i, s, b, r, np.array(ts), np.array(ls, dtype=np.int64)))
    return specs


def random_int_cube(seed: int, lines: int, samples: int, bands: int, hi: int = 16) -> np.ndarray:
    """Small BIL cube of uniform integers in [0, hi) (uint16), for exact tests."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, hi, size=(lines, bands, samples)).astype(np.uint16)


def score_sample(seed: int, n: int, bands: int = 270, nan_frac: float = 0.0) -> np.ndarray:
    """Seeded FP32 stand-ins for a cube's anomaly scores, for the transmission
    stage: chi-square-like background draws (gamma with shape bands/2, scale
    2), one in two thousand pixels a hundred times larger, exact zeros at a
    few places, and optionally NaN at a fraction nan_frac (a singular block's
    pixels).  Random numbers only; no part of the detector."""
    rng = np.random.default_rng(seed)
    d = rng.gamma(bands / 2.0, 2.0, size=n)
    hot = rng.random(n) < 5e-4
    d[hot] *= 100.0
    if n:
        d[rng.integers(0, n, size=max(1, n // 10000))] = 0.0
    if nan_frac > 0:
        d[rng.random(n) < nan_frac] = np.nan
    return d.astype(np.float32)


def raw_counts(seed: int, lines: int, bands: int, samples: int, bits: int = 12) -> np.ndarray:
    """Seeded uniform raw counts of a bits-bit sensor as uint16 BIL
    [lines][bands][samples] (the imager's raw 12-bit data, Section "System
    Implementation / Data Acquisition"), for the ingest binning."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << bits, size=(lines, bands, samples), dtype=np.uint16)
