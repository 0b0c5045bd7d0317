"""FP64 CPU oracle for global RX scoring -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP library and never
imports it.

What it computes (the paper, Section "System Implementation / Detection
Algorithm", Eq. 1): every band is a variable and every pixel a sample; the
mean vector mu and the B x B covariance Sigma are taken over all pixels of
the set (anomalies included); a pixel s scores
    delta = (s - mu)^T Sigma^{-1} (s - mu),
the squared Mahalanobis distance.  A threshold marks pixels whose score is
above a configurable value; the paper normalises scores so the set's maximum
is 1 before thresholding (same section).

Readings taken where the paper is silent:
  * covariance normaliser 1/(N - ddof), ddof = 0 by default;
  * optional ridge lambda = rho * tr(Sigma) / B added to the diagonal;
  * strict ">" for the threshold; relative mode compares delta / max(delta);
  * top-k ties go to the lower pixel index;
  * float input: a pixel with any NaN or infinite band is not part of the
    set (left out of mu, Sigma and N) and scores NaN; integer input cannot
    hold such values.

Algorithm chosen to differ from the GPU path on purpose: integer input gets
exact integer moments (Python ints, correctly rounded division); float input
gets a two-pass mean/centred-product in FP64; scores use an LU solve
(numpy.linalg.solve) rather than a Cholesky factor and a whitening product.
"""
from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------- layout
def pixels(cube: np.ndarray) -> np.ndarray:
    """BIL [lines][bands][samples] -> pixel rows [lines*samples][bands];
    pixel index p = line * samples + sample (push-broom lines of samples,
    Section "System Architecture / Data Acquisition")."""
    l, b, s = cube.shape
    return cube.transpose(0, 2, 1).reshape(l * s, b)


# ---------------------------------------------------------------- statistics
def int_moments(px: np.ndarray):
    """Exact first and second raw moments of integer pixel rows.

    Returns (n, s1, s2) with s1 = sum_p x_p (int64 [B]) and s2 = sum_p x_p x_p^T
    (int64 [B][B]).  s2 is formed by a float64 product of integer-valued
    arrays; it is exact while every partial sum stays below 2^53, which is
    checked here from the largest input value."""
    x = np.asarray(px)
    if not np.issubdtype(x.dtype, np.integer):
        raise TypeError("int_moments needs integer pixels")
    n = x.shape[0]
    vmax = int(x.max()) if x.size else 0
    if n * vmax * vmax >= 2 ** 53:
        raise OverflowError("block too large for an exact float64 second moment")
    xf = x.astype(np.float64)
    s2 = xf.T @ xf
    s1 = x.astype(np.int64).sum(axis=0)
    return n, s1, np.rint(s2).astype(np.int64)


def cov_from_int_moments(n: int, s1, s2, ddof: int = 0):
    """Mean and covariance from exact integer moments, each entry correctly
    rounded to float64:  mu_j = s1_j / n,
    Sigma_jk = (n * s2_jk - s1_j * s1_k) / (n * (n - ddof))."""
    b = len(s1)
    s1i = [int(v) for v in s1]
    den = n * (n - ddof)
    mu = np.array([v / n for v in s1i], dtype=np.float64)
    cov = np.empty((b, b), dtype=np.float64)
    for j in range(b):
        for k in range(j + 1):
            num = n * int(s2[j, k]) - s1i[j] * s1i[k]
            cov[j, k] = cov[k, j] = num / den
    return mu, cov


def float_stats(px: np.ndarray, ddof: int = 0):
    """Two-pass FP64 mean and covariance of pixel rows."""
    x = np.asarray(px, dtype=np.float64)
    n = x.shape[0]
    mu = x.sum(axis=0) / n
    d = x - mu[None, :]
    cov = (d.T @ d) / (n - ddof)
    return mu, cov


def stats(px: np.ndarray, ddof: int = 0):
    """Set statistics (mu, Sigma) of pixel rows: exact for integer input,
    two-pass FP64 otherwise."""
    if np.issubdtype(np.asarray(px).dtype, np.integer):
        n, s1, s2 = int_moments(px)
        return cov_from_int_moments(n, s1, s2, ddof)
    return float_stats(px, ddof)


def regularise(cov: np.ndarray, rho: float) -> np.ndarray:
    """Sigma + lambda I with lambda = rho * tr(Sigma) / B (rho = 0: unchanged)."""
    if rho == 0.0:
        return cov
    b = cov.shape[0]
    lam = rho * np.trace(cov) / b
    return cov + lam * np.eye(b)


# ---------------------------------------------------------------- score (Eq. 1)
def scores(px: np.ndarray, mu: np.ndarray, cov: np.ndarray, chunk: int = 1 << 16) -> np.ndarray:
    """delta_p = (x_p - mu)^T Sigma^{-1} (x_p - mu) for every pixel row, with
    Sigma^{-1} applied by an LU solve (numpy.linalg.solve), in FP64."""
    x = np.asarray(px)
    out = np.empty(x.shape[0], dtype=np.float64)
    for p0 in range(0, x.shape[0], chunk):
        d = x[p0:p0 + chunk].astype(np.float64) - mu[None, :]
        z = np.linalg.solve(cov, d.T)
        out[p0:p0 + chunk] = np.einsum("pk,kp->p", d, z)
    return out


def finite_pixels(px: np.ndarray) -> np.ndarray:
    """bool per pixel row: every band finite (always true for integers)."""
    x = np.asarray(px)
    if np.issubdtype(x.dtype, np.integer):
        return np.ones(x.shape[0], dtype=bool)
    return np.isfinite(x).all(axis=1)


def rx_batch(cube: np.ndarray, ddof: int = 0, rho: float = 0.0) -> np.ndarray:
    """Global RX over one set of lines: statistics of every finite pixel of
    the cube, then Eq. 1 for every pixel (NaN for the others).  Returns
    scores in pixel order."""
    px = pixels(cube)
    ok = finite_pixels(px)
    mu, cov = stats(px[ok], ddof)
    out = np.full(px.shape[0], np.nan)
    out[ok] = scores(px[ok], mu, regularise(cov, rho))
    return out


# ---------------------------------------------------------------- masks
def mask_abs(delta: np.ndarray, tau: float) -> np.ndarray:
    """Pixels whose score is strictly above tau (NaN scores are not marked)."""
    d = np.asarray(delta, dtype=np.float64)
    with np.errstate(invalid="ignore"):
        return np.where(np.isnan(d), False, d > tau)


def mask_rel(delta: np.ndarray, tau: float) -> np.ndarray:
    """Scores normalised so the set maximum is 1, then strictly above tau
    (the paper's flights use tau = 0.110).  Compared as delta > tau * max."""
    d = np.asarray(delta, dtype=np.float64)
    m = np.nanmax(d) if np.any(~np.isnan(d)) else np.nan
    return mask_abs(d, tau * m)


def mask_topk(delta: np.ndarray, k: int) -> np.ndarray:
    """The k largest scores; ties go to the lower pixel index; NaN never."""
    d = np.asarray(delta, dtype=np.float64)
    idx = np.arange(d.size)
    key = np.where(np.isnan(d), -np.inf, d)
    order = np.lexsort((idx, -key))
    valid = order[~np.isnan(d[order])][:k]
    m = np.zeros(d.size, dtype=bool)
    m[valid] = True
    return m


def pack_bits(mask: np.ndarray) -> np.ndarray:
    """Bit-pack a boolean mask: bit j of byte q is pixel 8q + j."""
    return np.packbits(np.asarray(mask, dtype=bool), bitorder="little")
