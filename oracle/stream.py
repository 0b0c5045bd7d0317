"""Line-block streaming form of the FP64 oracle -- TEST INFRASTRUCTURE ONLY.

The paper scores every 1000-line cube with statistics of that whole cube
(Section "System Implementation / Detection Algorithm") and proposes a
line-based detector to cut latency (Section "Discussion / Performance").  The
streaming reading used throughout: lines arrive in blocks; each block first
joins the statistics window, then every pixel of the block is scored with
the updated statistics ("update, then score": the set always includes the
pixels being scored, as in the paper).  The window is either cumulative
(window_lines = 0) or restarts every window_lines lines (1000 reproduces the
paper's per-cube detector when one block is one cube).

This is the plain definition, recomputed from scratch for every block:
exact integer moments for integer input, a two-pass FP64 pass over every
pixel kept in the window for float input, and an LU solve for the scores.
Float pixels with a NaN or infinite band are not part of the window (N
counts the others), score NaN and are counted in `nonfinite`; a block is
"notready" when N <= B without a ridge, or N <= ddof.

causal=True takes the other reading of the line-based detector: every block
is scored with the window as it was before the block joined it (a block that
starts a window has no statistics and is "notready").

one_pass=True scores every block of a push with the window as it was before
the push: with one block per push this is the causal reading above, and a
push of several blocks is scored as one unit against the earlier lines (the
statistics still update block by block).  A block whose window started
inside the push, at or before it, has no earlier statistics and is
"notready".
"""
from __future__ import annotations

import numpy as np

from . import rx


class RxStreamOracle:
    def __init__(self, bands: int, samples: int, ddof: int = 0, rho: float = 0.0,
                 window_lines: int = 0, block_lines: int = 0, causal: bool = False,
                 one_pass: bool = False):
        self.B, self.S = bands, samples
        self.causal = causal
        self.one_pass = one_pass
        self.ddof, self.rho = ddof, rho
        self.window_lines = window_lines
        self.block_lines = block_lines
        self.lines_seen = 0
        self.nonfinite = 0        # float pixels with a non-finite band, over every push
        self.status = []          # per processed block: "ok" | "notready" | "singular"
        self._reset()

    # -- window state
    def _reset(self):
        self.n = 0
        self.s1 = np.zeros(self.B, dtype=np.int64)
        self.s2 = np.zeros((self.B, self.B), dtype=np.int64)
        self.float_px = []        # kept window pixels for float input
        self.is_int = None

    def _blocks(self, n_lines: int):
        """Split a push of n_lines into blocks: at most block_lines each (the
        last one of a push may be short) and never crossing a window edge."""
        out = []
        pos = self.lines_seen
        left = n_lines
        while left > 0:
            take = left if self.block_lines <= 0 else min(left, self.block_lines)
            if self.window_lines > 0:
                to_edge = self.window_lines - (pos % self.window_lines)
                take = min(take, to_edge)
            out.append((pos, take))
            pos += take
            left -= take
        return out

    def stats(self):
        """(N, mu, Sigma) of the current window."""
        if self.is_int:
            mu, cov = rx.cov_from_int_moments(self.n, self.s1, self.s2, self.ddof)
        else:
            mu, cov = rx.float_stats(np.concatenate(self.float_px), self.ddof)
        return self.n, mu, cov

    def push(self, lines: np.ndarray) -> np.ndarray:
        """lines: BIL [n_lines][B][S].  Returns FP64 scores of every pixel of
        the pushed lines, in pixel order."""
        assert lines.ndim == 3 and lines.shape[1] == self.B and lines.shape[2] == self.S
        out = []
        off = 0
        # one_pass: the window before the push (None once a window has
        # started inside the push)
        before = self._state() if self.one_pass else None
        for pos, take in self._blocks(lines.shape[0]):
            if self.window_lines > 0 and pos % self.window_lines == 0:
                self._reset()
                before = None
            blk = lines[off:off + take]
            off += take
            px = rx.pixels(blk)
            is_int = np.issubdtype(px.dtype, np.integer)
            if self.one_pass:
                out.append(self._score_with(before, px))  # the window before the push
            elif self.causal:
                out.append(self._score_block(px))         # the window before the block
            if self.is_int is None:
                self.is_int = is_int
            if is_int:
                n, s1, s2 = rx.int_moments(px)
                self.n += n
                self.s1 += s1
                self.s2 += s2
            else:
                ok = rx.finite_pixels(px)
                self.float_px.append(px[ok].astype(np.float64))
                self.n += int(ok.sum())
                self.nonfinite += int((~ok).sum())
            self.lines_seen = pos + take
            if not self.causal and not self.one_pass:
                out.append(self._score_block(px))         # update, then score
        return np.concatenate(out) if out else np.zeros(0)

    def _state(self):
        """A copy of the window state (count, moments, kept float pixels)."""
        return (self.n, self.s1.copy(), self.s2.copy(), list(self.float_px), self.is_int)

    def _score_with(self, state, px):
        """Scores of px with the window `state` (from _state); None: no window."""
        if state is None:
            self.status.append("notready")
            return np.full(px.shape[0], np.nan)
        now = self._state()
        self.n, self.s1, self.s2, self.float_px, self.is_int = state
        try:
            return self._score_block(px)
        finally:
            self.n, self.s1, self.s2, self.float_px, self.is_int = now

    def _score_block(self, px):
        if (self.n <= self.B and self.rho == 0.0) or self.n <= self.ddof:
            self.status.append("notready")
            return np.full(px.shape[0], np.nan)
        n, mu, cov = self.stats()
        cov_r = rx.regularise(cov, self.rho)
        try:
            np.linalg.cholesky(cov_r)
        except np.linalg.LinAlgError:
            self.status.append("singular")
            return np.full(px.shape[0], np.nan)
        self.status.append("ok")
        ok = rx.finite_pixels(px)
        out = np.full(px.shape[0], np.nan)
        out[ok] = rx.scores(px[ok], mu, cov_r)
        return out


def float_stats_chunked(chunks, ddof: int = 0):
    """Two-pass FP64 statistics over a cube too large to hold in FP64 at
    once.  `chunks` is a zero-argument callable returning an iterator of
    pixel-row arrays; it is called twice (mean pass, centred-product pass)."""
    n = 0
    s = None
    for c in chunks():
        c = np.asarray(c, dtype=np.float64)
        s = c.sum(axis=0) if s is None else s + c.sum(axis=0)
        n += c.shape[0]
    mu = s / n
    m2 = None
    for c in chunks():
        d = np.asarray(c, dtype=np.float64) - mu[None, :]
        m2 = d.T @ d if m2 is None else m2 + d.T @ d
    return n, mu, m2 / (n - ddof)


# Operand formats of the low-precision products: (significand bits p,
# including the implicit one; exponent of the smallest normal).  Unit
# roundoff u = 2^-p: 2^-8 for BF16, 2^-11 for FP16, 2^-4 for OCP FP8 E4M3.
FORMATS = {"bf16": (8, -126), "fp16": (11, -14), "fp8": (4, -6)}


def rounding_spacing(v: np.ndarray, fmt: str) -> np.ndarray:
    """Gap between adjacent values of the format around v (the unit in the
    last place): 2^(floor(log2|v|) + 1 - p) in the normal range, the fixed
    subnormal gap 2^(emin + 1 - p) below it."""
    p, emin = FORMATS[fmt]
    a = np.abs(np.asarray(v, dtype=np.float64))
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, emin)
    return np.ldexp(1.0, (e + 1 - p).astype(np.int64))


def error_model_sd(px: np.ndarray, mu: np.ndarray, cov_r: np.ndarray, fmt: str, band_scale=None):
    """First-order standard deviation of the score error caused by rounding
    each centred input value d_k = x_k - mu_k to the operand format before
    the whitening product (the input-rounding term of the precision design;
    the score is Eq. 1, Section "System Implementation / Detection
    Algorithm").

    Linearised: delta(d + e) - delta(d) ~= 2 z^T e with z = Sigma_r^{-1} d.
    Round to nearest leaves an error spread evenly over one gap g_k of the
    format around the value, variance g_k^2 / 12, independently per band, so

        sd = 2 sqrt( sum_k z_k^2 g_k^2 / 12 ).

    band_scale (optional, powers of two): the values are rounded as
    d_k * band_scale_k (which moves them within the format's range; FP8's
    subnormals depend on it) and scaled back.  With relative error taken as
    uniform in [-u, u] instead, the same sum gives the cruder envelope
    (2u / sqrt 3) sqrt(sum_k d_k^2 z_k^2).  A model of the input rounding
    only: rounding of the whitening operand and of the covariance product
    adds to the measured error."""
    d = np.asarray(px, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]
    s = np.ones(d.shape[1]) if band_scale is None else np.asarray(band_scale, dtype=np.float64)
    g = rounding_spacing(d * s[None, :], fmt) / s[None, :]
    z = np.linalg.solve(cov_r, d.T).T
    return 2.0 * np.sqrt(np.sum(z * z * g * g, axis=1) / 12.0)


def error_model_bias(px: np.ndarray, mu: np.ndarray, cov_r: np.ndarray, fmt: str, band_scale=None):
    """Second-order mean of the same score error: the rounding error e also
    enters the score as e^T Sigma_r^{-1} e, which is never negative; with the
    errors independent and centred its expectation is
    sum_k (Sigma_r^{-1})_kk g_k^2 / 12.  Small beside error_model_sd for BF16
    and FP16; for FP8 E4M3 (u = 2^-4) it is a few tenths of it."""
    d = np.asarray(px, dtype=np.float64) - np.asarray(mu, dtype=np.float64)[None, :]
    s = np.ones(d.shape[1]) if band_scale is None else np.asarray(band_scale, dtype=np.float64)
    g = rounding_spacing(d * s[None, :], fmt) / s[None, :]
    dinv = np.diag(np.linalg.inv(cov_r))
    return np.sum(dinv[None, :] * g * g, axis=1) / 12.0
