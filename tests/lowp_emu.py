"""Host emulation of the low-precision whitening arithmetic (test support).

Reproduces, in numpy, what the whitening kernel computes for the 8-value
operand formats: FP32 centring with the mean split into hi + lo FP32 parts,
power-of-two band scales 2^-e_k (e_k = floor(log2 sigma_k)), row scales 2^f_i
(row maximum in [2^top, 2^(top+1))), round-to-nearest-even into BF16 / FP16 /
OCP FP8 E4M3 (saturating at 448), exact products, FP64 sums.  It checks the
kernel's quantisation and scaling, not the method: its inputs (W, mean,
covariance) come from the library under test."""
import numpy as np


def q_bf16(x):
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def q_f16(x):
    return np.asarray(x, dtype=np.float32).astype(np.float16).astype(np.float64)


def q_e4m3(x):
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    s = np.sign(x)
    a = np.abs(x)
    out = np.empty_like(a)
    sub = a < 2.0 ** -6
    out[sub] = np.rint(a[sub] * 512.0) / 512.0
    n = ~sub
    e = np.floor(np.log2(np.where(n, a, 1.0)))
    m = np.rint(np.where(n, a, 1.0) / 2.0 ** e * 8.0) / 8.0
    out[n] = (m * 2.0 ** e)[n]
    return s * np.minimum(out, 448.0)


QUANT = {"bf16": (q_bf16, 14), "fp16": (q_f16, 14), "fp8": (q_e4m3, 7)}


def operands(px, mean, cov_r, w, fmt, q=None):
    """The whitening kernel's operands for format fmt: the centred, band-scaled
    pixels dq [n][B] and the row- and band-scaled whitener wq [B][B], both
    rounded to the format (as float64 values), and the row exponents f
    (y_i = 2^f_i sum_j wq_ij dq_j).  q replaces the format's rounding."""
    qf, top = QUANT[fmt]
    q = q or qf
    v = np.diag(cov_r)
    sc = 1.0 / np.sqrt(v)
    e = np.frexp(1.0 / sc)[1] - 1                       # floor(log2 sigma_k)
    wt = np.ldexp(w, e[None, :])
    m = np.abs(wt).max(axis=1)
    f = np.where(m > 0, np.frexp(np.where(m > 0, m, 1.0))[1] - 1 - top, 0)
    wq = q(np.ldexp(w, e[None, :] - f[:, None]).astype(np.float32))
    mhi = mean.astype(np.float32)
    mlo = (mean - mhi.astype(np.float64)).astype(np.float32)
    d = (px.astype(np.float32) - mhi[None, :]) - mlo[None, :]
    dq = q((d * np.ldexp(np.float32(1.0), -e)[None, :].astype(np.float32)).astype(np.float32))
    return dq, wq, f


def emulate_scores(px, mean, cov_r, w, fmt, with_bound=False):
    """Scores the whitening kernel produces for format fmt, given the FP64
    mean, regularised covariance (for the band scales) and whitener W.
    with_bound: also return, per pixel, the largest difference the kernel's
    FP32 sums may make against these FP64 sums of the same operands.

    The bound: y_i sums B exact products (16- and 8-bit operands multiply
    exactly in FP32).  At most 2 u32 of error per FP32 addition (round to
    nearest, or toward zero inside the matrix cores) gives
    |dy_i| <= e_i = 2 B u32 m_i, m_i = sum_j |Wq_ij dq_j| 2^f_i, in any
    summation order.  Then |y_i^2 - yh_i^2| <= 2 |y_i| e_i + e_i^2, and
    squaring and summing the B squares in FP32 adds at most 2 (B + 1) u32
    delta <= 2 (B + 1) u32 sum_i |y_i| m_i.  With scale = sum_i |y_i| m_i:
    |delta - emu| <= 6 (B + 1) u32 scale + 4 B^2 u32^2 sum_i m_i^2.  A relative
    1e-6 covers the final FP32 score and the FP64 sums here."""
    dq, wq, f = operands(px, mean, cov_r, w, fmt)
    y = (dq @ wq.T) * np.ldexp(1.0, f)[None, :]
    delta = (y * y).sum(axis=1)
    if not with_bound:
        return delta
    B = px.shape[1]
    u = 2.0 ** -24
    mag = (np.abs(dq) @ np.abs(wq).T) * np.ldexp(1.0, f)[None, :]
    scale = (np.abs(y) * mag).sum(axis=1)
    bound = (6.0 * (B + 1) * u * scale + 4.0 * B * B * u * u * (mag * mag).sum(axis=1)
             + 1e-6 * np.maximum(delta, 1e-3 * B))
    return delta, bound


def fp8_clip_count(px, mean, cov_r):
    """Centred, band-scaled input values that E4M3 clips (|v| > 464), formed
    as the whitening kernel forms them (FP32 centring with the split mean,
    exact power-of-two band scale)."""
    sc = 1.0 / np.sqrt(np.diag(cov_r))
    e = np.frexp(1.0 / sc)[1] - 1                       # floor(log2 sigma_k), as in emulate_scores
    mhi = mean.astype(np.float32)
    mlo = (mean - mhi.astype(np.float64)).astype(np.float32)
    d = (px.astype(np.float32) - mhi[None, :]) - mlo[None, :]
    dq = (d * np.ldexp(np.float32(1.0), -e)[None, :].astype(np.float32)).astype(np.float32)
    return int(np.count_nonzero(np.abs(dq) > np.float32(464.0)))
