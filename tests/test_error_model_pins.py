"""Pins for the oracle's low-precision error model (oracle.stream.error_model_sd
and error_model_bias), CPU only.

The model predicts the spread of the score error (Eq. 1, Section "System
Implementation / Detection Algorithm") caused by rounding the centred inputs
to BF16, FP16 or FP8 E4M3 before the whitening product.  It is pinned by:
  * the formats' published value grids (the gap at 1.0 and in the subnormal
    range) and the one-band closed form;
  * an independent experiment: inputs rounded by round-to-nearest-even
    quantisers written from the bit layouts (tests/lowp_emu.py, no shared
    code with the model), scored exactly in FP64; the standardised error
    (observed - predicted mean) / predicted sd must have mean ~0 and mean
    square ~1 over thousands of pixels;
  * planted mistakes (a dropped factor, the covariance for its inverse, a gap
    one binade off, the variance of a uniform error over the wrong width, the
    second-order mean left out), each caught by one of the checks."""
import numpy as np
import pytest

from lowp_emu import q_bf16, q_e4m3, q_f16
from oracle import rx
from oracle import stream as ost
from paper_2602_13509_amd import synth

QUANT = {"bf16": q_bf16, "fp16": q_f16, "fp8": q_e4m3}


def test_format_gaps():
    # unit in the last place at 1.0: 2^(1 - p) with p = 8, 11, 4 significand bits
    assert ost.rounding_spacing(np.array([1.0]), "bf16")[0] == 2.0 ** -7
    assert ost.rounding_spacing(np.array([1.0]), "fp16")[0] == 2.0 ** -10
    assert ost.rounding_spacing(np.array([1.0]), "fp8")[0] == 2.0 ** -3
    assert ost.rounding_spacing(np.array([-3.0]), "fp8")[0] == 2.0 ** -2
    # subnormal steps: FP16 2^-24, E4M3 2^-9, below the smallest normal
    assert ost.rounding_spacing(np.array([2.0 ** -20]), "fp16")[0] == 2.0 ** -24
    assert ost.rounding_spacing(np.array([2.0 ** -8]), "fp8")[0] == 2.0 ** -9
    # the grids the quantisers realise have exactly these gaps
    for fmt, v in (("bf16", 1.0), ("fp16", 1.0), ("fp8", 1.0), ("fp8", 2.0 ** -8)):
        g = ost.rounding_spacing(np.array([v]), fmt)[0]
        assert QUANT[fmt](np.float32(v + 0.51 * g)) == v + g
        assert QUANT[fmt](np.float32(v + 0.49 * g)) == v


def test_one_band_closed_form():
    # B = 1: delta = d^2 / s2, d delta = 2 d e / s2 + e^2 / s2, e uniform over one gap g
    px = np.array([[3.0], [5.0], [10.5], [-2.0]])
    mu, cov = rx.stats(px)
    d = px[:, 0] - mu[0]
    for fmt in ("bf16", "fp16", "fp8"):
        g = ost.rounding_spacing(d, fmt)
        sd = ost.error_model_sd(px, mu, cov, fmt)
        bias = ost.error_model_bias(px, mu, cov, fmt)
        np.testing.assert_allclose(sd, 2 * np.abs(d) * g / np.sqrt(12) / cov[0, 0], rtol=1e-14)
        np.testing.assert_allclose(bias, g * g / 12 / cov[0, 0], rtol=1e-14)


def _experiment(seed, fmt, sd_fn=ost.error_model_sd, bias_fn=ost.error_model_bias):
    """Standardised score errors of quantised inputs over a 64 x 128 x 32
    Gaussian cube (the config-1 recipe), FP8 with per-band power-of-two
    scales 2^-floor(log2 sigma_k) as the whitening applies them."""
    g = synth.gauss_cube(seed, lines=64, samples=128, bands=32)
    px = rx.pixels(g.cube).astype(np.float64)
    mu, cov = rx.stats(px)
    scale = None
    if fmt == "fp8":
        e = np.floor(np.log2(np.sqrt(np.diag(cov))))
        scale = np.ldexp(1.0, (-e).astype(int))
    s = np.ones(px.shape[1]) if scale is None else scale
    d = px - mu[None, :]
    dq = QUANT[fmt]((d * s[None, :]).astype(np.float32)) / s[None, :]
    delta = np.einsum("pk,pk->p", d, np.linalg.solve(cov, d.T).T)
    delta_q = np.einsum("pk,pk->p", dq, np.linalg.solve(cov, dq.T).T)
    r = (delta_q - delta - bias_fn(px, mu, cov, fmt, band_scale=scale)) / sd_fn(px, mu, cov, fmt, band_scale=scale)
    return float(np.mean(r)), float(np.mean(r * r))


def _consistent(mean, msq):
    # 8192 pixels: the mean square of a unit-variance error has a sampling
    # sd of about sqrt(2 / 8192) = 0.016; the bounds leave room for the
    # linearisation and the quantisers' exactly representable values
    return abs(mean) <= 0.1 and 0.9 <= msq <= 1.15


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("seed", [5, 6])
def test_model_matches_quantised_scores(seed, fmt):
    mean, msq = _experiment(seed, fmt)
    assert _consistent(mean, msq), (fmt, seed, mean, msq)


# ---------------------------------------------------------------- planted mistakes
def _sd_mutant(kind):
    def f(px, mu, cov_r, fmt, band_scale=None):
        d = np.asarray(px, float) - mu[None, :]
        s = np.ones(d.shape[1]) if band_scale is None else band_scale
        g = ost.rounding_spacing(d * s[None, :], fmt) / s[None, :]
        if kind == "binade":
            g = 2 * g
        z = (d @ cov_r) if kind == "no inverse" else np.linalg.solve(cov_r, d.T).T
        v = np.sum(z * z * g * g, axis=1)
        if kind == "width":
            return 2 * np.sqrt(v / 3.0)           # uniform over [-g, g] instead of [-g/2, g/2]
        if kind == "factor 2":
            return np.sqrt(v / 12.0)
        return 2 * np.sqrt(v / 12.0)
    return f


SD_MUTANTS = ["factor 2", "no inverse", "binade", "width"]


@pytest.mark.parametrize("kind", SD_MUTANTS)
def test_sd_mutants_caught(kind):
    caught = False
    for fmt in ("bf16", "fp16"):
        mean, msq = _experiment(5, fmt, sd_fn=_sd_mutant(kind))
        caught |= not _consistent(mean, msq)
    assert caught, kind


def test_missing_second_order_mean_caught():
    mean, msq = _experiment(5, "fp8", bias_fn=lambda *a, **k: 0.0)
    assert not _consistent(mean, msq)
