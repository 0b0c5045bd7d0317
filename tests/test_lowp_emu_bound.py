"""The bound the low-precision whitening tests allow between the kernel and
the host emulation (FP32 sums against FP64 sums of the same operands) holds
for FP32 re-summations of the operands in several orders, and is far below
what a quantisation mistake makes (truncation instead of round-to-nearest-even,
the wrong 16-bit format, a mantissa bit short in FP8)."""
import numpy as np
import pytest

from lowp_emu import QUANT, emulate_scores, operands
from oracle import rx as orx
from paper_2602_13509_amd import synth


def setup(kind):
    B, S = 96, 64
    cube = (synth.sensor_cube(3, lines=4, samples=S, bands=B).cube if kind == "sensor"
            else synth.stress_cube(3, lines=4, samples=S, bands=B).cube)
    px = orx.pixels(cube)
    mu, cov = orx.stats(px)
    cov_r = cov + 1e-6 * np.trace(cov) / B * np.eye(B)
    w = np.linalg.inv(np.linalg.cholesky(cov_r))          # any whitener serves the emulation
    return px, mu, cov_r, w


def fp32_scores(dq, wq, f, order):
    """delta with every sum in FP32: y_i accumulated over j in the given
    order, then the squares summed in FP32."""
    n, B = dq.shape
    d32, w32 = dq.astype(np.float32), wq.astype(np.float32)
    acc = np.zeros((n, B), dtype=np.float32)
    for j in order:
        acc = acc + d32[:, j:j + 1] * w32[None, :, j]      # exact products, one FP32 rounding per addition
    y = acc * np.ldexp(np.float32(1.0), f).astype(np.float32)[None, :]
    s = np.zeros(n, dtype=np.float32)
    for i in order:
        s = s + y[:, i] * y[:, i]
    return s.astype(np.float64)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("kind", ["sensor", "stress"])
def test_fp32_resummations_stay_inside_the_bound(fmt, kind):
    px, mu, cov_r, w = setup(kind)
    emu, bound = emulate_scores(px, mu, cov_r, w, fmt, with_bound=True)
    dq, wq, f = operands(px, mu, cov_r, w, fmt)
    B = px.shape[1]
    for order in (range(B), range(B - 1, -1, -1), np.random.default_rng(0).permutation(B)):
        got = fp32_scores(dq, wq, f, order)
        assert np.all(np.abs(got - emu) <= bound)
    # blocked sums, as the matrix cores take them (numpy's FP32 product)
    y = (dq.astype(np.float32) @ wq.T.astype(np.float32)) * np.ldexp(np.float32(1.0), f).astype(np.float32)
    got = (y * y).sum(axis=1, dtype=np.float32).astype(np.float64)
    assert np.all(np.abs(got - emu) <= bound)


def q_bf16_trunc(x):
    f = np.asarray(x, dtype=np.float32)
    return (f.view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)


def q_e4m2(x):
    # one mantissa bit short: E4M3's exponent range, 2 fraction bits
    x = np.asarray(x, dtype=np.float32).astype(np.float64)
    a = np.abs(x)
    e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    e = np.maximum(e, -6.0)
    return np.sign(x) * np.minimum(np.rint(a / 2.0 ** e * 4.0) / 4.0 * 2.0 ** e, 448.0)


@pytest.mark.parametrize("fmt,wrong", [("bf16", q_bf16_trunc), ("bf16", QUANT["fp16"][0]), ("fp8", q_e4m2)])
@pytest.mark.parametrize("kind", ["sensor", "stress"])
def test_quantisation_mistakes_exceed_the_bound(fmt, wrong, kind):
    px, mu, cov_r, w = setup(kind)
    emu, bound = emulate_scores(px, mu, cov_r, w, fmt, with_bound=True)
    dq, wq, f = operands(px, mu, cov_r, w, fmt, q=wrong)
    y = (dq @ wq.T) * np.ldexp(1.0, f)[None, :]
    bad = (y * y).sum(axis=1)
    assert np.max(np.abs(bad - emu) / bound) > 10.0
