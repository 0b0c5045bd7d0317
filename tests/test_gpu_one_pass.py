"""One-pass scoring (RX_FLAG_ONE_PASS) on the GPU through the C ABI, against
the FP64 stream oracle in its one-pass mode: every block of a push is scored
with the window as it was before the push.  Pushes of several blocks, window
edges inside a push (the blocks from the edge on have no earlier window: NaN,
not ready), a push cut into two batches (more than 64 blocks), and one-block
pushes, which reduce to the causal reading."""
import numpy as np
import pytest

from gpu_util import assert_scores, oracle_stream_scores, say
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-9, 1e-11), "fp32": (1e-3, 1e-4), "bf16": (5e-2, 1e-2)}


def tol(prec, B):
    # The score sums B squared whitened terms with independent rounding
    # errors, so its relative error shrinks as 1/sqrt(B): below 270 bands the
    # 270-band BF16 bounds are scaled by sqrt(270 / B).
    f = max(1.0, (270.0 / B) ** 0.5) if prec == "bf16" else 1.0
    return TOL[prec][0] * f, TOL[prec][1] * f


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_pushes(rxm, cube, cfg, pushes, f64):
    st = rxm.RxStream(cfg)
    codes, l0 = [], 0
    x = dev(cube)
    for n in pushes:
        codes.append(st.rx_push_lines(x[l0:l0 + n]))
        l0 += n
    st.rx_sync()
    c = st.rx_get_counters()
    got = st.scores_host(f64=f64)
    stats = st.rx_get_stats()
    st.rx_destroy()
    return got, codes, c, stats


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("window_lines", [0, 16])
@pytest.mark.parametrize("S", [96, 128])
def test_one_pass_matches_oracle(rxm, prec, window_lines, S):
    L, B = 40, 40
    cube = synth.sensor_cube(41, lines=L, samples=S, bands=B).cube
    rho = 1e-6 if prec == "bf16" else 0.0
    pushes = [10, 14, 16]
    say(f"one-pass {prec} window {window_lines} S {S}")
    cfg = rxm.make_config(B, S, in_dtype=np.uint16, syrk=prec, whiten=prec, ridge_rel=rho, block_lines=8,
                          window_lines=window_lines, one_pass=True)
    got, codes, c, _ = run_pushes(rxm, cube, cfg, pushes, prec == "fp64")
    ref, o = oracle_stream_scores(cube, B, S, block_lines=8, window_lines=window_lines, rho=rho, pushes=pushes,
                                  one_pass=True)
    assert codes[0] == rxm.RX_E_NOTREADY                      # nothing before the first push
    assert c.notready_blocks == o.status.count("notready") >= 2
    assert c.singular_blocks == 0
    assert np.isnan(got[:10 * S]).all()
    assert_scores(got, ref, B, *tol(prec, B), label=f"one-pass {prec}")


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_one_pass_push_of_two_batches(rxm, prec):
    # 70 one-line blocks after an 8-line push: the launch takes at most 64
    # blocks, so the second batch must take the first batch's copy of the
    # window before the push, not the window after the first batch.
    L, B, S = 78, 24, 64
    cube = synth.sensor_cube(42, lines=L, samples=S, bands=B).cube
    rho = 1e-6 if prec == "bf16" else 0.0
    pushes = [8, 70]
    say(f"one-pass two batches {prec}")
    cfg = rxm.make_config(B, S, in_dtype=np.uint16, syrk=prec, whiten=prec, ridge_rel=rho, block_lines=1,
                          one_pass=True)
    got, codes, c, _ = run_pushes(rxm, cube, cfg, pushes, prec == "fp64")
    ref, o = oracle_stream_scores(cube, B, S, block_lines=1, rho=rho, pushes=pushes, one_pass=True)
    assert codes == [rxm.RX_E_NOTREADY, rxm.RX_OK]
    assert c.notready_blocks == o.status.count("notready") == 8
    assert_scores(got, ref, B, *tol(prec, B), label=f"one-pass two batches {prec}")


def test_one_pass_one_block_pushes_equal_causal(rxm):
    # One block per push: the window before the push is the window before the
    # block, so on the FP64 path (the same kernels) the scores equal the
    # causal mode's bit for bit.
    L, B, S, bl = 32, 40, 96, 4
    cube = synth.sensor_cube(43, lines=L, samples=S, bands=B).cube
    pushes = [bl] * (L // bl)
    mk = lambda **kw: rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64", block_lines=bl,
                                      window_lines=16, **kw)
    a, _, ca, sa = run_pushes(rxm, cube, mk(one_pass=True), pushes, True)
    b, _, cb, sb = run_pushes(rxm, cube, mk(causal=True), pushes, True)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert ca.notready_blocks == cb.notready_blocks
    assert sa[0] == sb[0] and np.array_equal(sa[1], sb[1]) and np.array_equal(sa[2], sb[2])


@pytest.mark.parametrize("B,S,window_lines", [(270, 640, 0), (270, 200, 12), (256, 96, 0), (100, 104, 12)])
def test_one_pass_single_read_kernel(rxm, B, S, window_lines):
    # BF16 products, 16-bit input with S % 8 == 0 and at most 272 bands: from
    # the second push on the window before the push is copied, and one kernel
    # forms each block's covariance partials and its scores from one read of
    # the lines (270 bands: two load rounds per wave; 200 and 104 samples: a
    # ragged last chunk).  With a 12-line window a block inside a push starts
    # a window: the same launch then centres it on its own shift and scores
    # it NaN.  Scores against the oracle, the statistics against the exact
    # integer covariance of the window; the third push is scored with
    # statistics the kernel formed.
    from oracle import rx as orx
    L, bl = 24, 4
    cube = synth.sensor_cube(44, lines=L, samples=S, bands=B).cube
    pushes = [8, 8, 8]
    say(f"one-pass single read B {B} S {S} window {window_lines}")
    cfg = rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6, block_lines=bl,
                          window_lines=window_lines, one_pass=True)
    got, codes, c, (n, mean, cov) = run_pushes(rxm, cube, cfg, pushes, False)
    ref, o = oracle_stream_scores(cube, B, S, block_lines=bl, window_lines=window_lines, rho=1e-6, pushes=pushes,
                                  one_pass=True)
    assert c.notready_blocks == o.status.count("notready")
    assert c.singular_blocks == 0
    assert_scores(got, ref, B, *tol("bf16", B), label=f"one-pass single read B={B} S={S}")
    w0 = 0 if window_lines == 0 else (L - 1) // window_lines * window_lines
    px = orx.pixels(cube[w0:])
    mu, cv = orx.stats(px)
    assert n == px.shape[0]
    assert np.max(np.abs(mean - mu)) <= 1e-12 * np.abs(mu).max()
    err = np.max(np.abs(cov - cv)) / np.abs(cv).max()
    say(f"  stats: max |cov err| / max|cov| = {err:.3e}")
    assert err <= 2e-2
