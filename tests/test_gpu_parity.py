"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Tolerances (rel_err = |d_gpu - d_ref| / max(d_ref, 1e-3 B)), fixed before the
first GPU run:
  FP64 path            max 1e-9, p99 1e-11   (stress cube: 1e-7 / 1e-9)
  FP32 path            max 1e-3, p99 1e-4
  BF16 SYRK + BF16 whitening with the 1e-6 ridge: max 5e-2, p99 1e-2
  FP16 / FP8 whitening: reported only (their errors are shown, not bounded)
Masks must agree bit for bit wherever the oracle score is farther than the
tolerance from the threshold (twice that in relative mode)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from gpu_util import assert_mask, assert_scores, err_summary, oracle_stream_scores, say
from oracle import rx as orx
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu

TOL = {"fp64": (1e-9, 1e-11), "fp32": (1e-3, 1e-4), "bf16": (5e-2, 1e-2)}


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_stream(rxm, cube, prec_s, prec_w, pushes=None, device_input=True, **cfgkw):
    B, S = cube.shape[1], cube.shape[2]
    cfg = rxm.make_config(B, S, in_dtype=cube.dtype, syrk=prec_s, whiten=prec_w, **cfgkw)
    st = rxm.RxStream(cfg)
    if pushes is None:
        pushes = [cube.shape[0]]
    l0 = 0
    for n in pushes:
        part = cube[l0:l0 + n]
        st.rx_push_lines(dev(part) if device_input else np.ascontiguousarray(part))
        l0 += n
    st.rx_sync(allow=(rxm.RX_E_SINGULAR,))
    return st


# ---------------------------------------------------------------------------- golden exact rationals
def test_golden_exact_rationals_fp64_path(rxm):
    path = os.path.join(os.path.dirname(__file__), "golden", "tiny_exact.json")
    for c in json.load(open(path)):
        cube = np.array(c["cube"], dtype=np.uint16)
        ref = np.array([float(Fraction(s)) for s in c["scores"]])
        rn, rd = c["ridge_rel"]
        say(f"golden B={c['bands']} S={c['samples']} L={c['lines']} ddof={c['ddof']}")
        st = run_stream(rxm, cube, "fp64", "fp64", ddof=c["ddof"], ridge_rel=rn / rd)
        got = st.scores_host(f64=True)
        assert_scores(got, ref, c["bands"], 1e-9, 1e-9, "golden fp64")


# ---------------------------------------------------------------------------- Gaussian cube, FP64
@pytest.mark.parametrize("seed", [0, 1])
def test_gauss_cube_fp64_scores_and_topk(rxm, seed):
    g = synth.gauss_cube(seed)
    say(f"gauss seed={seed} 64x128x32 f64")
    ref = orx.rx_batch(g.cube)
    st = run_stream(rxm, g.cube, "fp64", "fp64")
    m = st.mask_host(0.0, rxm.RX_THR_TOPK, 5)
    assert np.array_equal(np.flatnonzero(m), g.anomalies)
    got = st.scores_host(f64=True)
    assert_scores(got, ref, 32, *TOL["fp64"], label="gauss fp64")
    assert abs(got.mean() - 32) < 1e-8


def test_gauss_cube_mixed_paths(rxm):
    g = synth.gauss_cube(3)
    ref = orx.rx_batch(g.cube)
    for p in ("fp32", "bf16"):
        st = run_stream(rxm, g.cube, p, p)
        m = st.mask_host(0.0, rxm.RX_THR_TOPK, 5)      # the mask does not consume the scores
        assert np.array_equal(np.flatnonzero(m), g.anomalies)
        got = st.scores_host()
        say(f"gauss {p}: max/p99 rel {err_summary(got, ref, 32)}")
        if p == "fp32":
            assert_scores(got, ref, 32, *TOL["fp32"], label="gauss fp32")


# ---------------------------------------------------------------------------- sensor cube, several tiles + ragged tail
@pytest.mark.parametrize("samples", [200, 203])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_sensor_cube_blocks(rxm, prec, samples):
    B = 270
    cube = synth.sensor_cube(11, lines=90, samples=samples, bands=B).cube
    rho = 1e-6 if prec == "bf16" else 0.0
    say(f"sensor 90x{samples}x{B} u16 prec={prec} block_lines=40 rho={rho}")
    ref, _ = oracle_stream_scores(cube, B, samples, block_lines=40, rho=rho)
    st = run_stream(rxm, cube, prec, prec, block_lines=40, ridge_rel=rho)
    got = st.scores_host(f64=(prec == "fp64"))
    assert_scores(got, ref, B, *TOL[prec], label=f"sensor {prec} S={samples}")


@pytest.mark.parametrize("samples", [203, 640])
@pytest.mark.parametrize("whiten", ["bf16", "fp16"])
def test_fp16_covariance_product(rxm, samples, whiten):
    # FP16 operands in the covariance product (FP32 accumulation) at 270
    # bands with the 1e-6 ridge, against the oracle with the same ridge, at
    # the BF16 row's tolerance (FP16 rounds 8x finer than BF16).  640-sample
    # rows are whole 16-byte multiples and take the direct-to-LDS kernel;
    # 203-sample rows are not and take the register-staged one.  Three
    # blocks: several covariance splits per block and a short last block.
    B, BL = 270, 16
    lines = 40
    cube = synth.sensor_cube(31, lines=lines, samples=samples, bands=B).cube
    say(f"fp16 covariance: {lines}x{samples}x{B} u16, whitening {whiten}, blocks of {BL}, rho 1e-6")
    ref, o = oracle_stream_scores(cube, B, samples, block_lines=BL, rho=1e-6)
    st = run_stream(rxm, cube, "fp16", whiten, block_lines=BL, ridge_rel=1e-6)
    got = st.scores_host()
    assert_scores(got, ref, B, *TOL["bf16"], label=f"fp16 covariance + {whiten} whitening S={samples}")
    n, mu, cov = st.rx_get_stats()
    _, mu_r, cov_r = o.stats()
    err = np.max(np.abs(cov - cov_r)) / np.abs(cov_r).max()
    say(f"  fp16 covariance: max |cov err| / max|cov| = {err:.3e}")
    assert np.max(np.abs(mu - mu_r)) <= 1e-12 * np.abs(mu_r).max()
    assert err <= 2.5e-3      # the BF16 bound of the statistics test (2e-2) over 8: FP16 rounds 2^3 finer


def test_sensor_cube_host_input_and_push_split(rxm):
    B, S = 120, 96
    cube = synth.sensor_cube(12, lines=60, samples=S, bands=B).cube
    pushes = [7, 13, 40]
    ref, _ = oracle_stream_scores(cube, B, S, pushes=pushes)
    st = run_stream(rxm, cube, "fp64", "fp64", pushes=pushes, device_input=False)
    assert_scores(st.scores_host(f64=True), ref, B, *TOL["fp64"], label="host input, pushes 7/13/40")


def test_large_host_pushes_equal_device_pushes(rxm):
    # Host pushes of several 8 MiB copy chunks (three and five copy threads,
    # a ragged last chunk, chunk edges inside lines), back to back so that the
    # second push refills pinned buffers whose transfers are queued: the
    # scores and statistics equal those of the same lines pushed from device
    # memory, bit for bit.
    B, S = 270, 256
    cube = synth.sensor_cube(16, lines=400, samples=S, bands=B).cube
    pushes = [150, 250]
    say(f"large host pushes: {pushes} lines of {S}x{B} u16 ({cube.nbytes >> 20} MiB)")
    kw = dict(block_lines=50, ridge_rel=1e-6)
    a = run_stream(rxm, cube, "bf16", "bf16", pushes=pushes, device_input=False, **kw)
    b = run_stream(rxm, cube, "bf16", "bf16", pushes=pushes, device_input=True, **kw)
    got = a.scores_host()                     # pops the scores
    assert np.array_equal(got.view(np.uint32), b.scores_host().view(np.uint32))
    sa, sb = a.rx_get_stats(), b.rx_get_stats()
    assert sa[0] == sb[0] and np.array_equal(sa[1], sb[1]) and np.array_equal(sa[2], sb[2])
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=50, rho=1e-6, pushes=pushes)
    assert_scores(got, ref, B, *TOL["bf16"], label="large host pushes")
    a.rx_destroy()
    b.rx_destroy()


def test_window_reset_matches_independent_cubes(rxm):
    B, S = 64, 80
    cube = synth.sensor_cube(13, lines=75, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=10, window_lines=25)
    st = run_stream(rxm, cube, "fp64", "fp64", block_lines=10, window_lines=25)
    assert_scores(st.scores_host(f64=True), ref, B, *TOL["fp64"], label="window 25, blocks 10")


@pytest.mark.parametrize("B", [1, 2, 17, 31, 64, 65, 300])
def test_band_counts(rxm, B):
    S = 72
    cube = synth.sensor_cube(14, lines=12, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S)
    st = run_stream(rxm, cube, "fp64", "fp64")
    assert_scores(st.scores_host(f64=True), ref, B, *TOL["fp64"], label=f"B={B} fp64")
    st2 = run_stream(rxm, cube, "fp32", "fp32")
    assert_scores(st2.scores_host(), ref, B, *TOL["fp32"], label=f"B={B} fp32")


@pytest.mark.parametrize("B,S", [(16, 128), (100, 128), (200, 100), (272, 128), (288, 128), (289, 96),
                                 (320, 128), (320, 100)])
def test_band_counts_mixed_path(rxm, B, S):
    # The BF16 path across the factor kernel's tile counts (T = 1 .. 20: the
    # register-only sweep, the LDS overflow tiles from 273 bands, the largest
    # 320), the whitening kernel's 32-band step counts and both row
    # alignments (S % 8 == 0: 16-byte rows; S = 100, 8-byte rows), against
    # the FP64 oracle with the same ridge.  The score is a sum of B squared
    # whitened terms whose rounding errors are independent, so its relative
    # error shrinks as 1/sqrt(B): below 270 bands the 270-band BF16 bounds
    # are scaled by sqrt(270 / B).
    cube = synth.sensor_cube(15, lines=24, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=8, rho=1e-6)
    st = run_stream(rxm, cube, "bf16", "bf16", ridge_rel=1e-6, block_lines=8)
    f = max(1.0, (270.0 / B) ** 0.5)
    assert_scores(st.scores_host(), ref, B, TOL["bf16"][0] * f, TOL["bf16"][1] * f, label=f"B={B} S={S} bf16")


@pytest.mark.parametrize("S", [1, 3, 7, 65])
def test_narrow_lines_mixed_path(rxm, S):
    # Lines narrower than one 64-sample chunk or with a ragged chunk: the
    # register-staged covariance and the chunk whitening (element loads),
    # many lines per block.
    B = 30
    cube = synth.sensor_cube(16, lines=320, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=64, rho=1e-6)
    st = run_stream(rxm, cube, "bf16", "bf16", ridge_rel=1e-6, block_lines=64)
    f = (270.0 / B) ** 0.5                       # as in test_band_counts_mixed_path
    assert_scores(st.scores_host(), ref, B, TOL["bf16"][0] * f, TOL["bf16"][1] * f, label=f"S={S} bf16")


# ---------------------------------------------------------------------------- statistics and factor hooks
def test_stats_match_exact_integer_covariance(rxm):
    B, S = 270, 128
    cube = synth.sensor_cube(15, lines=30, samples=S, bands=B).cube
    px = orx.pixels(cube)
    mu, cov = orx.stats(px)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-5), ("bf16", 2e-2)):
        st = run_stream(rxm, cube, prec, prec, block_lines=8, ridge_rel=1e-6 if prec == "bf16" else 0.0)
        n, m, c = st.rx_get_stats()
        assert n == px.shape[0]
        assert np.max(np.abs(m - mu)) <= 1e-12 * np.abs(mu).max()
        err = np.max(np.abs(c - cov)) / np.abs(cov).max()
        say(f"  stats {prec}: max |cov err| / max|cov| = {err:.3e}")
        assert err <= tol


def test_whitener_inverts_regularised_covariance(rxm):
    B, S = 40, 64
    cube = synth.sensor_cube(16, lines=20, samples=S, bands=B).cube
    st = run_stream(rxm, cube, "fp64", "fp64", ridge_rel=1e-3)
    w = st.rx_get_whitener()
    assert np.all(np.triu(w, 1) == 0)
    _, mu, cov = st.rx_get_stats()
    cov_r = orx.regularise(cov, 1e-3)
    # W Sigma_r W^T = I  (whitened identity)
    assert np.max(np.abs(w @ cov_r @ w.T - np.eye(B))) <= 1e-10


def test_set_stats_roundtrip(rxm):
    B, S = 32, 64
    a = synth.sensor_cube(17, lines=20, samples=S, bands=B).cube
    b = synth.sensor_cube(18, lines=5, samples=S, bands=B).cube
    s1 = run_stream(rxm, a, "fp64", "fp64")
    n, m, c = s1.rx_get_stats()
    s1.scores_host(f64=True)
    s1.rx_push_lines(dev(b))
    want = s1.scores_host(f64=True)
    s2 = rxm.RxStream(rxm.make_config(B, S, syrk="fp64", whiten="fp64"))
    s2.rx_set_stats(n, m, c)
    s2.rx_push_lines(dev(b))
    got = s2.scores_host(f64=True)
    assert_scores(got, want, B, 1e-9, 1e-11, "restored stream")


# ---------------------------------------------------------------------------- degenerate cases
def test_not_ready_then_ready(rxm):
    B, S = 16, 4
    cube = synth.sensor_cube(19, lines=10, samples=S, bands=B).cube
    cfg = rxm.make_config(B, S, syrk="fp64", whiten="fp64")
    st = rxm.RxStream(cfg)
    r = st.rx_push_lines(dev(cube[:2]))               # N = 8 <= B
    assert r == rxm.RX_E_NOTREADY
    got = st.scores_host(f64=True)
    assert np.all(np.isnan(got))
    assert st.rx_push_lines(dev(cube[2:])) == rxm.RX_OK   # N = 40 > B
    ref, _ = oracle_stream_scores(cube, B, S, pushes=[2, 8])
    assert_scores(st.scores_host(f64=True), ref[8:], B, 1e-9, 1e-11, "after not-ready")


def test_constant_band_is_singular_without_ridge(rxm):
    B, S = 8, 32
    cube = synth.sensor_cube(20, lines=6, samples=S, bands=B).cube
    cube[:, 3, :] = 1000
    st = run_stream(rxm, cube, "fp64", "fp64")
    assert st.rx_get_counters().singular_blocks == 1
    assert np.all(np.isnan(st.scores_host(f64=True)))
    st2 = run_stream(rxm, cube, "fp64", "fp64", ridge_rel=1e-3)
    ref, _ = oracle_stream_scores(cube, B, S, rho=1e-3)
    assert_scores(st2.scores_host(f64=True), ref, B, 1e-9, 1e-11, "constant band + ridge")


def test_sync_reports_singular(rxm):
    B, S = 8, 32
    cube = synth.sensor_cube(21, lines=6, samples=S, bands=B).cube
    cube[:, 0, :] = 7
    cfg = rxm.make_config(B, S, syrk="fp64", whiten="fp64")
    st = rxm.RxStream(cfg)
    st.rx_push_lines(dev(cube))
    assert st.rx_sync(allow=(rxm.RX_E_SINGULAR,)) == rxm.RX_E_SINGULAR
    assert st.rx_sync() == rxm.RX_OK          # sticky error is cleared


# ---------------------------------------------------------------------------- masks
def test_masks_abs_rel_topk(rxm):
    B, S = 270, 128
    cube = synth.sensor_cube(22, lines=40, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S)
    for prec in ("fp64", "fp32"):
        st = run_stream(rxm, cube, prec, prec)
        tol = TOL[prec][0]
        tau = float(np.quantile(ref, 1 - 5e-4))
        assert_mask(st.mask_host(tau, rxm.RX_THR_ABS), ref, tau, tol, B, f"{prec} abs")
        assert_mask(st.mask_host(0.110, rxm.RX_THR_REL_MAX), ref, 0.110 * ref.max(), 2 * tol, B, f"{prec} rel")
        k = 7
        m = st.mask_host(0.0, rxm.RX_THR_TOPK, k)
        assert m.sum() == k
        order = np.lexsort((np.arange(ref.size), -ref))
        if ref[order[k - 1]] - ref[order[k]] > 2 * tol * ref[order[k - 1]]:
            assert np.array_equal(np.flatnonzero(m), np.sort(order[:k]))


def test_topk_ties_go_to_lower_index(rxm):
    # identical pixels produce exactly tied scores on the GPU
    B, S = 4, 64
    base = synth.sensor_cube(23, lines=3, samples=S, bands=B).cube
    base[1, :, 10] = base[0, :, 5] = base[2, :, 60] = np.array([4000, 10, 4000, 10], dtype=np.uint16)
    st = run_stream(rxm, base, "fp64", "fp64")
    m = st.mask_host(0.0, rxm.RX_THR_TOPK, 2)
    d = st.scores_host(f64=True)
    tied = np.flatnonzero(d == d.max())
    assert tied.size == 3
    assert np.array_equal(np.flatnonzero(m), tied[:2])


# ---------------------------------------------------------------------------- low precision on the stress cube
def test_stress_cube_precisions(rxm):
    B, S = 300, 128
    sc = synth.stress_cube(3, lines=40, samples=S, bands=B)
    ref, _ = oracle_stream_scores(sc.cube, B, S)
    st = run_stream(rxm, sc.cube, "fp64", "fp64")
    assert_scores(st.scores_host(f64=True), ref, B, 1e-7, 1e-9, "stress fp64")
    for w in ("fp16", "fp8"):
        st = run_stream(rxm, sc.cube, "fp64", w)
        got = st.scores_host()
        mx, p99 = err_summary(got, ref, B)
        say(f"  stress fp64 stats + {w} whitening: max rel {mx:.3e}, p99 rel {p99:.3e} (reported)")
        assert np.all(np.isfinite(got))


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
@pytest.mark.parametrize("kind", ["sensor", "stress"])
def test_lowp_whitening_matches_host_emulation(rxm, fmt, kind):
    # The kernel's quantisation (band/row power-of-two scales, RNE, FP8
    # saturation) and matrix-core accumulation against a numpy emulation of
    # the same arithmetic built from the library's own FP64 W and statistics.
    from lowp_emu import emulate_scores
    if kind == "sensor":
        B, S = 270, 128
        cube = synth.sensor_cube(25, lines=20, samples=S, bands=B).cube
    else:
        B, S = 300, 128
        cube = synth.stress_cube(4, lines=20, samples=S, bands=B).cube
    st = run_stream(rxm, cube, "fp64", fmt)
    got = st.scores_host()
    w = st.rx_get_whitener()
    n, mean, cov = st.rx_get_stats()
    # Allowed: the kernel's FP32 sums alone (the bound's derivation is in
    # emulate_scores), about 6 B u32 relative: far below one step of any of
    # the operand formats (2^-8 .. 2^-3 relative), so a quantisation mistake fails.
    emu, bound = emulate_scores(orx.pixels(cube), mean, cov, w, fmt, with_bound=True)
    e = np.abs(got - emu)
    say(f"  {kind} {fmt}: kernel vs emulation max |diff|/bound {np.max(e / bound):.3e}, "
        f"max rel {np.max(e / np.maximum(emu, 1e-3 * B)):.3e}")
    assert np.all(e <= bound)
    if fmt == "fp8":
        from lowp_emu import fp8_clip_count
        clipped = st.rx_get_counters().fp8_saturated
        say(f"  {kind} fp8: {clipped} operand values saturated")
        assert clipped == fp8_clip_count(orx.pixels(cube), mean, cov)


def test_determinism_bitwise(rxm):
    B, S = 270, 128
    cube = synth.sensor_cube(24, lines=30, samples=S, bands=B).cube
    a = run_stream(rxm, cube, "bf16", "bf16", block_lines=10, ridge_rel=1e-6).scores_host()
    b = run_stream(rxm, cube, "bf16", "bf16", block_lines=10, ridge_rel=1e-6).scores_host()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("fmt,B,S", [("bf16", 270, 200), ("fp16", 270, 200), ("fp8", 270, 200), ("fp8", 180, 200),
                                     ("bf16", 70, 100), ("bf16", 270, 100), ("fp8", 180, 100)])
def test_tile_whitening_equals_chunk_whitening_bitwise(rxm, fmt, B, S):
    # 16-bit rows with 8-byte aligned starts and S % 4 == 0 take the
    # 64-pixel tile kernel; the same lines pushed from a buffer offset by one
    # element take the chunk kernel.  Both centre, scale and round identically
    # and run the same matrix-core chains, so with FP64 statistics (computed
    # identically on both routes) the scores must match bit for bit.  S = 200
    # and S = 100 (S % 8 = 4, 8-byte rows like the imager's 900 samples)
    # leave a ragged last tile; 3 blocks put block boundaries inside
    # workgroup ranges.
    import torch
    cube = synth.sensor_cube(26, lines=90, samples=S, bands=B).cube
    say(f"tile vs chunk whitening {fmt}: 90x{S}x{B} u16, blocks of 40")
    a = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten=fmt, block_lines=40))
    a.rx_push_lines(dev(cube))
    flat = torch.empty(cube.size + 1, dtype=torch.int16, device="cuda")
    flat[1:].copy_(dev(cube.view(np.int16).reshape(-1)))
    off = flat[1:]
    assert off.data_ptr() % 16 == 2
    b = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten=fmt, block_lines=40))
    b.rx_push_lines(off.view(cube.shape))   # same bits; the library reads them as uint16
    a.rx_sync()
    b.rx_sync()
    sa, sb = a.scores_host(), b.scores_host()
    assert np.all(np.isfinite(sa))
    assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))


@pytest.mark.parametrize("syrk", ["bf16", "fp16", "fp32"])
def test_eight_byte_rows_equal_element_loads_bitwise(rxm, syrk):
    # 900-sample-like rows (S % 8 = 4): from an 8-byte aligned buffer the
    # register-staged covariance kernels and the tile whitening load 8 bytes
    # at a time; from a buffer offset by one element they load element by
    # element (and the whitening takes the chunk kernel).  Same values, same
    # arithmetic: the scores match bit for bit, one push and several.
    import torch
    B, S, BL = 70, 100, 30
    cube = synth.sensor_cube(48, lines=4 * BL, samples=S, bands=B).cube
    flat = torch.empty(cube.size + 1, dtype=torch.int16, device="cuda")
    flat[1:].copy_(dev(cube.view(np.int16).reshape(-1)))
    off = flat[1:].view(cube.shape)
    assert off.data_ptr() % 8 == 2
    x = dev(cube)
    cfg = dict(in_dtype=np.uint16, syrk=syrk, whiten="bf16", ridge_rel=1e-6, block_lines=BL)
    a = rxm.RxStream(rxm.make_config(B, S, **cfg))
    b = rxm.RxStream(rxm.make_config(B, S, **cfg))
    a.rx_push_lines(x[:BL])
    a.rx_push_lines(x[BL:])
    b.rx_push_lines(off[:BL])
    b.rx_push_lines(off[BL:])
    a.rx_sync()
    b.rx_sync()
    sa, sb = a.scores_host(), b.scores_host()
    assert np.all(np.isfinite(sa))
    assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))


def test_push_pattern_and_queue_mode_do_not_change_scores(rxm):
    # A lone one-block push to an idle stream runs on one HIP queue, other
    # pushes over three; switching between the two must not change a bit:
    # every block's arithmetic is fixed by the block, not by how it arrived.
    import torch
    B, S, BL = 64, 256, 16
    cube = synth.sensor_cube(41, lines=8 * BL, samples=S, bands=B).cube
    x = dev(cube)
    ref = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6,
                                       block_lines=BL))
    ref.rx_push_lines(x)
    ref.rx_sync()
    want = ref.scores_host()
    ref.rx_destroy()
    st = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6,
                                      block_lines=BL))
    l0 = 0
    for nb, sync in [(1, True), (1, False), (3, False), (1, True), (1, False), (1, False)]:
        st.rx_push_lines(x[l0:l0 + nb * BL])
        l0 += nb * BL
        if sync:
            st.rx_sync()
    st.rx_sync()
    got = st.scores_host()
    st.rx_destroy()
    assert l0 == cube.shape[0]
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_covariance_split_sharing_does_not_change_scores(rxm, fmt):
    # Launches with few covariance splits share each split among 2 or 4
    # workgroups (fragment columns dealt out among them); a launch with many
    # keeps one per split.  50-line blocks of 640 samples have 6 splits: the
    # 24-block push takes one workgroup per split, pushes of 1 to 6 blocks
    # four, the 11-block push two.  Scores must match bit for bit.
    B, S, BL = 150, 640, 50
    cube = synth.sensor_cube(43, lines=24 * BL, samples=S, bands=B).cube
    x = dev(cube)
    assert rxm.split_plan(rxm.make_config(B, S, in_dtype=np.uint16, syrk=fmt, whiten=fmt, block_lines=BL),
                          BL)[0] == 6

    def cfg():
        return rxm.make_config(B, S, in_dtype=np.uint16, syrk=fmt, whiten=fmt, ridge_rel=1e-6, block_lines=BL)
    ref = rxm.RxStream(cfg())
    ref.rx_push_lines(x)
    ref.rx_sync()
    want = ref.scores_host()
    ref.rx_destroy()
    st = rxm.RxStream(cfg())
    l0 = 0
    for nb in (1, 1, 5, 11, 6):
        st.rx_push_lines(x[l0:l0 + nb * BL])
        l0 += nb * BL
        st.rx_sync()
    got = st.scores_host()
    st.rx_destroy()
    assert l0 == cube.shape[0]
    assert np.all(np.isfinite(want))
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))


def test_resident_pushes_equal_device_pushes(rxm):
    # RX_LINES_RESIDENT orders a push against no caller stream; the lines are
    # the same, so are the scores, bit for bit, for one-block and multi-block
    # pushes, update-then-score and causal.  Other values are refused and the
    # stream stays usable.
    import torch
    B, S, BL = 96, 256, 16
    cube = synth.sensor_cube(47, lines=6 * BL, samples=S, bands=B).cube
    x = dev(cube)
    torch.cuda.synchronize()
    for causal in (False, True):
        def cfg():
            return rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6,
                                   block_lines=BL, causal=causal)
        a, b = rxm.RxStream(cfg()), rxm.RxStream(cfg())
        for l0, nb in ((0, 1), (BL, 3), (4 * BL, 1), (5 * BL, 1)):
            a.rx_push_lines(x[l0:l0 + nb * BL])
            b.rx_push_lines(x[l0:l0 + nb * BL], resident=True)
        a.rx_sync()
        b.rx_sync()
        sa, sb = a.scores_host(), b.scores_host()
        assert np.array_equal(sa.view(np.uint32), sb.view(np.uint32))
        assert np.isfinite(sa[-BL * S:]).all()
        a.rx_destroy()
        r = rxm.LIB.rx_push_lines(b.h, x.data_ptr(), BL, 3, None)
        assert r == rxm.RX_E_ARG, r
        b.rx_push_lines(x[:BL], resident=True)
        b.rx_sync()
        b.rx_destroy()


def test_relative_mask_maximum_over_pending_after_partial_pops(rxm):
    # The relative mask's maximum is over exactly the pending scores: after a
    # partial pop, after a push on top of a partly popped set, and after a
    # drain.  Every mask must equal delta > tau * max(pending), computed from
    # a twin stream's scores (bit-identical: same blocks, same arithmetic).
    B, S, BL = 48, 256, 12
    cube = synth.sensor_cube(43, lines=6 * BL, samples=S, bands=B).cube
    x = dev(cube)
    cfg = dict(in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6, block_lines=BL)
    st = rxm.RxStream(rxm.make_config(B, S, **cfg))
    tw = rxm.RxStream(rxm.make_config(B, S, **cfg))
    tau = 0.3

    def expect(sc):
        d = sc.astype(np.float64)
        return d > tau * np.nanmax(d)

    st.rx_push_lines(x[:2 * BL])
    tw.rx_push_lines(x[:2 * BL])
    tw.rx_sync()
    s_all = tw.scores_host()
    assert np.array_equal(st.mask_host(tau, rxm.RX_THR_REL_MAX), expect(s_all))
    cut = s_all.size // 3
    part = np.empty(cut, dtype=np.float32)
    assert st.rx_scores(part) == cut                      # partial pop
    assert np.array_equal(part.view(np.uint32), s_all[:cut].view(np.uint32))
    rest = s_all[cut:]
    assert np.array_equal(st.mask_host(tau, rxm.RX_THR_REL_MAX), expect(rest))
    st.rx_push_lines(x[2 * BL:3 * BL])                     # pushed on top of a partly popped set
    tw.rx_push_lines(x[2 * BL:3 * BL])
    tw.rx_sync()
    more = tw.scores_host()
    both = np.concatenate([rest, more])
    assert np.array_equal(st.mask_host(tau, rxm.RX_THR_REL_MAX), expect(both))
    assert np.array_equal(st.scores_host().view(np.uint32), both.view(np.uint32))   # drained
    st.rx_push_lines(x[3 * BL:6 * BL])                     # a fresh set
    tw.rx_push_lines(x[3 * BL:6 * BL])
    tw.rx_sync()
    last = tw.scores_host()
    assert np.array_equal(st.mask_host(tau, rxm.RX_THR_REL_MAX), expect(last))
    st.rx_destroy()
    tw.rx_destroy()


# ---------------------------------------------------------------------------- FP8 covariance product
def _fp8_block_product_emulation(cube):
    """Host emulation of one block's FP8 covariance operand: the shift c is
    the first line's band mean rounded to FP32, the band scale 2^-e puts the
    first line's largest |x - c| (FP32) at or below 224, the operand is the
    E4M3 rounding (saturating) of (x - c) 2^-e in FP32; returns the unscaled
    product sum_p q_a q_b / (s_a s_b) (exact in FP64), the shift, and the
    number of values beyond the format's range."""
    from lowp_emu import q_e4m3
    px = orx.pixels(cube).astype(np.float32)                     # [n][B]
    S = cube.shape[2]
    first = px[:S].astype(np.float64)
    c = (first.sum(axis=0) / S).astype(np.float32)
    m = np.max(np.abs(px[:S] - c[None, :]), axis=0).astype(np.float64)
    e = np.where(m > 0, np.frexp(m / 224.0)[1], 0)
    sc = np.ldexp(np.float32(1.0), -e).astype(np.float32)
    dv = (px - c[None, :]) * sc[None, :]
    clips = int(np.sum(np.abs(dv) > 464.0))
    q = q_e4m3(dv)
    prod = (q.T @ q) / np.outer(sc.astype(np.float64), sc.astype(np.float64))
    return prod, c.astype(np.float64), clips


@pytest.mark.parametrize("samples", [64, 203])
def test_fp8_covariance_product_matches_host_emulation(rxm, samples):
    # One block (a single split): the kernel's window statistics must equal
    # the emulated FP8 product with the merge's exact shift correction, to
    # FP32 accumulation rounding (far below one FP8 step), and its
    # saturation count must equal the emulated one.
    B, L = 64, 20
    cube = synth.sensor_cube(91, lines=L, samples=samples, bands=B).cube
    prod, c, clips = _fp8_block_product_emulation(cube)
    px = orx.pixels(cube).astype(np.float64)
    n = px.shape[0]
    mb = px.mean(axis=0)
    m2 = prod - n * np.outer(mb - c, mb - c)
    st = run_stream(rxm, cube, "fp8", "bf16", ridge_rel=1e-6)
    nn, mu, cov = st.rx_get_stats()
    assert nn == n
    got = cov * n
    scale = np.abs(prod).max()
    err = np.max(np.abs(got - m2)) / scale
    say(f"  fp8 covariance S={samples}: max |M2 - emulation| / max|product| = {err:.3e}; "
        f"{st.rx_get_counters().fp8_syrk_saturated} saturated (emulation {clips})")
    assert err <= 2.0 ** -24 * 512
    assert st.rx_get_counters().fp8_syrk_saturated == clips


def test_fp8_covariance_scores_reported(rxm):
    # FP8 operands in the covariance product at 270 bands, BF16 whitening,
    # against the oracle with the same ridge: reported, not bounded (parity
    # unpinned for FP8, as for FP8 whitening), except that every score is
    # finite and the implanted-material pixels stay at the top.
    B, S = 270, 640
    cube = synth.sensor_cube(92, lines=40, samples=S, bands=B).cube
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=20, rho=1e-6)
    st = run_stream(rxm, cube, "fp8", "bf16", block_lines=20, ridge_rel=1e-6)
    got = st.scores_host()
    mx, p99 = err_summary(got, ref, B)
    say(f"  fp8 covariance + bf16 whitening: max rel {mx:.3e}, p99 rel {p99:.3e} (reported); "
        f"{st.rx_get_counters().fp8_syrk_saturated} saturated")
    assert np.all(np.isfinite(got))
    top = np.argsort(-ref)[:10]
    assert np.all(got[top] > np.quantile(got, 0.99))
