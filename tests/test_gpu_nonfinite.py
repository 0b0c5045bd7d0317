"""Non-finite float input and FP8 saturation counts on the GPU, through the
C ABI, against the FP64 stream oracle.

A float pixel with a NaN or infinite band is left out of the statistics
(the window count N counts the others), scores NaN, is never marked, and is
counted; the oracle does the same from its own plain definition.  Planted
cases: scattered NaN / +-inf, a pixel in the first line of a block (the
centring shift), a whole line, a whole block (the window is then left as it
was) and a first block with no finite pixel (not ready without a ridge).

FP8 E4M3 whitening counts the centred, band-scaled input values beyond the
format's range (|v| > 464, stored as +-448).  With the window statistics set
to a huge N, unit-scale noise and planted values far outside the range, the
expected count is exactly the number of planted values; values that round
to 448 without clipping (|v| near 450) must not count."""
import numpy as np
import pytest

from gpu_util import assert_scores, oracle_stream_scores, say
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


def planted_cube(seed, dtype, L=24, B=40, S=96):
    cube = synth.sensor_cube(seed, lines=L, samples=S, bands=B).cube.astype(dtype)
    rng = np.random.default_rng(seed + 100)
    n = L * S
    for val, count in ((np.nan, 30), (np.inf, 5), (-np.inf, 5)):
        for p in rng.choice(n, size=count, replace=False):
            cube[p // S, rng.integers(B), p % S] = val
    cube[0, 7, 0] = np.nan            # first line of the first block
    cube[8, 0, 95] = np.inf           # first line of the second block (blocks of 8)
    cube[13, 3, :] = np.nan           # a whole line
    return cube


def run(rxm, cube, prec, pushes, **kw):
    B, S = cube.shape[1], cube.shape[2]
    st = rxm.RxStream(rxm.make_config(B, S, in_dtype=cube.dtype, syrk=prec, whiten=prec, **kw))
    l0 = 0
    for n in pushes:
        st.rx_push_lines(dev(cube[l0:l0 + n]))
        l0 += n
    st.rx_sync()
    return st


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("window_lines", [0, 16])
def test_nonfinite_pixels_left_out(rxm, dtype, prec, window_lines):
    cube = planted_cube(3, dtype)
    B, S = cube.shape[1], cube.shape[2]
    rho = 1e-6 if prec == "bf16" else 0.0
    pushes = [10, 14]
    say(f"non-finite pixels: {np.dtype(dtype).name} {prec} window {window_lines}")
    st = run(rxm, cube, prec, pushes, block_lines=8, window_lines=window_lines, ridge_rel=rho)
    c = st.rx_get_counters()
    n, mean, _ = st.rx_get_stats()
    m = st.mask_host(0.0, rxm.RX_THR_ABS)         # the mask does not consume the scores
    got = st.scores_host(f64=(prec == "fp64"))
    ref, o = oracle_stream_scores(cube, B, S, block_lines=8, window_lines=window_lines, rho=rho, pushes=pushes)
    assert c.nonfinite_px == o.nonfinite > 0
    assert c.window_px == n == o.n
    assert c.notready_blocks == 0
    _, mu_ref, _ = o.stats()
    assert np.max(np.abs(mean - mu_ref)) <= 1e-9 * np.max(np.abs(mu_ref))
    assert_scores(got, ref, B, *TOL[prec], label=f"{prec} with non-finite pixels")
    assert m.shape == ref.shape and not m[np.isnan(ref)].any() and m[~np.isnan(ref)].all()
    st.rx_destroy()


def test_block_without_finite_pixels_leaves_window_unchanged(rxm):
    L, B, S = 12, 16, 64
    cube = synth.sensor_cube(5, lines=L, samples=S, bands=B).cube.astype(np.float32)
    cube[4:8, 2, :] = np.nan                          # block 1 (lines 4..7) has no finite pixel
    st = run(rxm, cube, "fp64", [L], block_lines=4)
    c = st.rx_get_counters()
    got = st.scores_host(f64=True)
    ref, o = oracle_stream_scores(cube, B, S, block_lines=4)
    assert o.status == ["ok", "ok", "ok"]
    assert c.nonfinite_px == 4 * S and c.window_px == 8 * S and c.notready_blocks == 0
    assert np.isnan(got[4 * S:8 * S]).all()
    assert_scores(got, ref, B, *TOL["fp64"], label="block without finite pixels")
    st.rx_destroy()


def test_first_block_without_finite_pixels_is_not_ready(rxm):
    L, B, S = 12, 16, 64
    cube = synth.sensor_cube(6, lines=L, samples=S, bands=B).cube.astype(np.float64)
    cube[0:4, 0, :] = -np.inf
    st = run(rxm, cube, "fp64", [L], block_lines=4)
    c = st.rx_get_counters()
    got = st.scores_host(f64=True)
    ref, o = oracle_stream_scores(cube, B, S, block_lines=4)
    assert o.status == ["notready", "ok", "ok"]
    assert c.notready_blocks == 1 and c.window_px == 8 * S
    assert_scores(got, ref, B, *TOL["fp64"], label="first block not ready")
    st.rx_destroy()


@pytest.mark.parametrize("dtype", [np.uint16, np.float32])
def test_fp8_saturation_count(rxm, dtype):
    # 16-bit input takes the tile whitening kernel (S % 8 == 0, aligned rows),
    # float input the chunk kernel: both must count the same values.
    L, B, S = 16, 64, 128
    rng = np.random.default_rng(9)
    base = np.rint(2000.0 + 1.4 * rng.standard_normal((L, B, S)))
    cube = base.copy()
    far = [(0, 0, 0), (3, 10, 17), (3, 11, 17), (7, 63, 127), (9, 32, 64), (15, 5, 100), (15, 6, 101)]
    near = [(1, 1, 1), (5, 20, 30), (8, 40, 50), (12, 2, 3), (14, 60, 120)]
    for p in far:
        cube[p] = 4095.0                           # centred ~ 2095: clipped
    for p in near:
        cube[p] = 2450.0                           # centred ~ 450: rounds to 448, not clipped
    cube = cube.astype(dtype)
    cfg = rxm.make_config(B, S, in_dtype=dtype, syrk="fp64", whiten="fp8", bit_depth=12)
    st = rxm.RxStream(cfg)
    # a huge window with unit-scale spread: the block barely moves it, so the
    # band scale stays 1 (sigma ~ 1.41) and the centred values are x - 2000
    st.rx_set_stats(10 ** 9, np.full(B, 2000.0), 2.0 * np.eye(B))
    say(f"fp8 saturation count: {np.dtype(dtype).name}")
    st.rx_push_lines(dev(cube))
    st.rx_sync()
    assert st.rx_get_counters().fp8_saturated == len(far)
    got = st.scores_host()
    assert np.all(np.isfinite(got))
    st.rx_push_lines(dev(base.astype(dtype)))      # nothing beyond the range: the count stays
    st.rx_sync()
    assert st.rx_get_counters().fp8_saturated == len(far)
    st.rx_destroy()


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_many_pushes_in_flight_float_input(rxm, prec):
    # Twelve one-block pushes queued back to back (the caller's stream is not
    # made to wait, the input stays resident): the validity buffers alternate
    # by parity while earlier pushes' whitening may still read them.  Scores
    # do not depend on the push pattern, so they must equal those of one push
    # of the same lines bit for bit; the FP64 path is also held to the oracle.
    import torch
    cube = planted_cube(7, np.float32, L=48)
    B, S = cube.shape[1], cube.shape[2]
    x = dev(cube)
    rho = 1e-6 if prec == "bf16" else 0.0

    def run(pushes):
        st = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.float32, syrk=prec, whiten=prec, ridge_rel=rho,
                                          block_lines=4))
        l0 = 0
        for n in pushes:
            st.rx_push_lines(x[l0:l0 + n], guard=False)
            l0 += n
        st.rx_sync()
        torch.cuda.synchronize()
        c = st.rx_get_counters().nonfinite_px
        out = st.scores_host(f64=(prec == "fp64"))
        st.rx_destroy()
        return out, c

    a, ca = run([4] * 12)
    b, cb = run([48])
    assert np.array_equal(a.view(np.uint64 if prec == "fp64" else np.uint32),
                          b.view(np.uint64 if prec == "fp64" else np.uint32))
    ref, o = oracle_stream_scores(cube, B, S, block_lines=4, rho=rho, pushes=[4] * 12)
    assert ca == cb == o.nonfinite
    if prec == "fp64":
        assert_scores(a, ref, B, *TOL["fp64"], label="twelve pushes in flight")
