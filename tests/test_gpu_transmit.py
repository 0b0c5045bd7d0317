"""Transmission stage on the GPU through the C ABI, against the CPU oracle.

The codes are integers decided by floating point, and both sides take every
step in FP32 (correctly rounded square root and division, binary16 rounding
to nearest even), so codes, the header maximum, the decoded scores and the
receiver's threshold bits must all match bit for bit.  Inputs are seeded
score samples (never scores the GPU produced), at sizes from empty to the
2000 x 640 cube's 1 280 000 pixels, with ragged ends and NaN pixels.  The
stream-level entry point is checked against the buffer-level one on a
pushed cube, and its decoded scores against the FP64 scoring oracle."""
import numpy as np
import pytest

from gpu_util import assert_scores, oracle_stream_scores, say
from oracle import transmit as otx
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def run_gpu(rxm, d, tau):
    import torch
    n = d.size
    x = torch.from_numpy(d).cuda()
    codes = torch.zeros(max(n, 1), dtype=torch.int16, device="cuda")[:n]
    mslot = torch.full((1,), -1.0, dtype=torch.float32, device="cuda")
    delta = torch.zeros(max(n, 1), dtype=torch.float32, device="cuda")[:n]
    words = torch.zeros(max((n + 31) // 32, 1), dtype=torch.int32, device="cuda")
    rxm.tx_encode(x, codes, mslot)
    rxm.tx_decode(codes, mslot, tau, delta, words)
    torch.cuda.synchronize()
    bits = words.cpu().numpy().view(np.uint8)[:(n + 7) // 8]
    return (codes.cpu().numpy().view(np.uint16), np.float32(mslot.item()), delta.cpu().numpy(), bits)


@pytest.mark.parametrize("n,nan_frac", [(0, 0.0), (1, 0.0), (31, 0.0), (32, 0.0), (33, 0.01), (1000, 0.0),
                                        (1000003, 0.001), (1280000, 0.0)])
def test_encode_decode_bitwise(rxm, n, nan_frac):
    tau = 0.110
    d = synth.score_sample(n + 17, n, nan_frac=nan_frac)
    say(f"transmit n={n} nan_frac={nan_frac}")
    codes, m, delta, bits = run_gpu(rxm, d, tau)
    ref_codes, ref_m = otx.encode(d)
    ref_delta, ref_mask = otx.decode(ref_codes, ref_m, tau)
    assert m.view(np.uint32) == np.float32(ref_m).view(np.uint32)
    assert np.array_equal(codes, ref_codes)
    assert np.array_equal(delta.view(np.uint32), ref_delta.view(np.uint32))
    assert np.array_equal(bits, otx.pack_bits(ref_mask))


def test_all_zero_and_all_nan(rxm):
    for d in (np.zeros(100, np.float32), np.full(70, np.nan, np.float32)):
        codes, m, _, bits = run_gpu(rxm, d, 0.110)
        ref_codes, ref_m = otx.encode(d)
        assert m == ref_m == 0
        assert np.array_equal(codes, ref_codes)
        assert not bits.any()


def test_bad_arguments(rxm):
    import torch
    codes = torch.zeros(4, dtype=torch.int16, device="cuda")
    with pytest.raises(rxm.RxError) as e:
        rxm.tx_decode(codes, torch.zeros(1, device="cuda"), float("nan"))
    assert e.value.status == rxm.RX_E_ARG


def test_stream_encode_matches_buffer_encode_and_oracle(rxm):
    import torch
    B, S, L = 64, 128, 48
    cube = synth.sensor_cube(21, lines=L, samples=S, bands=B).cube
    cfg = rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6, block_lines=16)
    st = rxm.RxStream(cfg)
    st.rx_push_lines(torch.from_numpy(cube).cuda())
    n = L * S
    codes = torch.zeros(n, dtype=torch.int16, device="cuda")
    mslot = torch.zeros(1, dtype=torch.float32, device="cuda")
    assert st.rx_encode(codes, mslot) == n
    scores = st.scores_host()                     # pops what was just encoded
    torch.cuda.synchronize()
    codes2 = torch.zeros(n, dtype=torch.int16, device="cuda")
    mslot2 = torch.zeros(1, dtype=torch.float32, device="cuda")
    rxm.tx_encode(torch.from_numpy(scores).cuda(), codes2, mslot2)
    torch.cuda.synchronize()
    assert torch.equal(codes, codes2) and mslot.item() == mslot2.item()
    delta = torch.zeros(n, dtype=torch.float32, device="cuda")
    rxm.tx_decode(codes, mslot, 0.110, delta, None)
    torch.cuda.synchronize()
    ref, _ = oracle_stream_scores(cube, B, S, pushes=[16, 16, 16], rho=1e-6)
    # BF16 path tolerance plus the binary16 round trip (relative 2^-10)
    assert_scores(delta.cpu().numpy(), ref, B, 5e-2 + 2.0 ** -10, 1e-2 + 2.0 ** -10, "decoded vs FP64 oracle")
    st.rx_destroy()
