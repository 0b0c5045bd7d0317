"""Ingest band selection and binning on the GPU through the C ABI, against
the CPU oracle: integer sums, so every output must match bit for bit.
Shapes cover the 16-byte path (samples % 8 == 0), the per-sample path (the
imager's 900-sample lines), a misaligned input, an empty cube and the
paper's full 1000 x 300 x 900 cube binned 300 -> 280 -> 70.  A binned cube is
then scored on the FP64 path against the scoring oracle."""
import numpy as np
import pytest

from gpu_util import assert_scores, oracle_stream_scores, say
from oracle import binning as ob
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def gpu_bin(rxm, cube, b0, nb, k):
    import torch
    x = torch.from_numpy(cube).cuda()
    out = torch.zeros((cube.shape[0], nb // k, cube.shape[2]), dtype=torch.uint16, device="cuda")
    rxm.bin_bands(x, b0, nb, k, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("shape,b0,nb,k", [((7, 300, 640), 10, 280, 4), ((5, 300, 900), 10, 280, 4),
                                           ((3, 33, 17), 1, 30, 3), ((2, 40, 64), 0, 40, 1),
                                           ((4, 64, 128), 3, 48, 16), ((0, 300, 640), 10, 280, 4)])
def test_binning_bitwise(rxm, shape, b0, nb, k):
    cube = synth.raw_counts(sum(shape) + k, *shape)
    say(f"binning {shape} b0={b0} nb={nb} k={k}")
    got = gpu_bin(rxm, cube, b0, nb, k)
    assert np.array_equal(got.astype(np.int64), ob.bin_bands(cube, b0, nb, k))


def test_binning_misaligned_input(rxm):
    import torch
    cube = synth.raw_counts(9, 3, 24, 64)
    # the cube starts 2 bytes into a device buffer, so rows are not 16-byte aligned
    wide = torch.zeros((cube.size + 1,), dtype=torch.uint16, device="cuda")
    wide[1:] = torch.from_numpy(cube).cuda().reshape(-1)
    view = wide[1:].view(3, 24, 64)
    out = torch.zeros((3, 6, 64), dtype=torch.uint16, device="cuda")
    rxm.bin_bands(view, 0, 24, 4, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().astype(np.int64), ob.bin_bands(cube, 0, 24, 4))


def test_paper_cube_full_size(rxm):
    cube = synth.raw_counts(0, 1000, 300, 900)
    got = gpu_bin(rxm, cube, 10, 280, 4)
    assert got.shape == (1000, 70, 900)
    assert np.array_equal(got.astype(np.int64), ob.bin_bands(cube, 10, 280, 4))


def test_binning_argument_errors(rxm):
    import torch
    x = torch.zeros((2, 20, 16), dtype=torch.uint16, device="cuda")
    out = torch.zeros((2, 5, 16), dtype=torch.uint16, device="cuda")
    for b0, nb, k, bits in [(0, 20, 0, 12), (0, 18, 4, 12), (4, 20, 4, 12), (-1, 20, 4, 12), (0, 20, 20, 12),
                            (0, 20, 4, 0)]:
        with pytest.raises(rxm.RxError) as e:
            rxm.bin_bands(x, b0, nb, k, out, bit_depth=bits)
        assert e.value.status == rxm.RX_E_ARG, (b0, nb, k, bits)


def test_binned_cube_scores_fp64(rxm):
    import torch
    L, B, S = 64, 300, 128
    raw = synth.sensor_cube(13, lines=L, samples=S, bands=B).cube
    binned = ob.bin_bands(raw, 10, 280, 4).astype(np.uint16)
    x = torch.from_numpy(raw).cuda()
    out = torch.zeros((L, 70, S), dtype=torch.uint16, device="cuda")
    rxm.bin_bands(x, 10, 280, 4, out)
    cfg = rxm.make_config(70, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64", bit_depth=14)
    st = rxm.RxStream(cfg)
    st.rx_push_lines(out)
    st.rx_sync()
    got = st.scores_host(f64=True)
    ref, _ = oracle_stream_scores(binned, 70, S)
    assert_scores(got, ref, 70, 1e-9, 1e-11, "binned cube FP64 path")
    st.rx_destroy()
