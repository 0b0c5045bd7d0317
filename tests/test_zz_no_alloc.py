"""The allocation-free mask entry point (rx_mask_noalloc) against rx_mask,
through the C ABI: the same bits for every threshold mode, on two calls in
a row where the second has a smaller pending set (the shared working array
keeps the first call's contents, which must not leak into the second), and
the size limit refused on the host before anything is queued."""
import numpy as np
import pytest

from gpu_util import say
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def _both(rxm, st, tau, mode, k):
    import torch
    n = st.pending()
    nb = (n + 7) // 8
    a = torch.full((nb + 3,), 0xA5, dtype=torch.uint8, device="cuda")     # guard bytes past the end
    b = torch.full((nb + 3,), 0x5A, dtype=torch.uint8, device="cuda")
    assert st.rx_mask(tau, mode, k, a[:nb]) == n
    # an odd byte offset: the copy out of the working array takes any alignment
    off = torch.full((nb + 4,), 0x5A, dtype=torch.uint8, device="cuda")
    assert st.rx_mask_noalloc(tau, mode, k, off[1:nb + 1]) == n
    assert st.rx_mask_noalloc(tau, mode, k, b[:nb]) == n
    torch.cuda.synchronize()
    a, b, off = a.cpu().numpy(), b.cpu().numpy(), off.cpu().numpy()
    assert np.array_equal(a[:nb], b[:nb]), (mode, k)
    assert np.array_equal(a[:nb], off[1:nb + 1]), (mode, k)
    assert np.all(b[nb:] == 0x5A) and off[0] == 0x5A and np.all(off[nb + 1:] == 0x5A)   # nothing past the end
    return int(np.unpackbits(a[:nb], bitorder="little")[:n].sum())


@pytest.mark.parametrize("prec", ["bf16", "fp64"])
def test_noalloc_mask_equals_mask_on_two_calls(rxm, prec):
    import torch
    B, S = 96, 256
    big = synth.sensor_cube(71, lines=37, samples=S, bands=B).cube
    small = synth.sensor_cube(72, lines=5, samples=S, bands=B).cube
    st = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk=prec, whiten=prec,
                                      ridge_rel=1e-6 if prec == "bf16" else 0.0))
    for cube, label in ((big, "first (37 lines)"), (small, "second (5 lines)")):
        st.rx_push_lines(torch.from_numpy(cube).cuda())
        st.rx_sync()
        sc = st.scores_host(f64=(prec == "fp64"))
        st.rx_push_lines(torch.from_numpy(cube).cuda())   # the same lines again: pending = one push
        st.rx_sync()
        tau = float(np.quantile(sc, 0.99))
        marks = [_both(rxm, st, tau, rxm.RX_THR_ABS, 0), _both(rxm, st, 0.110, rxm.RX_THR_REL_MAX, 0),
                 _both(rxm, st, 0.0, rxm.RX_THR_TOPK, 7), _both(rxm, st, 0.0, rxm.RX_THR_TOPK, 0)]
        say(f"  {prec} {label}: {st.pending()} pending pixels, marked (abs, rel, top-7, top-0) {marks}")
        assert marks[2] == 7 and marks[3] == 0
        st.scores_host()                                   # drain for the next, smaller set
    st.rx_destroy()


def test_noalloc_mask_refuses_sets_past_its_limit(rxm):
    import torch
    B, S = 1, 1 << 16
    lines = (rxm.RX_MASK_NOALLOC_MAX_PX // S) + 1
    cube = np.random.default_rng(3).integers(0, 4096, size=(lines, B, S), dtype=np.uint16)
    st = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64"))
    st.rx_push_lines(torch.from_numpy(cube).cuda())
    st.rx_sync()
    n = st.pending()
    out = torch.zeros((n + 7) // 8, dtype=torch.uint8, device="cuda")
    with pytest.raises(rxm.RxError) as e:
        st.rx_mask_noalloc(1.0, rxm.RX_THR_ABS, 0, out)
    assert e.value.status == rxm.RX_E_ARG
    st.rx_destroy()
