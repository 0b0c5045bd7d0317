"""Causal scoring (RX_FLAG_CAUSAL) on the GPU through the C ABI, against the
FP64 stream oracle in its causal mode: every block is scored with the window
as it was before the block joined it.  Pushes of 10 and 14 lines in blocks of
8 make the first block of each push take the window before the push (the
extra snapshot slot); a 16-line reset window makes a block start a window in
the middle of a push (no statistics: NaN, not ready)."""
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


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("window_lines", [0, 16])
@pytest.mark.parametrize("S", [96, 128])
def test_causal_matches_oracle(rxm, prec, window_lines, S):
    L, B = 24, 40
    cube = synth.sensor_cube(31, lines=L, samples=S, bands=B).cube
    rho = 1e-6 if prec == "bf16" else 0.0
    pushes = [10, 14]
    say(f"causal {prec} window {window_lines} S {S}")
    cfg = rxm.make_config(B, S, in_dtype=np.uint16, syrk=prec, whiten=prec, ridge_rel=rho, block_lines=8,
                          window_lines=window_lines, causal=True)
    st = rxm.RxStream(cfg)
    codes = []
    l0 = 0
    for n in pushes:
        codes.append(st.rx_push_lines(dev(cube[l0:l0 + n])))
        l0 += n
    st.rx_sync()
    c = st.rx_get_counters()
    got = st.scores_host(f64=(prec == "fp64"))
    ref, o = oracle_stream_scores(cube, B, S, block_lines=8, window_lines=window_lines, rho=rho, pushes=pushes,
                                  causal=True)
    assert codes[0] == rxm.RX_E_NOTREADY                      # the first block has no window before it
    assert c.notready_blocks == o.status.count("notready") >= 1
    assert c.singular_blocks == 0
    assert np.isnan(got[:8 * S]).all()
    assert_scores(got, ref, B, *TOL[prec], label=f"causal {prec}")
    st.rx_destroy()


def test_causal_and_update_then_score_side_by_side(rxm):
    # The same cube through both readings on two streams, each against the
    # oracle in its own mode (one push, blocks of 4 lines).
    L, B, S = 16, 24, 64
    cube = synth.sensor_cube(32, lines=L, samples=S, bands=B).cube
    a = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64", block_lines=4,
                                     causal=True))
    b = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64", block_lines=4))
    a.rx_push_lines(dev(cube))
    b.rx_push_lines(dev(cube))
    a.rx_sync()
    b.rx_sync()
    ga, gb = a.scores_host(f64=True), b.scores_host(f64=True)
    ra, _ = oracle_stream_scores(cube, B, S, block_lines=4, causal=True)
    rb, _ = oracle_stream_scores(cube, B, S, block_lines=4)
    assert_scores(ga, ra, B, *TOL["fp64"], label="causal fp64")
    assert_scores(gb, rb, B, *TOL["fp64"], label="update-then-score fp64")
    a.rx_destroy()
    b.rx_destroy()


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp8"])
def test_causal_one_block_pushes(rxm, prec):
    # One-block pushes queued back to back (input resident, the caller's
    # stream not made to wait): from the second push on, the window-before
    # slot is copied from the previous push and the whitening starts without
    # waiting for the push's own statistics.  The scores must equal, bit for
    # bit, those of one push of all the lines (same blocks, slots formed in
    # the batch), and the FP64 / BF16 paths must match the oracle.
    import torch
    L, B, S, bl = 48, 64, 128, 4
    cube = synth.sensor_cube(33, lines=L, samples=S, bands=B).cube
    rho = 0.0 if prec == "fp64" else 1e-6
    syrk = "fp64" if prec in ("fp64", "fp8") else prec
    say(f"causal one-block pushes {prec}")
    x = dev(cube)

    def run(pushes):
        st = rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk=syrk, whiten=prec, ridge_rel=rho,
                                          block_lines=bl, window_lines=32, causal=True))
        l0 = 0
        for n in pushes:
            st.rx_push_lines(x[l0:l0 + n], guard=False)
            l0 += n
        st.rx_sync()
        torch.cuda.synchronize()
        c = st.rx_get_counters()
        out = st.scores_host(f64=(prec == "fp64"))
        st.rx_destroy()
        return out, c

    a, ca = run([bl] * (L // bl))
    b, cb = run([L])
    assert np.array_equal(a.view(np.uint64 if prec == "fp64" else np.uint32),
                          b.view(np.uint64 if prec == "fp64" else np.uint32))
    ref, o = oracle_stream_scores(cube, B, S, block_lines=bl, window_lines=32, rho=rho, pushes=[L], causal=True)
    assert ca.notready_blocks == cb.notready_blocks == o.status.count("notready") == 2
    if prec != "fp8":
        assert_scores(a, ref, B, *TOL[prec], label=f"causal one-block pushes {prec}")


def test_causal_after_set_stats_forms_the_slot_itself(rxm):
    # A checkpoint restored with rx_set_stats invalidates the copied slot: the
    # next causal push must score against the restored window (slot formed in
    # the batch).  Stream A pushes lines 0..15 then 16..31; stream B restores
    # A's statistics after line 15 and pushes 16..31: same scores on the FP64
    # path (up to the restore's rounding of mean * n and cov * n).
    L, B, S = 32, 40, 96
    cube = synth.sensor_cube(34, lines=L, samples=S, bands=B).cube
    x = dev(cube)
    mk = lambda: rxm.RxStream(rxm.make_config(B, S, in_dtype=np.uint16, syrk="fp64", whiten="fp64",
                                              block_lines=8, causal=True))
    a = mk()
    a.rx_push_lines(x[:16])
    a.rx_sync()
    n, mean, cov = a.rx_get_stats()
    a.scores_host(f64=True)
    a.rx_push_lines(x[16:])
    a.rx_sync()
    want = a.scores_host(f64=True)
    b = mk()
    b.rx_push_lines(x[:8])                 # a push first, so a copied slot would exist
    b.rx_sync()
    b.scores_host(f64=True)
    b.rx_set_stats(n, mean, cov)
    b.rx_push_lines(x[16:])
    b.rx_sync()
    got = b.scores_host(f64=True)
    assert n == 16 * S
    assert_scores(got, want, B, 1e-9, 1e-11, label="causal after rx_set_stats")
    ref, _ = oracle_stream_scores(cube, B, S, block_lines=8, causal=True, pushes=[16, 16])
    assert_scores(got, ref[16 * S:], B, 1e-9, 1e-11, label="causal after rx_set_stats vs oracle")
    a.rx_destroy()
    b.rx_destroy()
