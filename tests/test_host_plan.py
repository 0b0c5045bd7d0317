"""Host-side planning of the covariance product (no GPU needed).

The covariance kernels keep each split's raw band sums of 16-bit input as
exact 32-bit integers per thread; a thread adds 8 values per 64-sample chunk.
The split plan must keep 8 * 65535 * (chunks in a split) below 2^32 for every
block length, and leave the usual block sizes' plans (and so their
summation order and scores) as they are."""
import numpy as np
import pytest

from paper_2602_13509_amd import rx

U32 = 2 ** 32


@pytest.mark.parametrize("syrk", ["bf16", "fp16", "fp32", "fp64"])
@pytest.mark.parametrize("samples", [1, 63, 64, 640, 900, 1024, 4096])
def test_split_plan_never_overflows_raw_sums(syrk, samples):
    cfg = rx.make_config(270, samples, syrk=syrk)
    cpl = -(-samples // 64)
    for lines in (1, 7, 100, 128, 1000, 52428, 52429, 60000, 209715, 209716, 10 ** 6, 2 ** 31 - 1):
        ks, mc = rx.split_plan(cfg, lines)
        nch = lines * cpl
        assert ks >= 1 and mc >= 1
        assert ks * mc >= nch                      # the splits cover every chunk
        assert mc == -(-nch // ks)                 # and the largest holds ceil(nch / ks)
        assert 8 * 65535 * mc < U32, (lines, ks, mc)


def test_split_plan_of_usual_blocks_is_unchanged():
    # 100-line blocks of 640 samples: 11 splits of at most 91 chunks (the
    # whole-triangle kernels), 16 of at most 64 (the super-tile kernels);
    # up to 256 splits (about one per CU) the plan is ceil(chunks / per-split)
    assert rx.split_plan(rx.make_config(270, 640, syrk="bf16"), 100) == (11, 91)
    assert rx.split_plan(rx.make_config(270, 640, syrk="fp64"), 100) == (16, 63)
    for lines in (1, 16, 100, 500, 582, 1000, 2000, 2329, 5000):
        nch = lines * 10
        assert rx.split_plan(rx.make_config(270, 640, syrk="bf16"), lines)[0] == min(256, -(-nch // 91))
    # the paper's 1000-line cubes of 900 samples: 15 000 chunks, 165 splits
    assert rx.split_plan(rx.make_config(70, 900, syrk="bf16"), 1000) == (165, 91)
    # 209 716 lines: 2 097 160 chunks, which 256 splits could only hold with
    # 8193 chunks in one (past the bound); the plan takes 257 splits instead
    assert rx.split_plan(rx.make_config(270, 640, syrk="bf16"), 209715) == (256, 8192)
    ks, mc = rx.split_plan(rx.make_config(270, 640, syrk="bf16"), 209716)
    assert ks == 257 and mc <= 8192


def test_split_plan_rejects_bad_arguments():
    cfg = rx.make_config(270, 640)
    for lines in (0, -1, 2 ** 31):
        with pytest.raises(rx.RxError) as e:
            rx.split_plan(cfg, lines)
        assert e.value.status == rx.RX_E_ARG
    bad = rx.make_config(270, 640)
    bad.bands = 0
    with pytest.raises(rx.RxError):
        rx.split_plan(bad, 100)
