"""Serving through the C ABI: many streams of different widths and band
counts admitted on one server, their blocks batched into shared launches.

The property under test: a stream's scores are the same alone and in any
mix, bit for bit (every reduction of the path is fixed per block, never by
what shares the launch), and they match the FP64 oracle within the BF16
tolerance of the scoring tests."""
import numpy as np
import pytest

from gpu_util import assert_scores, oracle_stream_scores, say
from paper_2602_13509_amd import synth

pytestmark = pytest.mark.gpu

TOL_BF16 = (5e-2, 1e-2)


@pytest.fixture(scope="module")
def rxm():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2602_13509_amd import rx
    return rx


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def make_streams(seed):
    """(B, S, block sizes, cube) per stream; S = 204 rows are not 16-byte
    multiples, so that stream takes the register-staged kernels while the
    others take the direct-load and tile kernels in the same launches."""
    rng = np.random.default_rng(seed)
    shapes = [(120, 320), (200, 640), (270, 640), (300, 1024), (270, 320), (200, 204)]
    out = []
    for i, (B, S) in enumerate(shapes):
        blocks = [int(v) for v in rng.integers(16, 49, size=3)]
        cube = synth.sensor_cube(100 + i, lines=sum(blocks), samples=S, bands=B).cube
        out.append((B, S, blocks, cube))
    return out


def cfg_for(rxm, B, S, block_lines):
    return rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6,
                           block_lines=block_lines)


def test_served_mix_equals_alone_bitwise(rxm):
    import torch
    streams = make_streams(7)
    dcubes = [dev(c) for (_, _, _, c) in streams]

    # alone: one stream at a time, one push per block
    alone = []
    for (B, S, blocks, cube), dc in zip(streams, dcubes):
        st = rxm.RxStream(cfg_for(rxm, B, S, 0))
        l0 = 0
        for n in blocks:
            st.rx_push_lines(dc[l0:l0 + n])
            l0 += n
        st.rx_sync()
        alone.append(st.scores_host())
        st.rx_destroy()

    # mixed: every stream admitted on one server, blocks submitted in an
    # interleaved random order, stepped until drained
    srv = rxm.RxServer(8 << 30, 16)
    served = [rxm.RxStream(cfg_for(rxm, B, S, 64), server=srv) for (B, S, _, _) in streams]
    order = [(i, j) for i, s in enumerate(streams) for j in range(len(s[2]))]
    rng = np.random.default_rng(3)
    rng.shuffle(order)
    nxt = [0] * len(streams)
    starts = [np.concatenate([[0], np.cumsum(s[2])]) for s in streams]
    tag = 0
    for i, _ in order:                      # a stream's blocks keep their own order
        j = nxt[i]
        nxt[i] += 1
        l0, l1 = int(starts[i][j]), int(starts[i][j + 1])
        srv.rx_server_submit(served[i], dcubes[i][l0:l1], tag)
        tag += 1
    steps, done = 0, []
    while True:
        q, _, _ = srv.rx_server_queued()
        if q == 0:
            break
        n = srv.rx_server_step()
        steps += 1
        assert n >= 1
    done = srv.rx_server_poll(block=True)
    assert sorted(done) == list(range(tag))
    say(f"served mix: {len(streams)} streams, {tag} blocks in {steps} steps")
    torch.cuda.synchronize()
    for k, ((B, S, blocks, cube), st) in enumerate(zip(streams, served)):
        got = st.scores_host()
        assert got.shape == alone[k].shape
        assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), f"stream {k} (B={B}, S={S})"
        ref, _ = oracle_stream_scores(cube, B, S, pushes=blocks, rho=1e-6)
        assert_scores(got, ref, B, *TOL_BF16, label=f"served B={B} S={S}")
        st.rx_destroy()
    srv.rx_server_destroy()


def test_server_admission_by_budget_and_slots(rxm):
    cfg = cfg_for(rxm, 270, 640, 64)
    need = rxm.stream_footprint(cfg, 64)
    srv = rxm.RxServer(int(2.5 * need), 8)
    a = rxm.RxStream(cfg, server=srv)
    b = rxm.RxStream(cfg, server=srv)
    with pytest.raises(rxm.RxError) as e:
        rxm.RxStream(cfg, server=srv)
    assert e.value.status == rxm.RX_E_BUDGET
    _, _, used = srv.rx_server_queued()
    assert used == 2 * need
    a.rx_destroy()                          # frees its admission
    c = rxm.RxStream(cfg, server=srv)
    b.rx_destroy()
    c.rx_destroy()
    srv.rx_server_destroy()

    slots = rxm.RxServer(64 * need, 1)
    x = rxm.RxStream(cfg, server=slots)
    with pytest.raises(rxm.RxError) as e:
        rxm.RxStream(cfg, server=slots)
    assert e.value.status == rxm.RX_E_BUDGET
    x.rx_destroy()
    slots.rx_server_destroy()


def test_server_tags_in_launch_order_and_block_limit(rxm):
    B, S = 64, 128
    cube = synth.sensor_cube(31, lines=60, samples=S, bands=B).cube
    dc = dev(cube)
    srv = rxm.RxServer(1 << 30, 4)
    st = rxm.RxStream(cfg_for(rxm, B, S, 20), server=srv)
    with pytest.raises(rxm.RxError) as e:
        srv.rx_server_submit(st, dc[0:21], 99)           # longer than the stream's block limit
    assert e.value.status == rxm.RX_E_ARG
    for t in range(3):
        srv.rx_server_submit(st, dc[20 * t:20 * (t + 1)], 10 + t)
    assert srv.rx_server_step() == 1                     # one block per stream per step
    assert srv.rx_server_step() == 1
    assert srv.rx_server_step() == 1
    assert srv.rx_server_step() == 0
    assert srv.rx_server_poll(block=True) == [10, 11, 12]
    got = st.scores_host()
    ref, _ = oracle_stream_scores(cube, B, S, pushes=[20, 20, 20], rho=1e-6)
    assert_scores(got, ref, B, *TOL_BF16, label="served single stream")
    st.rx_destroy()
    srv.rx_server_destroy()


def test_served_mix_with_causal_and_float_streams(rxm):
    # Served streams batched into shared launches with the other readings:
    # causal scoring (its window-before slot formed in the batch on the
    # server, copied from the previous push when alone) and float input with
    # non-finite pixels (the validity pass joins the shared launches).  Every
    # stream must score bit for bit as alone; the FP64 ones match the oracle.
    import torch
    rng = np.random.default_rng(11)
    specs = []   # (B, S, dtype, prec, causal, blocks)
    for B, S, dt, prec, causal in [(200, 640, np.uint16, "bf16", True), (120, 320, np.float32, "fp64", False),
                                   (270, 640, np.uint16, "bf16", False), (64, 256, np.float32, "fp64", True),
                                   (96, 200, np.float64, "fp64", True)]:
        blocks = [int(v) for v in rng.integers(8, 25, size=4)]
        cube = synth.sensor_cube(200 + B, lines=sum(blocks), samples=S, bands=B).cube.astype(dt)
        if dt != np.uint16:
            n = cube.shape[0] * S
            for p in rng.choice(n, size=n // 50, replace=False):
                cube[p // S, rng.integers(B), p % S] = np.nan if p % 3 else np.inf
        specs.append((B, S, dt, prec, causal, blocks, cube))

    def cfg(B, S, dt, prec, causal, bl):
        return rxm.make_config(B, S, in_dtype=dt, syrk=prec, whiten=prec, ridge_rel=1e-6 if prec == "bf16" else 0.0,
                               block_lines=bl, causal=causal)

    dcubes = [dev(s[6]) for s in specs]
    alone = []
    for (B, S, dt, prec, causal, blocks, cube), dc in zip(specs, dcubes):
        st = rxm.RxStream(cfg(B, S, dt, prec, causal, 0))
        l0 = 0
        for n in blocks:
            st.rx_push_lines(dc[l0:l0 + n])
            l0 += n
        st.rx_sync()
        alone.append(st.scores_host(f64=(prec == "fp64")))
        st.rx_destroy()

    srv = rxm.RxServer(8 << 30, 16)
    served = [rxm.RxStream(cfg(B, S, dt, prec, causal, 64), server=srv) for (B, S, dt, prec, causal, _, _) in specs]
    order = [(i, j) for i, s in enumerate(specs) for j in range(len(s[5]))]
    rng.shuffle(order)
    nxt = [0] * len(specs)
    starts = [np.concatenate([[0], np.cumsum(s[5])]) for s in specs]
    tag = 0
    for i, _ in order:
        j = nxt[i]
        nxt[i] += 1
        srv.rx_server_submit(served[i], dcubes[i][int(starts[i][j]):int(starts[i][j + 1])], tag)
        tag += 1
    while srv.rx_server_queued()[0] > 0:
        srv.rx_server_step()
    assert sorted(srv.rx_server_poll(block=True)) == list(range(tag))
    torch.cuda.synchronize()
    for k, ((B, S, dt, prec, causal, blocks, cube), st) in enumerate(zip(specs, served)):
        got = st.scores_host(f64=(prec == "fp64"))
        w = np.uint64 if prec == "fp64" else np.uint32
        assert np.array_equal(got.view(w), alone[k].view(w)), f"stream {k} (B={B}, S={S}, causal={causal})"
        if prec == "fp64":
            ref, _ = oracle_stream_scores(cube, B, S, pushes=blocks, causal=causal)
            assert_scores(got, ref, B, 1e-9, 1e-11, label=f"served B={B} S={S} causal={causal}")
        st.rx_destroy()
    srv.rx_server_destroy()


def test_straddling_submit_is_refused_and_the_server_stays_consistent(rxm):
    # A block that would cross its stream's window edge is refused at
    # submission (nothing is queued, no stream changes); the streams already
    # queued on the server, including the refused stream's earlier blocks,
    # still produce exactly their scores alone.
    B, S, W = 64, 128, 40
    a_cube = synth.sensor_cube(61, lines=60, samples=S, bands=B).cube
    b_cube = synth.sensor_cube(62, lines=48, samples=S, bands=B).cube
    da, db = dev(a_cube), dev(b_cube)

    def cfg(win):
        return rxm.make_config(B, S, in_dtype=np.uint16, syrk="bf16", whiten="bf16", ridge_rel=1e-6,
                               block_lines=32, window_lines=win)

    alone_a = rxm.RxStream(cfg(W))
    for l0, n in ((0, 24), (24, 16), (40, 20)):
        alone_a.rx_push_lines(da[l0:l0 + n])
    alone_a.rx_sync()
    want_a = alone_a.scores_host()
    alone_a.rx_destroy()
    alone_b = rxm.RxStream(cfg(0))
    for l0, n in ((0, 16), (16, 32)):
        alone_b.rx_push_lines(db[l0:l0 + n])
    alone_b.rx_sync()
    want_b = alone_b.scores_host()
    alone_b.rx_destroy()

    srv = rxm.RxServer(1 << 30, 4)
    sa = rxm.RxStream(cfg(W), server=srv)
    sb = rxm.RxStream(cfg(0), server=srv)
    srv.rx_server_submit(sa, da[0:24], 0)
    srv.rx_server_submit(sb, db[0:16], 1)
    with pytest.raises(rxm.RxError) as e:           # lines 24..48 would cross the edge at 40
        srv.rx_server_submit(sa, da[24:48], 2)
    assert e.value.status == rxm.RX_E_ARG
    assert srv.rx_server_queued()[0] == 2
    srv.rx_server_submit(sa, da[24:40], 3)          # up to the edge
    srv.rx_server_submit(sa, da[40:60], 4)          # the next window
    srv.rx_server_submit(sb, db[16:48], 5)
    done = []
    while len(done) < 5:
        srv.rx_server_step()
        done += srv.rx_server_poll(block=True)
    assert sorted(done) == [0, 1, 3, 4, 5]
    got_a, got_b = sa.scores_host(), sb.scores_host()
    sa.rx_destroy()
    sb.rx_destroy()
    srv.rx_server_destroy()
    assert np.array_equal(got_a.view(np.uint32), want_a.view(np.uint32))
    assert np.array_equal(got_b.view(np.uint32), want_b.view(np.uint32))


def test_request_loop_mix_equals_alone_bitwise(rxm):
    # The library's own request loop (rx_server_start) steps the server while
    # blocks are submitted from this thread in an interleaved random order,
    # with pauses so that some steps run while others are queued.  Every
    # block is stamped done on the library clock, after its submission; the
    # scores equal the streams' alone runs bit for bit.
    import time
    import torch
    streams = make_streams(17)
    dcubes = [dev(c) for (_, _, _, c) in streams]
    alone = []
    for (B, S, blocks, cube), dc in zip(streams, dcubes):
        st = rxm.RxStream(cfg_for(rxm, B, S, 0))
        l0 = 0
        for n in blocks:
            st.rx_push_lines(dc[l0:l0 + n])
            l0 += n
        st.rx_sync()
        alone.append(st.scores_host())
        st.rx_destroy()
    srv = rxm.RxServer(8 << 30, 16)
    served = [rxm.RxStream(cfg_for(rxm, B, S, 64), server=srv) for (B, S, _, _) in streams]
    order = [(i, j) for i, s in enumerate(streams) for j in range(len(s[2]))]
    rng = np.random.default_rng(5)
    rng.shuffle(order)
    starts = [np.concatenate([[0], np.cumsum(s[2])]) for s in streams]
    nxt = [0] * len(streams)
    with pytest.raises(rxm.RxError):
        srv.rx_server_start()
        srv.rx_server_start()                       # already running
    sub = {}
    for tag, (i, _) in enumerate(order):
        j = nxt[i]
        nxt[i] += 1
        sub[tag] = rxm.clock_ns()
        srv.rx_server_submit(served[i], dcubes[i][int(starts[i][j]):int(starts[i][j + 1])], tag)
        if tag % 4 == 3:
            time.sleep(0.002)
    with pytest.raises(rxm.RxError) as e:
        srv.rx_server_step()                        # the loop steps by itself
    assert e.value.status == rxm.RX_E_STATE
    tags, stamps = srv.rx_server_poll_ns(block=True)
    srv.rx_server_stop()
    assert sorted(tags) == list(range(len(order)))
    lat = [(t_done - sub[t]) * 1e-6 for t, t_done in zip(tags, stamps)]
    say(f"request loop: {len(order)} blocks, latency ms p50 {np.median(lat):.3f}, max {max(lat):.3f}")
    assert min(lat) > 0.0
    torch.cuda.synchronize()
    for k, ((B, S, blocks, cube), st) in enumerate(zip(streams, served)):
        got = st.scores_host()
        assert np.array_equal(got.view(np.uint32), alone[k].view(np.uint32)), f"stream {k} (B={B}, S={S})"
        st.rx_destroy()
    srv.rx_server_destroy()


def test_served_one_pass_streams(rxm):
    # One-pass scoring on the server: every submitted block is a push of its
    # own, scored with the window before it (its slot formed in the step and
    # factored there).  The FP64 stream scores bit for bit as the same
    # stream alone pushing the same blocks (whose window-before slot is
    # copied from the previous push) and matches the oracle's one-pass mode;
    # the BF16 stream matches the oracle within the BF16 bounds (scaled by
    # sqrt(270 / B) below 270 bands); an update-then-score stream shares the
    # launches.
    import torch
    rng = np.random.default_rng(13)
    specs = []   # (B, S, prec, one_pass, blocks, cube)
    for B, S, prec, op in [(96, 200, "fp64", True), (120, 320, "bf16", True), (64, 256, "fp64", False)]:
        blocks = [int(v) for v in rng.integers(8, 25, size=5)]
        cube = synth.sensor_cube(300 + B, lines=sum(blocks), samples=S, bands=B).cube
        specs.append((B, S, prec, op, blocks, cube))

    def cfg(B, S, prec, op, bl):
        return rxm.make_config(B, S, in_dtype=np.uint16, syrk=prec, whiten=prec,
                               ridge_rel=1e-6 if prec == "bf16" else 0.0, block_lines=bl, one_pass=op)

    dcubes = [dev(s[5]) for s in specs]
    alone = []
    for (B, S, prec, op, blocks, cube), dc in zip(specs, dcubes):
        st = rxm.RxStream(cfg(B, S, prec, op, 0))
        l0 = 0
        for n in blocks:
            st.rx_push_lines(dc[l0:l0 + n])
            l0 += n
        st.rx_sync()
        alone.append(st.scores_host(f64=(prec == "fp64")))
        st.rx_destroy()
    srv = rxm.RxServer(8 << 30, 16)
    served = [rxm.RxStream(cfg(B, S, prec, op, 64), server=srv) for (B, S, prec, op, _, _) in specs]
    order = [(i, j) for i, s in enumerate(specs) for j in range(len(s[4]))]
    rng.shuffle(order)
    nxt = [0] * len(specs)
    starts = [np.concatenate([[0], np.cumsum(s[4])]) for s in specs]
    tag = 0
    for i, _ in order:
        j = nxt[i]
        nxt[i] += 1
        srv.rx_server_submit(served[i], dcubes[i][int(starts[i][j]):int(starts[i][j + 1])], tag)
        tag += 1
    while srv.rx_server_queued()[0] > 0:
        srv.rx_server_step()
    assert sorted(srv.rx_server_poll(block=True)) == list(range(tag))
    torch.cuda.synchronize()
    for k, ((B, S, prec, op, blocks, cube), st) in enumerate(zip(specs, served)):
        got = st.scores_host(f64=(prec == "fp64"))
        rho = 1e-6 if prec == "bf16" else 0.0
        ref, o = oracle_stream_scores(cube, B, S, rho=rho, pushes=blocks, one_pass=op)
        assert st.rx_get_counters().notready_blocks == o.status.count("notready")
        if prec == "fp64":
            assert np.array_equal(got.view(np.uint64), alone[k].view(np.uint64)), f"stream {k} (B={B}, one_pass={op})"
            assert_scores(got, ref, B, 1e-9, 1e-11, label=f"served B={B} one_pass={op}")
        else:
            f = max(1.0, (270.0 / B) ** 0.5)
            assert_scores(got, ref, B, 5e-2 * f, 1e-2 * f, label=f"served B={B} one_pass={op} bf16")
        st.rx_destroy()
    srv.rx_server_destroy()
