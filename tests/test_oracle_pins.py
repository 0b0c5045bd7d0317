"""Pins for the FP64 oracle: each test fixes part of it by something other
than the oracle itself -- exact rationals, closed forms, identities of Eq. 1
(paper, Section "System Implementation / Detection Algorithm"), the
band-transform invariance the paper states (Section "System Architecture /
Data Acquisition"), brute force and library special cases.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats as sstats

from oracle import brute, rx
from oracle.stream import RxStreamOracle, float_stats_chunked
from paper_2602_13509_amd import synth


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def _tiny_int_px(seed, n, b, hi=9):
    rng = np.random.default_rng(seed)
    while True:
        px = rng.integers(0, hi, size=(n, b))
        mu, cov = rx.stats(px)
        if np.linalg.matrix_rank(cov) == b:
            return px


# ---------------------------------------------------------------- P1 exact rationals
@pytest.mark.parametrize("seed,n,b", [(0, 12, 1), (1, 20, 2), (2, 24, 3), (3, 40, 5), (4, 64, 6)])
def test_p1_brute_force_rationals(seed, n, b):
    px = _tiny_int_px(seed, n, b)
    exact = [float(v) for v in brute.exact_scores(px.tolist())]
    got = rx.scores(px, *rx.stats(px))
    assert _rel(got, exact) <= 1e-13


@pytest.mark.parametrize("ddof", [0, 1])
def test_p1_brute_force_ridge_and_ddof(ddof):
    px = _tiny_int_px(7, 30, 4)
    exact = [float(v) for v in brute.exact_scores(px.tolist(), ddof=ddof, ridge_num=1, ridge_den=10)]
    mu, cov = rx.stats(px, ddof)
    got = rx.scores(px, mu, rx.regularise(cov, 0.1))
    assert _rel(got, exact) <= 1e-13


def test_p1_exact_integer_covariance():
    px = _tiny_int_px(11, 50, 6, hi=4096)
    mu_f, cov_f = brute.exact_stats(px.tolist())
    mu, cov = rx.stats(px)
    # the integer path rounds each entry correctly: equal to the rounded rational
    assert all(mu[j] == float(mu_f[j]) for j in range(6))
    assert all(cov[j, k] == float(cov_f[j][k]) for j in range(6) for k in range(6))


# ---------------------------------------------------------------- P2 closed forms
def test_p2_single_band_closed_form():
    rng = np.random.default_rng(3)
    x = rng.normal(5.0, 2.0, size=(500, 1))
    m = sum(x[:, 0]) / len(x)
    var = sum((v - m) ** 2 for v in x[:, 0]) / len(x)
    want = [(v - m) ** 2 / var for v in x[:, 0]]
    got = rx.scores(x, *rx.stats(x))
    assert _rel(got, want) <= 1e-12


def test_p2_two_band_adjugate():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(300, 2)) @ np.array([[1.0, 0.3], [0.0, 0.5]])
    mu, cov = rx.stats(x)
    a, bb, c = cov[0, 0], cov[0, 1], cov[1, 1]
    d1, d2 = x[:, 0] - mu[0], x[:, 1] - mu[1]
    want = (c * d1 * d1 - 2 * bb * d1 * d2 + a * d2 * d2) / (a * c - bb * bb)
    assert _rel(rx.scores(x, mu, cov), want) <= 1e-12


# ---------------------------------------------------------------- P3 leverage identity
@pytest.mark.parametrize("b", [1, 3, 8, 20])
def test_p3_n_equals_b_plus_one(b):
    # N = B+1 points in general position: the hat matrix of [1 X] is I, so every
    # pixel sits at leverage 1 and delta_p = N*h_pp - 1 = B exactly.
    rng = np.random.default_rng(b)
    x = rng.normal(size=(b + 1, b))
    d = rx.scores(x, *rx.stats(x))
    assert np.max(np.abs(d - b)) <= 1e-9 * b


# ---------------------------------------------------------------- P4 mean score
@pytest.mark.parametrize("seed", [0, 1])
def test_p4_mean_score_equals_bands(seed):
    g = synth.gauss_cube(seed)
    d = rx.rx_batch(g.cube)
    assert abs(d.mean() - 32) <= 1e-9


def test_p4_mean_score_equals_bands_integer_cube():
    c = synth.sensor_cube(1, lines=8, samples=64, bands=40)
    d = rx.rx_batch(c.cube)
    assert abs(d.mean() - 40) <= 1e-8


def test_p4_mean_score_with_ridge_spectral_sum():
    g = synth.gauss_cube(2, lines=16, samples=64, bands=24)
    px = rx.pixels(g.cube)
    mu, cov = rx.stats(px)
    rho = 1e-2
    lam = rho * np.trace(cov) / 24
    want = np.sum(np.linalg.eigvalsh(cov) / (np.linalg.eigvalsh(cov) + lam))
    d = rx.scores(px, mu, rx.regularise(cov, rho))
    assert abs(d.mean() - want) <= 1e-9 * want


# ---------------------------------------------------------------- P5 bound
def test_p5_leverage_bound():
    g = synth.gauss_cube(5, lines=4, samples=16, bands=12)
    d = rx.rx_batch(g.cube)
    n = d.size
    assert d.min() >= -1e-12 and d.max() <= n - 1 + 1e-9


def test_p5_bound_reached_by_lone_outlier():
    # all pixels equal except one outlier along one band direction plus
    # independent noise in the others: the outlier's leverage tends to 1.
    rng = np.random.default_rng(9)
    x = rng.normal(size=(200, 3)) * 1e-6
    x[17, 0] += 1.0
    d = rx.scores(x, *rx.stats(x))
    assert d.max() <= 199 + 1e-6 and d[17] > 150


# ---------------------------------------------------------------- P6 zero at the mean
def test_p6_zero_at_mean():
    rng = np.random.default_rng(6)
    c = rng.normal(size=7)
    v = rng.normal(size=(9, 7))
    x = np.vstack([c + v, c - v, c[None, :]])
    d = rx.scores(x, *rx.stats(x))
    assert abs(d[-1]) <= 1e-20 + 1e-12 * d[:-1].max()


# ---------------------------------------------------------------- P7 band transform
def test_p7_affine_band_transform_invariance():
    g = synth.gauss_cube(7, lines=16, samples=32, bands=10)
    px = rx.pixels(g.cube)
    rng = np.random.default_rng(70)
    a = rng.normal(size=(10, 10)) + 3 * np.eye(10)
    t = rng.normal(size=10)
    d0 = rx.scores(px, *rx.stats(px))
    y = px @ a.T + t
    d1 = rx.scores(y, *rx.stats(y))
    assert _rel(d1, d0) <= 1e-8


def test_p7_orthogonal_scaled_transform_with_ridge():
    g = synth.gauss_cube(8, lines=16, samples=32, bands=10)
    px = rx.pixels(g.cube)
    q = np.linalg.qr(np.random.default_rng(80).normal(size=(10, 10)))[0]
    y = 3.5 * px @ q.T + 1.0
    for p in (px, y):
        mu, cov = rx.stats(p)
        if p is px:
            d0 = rx.scores(p, mu, rx.regularise(cov, 1e-3))
        else:
            d1 = rx.scores(p, mu, rx.regularise(cov, 1e-3))
    assert _rel(d1, d0) <= 1e-9


# ---------------------------------------------------------------- P8/P9 streaming
def test_p8_push_split_invariance_exact():
    cube = synth.sensor_cube(3, lines=40, samples=24, bands=16).cube
    finals = []
    for step in (1, 7, 40):
        o = RxStreamOracle(16, 24)
        for l0 in range(0, 40, step):
            o.push(cube[l0:l0 + step])
        finals.append((o.n, o.s1.copy(), o.s2.copy()))
    for f in finals[1:]:
        assert f[0] == finals[0][0]
        assert np.array_equal(f[1], finals[0][1]) and np.array_equal(f[2], finals[0][2])


def test_p8_pixel_order_invariance_exact():
    cube = synth.sensor_cube(4, lines=6, samples=20, bands=12).cube
    px = rx.pixels(cube)
    perm = np.random.default_rng(1).permutation(px.shape[0])
    assert all(np.array_equal(a, b) for a, b in zip(rx.int_moments(px), rx.int_moments(px[perm])))


def test_p9_stream_one_block_equals_batch():
    cube = synth.sensor_cube(5, lines=10, samples=32, bands=20).cube
    o = RxStreamOracle(20, 32)
    assert np.array_equal(o.push(cube), rx.rx_batch(cube))


def test_p9_reset_window_equals_independent_cubes():
    cube = synth.sensor_cube(6, lines=30, samples=16, bands=8).cube
    o = RxStreamOracle(8, 16, window_lines=10)
    got = np.concatenate([o.push(cube[i:i + 10]) for i in range(0, 30, 10)])
    want = np.concatenate([rx.rx_batch(cube[i:i + 10]) for i in range(0, 30, 10)])
    assert np.array_equal(got, want)


def test_p9_block_lines_split_matches_per_block_pushes():
    cube = synth.sensor_cube(7, lines=25, samples=16, bands=8).cube
    a = RxStreamOracle(8, 16, block_lines=10)
    got = a.push(cube)
    b = RxStreamOracle(8, 16)
    want = np.concatenate([b.push(cube[0:10]), b.push(cube[10:20]), b.push(cube[20:25])])
    assert np.array_equal(got, want)


def test_stream_update_then_score_prefix():
    # block k is scored with the statistics of blocks 0..k (cumulative window)
    cube = synth.sensor_cube(8, lines=12, samples=16, bands=6).cube
    o = RxStreamOracle(6, 16, block_lines=4)
    got = o.push(cube)
    for k in range(3):
        px_all = rx.pixels(cube[: 4 * (k + 1)])
        mu, cov = rx.stats(px_all)
        want = rx.scores(rx.pixels(cube[4 * k: 4 * (k + 1)]), mu, cov)
        assert _rel(got[64 * k: 64 * (k + 1)], want) <= 1e-12


def test_stream_notready_and_singular():
    o = RxStreamOracle(8, 4)                 # 4 pixels per line, B = 8
    c = synth.random_int_cube(0, 2, 4, 8, hi=100)
    d = o.push(c)                             # N = 8 <= B
    assert np.all(np.isnan(d)) and o.status == ["notready"]
    c2 = synth.random_int_cube(1, 10, 4, 8, hi=100)
    c2[:, 3, :] = 5                           # constant band
    o2 = RxStreamOracle(8, 4)
    d2 = o2.push(c2)
    assert np.all(np.isnan(d2)) and o2.status == ["singular"]
    o3 = RxStreamOracle(8, 4, rho=1e-3)       # ridge lifts the constant band
    assert np.all(np.isfinite(o3.push(c2))) and o3.status == ["ok"]


def test_float_stats_chunked_matches_two_pass():
    s = synth.stress_cube(1, lines=12, samples=32, bands=20)
    px = rx.pixels(s.cube)
    n, mu, cov = float_stats_chunked(lambda: (px[i:i + 50] for i in range(0, px.shape[0], 50)))
    mu2, cov2 = rx.float_stats(px)
    assert n == px.shape[0]
    assert _rel(mu, mu2) <= 1e-12 and np.max(np.abs(cov - cov2)) <= 1e-10 * np.abs(cov2).max()


# ---------------------------------------------------------------- P10 anomalies rank first
@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_p10_implanted_anomalies_rank_first(seed):
    g = synth.gauss_cube(seed)
    d = rx.rx_batch(g.cube)
    top = np.flatnonzero(rx.mask_topk(d, 5))
    assert np.array_equal(top, g.anomalies)


# ---------------------------------------------------------------- P12 Beta law (statistical)
def test_p12_in_sample_beta_law():
    g = synth.gauss_cube(12, lines=64, samples=128, bands=32, n_anomalies=0)
    d = rx.rx_batch(g.cube)
    n, b = d.size, 32
    u = n * d / (n - 1) ** 2
    ks = sstats.kstest(u, sstats.beta(b / 2, (n - b - 1) / 2).cdf)
    assert ks.pvalue > 1e-3


# ---------------------------------------------------------------- P13 library special case
def test_p13_numpy_inverse_matches_gauss_jordan():
    rng = np.random.default_rng(13)
    a = rng.integers(-5, 6, size=(6, 6))
    spd = a @ a.T + 6 * np.eye(6, dtype=np.int64)
    gj = brute.gauss_jordan_inverse([[Fraction(int(v)) for v in row] for row in spd])
    inv = np.linalg.inv(spd.astype(float))
    assert np.max(np.abs(inv - np.array([[float(v) for v in r] for r in gj]))) <= 1e-14
    l = np.linalg.cholesky(spd.astype(float))
    assert np.max(np.abs(l @ l.T - spd)) <= 1e-12


# ---------------------------------------------------------------- P14/P15
def test_p14_ddof_relation():
    g = synth.gauss_cube(14, lines=8, samples=32, bands=16)
    px = rx.pixels(g.cube)
    n = px.shape[0]
    d0 = rx.scores(px, *rx.stats(px, 0))
    d1 = rx.scores(px, *rx.stats(px, 1))
    assert _rel(d1, d0 * (n - 1) / n) <= 1e-10


def test_p15_scale_invariance_with_ridge():
    g = synth.gauss_cube(15, lines=8, samples=32, bands=16)
    px = rx.pixels(g.cube)
    out = []
    for c in (1.0, 1234.5):
        mu, cov = rx.stats(c * px)
        out.append(rx.scores(c * px, mu, rx.regularise(cov, 1e-4)))
    assert _rel(out[1], out[0]) <= 1e-9


# ---------------------------------------------------------------- masks
def test_masks_against_loops():
    d = np.array([0.5, 2.0, 2.0, np.nan, 1.0, 3.0, 3.0, 0.1, 2.0])
    assert rx.mask_abs(d, 2.0).tolist() == [v > 2.0 if v == v else False for v in d]
    m = max(v for v in d if v == v)
    assert rx.mask_rel(d, 0.5).tolist() == [(v > 0.5 * m) if v == v else False for v in d]
    # top-3: the two 3.0 then the lowest-index 2.0 (pixel 1)
    assert np.flatnonzero(rx.mask_topk(d, 3)).tolist() == [1, 5, 6]
    assert np.flatnonzero(rx.mask_topk(d, 4)).tolist() == [1, 2, 5, 6]


def test_pack_bits_order():
    m = np.zeros(11, dtype=bool)
    m[[0, 3, 8, 10]] = True
    assert rx.pack_bits(m).tolist() == [0b00001001, 0b00000101]


# ---------------------------------------------------------------- generators
def test_generators_deterministic():
    a = synth.sensor_cube(3, lines=5, samples=16, bands=30)
    b = synth.sensor_cube(3, lines=5, samples=16, bands=30)
    c = synth.sensor_cube(4, lines=5, samples=16, bands=30)
    assert np.array_equal(a.cube, b.cube) and not np.array_equal(a.cube, c.cube)
    assert np.array_equal(synth.gauss_cube(1).cube, synth.gauss_cube(1).cube)
    assert np.array_equal(synth.stress_cube(2, 4, 8, 12).cube, synth.stress_cube(2, 4, 8, 12).cube)


def test_generator_shapes_and_ranges():
    s = synth.sensor_cube(0, lines=40, samples=100, bands=50)
    assert s.cube.dtype == np.uint16 and s.cube.shape == (40, 50, 100)
    assert s.cube.max() <= 4095 and len(s.anomalies) == 2
    st = synth.stress_cube(0, lines=4, samples=8, bands=30)
    assert st.cube.dtype == np.float32
    assert np.isclose(st.gains.max() / st.gains.min(), 1e3)
    assert np.isclose(st.core_eigs.max() / st.core_eigs.min(), 1e6)


def test_gauss_generator_moments():
    g = synth.gauss_cube(21, lines=256, samples=128, bands=8, n_anomalies=0)
    px = synth.bil_to_pixels(g.cube)
    assert np.max(np.abs(px.mean(axis=0) - g.mean)) < 5 * np.sqrt(np.max(np.diag(g.cov)) / px.shape[0])
    emp = np.cov(px.T, bias=True)
    assert np.max(np.abs(emp - g.cov)) < 0.05 * np.max(np.abs(g.cov))


def test_served_stream_specs():
    sp = synth.served_streams(0)
    assert len(sp) == 16
    assert {(s.samples, s.bands) for s in sp[:12]} == {(a, b) for a in (320, 640, 1024) for b in (120, 200, 270, 300)}
    for s in sp:
        assert 100 <= s.rate_lines_per_s <= 400
        assert np.all(np.diff(s.arrivals) > 0) and s.arrivals[-1] <= 30.0
        assert s.block_lines.min() >= 16 and s.block_lines.max() <= 128


# ---------------------------------------------------------------- non-finite float pixels
@pytest.mark.parametrize("block_lines", [0, 2])
def test_nonfinite_pixels_are_not_part_of_the_set(block_lines):
    # Float input holding small integers, with NaN / +-inf planted in some
    # pixels (one of them in the first line): every other pixel must score
    # exactly what the exact-rational brute force gives over the finite
    # pixels pushed so far, the planted ones NaN, and the count must match.
    L, B, S = 6, 3, 8
    rng = np.random.default_rng(5)
    cube = rng.integers(0, 9, size=(L, B, S)).astype(np.float64)
    bad = {(0, 0, 1): np.nan, (1, 2, 5): np.inf, (3, 1, 0): -np.inf, (4, 0, 7): np.nan, (4, 2, 7): np.nan}
    for (l, b, s), v in bad.items():
        cube[l, b, s] = v
    o = RxStreamOracle(B, S, block_lines=block_lines)
    got = o.push(cube)
    px = rx.pixels(cube)
    fin = np.isfinite(px).all(axis=1)
    assert o.nonfinite == int((~fin).sum()) == 4            # (4, 0, 7) and (4, 2, 7) are one pixel
    assert np.array_equal(np.isnan(got), ~fin)
    step = (block_lines or L) * S
    for p0 in range(0, L * S, step):
        seen = px[:p0 + step][fin[:p0 + step]]
        exact = [float(v) for v in brute.exact_scores(seen.astype(np.int64).tolist())]
        want = np.full(step, np.nan)
        want[fin[p0:p0 + step]] = exact[len(exact) - int(fin[p0:p0 + step].sum()):]
        ok = fin[p0:p0 + step]
        assert _rel(got[p0:p0 + step][ok], want[ok]) <= 1e-12
    assert o.n == int(fin.sum())


def test_nonfinite_batch_equals_set_without_them():
    rng = np.random.default_rng(6)
    cube = rng.normal(size=(5, 4, 9))
    cube[2, 1, 3] = np.nan
    cube[0, 3, 8] = -np.inf
    px = rx.pixels(cube)
    fin = np.isfinite(px).all(axis=1)
    got = rx.rx_batch(cube)
    kept = px[fin]
    # the set without the non-finite pixels, scored by the closed form
    # delta = N h_pp - 1 of the hat matrix of [1 X] (ddof 0, no ridge)
    x1 = np.hstack([np.ones((kept.shape[0], 1)), kept])
    h = np.diag(x1 @ np.linalg.pinv(x1))
    assert np.array_equal(np.isnan(got), ~fin)
    assert _rel(got[fin], kept.shape[0] * h - 1.0) <= 1e-9


# ---------------------------------------------------------------- causal scoring
@pytest.mark.parametrize("window_lines", [0, 4])
def test_causal_blocks_scored_with_the_window_before_them(window_lines):
    # Each block's scores equal exact-rational quadratic forms with the mean
    # and covariance of the window's earlier lines only (Gauss-Jordan
    # inverse); a block that starts a window has none and is not ready.
    L, B, S, bl = 8, 3, 6, 2
    cube = np.random.default_rng(8).integers(0, 9, size=(L, B, S)).astype(np.uint16)
    o = RxStreamOracle(B, S, block_lines=bl, window_lines=window_lines, causal=True)
    got = np.concatenate([o.push(cube[:4]), o.push(cube[4:])])
    px = rx.pixels(cube)
    want_status = []
    for l0 in range(0, L, bl):
        w0 = 0 if window_lines == 0 else (l0 // window_lines) * window_lines
        prev = px[w0 * S:l0 * S]
        blk = slice(l0 * S, (l0 + bl) * S)
        if prev.shape[0] <= B:
            want_status.append("notready")
            assert np.isnan(got[blk]).all()
            continue
        want_status.append("ok")
        mu, cov = brute.exact_stats(prev.tolist())
        inv = brute.gauss_jordan_inverse(cov)
        exact = []
        for p in px[blk]:
            d = [int(p[j]) - mu[j] for j in range(B)]
            exact.append(float(sum(d[i] * inv[i][j] * d[j] for i in range(B) for j in range(B))))
        assert _rel(got[blk], exact) <= 1e-12
    assert o.status == want_status


# ---------------------------------------------------------------- one-pass scoring
@pytest.mark.parametrize("window_lines", [0, 6])
def test_one_pass_blocks_scored_with_the_window_before_the_push(window_lines):
    # Every block of a push is scored with exact-rational quadratic forms over
    # the lines of the window that came before the push (Gauss-Jordan
    # inverse); a block whose window started inside the push, at or before
    # it, has no earlier statistics and is not ready.  Pushes of 3, 5 and 4
    # lines in blocks of at most 2 lines.
    L, B, S, bl = 12, 3, 5, 2
    cube = np.random.default_rng(11).integers(0, 9, size=(L, B, S)).astype(np.uint16)
    o = RxStreamOracle(B, S, block_lines=bl, window_lines=window_lines, one_pass=True)
    pushes = [(0, 3), (3, 8), (8, 12)]
    got = np.concatenate([o.push(cube[a:b]) for a, b in pushes])
    px = rx.pixels(cube)
    want_status = []
    for a, b in pushes:
        w0 = 0 if window_lines == 0 else (a // window_lines) * window_lines
        prev = px[w0 * S:a * S]
        l0 = a
        while l0 < b:
            take = min(bl, b - l0)
            if window_lines:
                take = min(take, window_lines - l0 % window_lines)
            blk = slice(l0 * S, (l0 + take) * S)
            reset_inside = window_lines and any(l % window_lines == 0 for l in range(a, l0 + 1))
            if reset_inside or prev.shape[0] <= B:
                want_status.append("notready")
                assert np.isnan(got[blk]).all()
            else:
                want_status.append("ok")
                mu, cov = brute.exact_stats(prev.tolist())
                inv = brute.gauss_jordan_inverse(cov)
                exact = []
                for p in px[blk]:
                    d = [int(p[j]) - mu[j] for j in range(B)]
                    exact.append(float(sum(d[i] * inv[i][j] * d[j] for i in range(B) for j in range(B))))
                assert _rel(got[blk], exact) <= 1e-12
            l0 += take
    assert o.status == want_status


def test_one_pass_with_one_block_pushes_is_the_causal_reading():
    # one block per push: the window before the push is the window before the
    # block, so both modes give the same scores (the causal mode is pinned
    # against exact rationals above)
    L, B, S, bl = 10, 4, 7, 2
    cube = np.random.default_rng(12).integers(0, 50, size=(L, B, S)).astype(np.uint16)
    a = RxStreamOracle(B, S, block_lines=bl, window_lines=6, one_pass=True, rho=1e-3)
    c = RxStreamOracle(B, S, block_lines=bl, window_lines=6, causal=True, rho=1e-3)
    ga = np.concatenate([a.push(cube[i:i + bl]) for i in range(0, L, bl)])
    gc = c.push(cube)
    assert np.array_equal(np.isnan(ga), np.isnan(gc))
    assert np.array_equal(ga[~np.isnan(ga)], gc[~np.isnan(gc)])
    assert a.status == c.status
