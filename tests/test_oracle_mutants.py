"""Planted mistakes: each mutant is a plausible error in the oracle (a dropped
term, a wrong index, a transposed operand, an off-by-one, a wrong sign) and
must be caught by at least one pin.  The mistakes are planted in copies of
oracle functions on the CPU; the real oracle must pass every check."""
import numpy as np
import pytest

from oracle import brute, rx
from paper_2602_13509_amd import synth


class Impl:
    """The pieces of the oracle the pins exercise, swappable one by one."""

    def __init__(self, **over):
        self.pixels = over.get("pixels", rx.pixels)
        self.stats = over.get("stats", rx.stats)
        self.scores = over.get("scores", rx.scores)
        self.regularise = over.get("regularise", rx.regularise)
        self.topk = over.get("topk", rx.mask_topk)

    def batch(self, cube, rho=0.0):
        px = self.pixels(cube)
        mu, cov = self.stats(px)
        return self.scores(px, mu, self.regularise(cov, rho))


# ---------------------------------------------------------------- checks
def chk_brute(im):
    rng = np.random.default_rng(3)
    px = rng.integers(0, 9, size=(30, 4))
    exact = np.array([float(v) for v in brute.exact_scores(px.tolist())])
    cube = px.reshape(1, 30, 4).transpose(0, 2, 1)
    return np.allclose(im.batch(cube), exact, rtol=1e-12, atol=0)


def chk_mean_is_b(im):
    c = synth.sensor_cube(2, lines=6, samples=32, bands=12).cube
    return abs(im.batch(c).mean() - 12) < 1e-8


def chk_zero_at_mean(im):
    rng = np.random.default_rng(6)
    c, v = rng.normal(size=5) + 3.0, rng.normal(size=(7, 5))
    x = np.vstack([c + v, c - v, c[None, :]])
    cube = x.reshape(1, 15, 5).transpose(0, 2, 1)
    d = im.batch(cube)
    return abs(d[-1]) < 1e-10


def chk_affine(im):
    g = synth.gauss_cube(7, lines=8, samples=16, bands=6)
    rng = np.random.default_rng(1)
    a, t = rng.normal(size=(6, 6)) + 3 * np.eye(6), rng.normal(size=6)
    y = np.einsum("ij,ljs->lis", a, g.cube) + t[None, :, None]
    return np.allclose(im.batch(g.cube), im.batch(y), rtol=1e-8)


def chk_ridge_mean(im):
    g = synth.gauss_cube(2, lines=8, samples=32, bands=10)
    px = rx.pixels(g.cube)
    mu, cov = rx.stats(px)
    lam = 1e-2 * np.trace(cov) / 10
    ev = np.linalg.eigvalsh(cov)
    return abs(im.batch(g.cube, rho=1e-2).mean() - np.sum(ev / (ev + lam))) < 1e-8


def chk_anomalies_first(im):
    g = synth.gauss_cube(0)
    return np.array_equal(np.flatnonzero(im.topk(im.batch(g.cube), 5)), g.anomalies)


def chk_tie_rule(im):
    d = np.array([1.0, 2.0, 2.0, 0.0])
    return np.flatnonzero(im.topk(d, 1)).tolist() == [1]


CHECKS = [chk_brute, chk_mean_is_b, chk_zero_at_mean, chk_affine, chk_ridge_mean,
          chk_anomalies_first, chk_tie_rule]


def _run(im):
    out = {}
    for c in CHECKS:
        try:
            out[c.__name__] = bool(c(im))
        except Exception:
            out[c.__name__] = False
    return out


# ---------------------------------------------------------------- mutants
def scores_no_inverse(px, mu, cov):
    d = np.asarray(px, float) - mu
    return np.einsum("pk,kj,pj->p", d, cov, d)


def scores_no_centring(px, mu, cov):
    x = np.asarray(px, float)
    return np.einsum("pk,kp->p", x, np.linalg.solve(cov, x.T))


def scores_transposed_solve(px, mu, cov):
    d = np.asarray(px, float) - mu
    z = np.linalg.solve(cov, d.T)
    return np.einsum("pk,kp->p", d[::-1], z)       # pairs pixel p with pixel N-1-p


def stats_ddof_off_by_one(px):
    return rx.stats(px, ddof=1)


def stats_wrong_cross_term(px):
    if not np.issubdtype(np.asarray(px).dtype, np.integer):
        return rx.stats(px)
    n, s1, s2 = rx.int_moments(px)
    b = len(s1)
    mu = s1 / n
    cov = np.array([[(n * int(s2[j, k]) - int(s1[j]) * int(s1[j])) / (n * n) for k in range(b)]
                    for j in range(b)])
    return mu, (cov + cov.T) / 2


def regularise_wrong_sign(cov, rho):
    return cov - rho * np.trace(cov) / cov.shape[0] * np.eye(cov.shape[0])


def pixels_missing_transpose(cube):
    l, b, s = cube.shape
    return cube.reshape(l * s, b)


def topk_ties_high(d, k):
    d = np.asarray(d, float)
    order = np.lexsort((-np.arange(d.size), -d))[:k]
    m = np.zeros(d.size, bool)
    m[order] = True
    return m


MUTANTS = {
    "dropped inverse": dict(scores=scores_no_inverse),
    "dropped centring": dict(scores=scores_no_centring),
    "transposed operand": dict(scores=scores_transposed_solve),
    "ddof off by one": dict(stats=stats_ddof_off_by_one),
    "wrong cross index": dict(stats=stats_wrong_cross_term),
    "ridge sign": dict(regularise=regularise_wrong_sign),
    "pixel layout": dict(pixels=pixels_missing_transpose),
    "tie order": dict(topk=topk_ties_high),
}


def test_real_oracle_passes_every_check():
    res = _run(Impl())
    assert all(res.values()), res


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_each_planted_mistake_is_caught(name):
    res = _run(Impl(**MUTANTS[name]))
    assert not all(res.values()), f"mutant '{name}' passed every pin: {res}"


# ---------------------------------------------------------------- stream oracle: causal scoring, non-finite pixels
from oracle.stream import RxStreamOracle  # noqa: E402


def chk_causal_exact(cls):
    """Causal block scores = exact-rational forms over the earlier lines."""
    L, B, S, bl = 6, 3, 6, 2
    cube = np.random.default_rng(8).integers(0, 9, size=(L, B, S)).astype(np.uint16)
    o = cls(B, S, block_lines=bl, causal=True)
    got = o.push(cube)
    px = rx.pixels(cube)
    for l0 in range(bl, L, bl):
        prev = px[:l0 * S]
        mu, cov = brute.exact_stats(prev.tolist())
        inv = brute.gauss_jordan_inverse(cov)
        for p in range(l0 * S, (l0 + bl) * S):
            d = [int(px[p, j]) - mu[j] for j in range(B)]
            want = float(sum(d[i] * inv[i][j] * d[j] for i in range(B) for j in range(B)))
            if not abs(got[p] - want) <= 1e-12 * max(abs(want), 1e-300):
                return False
    return np.isnan(got[:bl * S]).all()


def chk_nonfinite_exact(cls):
    """Finite pixels score as the exact-rational set without the others."""
    L, B, S = 4, 3, 8
    cube = np.random.default_rng(5).integers(0, 9, size=(L, B, S)).astype(np.float64)
    cube[1, 2, 5] = np.inf
    cube[3, 0, 0] = np.nan
    o = cls(B, S)
    got = o.push(cube)
    px = rx.pixels(cube)
    fin = np.isfinite(px).all(axis=1)
    exact = np.array([float(v) for v in brute.exact_scores(px[fin].astype(np.int64).tolist())])
    return (np.array_equal(np.isnan(got), ~fin) and o.nonfinite == 2
            and np.allclose(got[fin], exact, rtol=1e-12, atol=0))


class CausalUsesUpdatedWindow(RxStreamOracle):
    """Mistake: the causal flag ignored (the block joins the window first)."""
    def __init__(self, *a, causal=False, **k):
        super().__init__(*a, causal=False, **k)


class NonfiniteStillCounted(RxStreamOracle):
    """Mistake: non-finite pixels left out of the sums but still counted in N."""
    def _score_block(self, px):
        self.n += int((~rx.finite_pixels(px)).sum())
        try:
            return super()._score_block(px)
        finally:
            self.n -= int((~rx.finite_pixels(px)).sum())

    def stats(self):
        n, mu, cov = super().stats()
        kept = np.concatenate(self.float_px)
        d = kept - mu[None, :]
        return n, mu, (d.T @ d) / self.n


class NonfiniteScoredFinite(RxStreamOracle):
    """Mistake: non-finite pixels excluded from the statistics but their
    scores computed anyway (inf / nan arithmetic) instead of NaN."""
    def _score_block(self, px):
        out = super()._score_block(px)
        bad = ~rx.finite_pixels(px)
        out[bad] = 0.0
        return out


def test_stream_oracle_passes_its_new_pins():
    assert chk_causal_exact(RxStreamOracle)
    assert chk_nonfinite_exact(RxStreamOracle)


@pytest.mark.parametrize("cls,chk", [(CausalUsesUpdatedWindow, chk_causal_exact),
                                     (NonfiniteStillCounted, chk_nonfinite_exact),
                                     (NonfiniteScoredFinite, chk_nonfinite_exact)])
def test_stream_oracle_mutants_caught(cls, chk):
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        assert not chk(cls)
