"""Exact-rational brute force for tiny integer cubes -- TEST INFRASTRUCTURE ONLY.

Only tests and fixture scripts may use it.  It recomputes Eq. 1 of the
paper (Section "System Implementation / Detection Algorithm") with Python
Fractions: exact mean, exact covariance with normaliser 1/(N - ddof), an
explicit inverse by Gauss-Jordan elimination, and exact quadratic forms.
It uses no floating point at all, so it pins the FP64 oracle independently.
"""
from __future__ import annotations

from fractions import Fraction


def exact_stats(px, ddof: int = 0):
    """px: list of integer pixel rows.  Returns (mu, Sigma) as Fractions."""
    n = len(px)
    b = len(px[0])
    mu = [Fraction(sum(int(p[j]) for p in px), n) for j in range(b)]
    cov = [[Fraction(0)] * b for _ in range(b)]
    for j in range(b):
        for k in range(b):
            s = sum((int(p[j]) - mu[j]) * (int(p[k]) - mu[k]) for p in px)
            cov[j][k] = s / (n - ddof)
    return mu, cov


def gauss_jordan_inverse(a):
    """Inverse of a square matrix of Fractions by Gauss-Jordan elimination
    with row pivoting on the first non-zero entry.  Raises ZeroDivisionError
    for a singular matrix."""
    n = len(a)
    m = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(a)]
    for c in range(n):
        piv = next((r for r in range(c, n) if m[r][c] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular matrix")
        m[c], m[piv] = m[piv], m[c]
        inv_p = 1 / m[c][c]
        m[c] = [v * inv_p for v in m[c]]
        for r in range(n):
            if r != c and m[r][c] != 0:
                f = m[r][c]
                m[r] = [vr - f * vc for vr, vc in zip(m[r], m[c])]
    return [row[n:] for row in m]


def exact_scores(px, ddof: int = 0, ridge_num: int = 0, ridge_den: int = 1):
    """Exact delta_p for every pixel row.  Optional ridge
    lambda = (ridge_num/ridge_den) * tr(Sigma) / B, added to the diagonal."""
    mu, cov = exact_stats(px, ddof)
    b = len(mu)
    if ridge_num:
        lam = Fraction(ridge_num, ridge_den) * sum(cov[k][k] for k in range(b)) / b
        cov = [[cov[i][j] + (lam if i == j else 0) for j in range(b)] for i in range(b)]
    inv = gauss_jordan_inverse(cov)
    out = []
    for p in px:
        d = [int(p[j]) - mu[j] for j in range(b)]
        out.append(sum(d[i] * inv[i][j] * d[j] for i in range(b) for j in range(b)))
    return out
