"""Pins of the oracle's weighted-quadrature solves against a from-scratch high-precision
computation of the same definition.

The reference below evaluates everything at 40 significant digits with its own routines
(Gauss-Legendre nodes by Newton's method on the three-term recurrence, B-splines by the
Cox-de Boor recursion, Gram integrals by Gauss quadrature) and takes the minimum-norm
solution of the exactness conditions in their original form: sum_q w_q B_j^(a)(x_q) =
int B_i^(a) B_j^(a) for every j overlapping the test function (Section 1, weighted
quadrature; Section 2.2 steps 1 and 5), one redundant condition dropped for a = 1.  The
oracle solves the row-scaled system, and for a = 1 the equivalent system on the
derivative space's B-splines, in FP64; this checks that both choices leave the weights
at full FP64 accuracy at the highest degrees, where the weights are least well fixed.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle.spline import Line, insert_knot_int, support, wq_rule

DPS = 40


def _legendre_mp(n):
    xs, ws = [], []
    for k in range(1, n + 1):
        x = mp.cos(mp.pi * (k - mp.mpf(1) / 4) / (n + mp.mpf(1) / 2))
        for _ in range(200):
            p0, p1 = mp.mpf(1), x
            for m in range(2, n + 1):
                p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
            dp = n * (x * p1 - p0) / (x * x - 1)
            dx = p1 / dp
            x -= dx
            if abs(dx) < mp.mpf(10) ** (-DPS + 3):
                break
        xs.append(x)
        ws.append(2 / ((1 - x * x) * dp * dp))
    order = sorted(range(n), key=lambda k: xs[k])
    return [xs[k] for k in order], [ws[k] for k in order]


def _bsp(t, p, i, x):
    if p == 0:
        if t[i] <= x < t[i + 1]:
            return mp.mpf(1)
        return mp.mpf(1) if (x == t[-1] and t[i] < t[i + 1] == t[-1]) else mp.mpf(0)
    v = mp.mpf(0)
    if t[i + p] != t[i]:
        v += (x - t[i]) / (t[i + p] - t[i]) * _bsp(t, p - 1, i, x)
    if t[i + p + 1] != t[i + 1]:
        v += (t[i + p + 1] - x) / (t[i + p + 1] - t[i + 1]) * _bsp(t, p - 1, i + 1, x)
    return v


def _dbsp(t, p, i, x):
    v = mp.mpf(0)
    if t[i + p] != t[i]:
        v += p / (t[i + p] - t[i]) * _bsp(t, p - 1, i, x)
    if t[i + p + 1] != t[i + 1]:
        v -= p / (t[i + p + 1] - t[i + 1]) * _bsp(t, p - 1, i + 1, x)
    return v


def reference_rule(nel, p, tk, pts, i, a):
    """40-digit minimum-norm weights of test function i (integer knots tk) at the points
    pts = [(element, gauss index)], rounded to FP64."""
    with mp.workdps(DPS):
        h = mp.mpf(1) / nel
        t = [mp.mpf(int(k)) * h for k in tk]
        gx, gw = _legendre_mp(p + 1)
        coord = lambda e, g: (e + (1 + gx[g]) / 2) * h            # noqa: E731
        f = (lambda j, x: _bsp(t, p, j, x)) if a == 0 else (lambda j, x: _dbsp(t, p, j, x))
        sa, sb = support(tk, p, i)
        J = [j for j in range(len(tk) - p - 1) if max(sa, support(tk, p, j)[0]) < min(sb, support(tk, p, j)[1])]
        rows, rhs = [], []
        for j in J:
            rows.append([f(j, coord(e, g)) for (e, g) in pts])
            lo, hi = max(sa, support(tk, p, j)[0]), min(sb, support(tk, p, j)[1])
            rhs.append(sum(gw[g] * h / 2 * f(i, coord(e, g)) * f(j, coord(e, g))
                           for e in range(lo, hi) for g in range(p + 1)))
        if a == 1:                      # the conditions sum to zero: drop one
            rows, rhs = rows[:-1], rhs[:-1]
        A = mp.matrix(rows)
        y = mp.lu_solve(A * A.T, mp.matrix(rhs))
        return np.array([float(v) for v in A.T * y])


@pytest.mark.parametrize("p", [2, 4, 5, 6])
def test_wq_weights_match_high_precision(p):
    """Every rule of a 16-element direction that is not a plain Gauss rule (boundary,
    near-boundary and translation-invariant interior functions)."""
    line = Line(16, p)
    for i in range(line.n):
        sa, sb = support(line.tk, p, i)
        if all(e in line.full_gauss_elems for e in range(sa, sb)):
            continue
        for a in (0, 1):
            Q, w = wq_rule(line, line.tk, line.X, line.full_gauss_elems, i, a)
            ref = reference_rule(line.nel, p, line.tk, Q, i, a)
            err = np.abs(w - ref).max() / np.abs(ref).max()
            assert err <= 1e-13, (p, i, a, err)


@pytest.mark.parametrize("p", [5, 6])
def test_refined_rule_matches_high_precision(p):
    """A refined-space rule of a DWQ construction (break at knot s raised to multiplicity
    p+1, full Gauss points in the element above it) against the same reference."""
    line = Line(16, p)
    s = 8
    tkr = insert_knot_int(line.tk, s, p)
    full = set(line.full_gauss_elems) | {s}
    pts = sorted(set(line.X) | {(s, g) for g in range(p + 1)}, key=lambda eg: (eg[0], line.gxi[eg[1]]))
    # refined functions on the high side whose support holds more than the element s
    ks = [k for k in range(len(tkr) - p - 1) if support(tkr, p, k)[0] >= s and support(tkr, p, k)[1] - support(tkr, p, k)[0] > 1]
    for k in ks[:3]:
        for a in (0, 1):
            Q, w = wq_rule(line, tkr, pts, full, k, a)
            ref = reference_rule(line.nel, p, tkr, Q, k, a)
            err = np.abs(w - ref).max() / np.abs(ref).max()
            assert err <= 1e-13, (p, k, a, err)
