"""Pins of the oracle's univariate layer: Gauss rules, B-splines, WQ and DWQ rules.

Each check compares the oracle against something fixed outside it: closed forms
(truncated-power cardinal B-splines, hat functions, the p=1 stencils), polynomial
exactness, symmetry of the construction, or an independent higher-order quadrature.
"""
import math

import numpy as np
import pytest

from oracle.spline import (Line, Rules1D, bspline, bspline_all, dwq_rule, gauss_legendre,
                           insert_knot_int, subdivision_row, support)


def cardinal_deriv(m, x, r):
    """r-th derivative of the cardinal B-spline of degree m (truncated powers)."""
    x = np.asarray(x, dtype=np.float64)
    deg = m - r
    out = np.zeros_like(x)
    for k in range(m + 2):
        out += (-1) ** k * math.comb(m + 1, k) * np.where(x - k > 0, (x - k) ** deg, 0.0)
    return out / math.factorial(deg)


def fine_gram(line, tk, i, j, a, npts=10):
    """int B_i^(a) B_j^(a) with an npts-point Gauss rule per element (independent order)."""
    return fine_gram_matrix(line, tk, a, npts)[i, j]


_FG = {}


def fine_gram_matrix(line, tk, a, npts=10):
    key = (line.nel, line.p, tuple(tk), a, npts)
    if key not in _FG:
        xi, w = gauss_legendre(npts)
        t = line.knot_coord(tk)
        x = np.concatenate([line.lo + (e + (1 + xi) / 2) * line.h for e in range(line.nel)])
        wx = np.tile(w * line.h / 2, line.nel)
        B = np.array([bspline(t, line.p, i, x, a) for i in range(len(tk) - line.p - 1)])
        _FG[key] = (B * wx) @ B.T
    return _FG[key]


def wq_matrix(line, rules, a):
    """A[i, j] = sum_q w^(aa)_{i,q} B_j^(a)(x_q) (kappa = 1)."""
    t = line.knot_coord(line.tk)
    A = np.zeros((line.n, line.n))
    for i in range(line.n):
        Q, w = rules.rule[a][i]
        xq = line.coord(Q)
        for j in range(line.n):
            A[i, j] = np.sum(w * bspline(t, line.p, j, xq, a))
    return A


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("n", range(1, 9))
def test_gauss_exact_degree(n):
    xi, w = gauss_legendre(n)
    for k in range(2 * n):
        exact = 2.0 / (k + 1) if k % 2 == 0 else 0.0
        assert abs(np.sum(w * xi ** k) - exact) < 1e-14
    # degree 2n is not integrated exactly (the rule really has n points)
    assert abs(np.sum(w * xi ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def test_gauss_closed_form_nodes():
    xi, w = gauss_legendre(2)
    assert np.allclose(xi, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    xi, w = gauss_legendre(3)
    assert np.allclose(xi, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)


@pytest.mark.parametrize("p", range(1, 7))
def test_basis_cardinal_interior(p):
    line = Line(3 * p + 3, p)
    t = line.knot_coord(line.tk)
    x = np.random.default_rng(p).uniform(0, 1, 400)
    for j in range(p, line.n - p):
        y = (x - line.lo) / line.h - (j - p)
        ins = (y > 0) & (y < p + 1)
        assert np.all(bspline(t, p, j, x[~ins]) == 0.0)
        assert np.allclose(bspline(t, p, j, x[ins]), cardinal_deriv(p, y[ins], 0), rtol=0, atol=1e-12)
        assert np.allclose(bspline(t, p, j, x[ins], 1), cardinal_deriv(p, y[ins], 1) / line.h,
                           rtol=0, atol=1e-11 / line.h)


@pytest.mark.parametrize("p", range(1, 7))
def test_basis_partition_and_vectorised(p):
    line = Line(7, p)
    t = line.knot_coord(line.tk)
    x = np.concatenate([np.random.default_rng(0).uniform(0, 1, 300), [0.0, 1.0]])
    B, dB = bspline_all(t, p, x)
    assert np.allclose(B.sum(0), 1.0, atol=1e-14)
    assert np.allclose(dB.sum(0), 0.0, atol=1e-10)
    assert np.all(B >= -1e-15)
    for i in range(line.n):
        assert np.array_equal(B[i], bspline(t, p, i, x))


def test_basis_boundary_closed_forms():
    h = 1 / 5
    line = Line(5, 1)
    t = line.knot_coord(line.tk)
    x = np.linspace(0, h, 7)[:-1]
    assert np.allclose(bspline(t, 1, 0, x), 1 - x / h, atol=1e-15)
    line = Line(5, 2)
    t = line.knot_coord(line.tk)
    assert np.allclose(bspline(t, 2, 0, x), (1 - x / h) ** 2, atol=1e-15)
    assert np.allclose(bspline(t, 2, 0, x, 1), -2 * (1 - x / h) / h, atol=1e-12)
    assert bspline(t, 2, line.n - 1, np.array([1.0]))[0] == 1.0


def test_basis_derivative_vs_difference():
    line = Line(6, 4)
    t = line.knot_coord(line.tk)
    x = np.random.default_rng(3).uniform(0.01, 0.99, 50)
    eps = 1e-6
    for i in range(line.n):
        fd = (bspline(t, 4, i, x + eps) - bspline(t, 4, i, x - eps)) / (2 * eps)
        assert np.allclose(bspline(t, 4, i, x, 1), fd, atol=1e-6)


# ------------------------------------------------------------------------------------------
def test_p1_closed_forms():
    """1D p=1: mass h/6 [1 4 1], boundary h/6 [2 1]; stiffness (1/h)[-1 2 -1], boundary (1/h)[1 -1]."""
    line = Line(8, 1)
    r = Rules1D(line)
    M = wq_matrix(line, r, 0)
    K = wq_matrix(line, r, 1)
    h = line.h
    for i in range(1, line.n - 1):
        assert np.allclose(M[i, i - 1:i + 2], h / 6 * np.array([1, 4, 1]), atol=1e-15)
        assert np.allclose(K[i, i - 1:i + 2], np.array([-1, 2, -1]) / h, atol=1e-12)
    assert np.allclose(M[0, :2], h / 6 * np.array([2, 1]), atol=1e-15)
    assert np.allclose(K[0, :2], np.array([1, -1]) / h, atol=1e-12)
    assert np.allclose(M[-1, -2:], h / 6 * np.array([1, 2]), atol=1e-15)


@pytest.mark.parametrize("p", range(2, 7))
def test_interior_stencils_cardinal(p):
    """Interior mass row = h N_{2p+1}(p+1+k), stiffness row = -N''_{2p+1}(p+1+k)/h."""
    line = Line(4 * p + 4, p)
    r = Rules1D(line)
    M = wq_matrix(line, r, 0)
    K = wq_matrix(line, r, 1)
    k = np.arange(-p, p + 1)
    ms = line.h * cardinal_deriv(2 * p + 1, p + 1 + k, 0)
    ks = -cardinal_deriv(2 * p + 1, p + 1 + k, 2) / line.h
    for i in range(2 * p, line.n - 2 * p):
        assert np.allclose(M[i, i - p:i + p + 1], ms, rtol=1e-12, atol=1e-16)
        assert np.allclose(K[i, i - p:i + p + 1], ks, rtol=1e-11, atol=1e-11 * np.abs(ks).max())
    if p == 2:
        assert np.allclose(ms / line.h, np.array([1, 26, 66, 26, 1]) / 120, atol=1e-15)


@pytest.mark.parametrize("p", range(1, 7))
def test_wq_exact_all_rows(p):
    """Every rule (boundary rows too) integrates B_i^(a) B_j^(a) exactly (10-point reference)."""
    line = Line(2 * p + 5, p)
    r = Rules1D(line)
    for a in (0, 1):
        A = wq_matrix(line, r, a)
        G = fine_gram_matrix(line, line.tk, a)
        assert np.abs(A - G).max() <= 1e-13 * np.abs(G).max()


@pytest.mark.parametrize("p", range(1, 7))
def test_wq_layout_and_structure(p):
    nel = 4 * p + 4
    line = Line(nel, p)
    r = Rules1D(line)
    assert len(line.X) == (2 * nel + 2 * p - 2 if p > 1 else 2 * nel)
    # every WQ point is a Gauss point of its element
    for (e, g) in line.X:
        assert 0 <= g <= p
    t = line.knot_coord(line.tk)
    for a in (0, 1):
        for i in range(line.n):
            Q, w = r.rule[a][i]
            sa, sb = support(line.tk, p, i)
            assert all(sa <= e < sb for (e, _) in Q)
            # mirror symmetry
            Qm, wm = r.rule[a][line.n - 1 - i]
            assert len(Qm) == len(Q)
            # mirror x -> 1-x: B_j^(a) picks up (-1)^a, so the weights do too
            assert np.allclose(wm[::-1], (-1) ** a * w, atol=1e-13 * np.abs(w).max())
            if all(e in line.full_gauss_elems for e in range(sa, sb)):
                # Gauss weights used directly
                xq = line.coord(Q)
                om = np.array([line.gauss_weight(g) for (_, g) in Q])
                assert np.allclose(w, om * bspline(t, p, i, xq, a), atol=1e-15)
            else:
                # minimum norm: w lies in the row space of the exactness system
                J = [j for j in range(line.n) if max(sa, support(line.tk, p, j)[0]) < min(sb, support(line.tk, p, j)[1])]
                A = np.array([bspline(t, p, j, line.coord(Q), a) for j in J])
                y = np.linalg.lstsq(A.T, w, rcond=None)[0]
                assert np.linalg.norm(A.T @ y - w) <= 1e-10 * np.linalg.norm(w)
        # translation invariance of interior rules
        ref = r.rule[a][2 * p][1]
        for i in range(2 * p, line.n - 2 * p):
            assert np.allclose(r.rule[a][i][1], ref, rtol=0, atol=1e-11 * np.abs(ref).max())
    if p == 1:
        assert line.full_gauss_elems == set(range(nel))


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("p", range(1, 6))
def test_subdivision_identity(p):
    line = Line(3 * p + 3, p)
    s = line.nel // 2
    tkr = insert_knot_int(line.tk, s, p)
    assert np.sum(tkr == s) == p + 1
    t, tr = line.knot_coord(line.tk), line.knot_coord(tkr)
    x = np.random.default_rng(p).uniform(0, 1, 200)
    nref = len(tkr) - p - 1
    for i in range(line.n):
        S = subdivision_row(line, line.tk, tkr, i)
        rec = sum(S[k] * bspline(tr, p, k, x) for k in range(nref))
        assert np.allclose(rec, bspline(t, p, i, x), atol=1e-13)


@pytest.mark.parametrize("p", range(1, 7))
def test_dwq_one_sided_exactness(p):
    """The DWQ rule integrates B_i^(a) B_j^(a) over its side only; both sides sum to the whole."""
    line = Line(3 * p + 3, p)
    t = line.knot_coord(line.tk)
    xi, wg = gauss_legendre(10)
    i = line.n // 2
    sa, sb = support(line.tk, p, i)
    for s in range(sa + 1, sb):
        for a in (0, 1):
            tot = {}
            for high in (True, False):
                Q, w = dwq_rule(line, i, s, high, a)
                side = range(s, sb) if high else range(sa, s)
                assert all(e in side for (e, _) in Q)
                estar = s if high else s - 1
                assert {(estar, g) for g in range(p + 1)} <= set(Q)
                xq = line.coord(Q)
                for j in range(line.n):
                    ref = 0.0
                    for e in side:
                        x = line.lo + (e + (1 + xi) / 2) * line.h
                        ref += np.sum(wg * line.h / 2 * bspline(t, p, i, x, a) * bspline(t, p, j, x, a))
                    got = np.sum(w * bspline(t, p, j, xq, a))
                    scale = abs(fine_gram(line, line.tk, i, i, a))
                    assert abs(got - ref) <= 1e-12 * scale
                    tot[j] = tot.get(j, 0.0) + got
            for j in range(line.n):
                assert abs(tot[j] - fine_gram(line, line.tk, i, j, a)) <= 1e-12 * abs(fine_gram(line, line.tk, i, i, a))


# smallest positive Gauss-Legendre node of order p+1 (tabulated values, 6 digits)
ZETA = {2: 0.774597, 3: 0.339981, 4: 0.538469, 5: 0.238619, 6: 0.405845}


@pytest.mark.parametrize("p", range(2, 7))
def test_kept_pair_is_nearest_midpoint_pair(p):
    """Reading of the point layout (Section 2.2, layout paragraph): an element that is
    neither the first nor the last of its direction keeps the Gauss pair +-zeta_p around
    its midpoint, zeta_p the smallest positive node of the (p+1)-point rule; the boundary
    elements keep all p+1 points."""
    line = Line(6, p)
    for e in range(1, line.nel - 1):
        xi = np.array([line.gxi[g] for g in line.kept[e]])
        assert np.allclose(xi, [-ZETA[p], ZETA[p]], rtol=0, atol=1e-6)
        x = line.coord([(e, g) for g in line.kept[e]])
        mid = line.lo + (e + 0.5) * line.h
        assert np.allclose(x, [mid - ZETA[p] * line.h / 2, mid + ZETA[p] * line.h / 2], rtol=0, atol=1e-6 * line.h)
    for e in (0, line.nel - 1):
        assert line.kept[e] == list(range(p + 1))
