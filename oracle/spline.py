"""Univariate B-splines, Gauss rules and the weighted-quadrature point layout (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Basis (Section 1 and Section 2 opening paragraph): degree p, maximal smoothness
C^{p-1}, open knot vectors, identity map.  Knots are kept as integers counting
element boundaries (0..nel), so supports and splits are exact integer ranges; the
coordinate of knot k is lo + k*h.

Point layout (Section 2.2, paragraph after Fig. 3: WQ points are picked among the
element Gauss points).  Reading used here: the two boundary elements of each
direction, and every element when p = 1, keep all p+1 Gauss points; every other
element keeps the symmetric pair of Gauss points closest to the element midpoint
(excluding a node at the midpoint).  With two points per interior element each
maximally smooth test function has 2p+2 points for its 2p+1 exactness conditions.
"""
from __future__ import annotations

import numpy as np


def gauss_legendre(npts: int):
    """Gauss-Legendre nodes (ascending) and weights on [-1, 1] (library routine)."""
    xi, w = np.polynomial.legendre.leggauss(npts)
    return np.asarray(xi, dtype=np.float64), np.asarray(w, dtype=np.float64)


def open_knots_int(nel: int, p: int) -> np.ndarray:
    """Open uniform knot vector in element-boundary units: 0 (p+1 times), 1..nel-1, nel (p+1 times)."""
    return np.array([0] * (p + 1) + list(range(1, nel)) + [nel] * (p + 1), dtype=np.int64)


def insert_knot_int(tk: np.ndarray, s: int, p: int) -> np.ndarray:
    """Raise the multiplicity of interior knot s to p+1 (a C^-1 break, Section 2.2 step 3)."""
    mult = int(np.sum(tk == s))
    assert mult >= 1
    pos = int(np.searchsorted(tk, s, side="right"))
    return np.concatenate([tk[:pos], np.full(p + 1 - mult, s, dtype=np.int64), tk[pos:]])


class Line:
    """One parametric direction: nel uniform elements on [lo, hi], degree p."""

    def __init__(self, nel: int, p: int, lo: float = 0.0, hi: float = 1.0):
        self.nel, self.p, self.lo, self.hi = int(nel), int(p), float(lo), float(hi)
        self.h = (self.hi - self.lo) / self.nel
        self.tk = open_knots_int(self.nel, self.p)
        self.n = self.nel + self.p
        self.gxi, self.gw = gauss_legendre(self.p + 1)
        # WQ layout: Gauss indices kept per element
        self.kept = [self._kept(e) for e in range(self.nel)]
        self.full_gauss_elems = {e for e in range(self.nel) if len(self.kept[e]) == self.p + 1}
        # global WQ point list X as (element, gauss index), ascending in coordinate
        self.X = [(e, g) for e in range(self.nel) for g in self.kept[e]]
        self.xidx = {eg: k for k, eg in enumerate(self.X)}

    # --- geometry -----------------------------------------------------------------
    def knot_coord(self, k):
        return self.lo + np.asarray(k, dtype=np.float64) * self.h

    def gauss_coord(self, e: int, g):
        return self.lo + (e + (1.0 + self.gxi[g]) / 2.0) * self.h

    def gauss_weight(self, g):
        return self.gw[g] * self.h / 2.0

    def coord(self, pts):
        return np.array([self.gauss_coord(e, g) for (e, g) in pts], dtype=np.float64)

    def _kept(self, e: int):
        p = self.p
        if e == 0 or e == self.nel - 1 or p == 1:
            return list(range(p + 1))
        pos = [g for g in range(p + 1) if self.gxi[g] > 1e-14]
        gz = min(pos, key=lambda g: self.gxi[g])
        return sorted([p - gz, gz])          # the node and its mirror image

    @property
    def Xcoord(self):
        return self.coord(self.X)


# ----------------------------------------------------------------------------------------
# Cox-de Boor
# ----------------------------------------------------------------------------------------
def _cdb(t: np.ndarray, i: int, k: int, x: np.ndarray) -> np.ndarray:
    """B_{i,k}(x) by the Cox-de Boor recursion; right-continuous, right end included."""
    if k == 0:
        r = ((t[i] <= x) & (x < t[i + 1])).astype(np.float64)
        if t[i] < t[i + 1] and t[i + 1] == t[-1]:
            r[x == t[-1]] = 1.0
        return r
    out = np.zeros_like(x, dtype=np.float64)
    if t[i + k] != t[i]:
        out = out + (x - t[i]) / (t[i + k] - t[i]) * _cdb(t, i, k - 1, x)
    if t[i + k + 1] != t[i + 1]:
        out = out + (t[i + k + 1] - x) / (t[i + k + 1] - t[i + 1]) * _cdb(t, i + 1, k - 1, x)
    return out


def bspline(t: np.ndarray, p: int, i: int, x, deriv: int = 0) -> np.ndarray:
    """B_i (deriv=0) or B_i' (deriv=1) of degree p over float knots t at points x."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    if deriv == 0:
        return _cdb(t, i, p, x)
    assert deriv == 1 and p >= 1
    out = np.zeros_like(x)
    if t[i + p] != t[i]:
        out += p / (t[i + p] - t[i]) * _cdb(t, i, p - 1, x)
    if t[i + p + 1] != t[i + 1]:
        out -= p / (t[i + p + 1] - t[i + 1]) * _cdb(t, i + 1, p - 1, x)
    return out


def bspline_all(t: np.ndarray, p: int, x):
    """All B_j and B_j' (j = 0..len(t)-p-2) at points x: two arrays (nfun, len(x)).

    The same Cox-de Boor recursion as bspline(), evaluated degree by degree for every
    function at once (0/0 terms dropped)."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(t) - 1
    N = ((t[:m, None] <= x[None, :]) & (x[None, :] < t[1:, None])).astype(np.float64)
    last = np.nonzero(t[:m] < t[1:])[0][-1]
    N[last, x == t[-1]] = 1.0

    def ratio(num, den):
        out = np.zeros_like(num)
        ok = den != 0.0
        out[ok] = num[ok] / np.broadcast_to(den, num.shape)[ok]
        return out

    prev = None
    for k in range(1, p + 1):
        j = np.arange(m - k)
        left = ratio(x[None, :] - t[j, None], (t[j + k] - t[j])[:, None] + 0 * x[None, :]) * N[j]
        right = ratio(t[j + k + 1, None] - x[None, :], (t[j + k + 1] - t[j + 1])[:, None] + 0 * x[None, :]) * N[j + 1]
        prev = N
        N = left + right
    nf = len(t) - p - 1
    j = np.arange(nf)
    dl = np.where(t[j + p] != t[j], p / np.where(t[j + p] != t[j], t[j + p] - t[j], 1.0), 0.0)
    dr = np.where(t[j + p + 1] != t[j + 1], p / np.where(t[j + p + 1] != t[j + 1], t[j + p + 1] - t[j + 1], 1.0), 0.0)
    dN = dl[:, None] * prev[j] - dr[:, None] * prev[j + 1]
    return N[:nf], dN


def support(tk: np.ndarray, p: int, i: int):
    """Element range [a, b) (integers) of supp B_i."""
    return int(tk[i]), int(tk[i + p + 1])


# ----------------------------------------------------------------------------------------
# weighted quadrature (Section 1, WQ ingredient; Section 2.2 steps 1 and 5)
# ----------------------------------------------------------------------------------------
def exact_gram(line: Line, tk: np.ndarray, i: int, j: int, a: int) -> float:
    """int B_i^(a) B_j^(a) over the common support, by (p+1)-point Gauss per element (exact)."""
    return _gram(line, tk, i, a, lambda t, x: bspline(t, line.p, j, x, a), support(tk, line.p, j))


def _gram(line: Line, tk: np.ndarray, i: int, at: int, fn, sup) -> float:
    """int B_i^(at) fn over supp B_i intersected with sup (element range), (p+1)-point Gauss per
    element; exact when fn is a piecewise polynomial of degree <= p on the elements."""
    p = line.p
    t = line.knot_coord(tk)
    ai, bi = support(tk, p, i)
    s = 0.0
    g = np.arange(p + 1)
    for e in range(max(ai, sup[0]), min(bi, sup[1])):
        x = line.gauss_coord(e, g)
        s += float(np.sum(line.gauss_weight(g) * bspline(t, p, i, x, at) * fn(t, x)))
    return s


def rule_orders(a):
    """(test derivative order, trial derivative order) of a rule family: 0 = (0, 0) mass,
    1 = (1, 1) stiffness, (1, 0) and (0, 1) the mixed families of a full coefficient tensor."""
    return (a, a) if a in (0, 1) else (int(a[0]), int(a[1]))


def exactness_system(line: Line, tk: np.ndarray, i: int, a, xq: np.ndarray):
    """Exactness conditions of the rule of test function i at points xq: (A, b), one row
    per condition, A[c, q] = (condition function c)(x_q).  a: family (rule_orders), test
    derivative order at and trial derivative order ac.

    ac = 0: the conditions are sum_q w_q B_j(x_q) = int B_i^(at) B_j for every j whose support
    overlaps supp B_i in positive measure.
    ac = 1: the conditions sum_q w_q B_j'(x_q) = int B_i^(at) B_j' for those j span, on supp B_i,
    the same space as the degree p-1 B-splines N_k over the same knots that are nonzero
    there (each B_j' is a combination of N_j and N_{j+1}; the B_j' lose one dimension
    because they sum to zero on the support).  Imposing sum_q w_q N_k(x_q) = int B_i^(at) N_k
    for those k therefore gives the same set of admissible weights, with one condition
    per dimension instead of a redundant one."""
    p = line.p
    at, ac = rule_orders(a)
    t = line.knot_coord(tk)
    sa, sb = support(tk, p, i)
    if ac == 0:
        J = [j for j in range(len(tk) - p - 1)
             if max(sa, support(tk, p, j)[0]) < min(sb, support(tk, p, j)[1])]
        A = np.array([bspline(t, p, j, xq) for j in J])
        b = np.array([_gram(line, tk, i, at, lambda tt, x, j=j: bspline(tt, p, j, x), support(tk, p, j))
                      for j in J])
        return A, b
    K = [k for k in range(len(tk) - p) if tk[k] < tk[k + p] and max(sa, tk[k]) < min(sb, tk[k + p])]
    A = np.array([bspline(t, p - 1, k, xq) for k in K])
    b = np.array([_gram(line, tk, i, at, lambda tt, x, k=k: bspline(tt, p - 1, k, x), (int(tk[k]), int(tk[k + p])))
                  for k in K])
    return A, b


def wq_rule(line: Line, tk: np.ndarray, pts, full_gauss: set, i: int, a: int):
    """Weighted-quadrature rule of test function i (knots tk) for family a (rule_orders).

    pts: the global point list ((element, gauss index), ascending); full_gauss: the
    elements that keep all their Gauss points.  Returns (list of points, weights).

    Conditions: sum_q w_q B_j^(a)(x_q) = int B_i^(a) B_j^(a) for every j whose support
    overlaps supp B_i in a set of positive measure.  If every element of supp B_i
    keeps all Gauss points, the Gauss weights times B_i^(a) are used directly
    (Section 2.2, last paragraph).  Otherwise the rule is the minimum-Euclidean-norm
    solution of the (consistent, underdetermined) system after scaling each condition
    to unit norm (the solution does not depend on that scaling; it only removes the
    spread of the rows' magnitudes from the conditioning): with the QR factorization
    A^T = Q R (full row rank), w = Q R^-T b is the solution in the row space of A.  For
    a = 1 the conditions are posed on the derivative space's own B-splines
    (`exactness_system`), which fixes the same weights without the redundant condition.
    """
    p = line.p
    t = line.knot_coord(tk)
    sa, sb = support(tk, p, i)
    Q = [(e, g) for (e, g) in pts if sa <= e < sb]
    xq = line.coord(Q)
    if all(e in full_gauss for e in range(sa, sb)):
        wg = np.array([line.gauss_weight(g) for (_, g) in Q])
        return Q, wg * bspline(t, p, i, xq, rule_orders(a)[0])
    A, b = exactness_system(line, tk, i, a, xq)
    s = 1.0 / np.linalg.norm(A, axis=1)
    Qf, Rf = np.linalg.qr((A * s[:, None]).T)
    w = Qf @ np.linalg.solve(Rf.T, b * s)
    return Q, w


class Rules1D:
    """All standard WQ rules of one direction: rule[a][i] = (points, weights); the mixed
    families (1, 0) and (0, 1) on demand through family()."""

    def __init__(self, line: Line):
        self.line = line
        self.rule = [[wq_rule(line, line.tk, line.X, line.full_gauss_elems, i, a)
                      for i in range(line.n)] for a in (0, 1)]
        self._mixed = {}

    def family(self, a, i):
        if a in (0, 1):
            return self.rule[a][i]
        key = (rule_orders(a), i)
        if key not in self._mixed:
            self._mixed[key] = wq_rule(self.line, self.line.tk, self.line.X, self.line.full_gauss_elems, i, a)
        return self._mixed[key]


# ----------------------------------------------------------------------------------------
# discontinuous weighted quadrature (Section 2.2 steps 3-6)
# ----------------------------------------------------------------------------------------
def subdivision_row(line: Line, tk: np.ndarray, tkr: np.ndarray, i: int) -> np.ndarray:
    """Coefficients S_ik with B_i = sum_k S_ik Btilde_k (refined knots tkr).

    B_i lies in the refined space and only refined functions whose support lies in
    supp B_i take part, so least squares over those functions at p+2 points per
    element of supp B_i reproduces B_i exactly."""
    p = line.p
    t, tr = line.knot_coord(tk), line.knot_coord(tkr)
    sa, sb = support(tk, p, i)
    u = (np.arange(p + 2) + 0.5) / (p + 2)
    x = np.concatenate([line.lo + (e + u) * line.h for e in range(sa, sb)])
    nref = len(tkr) - p - 1
    inside = [k for k in range(nref) if sa <= support(tkr, p, k)[0] and support(tkr, p, k)[1] <= sb]
    A = np.array([bspline(tr, p, k, x) for k in inside]).T
    S = np.zeros(nref)
    S[inside] = np.linalg.lstsq(A, bspline(t, p, i, x), rcond=None)[0]
    return S


def dwq_rule(line: Line, i: int, s: int, high: bool, a: int):
    """One-sided DWQ rule of test function i with an artificial break at knot s.

    Step 3: insert s until it has multiplicity p+1 and keep S.  Step 4 (reading):
    the nested points are all Gauss points of the element next to the break on
    the kept side.  Step 5: WQ weights of every refined function on the kept side
    inside supp B_i.  Step 6: w = sum_k S_ik wtilde_k on the kept side; the other
    side gets no points (zero weights).  Returns (points, weights), points on the
    kept side only.
    """
    p = line.p
    tkr = insert_knot_int(line.tk, s, p)
    S = subdivision_row(line, line.tk, tkr, i)
    estar = s if high else s - 1
    full = set(line.full_gauss_elems) | {estar}
    pts = sorted(set(line.X) | {(estar, g) for g in range(p + 1)},
                 key=lambda eg: (eg[0], line.gxi[eg[1]]))
    sa, sb = support(line.tk, p, i)
    lo_side, hi_side = (s, sb) if high else (sa, s)
    acc = {}
    for k in range(len(tkr) - p - 1):
        ka, kb = support(tkr, p, k)
        if ka >= kb or not (lo_side <= ka and kb <= hi_side):
            continue
        Qk, wk = wq_rule(line, tkr, pts, full, k, a)
        for q, wq in zip(Qk, wk):
            acc[q] = acc.get(q, 0.0) + S[k] * wq
    Q = sorted(acc, key=lambda eg: (eg[0], line.gxi[eg[1]]))
    return Q, np.array([acc[q] for q in Q])
