"""L2 projection with extended B-splines on a cut background mesh (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 3.1 forms the mass matrix of the active functions on the fictitious domain and
projects a target function f onto the spline space; extended B-splines keep the system
well conditioned; the relative L2 error of the projection measures accuracy (Section
3.2).  Readings used here (the paper defers the details to the cited works):

  * Load vector: b_I = sum over the quadrature parts of row I (WQ / DWQ box, element Gauss
    remainder, octree cut cells) of W_I(q) f(x_q): the points and test weights of the mass
    row, with f in place of the coefficient and no trial function.
  * Inner functions: active functions whose support contains at least one interior
    element; the other active functions are outer.
  * Extension (extended B-splines after Hoellig, in the form for open knot vectors): the
    root element of an outer function j is the interior element l nearest to it, measured
    between the element's centre l + 1/2 and the centre j - p/2 + 1/2 of the support of B_j
    in element units (so |l + p/2 - j|, Euclidean over the three directions), the first in
    lexicographic order on ties.  The functions supported on l, l + {0..p}^3, are all inner;
    they are B_j's array.  B_j enters the basis through them with the coefficients
    e_{i,j} = lambda_j(P_i), P_i the polynomial piece of B_i on the root element and lambda_j
    the dual functional of B_j (the B-spline coefficient of a polynomial w.r.t. B_j).  These
    reproduce every polynomial of degree p in each variable: a polynomial's coefficients on
    outer functions follow from those on inner ones.  On uniform knots they are Lagrange
    extrapolation weights in the index, prod_d L_{i_d - l_d}(j_d - l_d).  The extended basis is
    B_i + sum_j e_{i,j} B_j over the outer j that use inner i; E (active x inner) maps its
    coefficients to the active coefficients.
  * System: E^T M E c = E^T b with M the mass matrix (kappa = 1); u = E c.
  * Error: ||u_h - f||^2 and ||f||^2 over Omega with the (p+1)^3 Gauss rule on interior
    elements and the octree points on cut elements (the points of the conventional
    assembly).
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from functools import lru_cache

import numpy as np

from .domain import CUT, IN, OUT
from .spline import bspline


def _knots(nel: int, p: int):
    """Open uniform knots in element units (integers)."""
    return [min(max(k - p, 0), nel) for k in range(nel + 2 * p + 1)]


@lru_cache(maxsize=None)
def _piece(nel: int, p: int, i: int, s: int):
    """Coefficients (ascending powers of x, exact fractions) of the polynomial that equals
    B_i on the knot span [t_s, t_{s+1}], element units: the Cox-de Boor recursion carried out
    on polynomials, 0/0 terms dropped."""
    t = _knots(nel, p)

    def rec(i, k):
        if k == 0:
            return [Fraction(1 if i == s else 0)]
        out = [Fraction(0)] * (k + 1)
        d1 = t[i + k] - t[i]
        if d1 != 0:                                   # (x - t_i) / d1 * B_{i,k-1}
            for n, c in enumerate(rec(i, k - 1)):
                out[n + 1] += c / d1
                out[n] -= c * t[i] / d1
        d2 = t[i + k + 1] - t[i + 1]
        if d2 != 0:                                   # (t_{i+k+1} - x) / d2 * B_{i+1,k-1}
            for n, c in enumerate(rec(i + 1, k - 1)):
                out[n] += c * t[i + k + 1] / d2
                out[n + 1] -= c / d2
        return out

    return tuple(rec(i, p))


def _poly_at(c, x):
    v = Fraction(0)
    for a in reversed(c):
        v = v * x + a
    return v


def _solve_exact(A, b):
    """Gaussian elimination over fractions (A regular)."""
    n = len(b)
    M = [list(A[r]) + [b[r]] for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [a - f * c for a, c in zip(M[r], M[col])]
    return [M[r][n] / M[r][r] for r in range(n)]


@lru_cache(maxsize=None)
def _dual(nel: int, p: int, l: int, m: int, j: int) -> float:
    P = _piece(nel, p, m, l + p)                      # element l is the span [t_{l+p}, t_{l+p+1}]
    e = max(j - p, 0)                                 # an element in the support of B_j
    xs = [e + Fraction(r + 1, p + 2) for r in range(p + 1)]
    A = [[_poly_at(_piece(nel, p, e + k, e + p), x) for k in range(p + 1)] for x in xs]
    sol = _solve_exact(A, [_poly_at(P, x) for x in xs])
    return float(sol[j - e])


def dual_coefficient(line, l: int, m: int, j: int) -> float:
    """lambda_j(P): the coefficient of B_j in the B-spline expansion of P, the polynomial that
    equals B_m on element l.  On an element e in the support of B_j only B_e..B_{e+p} are
    nonzero, so the coefficient follows from interpolating P at p+1 points of e; everything is
    exact rational arithmetic in element units (B-spline coefficients do not change under an
    affine change of the parameter)."""
    return _dual(line.nel, line.p, int(l), int(m), int(j))


class Projection:
    """Load vector, extension operator, projection and error for one Problem."""

    def __init__(self, problem):
        self.P = problem
        self.dom = problem.dom
        self.p = problem.p

    # --- load vector ----------------------------------------------------------------------
    def load_vector(self, f_fn, share=(0, 1), rows=None) -> np.ndarray:
        """b (n_active); share = (k, n): only every n-th row from the k-th; rows: only these
        active rows (the other entries stay zero)."""
        dom = self.dom
        b = np.zeros(dom.n_active)
        todo = range(dom.n_active) if rows is None else sorted(set(int(r) for r in rows))
        for c, r in enumerate(todo):
            if c % share[1] != share[0]:
                continue
            I = dom.unlex(dom.active_lex[r])
            for part in self.P.row_parts(I):
                if part["xyz"].shape[0]:
                    b[r] += float(np.sum(part["wM"] * f_fn(part["xyz"])))
        return b

    # --- extension ------------------------------------------------------------------------
    def inner_mask(self) -> np.ndarray:
        """(n_active,) True for inner functions."""
        dom = self.dom
        out = np.zeros(dom.n_active, dtype=bool)
        for r, k in enumerate(dom.active_lex):
            I = dom.unlex(k)
            out[r] = bool(np.any(dom.ecls[dom.support_slices(I)] == IN))
        return out

    def arrays(self):
        """{outer active index: root element l (3-tuple)}."""
        dom, p = self.dom, self.p
        inner = self.inner_mask()
        cand = np.argwhere(dom.ecls == IN)                  # lexicographic order
        if len(cand) == 0 and not inner.all():
            raise ValueError("no interior element: the mesh is too coarse for the extension")
        out = {}
        for r, k in enumerate(dom.active_lex):
            if inner[r]:
                continue
            j = np.array(dom.unlex(k))
            d2 = np.sum((2 * cand + p - 2 * j) ** 2, axis=1)   # 4 |l + p/2 - j|^2, exact
            out[r] = tuple(int(v) for v in cand[int(np.argmin(d2))])
        return out

    def extension(self) -> np.ndarray:
        """E (n_active x n_inner), dense."""
        dom, p = self.dom, self.p
        inner = self.inner_mask()
        inner_idx = -np.ones(dom.n_active, dtype=np.int64)
        inner_idx[inner] = np.arange(int(inner.sum()))
        lex2act = dom.lex_to_active
        E = np.zeros((dom.n_active, int(inner.sum())))
        E[np.nonzero(inner)[0], inner_idx[inner]] = 1.0
        lines = self.P.lines
        for r, l in self.arrays().items():
            j = dom.unlex(dom.active_lex[r])
            lam = [[dual_coefficient(lines[d], l[d], l[d] + a, j[d]) for a in range(p + 1)] for d in range(3)]
            for a in itertools.product(range(p + 1), repeat=3):
                i = tuple(l[d] + a[d] for d in range(3))
                ri = lex2act[dom.lex(i)]
                E[r, inner_idx[ri]] += lam[0][a[0]] * lam[1][a[1]] * lam[2][a[2]]
        return E

    # --- projection -----------------------------------------------------------------------
    def dense_mass(self, M_vals) -> np.ndarray:
        rp = self.P.row_ptr()
        cols = self.P.csr_cols()
        n = self.dom.n_active
        A = np.zeros((n, n))
        for r in range(n):
            A[r, cols[rp[r]:rp[r + 1]]] = M_vals[rp[r]:rp[r + 1]]
        return A

    def solve(self, M_vals, b) -> np.ndarray:
        """u = E c with E^T M E c = E^T b (dense direct solve)."""
        E = self.extension()
        A = E.T @ self.dense_mass(M_vals) @ E
        c = np.linalg.solve(A, E.T @ b)
        return E @ c

    # --- error ----------------------------------------------------------------------------
    def l2_error(self, u, f_fn):
        """(sum w (u_h - f)^2, sum w f^2) over interior elements (Gauss) and cut elements (octree)."""
        dom, p = self.dom, self.p
        lines = self.P.lines
        sl = self.P.slots(with_octree=False)
        coef = np.zeros(dom.nfun)
        for r, k in enumerate(dom.active_lex):
            coef[dom.unlex(k)] = u[r]
        err2 = 0.0
        fn2 = 0.0
        for e in itertools.product(*map(range, dom.nel)):
            if dom.ecls[e] == IN:
                x, w = self.P._element_gauss_points(e)
            elif dom.ecls[e] == CUT:
                x, w = sl.octree(e)
            else:
                continue
            if len(w) == 0:
                continue
            B = [np.array([bspline(lines[d].knot_coord(lines[d].tk), p, e[d] + a, x[:, d]) for a in range(p + 1)])
                 for d in range(3)]
            c = coef[e[0]:e[0] + p + 1, e[1]:e[1] + p + 1, e[2]:e[2] + p + 1]
            uh = np.einsum("abc,ap,bp,cp->p", c, B[0], B[1], B[2])
            fv = f_fn(x)
            err2 += float(np.sum(w * (uh - fv) ** 2))
            fn2 += float(np.sum(w * fv ** 2))
        return err2, fn2
