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
  * Extension (after Hoellig's weighted extended B-splines): for an outer index j the array
    l + {0..p}^3 of inner indices whose centre l + p/2 is closest to j in the Euclidean
    norm, the first such l in lexicographic order on ties; the outer function enters the
    basis through the inner functions of its array with the coefficients
    e_{i,j} = prod_d L_{i_d - l_d}(j_d - l_d), L_a the Lagrange polynomials on the nodes
    0..p (they reproduce polynomials of degree p in the index).  The extended basis is
    B_i + sum_j e_{i,j} B_j over the outer j that use inner i; E (active x inner) maps
    its coefficients to the active coefficients.
  * System: E^T M E c = E^T b with M the mass matrix (kappa = 1); u = E c.
  * Error: ||u_h - f||^2 and ||f||^2 over Omega with the (p+1)^3 Gauss rule on interior
    elements and the octree points on cut elements (the points of the conventional
    assembly).
"""
from __future__ import annotations

import itertools

import numpy as np

from .domain import CUT, IN, OUT
from .spline import bspline


def lagrange_weights(p: int, x: float) -> np.ndarray:
    """L_a(x), a = 0..p, Lagrange polynomials on the integer nodes 0..p."""
    out = np.ones(p + 1)
    for a in range(p + 1):
        for m in range(p + 1):
            if m != a:
                out[a] *= (x - m) / (a - m)
    return out


class Projection:
    """Load vector, extension operator, projection and error for one Problem."""

    def __init__(self, problem):
        self.P = problem
        self.dom = problem.dom
        self.p = problem.p

    # --- load vector ----------------------------------------------------------------------
    def load_vector(self, f_fn, share=(0, 1)) -> np.ndarray:
        """b (n_active); share = (k, n): only every n-th row from the k-th (the rest zero)."""
        dom = self.dom
        b = np.zeros(dom.n_active)
        for r, k in enumerate(dom.active_lex):
            if r % share[1] != share[0]:
                continue
            I = dom.unlex(k)
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
        """{outer active index: base l (3-tuple)} of the extension arrays."""
        dom, p = self.dom, self.p
        nf = dom.nfun
        inner = self.inner_mask()
        ind = np.zeros(nf, dtype=np.int64)
        for r, k in enumerate(dom.active_lex):
            if inner[r]:
                ind[dom.unlex(k)] = 1
        # blocks l + {0..p}^3 that are all inner: box sums of the indicator
        S = np.zeros(tuple(n + 1 for n in nf), dtype=np.int64)
        S[1:, 1:, 1:] = ind.cumsum(0).cumsum(1).cumsum(2)
        L = [np.arange(n - p) for n in nf]
        l0, l1, l2 = np.meshgrid(*L, indexing="ij")
        tot = np.zeros(l0.shape, dtype=np.int64)
        for bits in itertools.product((0, 1), repeat=3):
            idx = tuple((l + (p + 1) * bt) for l, bt in zip((l0, l1, l2), bits))
            tot += (-1) ** (3 - sum(bits)) * S[idx]
        cand = np.argwhere(tot == (p + 1) ** 3)           # lexicographic order
        if len(cand) == 0:
            raise ValueError("no array of inner functions: the mesh is too coarse for the extension")
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
        for r, l in self.arrays().items():
            j = dom.unlex(dom.active_lex[r])
            lam = [lagrange_weights(p, j[d] - l[d]) for d in range(3)]
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
