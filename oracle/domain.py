"""Function types, DWQ split search, octree cut integration and slot layout (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings used (the paper leaves these open):
  * Box test (Section 2.1 defines the types through the overlap of a support with
    the closed domain, in measure): a box is interior if max phi <= 0 on it,
    exterior if min phi >= 0, cut otherwise.  Plane and ball use the exact box
    extrema; the torus uses the conservative 1-Lipschitz test
    |phi(centre)| >= half-diagonal.
  * Function I is exterior if all elements of its support are exterior, interior
    if all are interior, cut otherwise (Section 2.1).  Active = not exterior,
    numbered lexicographically (first index slowest).  Row I's pattern holds every
    active J with max_d |I_d - J_d| <= p, ascending.
  * Split (Section 2.2 step 2 and the 3D paragraph after Fig. 3): candidates are a
    direction d, an interior knot s of supp B_I in d and a side; the candidate box
    is supp B_I with direction d restricted to the chosen side.  It is valid when
    every element in it is interior; the valid box with most elements wins, the
    first strict maximum in the order d ascending, s ascending, high side before low.
  * Cut elements (stand-in for the sub-element scheme the paper cites, Section
    2.2 first paragraph): recursive 2x2x2 bisection to depth L; interior cells at
    any depth and cut cells at depth L carry a (p+1)^3 Gauss rule, the latter with
    weight 0 at points where phi >= 0; exterior cells are dropped.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .spline import gauss_legendre

OUT, IN, CUT = 0, 1, 2


# ----------------------------------------------------------------------------------------
# level set
# ----------------------------------------------------------------------------------------
def phi(ls, x: np.ndarray) -> np.ndarray:
    """Signed distance-type level set at points x (N,3); Omega = {phi < 0}."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    if ls.kind == 0:
        return -np.ones(len(x))
    if ls.kind == 1:
        n = np.asarray(ls.n, dtype=np.float64)
        return (x @ n - ls.r0) / np.linalg.norm(n)
    c = np.asarray(ls.c, dtype=np.float64)
    if ls.kind == 2:
        return np.linalg.norm(x - c, axis=1) - ls.r0
    if ls.kind == 3:
        rho = np.hypot(x[:, 0] - c[0], x[:, 1] - c[1])
        return np.hypot(rho - ls.r0, x[:, 2] - c[2]) - ls.r1
    raise ValueError(ls.kind)


def classify_box(ls, lo, hi) -> int:
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    if ls.kind == 0:
        return IN
    if ls.kind == 1:
        corners = np.array(list(itertools.product(*zip(lo, hi))))
        v = phi(ls, corners)
        vmin, vmax = v.min(), v.max()
    elif ls.kind == 2:
        c = np.asarray(ls.c, dtype=np.float64)
        near = np.clip(c, lo, hi)
        far = np.where(np.abs(lo - c) > np.abs(hi - c), lo, hi)
        vmin = float(np.linalg.norm(near - c)) - ls.r0
        vmax = float(np.linalg.norm(far - c)) - ls.r0
    elif ls.kind == 3:
        mid = 0.5 * (lo + hi)
        hd = 0.5 * float(np.linalg.norm(hi - lo))
        v = float(phi(ls, mid[None])[0])
        vmin, vmax = v - hd, v + hd
    else:
        raise ValueError(ls.kind)
    if vmax <= 0.0:
        return IN
    if vmin >= 0.0:
        return OUT
    return CUT


# ----------------------------------------------------------------------------------------
# mesh-level classification
# ----------------------------------------------------------------------------------------
class Domain:
    """Element / function types, active numbering, pattern and splits for one workload."""

    def __init__(self, lines, ls, hybrid_gauss=False):
        self.lines, self.ls = lines, ls
        self.hybrid_gauss = hybrid_gauss
        self.p = lines[0].p
        p = self.p
        self.nel = tuple(l.nel for l in lines)
        self.nfun = tuple(l.n for l in lines)
        ne, nf = self.nel, self.nfun
        self.ecls = np.empty(ne, dtype=np.int8)
        for e in itertools.product(*map(range, ne)):
            lo = [lines[d].lo + e[d] * lines[d].h for d in range(3)]
            hi = [lines[d].lo + (e[d] + 1) * lines[d].h for d in range(3)]
            self.ecls[e] = classify_box(ls, lo, hi)
        self.fcls = np.empty(nf, dtype=np.int8)
        for I in itertools.product(*map(range, nf)):
            sub = self.ecls[self.support_slices(I)]
            if np.all(sub == OUT):
                self.fcls[I] = OUT
            elif np.all(sub == IN):
                self.fcls[I] = IN
            else:
                self.fcls[I] = CUT
        act = (self.fcls != OUT).ravel()
        self.active_lex = np.nonzero(act)[0]                # active index -> lexicographic
        self.lex_to_active = -np.ones(act.size, dtype=np.int64)
        self.lex_to_active[self.active_lex] = np.arange(self.active_lex.size)
        self.n_active = int(self.active_lex.size)
        self._split = {}
        self._Eg = None

    # --- helpers ----------------------------------------------------------------------
    def support_range(self, I, d):
        p = self.p
        return max(I[d] - p, 0), min(I[d], self.nel[d] - 1)     # inclusive element range

    def support_slices(self, I):
        return tuple(slice(self.support_range(I, d)[0], self.support_range(I, d)[1] + 1)
                     for d in range(3))

    def lex(self, I):
        return (I[0] * self.nfun[1] + I[1]) * self.nfun[2] + I[2]

    def unlex(self, k):
        k = int(k)
        return (k // (self.nfun[1] * self.nfun[2]), (k // self.nfun[2]) % self.nfun[1], k % self.nfun[2])

    def pattern(self, I):
        """Active J (as lexicographic triples) of row I, ascending."""
        p = self.p
        rng = [range(max(I[d] - p, 0), min(I[d] + p, self.nfun[d] - 1) + 1) for d in range(3)]
        return [J for J in itertools.product(*rng) if self.fcls[J] != OUT]

    def row_ptr(self):
        """CSR row pointer: counts of active J in each active row's window (box sums)."""
        p = self.p
        act = (self.fcls != OUT).astype(np.int64)
        S = np.zeros(tuple(n + 1 for n in self.nfun), dtype=np.int64)
        S[1:, 1:, 1:] = act.cumsum(0).cumsum(1).cumsum(2)
        I = np.array([self.unlex(k) for k in self.active_lex]).reshape(-1, 3)
        lo = np.maximum(I - p, 0)
        hi = np.minimum(I + p + 1, np.array(self.nfun))
        cnt = np.zeros(len(I), dtype=np.int64)
        for b in itertools.product((0, 1), repeat=3):
            idx = tuple(np.where(b[d], hi[:, d], lo[:, d]) for d in range(3))
            cnt += (-1) ** (3 - sum(b)) * S[idx]
        return np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)

    # --- split search -------------------------------------------------------------------
    def split(self, I):
        """(d, s, high, box) for a cut function, or None when no candidate is valid.

        box = ((lo1,hi1),(lo2,hi2),(lo3,hi3)) inclusive element ranges.  In the Hybrid Gauss
        scheme (Section 3.1, the compared schemes) no cut function gets a box: its whole
        regular support is integrated element by element with Gauss rules."""
        if self.hybrid_gauss:
            return None
        if I in self._split:
            return self._split[I]
        best, best_count = None, 0
        rng = [self.support_range(I, d) for d in range(3)]
        for d in range(3):
            lo, hi = rng[d]
            for s in range(lo + 1, hi + 1):
                for high in (True, False):
                    box = list(rng)
                    box[d] = (s, hi) if high else (lo, s - 1)
                    sub = self.ecls[tuple(slice(a, b + 1) for (a, b) in box)]
                    if np.all(sub == IN) and sub.size > best_count:
                        best, best_count = (d, s, high, tuple(box)), sub.size
        self._split[I] = best
        return best

    # --- element Gauss blocks -------------------------------------------------------------
    def gauss_block_elements(self):
        """Interior elements lying in the support of at least one cut function, lexicographic."""
        if self._Eg is None:
            mark = np.zeros(self.nel, dtype=bool)
            for I in zip(*np.nonzero(self.fcls == CUT)):
                sl = self.support_slices(I)
                mark[sl] |= self.ecls[sl] == IN
            self._Eg = [tuple(int(v) for v in e) for e in zip(*np.nonzero(mark))]
        return self._Eg

    def cut_elements(self):
        return [tuple(int(v) for v in e) for e in zip(*np.nonzero(self.ecls == CUT))]


# ----------------------------------------------------------------------------------------
# octree cut integration
# ----------------------------------------------------------------------------------------
def octree_points(lines, ls, e, levels: int):
    """Quadrature points and weights of cut element e: ((P,3) coords, (P,) weights).

    Cells are visited depth first, children in lexicographic order of their offset
    (first direction slowest); each cell's points are in lexicographic Gauss order."""
    p = lines[0].p
    gxi, gw = lines[0].gxi, lines[0].gw
    xs, ws = [], []

    def emit(lo, size, indicator):
        c1 = [lo[d] + (1.0 + gxi) / 2.0 * size[d] for d in range(3)]
        w1 = [gw * size[d] / 2.0 for d in range(3)]
        pts = np.stack(np.meshgrid(*c1, indexing="ij"), -1).reshape(-1, 3)
        w = np.einsum("a,b,c->abc", *w1).ravel()
        if indicator:
            w = np.where(phi(ls, pts) < 0.0, w, 0.0)
        xs.append(pts)
        ws.append(w)

    def rec(depth, off):
        scale = 2 ** depth
        lo = [lines[d].lo + (e[d] * scale + off[d]) * (lines[d].h / scale) for d in range(3)]
        size = [lines[d].h / scale for d in range(3)]
        hi = [lo[d] + size[d] for d in range(3)]
        c = classify_box(ls, lo, hi) if depth > 0 else CUT
        if c == OUT:
            return
        if c == IN:
            emit(lo, size, False)
        elif depth == levels:
            emit(lo, size, True)
        else:
            for b in itertools.product((0, 1), repeat=3):
                rec(depth + 1, tuple(2 * off[d] + b[d] for d in range(3)))

    rec(0, (0, 0, 0))
    if not xs:
        return np.zeros((0, 3)), np.zeros(0)
    return np.concatenate(xs), np.concatenate(ws)


def fitted_rule(lines, e, pts, w):
    """A rule of NK^3 = (2p+1)^3 points for cut element e that integrates every polynomial of
    degree <= 2p in each variable as the octree rule (pts, w) does: the tensor Gauss-Legendre
    points of NK nodes on the element, weights from the Legendre moments of the octree rule
    (m = (V x V x V) w_fit, V[k][g] = L_k(node g), solved direction by direction).  The
    products B_a B_b and their gradients' products lie in that space, so with kappa = 1 the cut
    element's matrices are the octree's."""
    p = lines[0].p
    nk = 2 * p + 1
    xi, _ = gauss_legendre(nk)
    V = np.polynomial.legendre.legvander(xi, 2 * p).T                 # [k][g]
    lo = [lines[d].lo + e[d] * lines[d].h for d in range(3)]
    t = [2.0 * (pts[:, d] - lo[d]) / lines[d].h - 1.0 for d in range(3)]
    L = [np.polynomial.legendre.legvander(t[d], 2 * p) for d in range(3)]   # [q][k]
    m = np.einsum("q,qa,qb,qc->abc", w, L[0], L[1], L[2])
    Vi = np.linalg.inv(V)
    wf = np.einsum("ai,bj,ck,ijk->abc", Vi, Vi, Vi, m).ravel()          # Vi[g][k]
    c1 = [lo[d] + (1.0 + xi) / 2.0 * lines[d].h for d in range(3)]
    xf = np.stack(np.meshgrid(*c1, indexing="ij"), -1).reshape(-1, 3)
    return xf, wf


# ----------------------------------------------------------------------------------------
# slot layout (kappa input / dL/dkappa output)
# ----------------------------------------------------------------------------------------
class Slots:
    """Enumeration of the quadrature points at which kappa is an input.

    [grid]   X1 x X2 x X3, lexicographic (x1 slowest);
    [blocks] for every element of Domain.gauss_block_elements() in order, its
             (p+1)^3 Gauss points, lexicographic; a Gauss point all of whose
             coordinates are WQ points is always addressed through the grid, so its
             block entry is never used;
    [octree] for every cut element in lexicographic order, its octree points in
             the order of octree_points() (fit = True: the NK^3 points of its fitted rule,
             fitted_rule()).
    """

    def __init__(self, lines, dom: Domain, levels: int, fit: bool = False):
        self.lines, self.dom, self.levels, self.fit = lines, dom, levels, fit
        p = lines[0].p
        self.nx = tuple(len(l.X) for l in lines)
        self.n_grid = int(np.prod(self.nx))
        self.Eg = dom.gauss_block_elements()
        self.block_of = {e: b for b, e in enumerate(self.Eg)}
        self.npe = (p + 1) ** 3
        self.base_block = self.n_grid
        self.base_oct = self.n_grid + len(self.Eg) * self.npe
        self.cut = dom.cut_elements()
        self._oct = {}
        self.oct_base = {}
        self.n_slots = None

    def enumerate_octree(self):
        """Fix the octree slot ranges (builds the octree of every cut element)."""
        if self.n_slots is None:
            nxt = self.base_oct
            for e in self.cut:
                _, w = self.octree(e)
                self.oct_base[e] = nxt
                nxt += len(w)
            self.n_slots = nxt
        return self

    def octree(self, e):
        if e not in self._oct:
            pts, w = octree_points(self.lines, self.dom.ls, e, self.levels)
            self._oct[e] = fitted_rule(self.lines, e, pts, w) if self.fit else (pts, w)
        return self._oct[e]

    def gauss_slot(self, eg):
        """Slot of the Gauss point eg = ((e1,g1),(e2,g2),(e3,g3))."""
        xi = [self.lines[d].xidx.get(eg[d]) for d in range(3)]
        if all(v is not None for v in xi):
            return (xi[0] * self.nx[1] + xi[1]) * self.nx[2] + xi[2]
        e = tuple(eg[d][0] for d in range(3))
        g = tuple(eg[d][1] for d in range(3))
        p1 = self.lines[0].p + 1
        return self.base_block + self.block_of[e] * self.npe + (g[0] * p1 + g[1]) * p1 + g[2]

    def coords(self):
        """(n_slots, 3) coordinates of every slot."""
        out = np.empty((self.n_slots, 3))
        X = [l.Xcoord for l in self.lines]
        out[:self.n_grid] = np.stack(np.meshgrid(*X, indexing="ij"), -1).reshape(-1, 3)
        p1 = self.lines[0].p + 1
        for b, e in enumerate(self.Eg):
            c = [self.lines[d].gauss_coord(e[d], np.arange(p1)) for d in range(3)]
            out[self.base_block + b * self.npe: self.base_block + (b + 1) * self.npe] = \
                np.stack(np.meshgrid(*c, indexing="ij"), -1).reshape(-1, 3)
        for e, base in self.oct_base.items():
            pts, _ = self.octree(e)
            out[base:base + len(pts)] = pts
        return out
