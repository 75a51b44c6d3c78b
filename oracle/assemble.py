"""Matrix entries as direct sums over quadrature points (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Row I of the mass matrix M and the stiffness matrix K (same coefficient kappa for
both; the paper forms mass matrices, Section 3.1, the stiffness rules follow the
same weighted-quadrature construction with derivative test and trial functions):

  M_IJ = sum_parts sum_q W_I(q) kappa(x_q) B_J(x_q)
  K_IJ = sum_parts sum_q sum_k W_I^(k)(q) kappa(x_q) d_k B_J(x_q)

Parts (domain splitting of Eq. (1) and the caption of Fig. 3):
  interior I        : tensor WQ rule, W_I = prod_d w^00_{I_d}, W_I^(k) uses w^11 in
                      direction k and w^00 in the others (Section 1, WQ; Section 2.2 step 1);
  cut I, split box  : the same with direction d replaced by the one-sided DWQ rule
                      (Section 2.2 steps 2-6);
  cut I, interior elements of supp B_I outside the box: element Gauss,
                      W_I = omega_g B_I(x_g), W_I^(k) = omega_g d_k B_I(x_g);
  cut I, cut elements of supp B_I: octree points with the same Gauss-type weights.
Each entry is a direct sum over the part's points (no sum factorization).  For
points of an element e, B_J vanishes unless e_d <= J_d <= e_d + p in every
direction, so only those J are evaluated there.

Conventional assembly (the paper's "Standard Gauss (Ref)", Section 3.1): loop over
interior elements with (p+1)^3 Gauss points and over cut elements with their octree
points, local matrices added into the same pattern.

Adjoint: for L = sum_IJ (GM_IJ M_IJ + GK_IJ K_IJ), dL/dkappa at a slot is the sum,
over every (row, part, point) that uses the slot, of
W_I(q) sum_J GM_IJ B_J(x_q) + sum_k W_I^(k)(q) sum_J GK_IJ d_k B_J(x_q).
"""
from __future__ import annotations

import itertools

import numpy as np

from .domain import CUT, IN, OUT, Domain, Slots
from .spline import Line, Rules1D, bspline, bspline_all, dwq_rule

MASS, STIFF = 1, 2


class Problem:
    """Everything the oracle derives from a workload (lazily where it is costly)."""

    def __init__(self, wl, hybrid_gauss=False):
        self.wl = wl
        p = wl.degree
        self.p = p
        cache = {}
        self.lines = []
        for d in range(3):
            key = (wl.nel[d], wl.lo[d], wl.hi[d])
            if key not in cache:
                cache[key] = Line(wl.nel[d], p, wl.lo[d], wl.hi[d])
            self.lines.append(cache[key])
        rcache = {}
        self.rules = []
        for l in self.lines:
            if id(l) not in rcache:
                rcache[id(l)] = Rules1D(l)
            self.rules.append(rcache[id(l)])
        self.dom = Domain(self.lines, wl.levelset, hybrid_gauss)
        self._slots = None
        self._dwq = {}
        self._rowptr = None

    # --- derived data ---------------------------------------------------------------
    def slots(self, with_octree=True) -> Slots:
        if self._slots is None:
            self._slots = Slots(self.lines, self.dom, self.wl.octree_levels,
                                fit=getattr(self.wl, "cut_rule", "octree") == "fit")
        if with_octree:
            self._slots.enumerate_octree()
        return self._slots

    def row_ptr(self):
        if self._rowptr is None:
            self._rowptr = self.dom.row_ptr()
        return self._rowptr

    def dwq(self, d, i, s, high, a):
        key = (d, i, s, high, a)
        if key not in self._dwq:
            self._dwq[key] = dwq_rule(self.lines[d], i, s, high, a)
        return self._dwq[key]

    # --- basis helpers -------------------------------------------------------------------
    def b1d(self, d, j, x, a=0):
        l = self.lines[d]
        return bspline(l.knot_coord(l.tk), self.p, j, x, a)

    # --- quadrature parts of one row ----------------------------------------------------
    def _tensor_part(self, rule_pts, rule_w0, rule_w1, slots):
        """Tensor-product part from 1D (points, w00, w11) per direction."""
        n = [len(r) for r in rule_pts]
        x1 = [self.lines[d].coord(rule_pts[d]) for d in range(3)]
        xyz = np.stack(np.meshgrid(*x1, indexing="ij"), -1).reshape(-1, 3)
        wM = np.einsum("a,b,c->abc", *rule_w0).ravel()
        wK = np.stack([np.einsum("a,b,c->abc", *[rule_w1[d] if d == k else rule_w0[d]
                                                for d in range(3)]).ravel()
                       for k in range(3)], axis=1)
        slot = None
        if slots is not None:
            slot = np.array([slots.gauss_slot(eg) for eg in itertools.product(*rule_pts)],
                            dtype=np.int64)
        return dict(xyz=xyz, wM=wM, wK=wK, slot=slot, elem=None)

    def _element_gauss_part(self, I, e, slots):
        p = self.p
        g = np.arange(p + 1)
        x1 = [self.lines[d].gauss_coord(e[d], g) for d in range(3)]
        w1 = [self.lines[d].gauss_weight(g) for d in range(3)]
        b = [self.b1d(d, I[d], x1[d]) for d in range(3)]
        db = [self.b1d(d, I[d], x1[d], 1) for d in range(3)]
        xyz = np.stack(np.meshgrid(*x1, indexing="ij"), -1).reshape(-1, 3)
        om = np.einsum("a,b,c->abc", *w1).ravel()
        BI = np.einsum("a,b,c->abc", *b).ravel()
        dBI = np.stack([np.einsum("a,b,c->abc", *[db[d] if d == k else b[d] for d in range(3)]).ravel()
                        for k in range(3)], axis=1)
        slot = None
        if slots is not None:
            slot = np.array([slots.gauss_slot(((e[0], a), (e[1], bb), (e[2], c)))
                             for a, bb, c in itertools.product(g, g, g)], dtype=np.int64)
        return dict(xyz=xyz, wM=om * BI, wK=om[:, None] * dBI, slot=slot, elem=e)

    def _octree_part(self, I, e, slots):
        pts, w = slots.octree(e)
        b = [self.b1d(d, I[d], pts[:, d]) for d in range(3)]
        db = [self.b1d(d, I[d], pts[:, d], 1) for d in range(3)]
        BI = b[0] * b[1] * b[2]
        dBI = np.stack([db[0] * b[1] * b[2], b[0] * db[1] * b[2], b[0] * b[1] * db[2]], axis=1)
        slot = None
        if e in slots.oct_base:
            slot = slots.oct_base[e] + np.arange(len(w))
        return dict(xyz=pts, wM=w * BI, wK=w[:, None] * dBI, slot=slot, elem=e)

    def regular_part(self, I, slots=None):
        """The WQ (interior row) or DWQ-box (cut row) tensor part, or None."""
        dom = self.dom
        c = dom.fcls[I]
        if c == OUT:
            return None
        if c == IN:
            pts = [self.rules[d].rule[0][I[d]][0] for d in range(3)]
            w0 = [self.rules[d].rule[0][I[d]][1] for d in range(3)]
            w1 = [self.rules[d].rule[1][I[d]][1] for d in range(3)]
            return self._tensor_part(pts, w0, w1, slots)
        sp = dom.split(I)
        if sp is None:
            return None
        d0, s, high, _ = sp
        pts, w0, w1 = [], [], []
        for d in range(3):
            if d == d0:
                q0, v0 = self.dwq(d, I[d], s, high, 0)
                q1, v1 = self.dwq(d, I[d], s, high, 1)
                assert q0 == q1
                pts.append(q0); w0.append(v0); w1.append(v1)
            else:
                pts.append(self.rules[d].rule[0][I[d]][0])
                w0.append(self.rules[d].rule[0][I[d]][1])
                w1.append(self.rules[d].rule[1][I[d]][1])
        return self._tensor_part(pts, w0, w1, slots)

    def remainder_elements(self, I):
        """Interior elements of supp B_I handled by element Gauss (cut rows only)."""
        dom = self.dom
        if dom.fcls[I] != CUT:
            return []
        sp = dom.split(I)
        box = sp[3] if sp is not None else None
        rng = [range(dom.support_range(I, d)[0], dom.support_range(I, d)[1] + 1) for d in range(3)]
        out = []
        for e in itertools.product(*rng):
            if dom.ecls[e] != IN:
                continue
            if box is not None and all(box[d][0] <= e[d] <= box[d][1] for d in range(3)):
                continue
            out.append(e)
        return out

    def cut_elements_of(self, I):
        dom = self.dom
        rng = [range(dom.support_range(I, d)[0], dom.support_range(I, d)[1] + 1) for d in range(3)]
        return [e for e in itertools.product(*rng) if dom.ecls[e] == CUT]

    def row_parts(self, I, slots=None, include_cut_elements=True):
        parts = []
        reg = self.regular_part(I, slots)
        if reg is not None:
            parts.append(reg)
        for e in self.remainder_elements(I):
            parts.append(self._element_gauss_part(I, e, slots))
        if include_cut_elements and self.dom.fcls[I] == CUT:
            sl = slots if slots is not None else self.slots(with_octree=False)
            for e in self.cut_elements_of(I):
                parts.append(self._octree_part(I, e, sl))
        return parts

    # --- trial functions at a part's points ---------------------------------------------
    def _basis_1d(self, d, x, jr):
        """B_j and B_j' for j in range jr at coordinates x (evaluated once per distinct x)."""
        l = self.lines[d]
        u, inv = np.unique(x, return_inverse=True)
        B, dB = bspline_all(l.knot_coord(l.tk), self.p, u)
        return B[jr.start:jr.stop][:, inv], dB[jr.start:jr.stop][:, inv]

    def _trial(self, I, part):
        """(list of J, B_J values (nJ,P), d_k B_J values (3,nJ,P))."""
        p = self.p
        x = part["xyz"]
        if part["elem"] is not None:
            e = part["elem"]
            rng = [range(e[d], e[d] + p + 1) for d in range(3)]
        else:
            rng = [range(max(I[d] - p, 0), min(I[d] + p, self.dom.nfun[d] - 1) + 1) for d in range(3)]
        bb = [self._basis_1d(d, x[:, d], rng[d]) for d in range(3)]
        b = [v[0] for v in bb]
        db = [v[1] for v in bb]
        P = x.shape[0]

        def outer(f0, f1, f2):
            return (f0[:, None, None, :] * f1[None, :, None, :] * f2[None, None, :, :]).reshape(-1, P)

        J = list(itertools.product(*rng))
        BJ = outer(b[0], b[1], b[2])
        dBJ = np.stack([outer(db[0], b[1], b[2]), outer(b[0], db[1], b[2]), outer(b[0], b[1], db[2])])
        return J, BJ, dBJ

    # --- one row -----------------------------------------------------------------------
    def assemble_row(self, I, kappa_fn, parts=None):
        """(pattern J list, M row, K row) by direct sums over every part of row I."""
        pat = self.dom.pattern(I)
        pos = {J: k for k, J in enumerate(pat)}
        M = np.zeros(len(pat))
        K = np.zeros(len(pat))
        for part in (parts if parts is not None else self.row_parts(I)):
            if part["xyz"].shape[0] == 0:
                continue
            kap = kappa_fn(part["xyz"])
            J, BJ, dBJ = self._trial(I, part)
            m = BJ @ (part["wM"] * kap)
            k = sum(dBJ[c] @ (part["wK"][:, c] * kap) for c in range(3))
            for jj, Jt in enumerate(J):
                if Jt in pos:
                    M[pos[Jt]] += m[jj]
                    K[pos[Jt]] += k[jj]
                else:
                    assert m[jj] == 0.0 and k[jj] == 0.0
        return pat, M, K

    def assemble_rows(self, rows_active, kappa_fn):
        """Rows given by active index: list of (pattern, M, K)."""
        return [self.assemble_row(self.dom.unlex(self.dom.active_lex[r]), kappa_fn)
                for r in rows_active]

    # --- whole matrices ---------------------------------------------------------------------
    def _csr_pos(self, row_ptr, cols, ra, cb):
        s, e = row_ptr[ra], row_ptr[ra + 1]
        k = np.searchsorted(cols[s:e], cb)
        assert np.all(cols[s:e][k] == cb)
        return s + k

    def csr_cols(self):
        dom = self.dom
        cols = []
        for k in dom.active_lex:
            cols.extend(dom.lex_to_active[dom.lex(J)] for J in dom.pattern(dom.unlex(k)))
        return np.array(cols, dtype=np.int64)

    def _element_tables(self, e, x):
        """Functions supported on element e and their values / gradients at points x."""
        p = self.p
        dom = self.dom
        rng = [range(e[d], e[d] + p + 1) for d in range(3)]
        bb = [self._basis_1d(d, x[:, d], rng[d]) for d in range(3)]
        b = [v[0] for v in bb]
        db = [v[1] for v in bb]
        P = x.shape[0]

        def outer(f0, f1, f2):
            return (f0[:, None, None, :] * f1[None, :, None, :] * f2[None, None, :, :]).reshape(-1, P)

        Phi = outer(b[0], b[1], b[2])
        dPhi = [outer(db[0], b[1], b[2]), outer(b[0], db[1], b[2]), outer(b[0], b[1], db[2])]
        funcs = list(itertools.product(*rng))
        act = np.array([dom.lex_to_active[dom.lex(f)] for f in funcs])
        return funcs, act, Phi, dPhi

    def _add_element_local(self, e, x, w, kappa_fn, row_ptr, cols, M, K, rows_filter=None):
        """Element-loop contribution sum_g w_g kappa B_a B_b (and gradients) for a, b on e."""
        if x.shape[0] == 0:
            return
        kap = kappa_fn(x)
        funcs, act, Phi, dPhi = self._element_tables(e, x)
        wk = w * kap
        Lm = (Phi * wk) @ Phi.T
        Lk = sum((dPhi[c] * wk) @ dPhi[c].T for c in range(3))
        ok = act >= 0
        for ia, f in enumerate(funcs):
            if act[ia] < 0 or (rows_filter is not None and f not in rows_filter):
                continue
            posn = self._csr_pos(row_ptr, cols, act[ia], act[ok])
            M[posn] += Lm[ia, ok]
            K[posn] += Lk[ia, ok]

    def _element_gauss_points(self, e):
        p = self.p
        g = np.arange(p + 1)
        x1 = [self.lines[d].gauss_coord(e[d], g) for d in range(3)]
        w1 = [self.lines[d].gauss_weight(g) for d in range(3)]
        x = np.stack(np.meshgrid(*x1, indexing="ij"), -1).reshape(-1, 3)
        return x, np.einsum("a,b,c->abc", *w1).ravel()

    def remainder_rows_by_element(self):
        """element -> set of cut rows (triples) that integrate it by element Gauss."""
        out = {}
        for I in zip(*np.nonzero(self.dom.fcls == CUT)):
            I = tuple(int(v) for v in I)
            for e in self.remainder_elements(I):
                out.setdefault(e, set()).add(I)
        return out

    def assemble_full_wq(self, kappa_fn, share=(0, 1)):
        """Whole WQ/DWQ matrices (CSR values over row_ptr / csr_cols).

        Regular parts row by row; remainder-element and cut-element parts are the same
        sums grouped by element (each element's points serve all rows that use them).
        share = (k, n): only every n-th row and element starting at the k-th; the n
        shares sum to the whole matrices (lets a caller spread the loops over processes)."""
        k0, ns = share
        dom = self.dom
        row_ptr = self.row_ptr()
        cols = self.csr_cols()
        M = np.zeros(row_ptr[-1])
        K = np.zeros(row_ptr[-1])
        for r, k in enumerate(dom.active_lex):
            if r % ns != k0:
                continue
            I = dom.unlex(k)
            reg = self.regular_part(I)
            if reg is None:
                continue
            _, m, kk = self.assemble_row(I, kappa_fn, parts=[reg])
            M[row_ptr[r]:row_ptr[r + 1]] += m
            K[row_ptr[r]:row_ptr[r + 1]] += kk
        for c, (e, rows) in enumerate(self.remainder_rows_by_element().items()):
            if c % ns != k0:
                continue
            x, w = self._element_gauss_points(e)
            self._add_element_local(e, x, w, kappa_fn, row_ptr, cols, M, K, rows_filter=rows)
        sl = self.slots(with_octree=False)
        for c, e in enumerate(dom.cut_elements()):
            if c % ns != k0:
                continue
            x, w = sl.octree(e)
            self._add_element_local(e, x, w, kappa_fn, row_ptr, cols, M, K)
        return M, K

    def assemble_full_gauss(self, kappa_fn):
        """Conventional element loop: Gauss on interior elements, octree on cut elements."""
        dom = self.dom
        row_ptr = self.row_ptr()
        cols = self.csr_cols()
        M = np.zeros(row_ptr[-1])
        K = np.zeros(row_ptr[-1])
        sl = self.slots(with_octree=False)
        for e in itertools.product(*map(range, dom.nel)):
            if dom.ecls[e] == IN:
                x, w = self._element_gauss_points(e)
            elif dom.ecls[e] == CUT:
                x, w = sl.octree(e)
            else:
                continue
            self._add_element_local(e, x, w, kappa_fn, row_ptr, cols, M, K)
        return M, K

    # --- adjoint --------------------------------------------------------------------------
    def _adjoint_element(self, e, x, w, slot, GM, GK, row_ptr, cols, dk, rows_filter=None):
        """dk[slot_g] += w_g sum_{a,b} (GM_ab B_a B_b + GK_ab grad B_a . grad B_b)(x_g)."""
        if x.shape[0] == 0:
            return
        funcs, act, Phi, dPhi = self._element_tables(e, x)
        n = len(funcs)
        gm = np.zeros((n, n)); gk = np.zeros((n, n))
        ok = act >= 0
        for ia, f in enumerate(funcs):
            if act[ia] < 0 or (rows_filter is not None and f not in rows_filter):
                continue
            posn = self._csr_pos(row_ptr, cols, act[ia], act[ok])
            if GM is not None:
                gm[ia, ok] = GM[posn]
            if GK is not None:
                gk[ia, ok] = GK[posn]
        contrib = np.sum(Phi * (gm @ Phi), axis=0)
        contrib += sum(np.sum(dPhi[c] * (gk @ dPhi[c]), axis=0) for c in range(3))
        np.add.at(dk, slot, w * contrib)

    def adjoint(self, GM, GK, share=(0, 1)):
        """dL/dkappa over all slots for cotangents GM, GK given as CSR value arrays (or None).

        Regular parts row by row; element parts grouped by element as in assemble_full_wq
        (share as there: the n shares sum to the whole gradient)."""
        k0, ns = share
        dom = self.dom
        sl = self.slots(with_octree=True)
        row_ptr = self.row_ptr()
        cols = self.csr_cols()
        dk = np.zeros(sl.n_slots)
        for r, k in enumerate(dom.active_lex):
            if r % ns != k0:
                continue
            I = dom.unlex(k)
            part = self.regular_part(I, slots=sl)
            if part is None:
                continue
            self._adjoint_rowpart(I, part, GM, GK, row_ptr[r], row_ptr[r + 1], dk)
        p1 = self.p + 1
        for ce, (e, rows) in enumerate(self.remainder_rows_by_element().items()):
            if ce % ns != k0:
                continue
            x, w = self._element_gauss_points(e)
            slot = np.array([sl.gauss_slot(((e[0], a), (e[1], b), (e[2], c)))
                             for a, b, c in itertools.product(range(p1), repeat=3)])
            self._adjoint_element(e, x, w, slot, GM, GK, row_ptr, cols, dk, rows_filter=rows)
        for c, e in enumerate(dom.cut_elements()):
            if c % ns != k0:
                continue
            x, w = sl.octree(e)
            slot = sl.oct_base[e] + np.arange(len(w))
            self._adjoint_element(e, x, w, slot, GM, GK, row_ptr, cols, dk)
        return dk

    def _adjoint_rowpart(self, I, part, GM, GK, s, t, dk):
        pat = self.dom.pattern(I)
        pos = {J: c for c, J in enumerate(pat)}
        gm = GM[s:t] if GM is not None else np.zeros(len(pat))
        gk = GK[s:t] if GK is not None else np.zeros(len(pat))
        J, BJ, dBJ = self._trial(I, part)
        sel = np.array([pos.get(Jt, -1) for Jt in J])
        okj = sel >= 0
        gmJ = np.zeros(len(J)); gkJ = np.zeros(len(J))
        gmJ[okj] = gm[sel[okj]]; gkJ[okj] = gk[sel[okj]]
        contrib = part["wM"] * (gmJ @ BJ) + sum(part["wK"][:, c] * (gkJ @ dBJ[c]) for c in range(3))
        np.add.at(dk, part["slot"], contrib)

    def adjoint_rows(self, rows_active, GM_rows, GK_rows):
        """dL/dkappa restricted to the listed rows (every part of each row, row by row).

        GM_rows / GK_rows: per listed row, the cotangent values over its pattern."""
        sl = self.slots(with_octree=True)
        dk = np.zeros(sl.n_slots)
        for r, gm, gk in zip(rows_active, GM_rows, GK_rows):
            I = self.dom.unlex(self.dom.active_lex[r])
            for part in self.row_parts(I, slots=sl):
                if part["xyz"].shape[0]:
                    self._adjoint_rowpart(I, part, gm, gk, 0, len(gm), dk)
        return dk


def kappa_numpy(wl):
    """kappa of a workload as a numpy callable (evaluated through the input module)."""
    import torch
    from workloads import kappa_at

    def f(xyz):
        return kappa_at(wl, torch.as_tensor(np.asarray(xyz, dtype=np.float64))).numpy()
    return f
