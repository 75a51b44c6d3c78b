"""Stiffness matrix with a full symmetric coefficient tensor (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2 takes the identity as the map from the parameter space to the background mesh and
notes that this loses no generality.  Under a geometry map F the Laplacian stiffness becomes,
in parameter coordinates,

  K_IJ = int_Omega grad B_I . C grad B_J,   C = |det DF| DF^-1 DF^-T (times a material
                                             coefficient),

a full symmetric 3 x 3 coefficient tensor; the mass matrix only changes its scalar
coefficient (|det DF| kappa), which the scalar path already takes.  Written out,
grad B_I . C grad B_J = sum_{d,e} C_de d_d B_I d_e B_J: nine terms.

Weighted quadrature (Section 1; readings as for the scalar stiffness): the test function is
folded into 1D weights per direction, so term (d, e) uses in direction x the rule family
(x == d, x == e) = (test derivative order, trial derivative order): (0, 0) and (1, 1) as for
the scalar matrices, and the mixed families (1, 0) in direction d and (0, 1) in direction e
when d != e.  The mixed rules satisfy
  (1, 0): sum_q w_q B_j(x_q) = int B_i' B_j     for every j overlapping supp B_i,
  (0, 1): sum_q w_q B_j'(x_q) = int B_i B_j'    (posed on the degree p-1 B-splines, as the
                                                (1, 1) rule),
with the same points and the same minimum-norm solve (oracle/spline.py, exactness_system).
DWQ box rows use the one-sided rule of each family in the split direction (Section 2.2 steps
3-6, linear in the test function).  Remainder elements (element Gauss) and cut elements
(their cut rule) use w_q d_d B_I(x_q) as the weight of term (d, e), as in the scalar matrices.

Everything here is a direct sum over each part's points (no sum factorization).
"""
from __future__ import annotations

import itertools

import numpy as np

from .domain import CUT, IN, OUT


def family(x: int, d: int, e: int):
    """Rule family of direction x in term (d, e): 0, 1 or a mixed pair."""
    f = (int(x == d), int(x == e))
    return f[0] if f[0] == f[1] else f


def _tensor_weights(w_of_fam):
    """wT[q, d, e] over the tensor grid from per-direction weights w_of_fam[x][family]."""
    n = [len(w_of_fam[x][0]) for x in range(3)]
    wT = np.zeros((n[0] * n[1] * n[2], 3, 3))
    for d in range(3):
        for e in range(3):
            w = [w_of_fam[x][family(x, d, e)] for x in range(3)]
            wT[:, d, e] = np.einsum("a,b,c->abc", *w).ravel()
    return wT


FAMILIES = (0, 1, (1, 0), (0, 1))


def regular_part(P, I):
    """The WQ (interior row) or DWQ-box (cut row) part of row I with term weights, or None."""
    dom = P.dom
    c = dom.fcls[I]
    if c == OUT:
        return None
    if c == IN:
        pts = [P.rules[x].family(0, I[x])[0] for x in range(3)]
        wf = [{f: P.rules[x].family(f, I[x])[1] for f in FAMILIES} for x in range(3)]
    else:
        sp = dom.split(I)
        if sp is None:
            return None
        d0, s, high, _ = sp
        pts, wf = [], []
        for x in range(3):
            if x == d0:
                rr = {f: P.dwq(x, I[x], s, high, f) for f in FAMILIES}
                assert all(rr[f][0] == rr[0][0] for f in FAMILIES)
                pts.append(rr[0][0])
                wf.append({f: rr[f][1] for f in FAMILIES})
            else:
                pts.append(P.rules[x].family(0, I[x])[0])
                wf.append({f: P.rules[x].family(f, I[x])[1] for f in FAMILIES})
    x1 = [P.lines[x].coord(pts[x]) for x in range(3)]
    xyz = np.stack(np.meshgrid(*x1, indexing="ij"), -1).reshape(-1, 3)
    return dict(xyz=xyz, wT=_tensor_weights(wf), elem=None)


def element_part(P, I, e, x, w):
    """Points x with weights w of element e: term (d, e') weight w d_d B_I."""
    b = [P.b1d(d, I[d], x[:, d]) for d in range(3)]
    db = [P.b1d(d, I[d], x[:, d], 1) for d in range(3)]
    dBI = np.stack([db[0] * b[1] * b[2], b[0] * db[1] * b[2], b[0] * b[1] * db[2]], axis=1)
    wT = np.repeat((w[:, None] * dBI)[:, :, None], 3, axis=2)
    return dict(xyz=x, wT=wT, elem=e)


def row_parts(P, I):
    parts = []
    reg = regular_part(P, I)
    if reg is not None:
        parts.append(reg)
    for e in P.remainder_elements(I):
        parts.append(element_part(P, I, e, *P._element_gauss_points(e)))
    if P.dom.fcls[I] == CUT:
        sl = P.slots(with_octree=False)
        for e in P.cut_elements_of(I):
            x, w = sl.octree(e)
            parts.append(element_part(P, I, e, x, w))
    return parts


def assemble_row(P, I, C_fn):
    """(pattern, K row): K_IJ = sum_parts sum_q sum_{d,e} wT[q,d,e] C_de(x_q) d_e B_J(x_q)."""
    pat = P.dom.pattern(I)
    pos = {J: k for k, J in enumerate(pat)}
    K = np.zeros(len(pat))
    for part in row_parts(P, I):
        if part["xyz"].shape[0] == 0:
            continue
        C = C_fn(part["xyz"])
        J, _, dBJ = P._trial(I, part)
        k = sum(dBJ[e] @ (part["wT"][:, d, e] * C[:, d, e]) for d in range(3) for e in range(3))
        for jj, Jt in enumerate(J):
            if Jt in pos:
                K[pos[Jt]] += k[jj]
            else:
                assert k[jj] == 0.0
    return pat, K


def assemble(P, C_fn, share=(0, 1), rows=None):
    """K values over the CSR pattern (row by row); share = (k, n) every n-th row from the
    k-th; rows: only these active rows."""
    dom = P.dom
    row_ptr = P.row_ptr()
    K = np.zeros(row_ptr[-1])
    todo = range(dom.n_active) if rows is None else sorted(set(int(r) for r in rows))
    for c, r in enumerate(todo):
        if c % share[1] != share[0]:
            continue
        _, k = assemble_row(P, dom.unlex(dom.active_lex[r]), C_fn)
        K[row_ptr[r]:row_ptr[r + 1]] = k
    return K


def assemble_gauss(P, C_fn):
    """Conventional element loop: element Gauss on interior elements, the cut rule on cut
    elements, local matrices sum_q w_q grad B_a . C grad B_b added into the pattern."""
    dom = P.dom
    row_ptr = P.row_ptr()
    cols = P.csr_cols()
    K = np.zeros(row_ptr[-1])
    sl = P.slots(with_octree=False)
    for e in itertools.product(*map(range, dom.nel)):
        if dom.ecls[e] == IN:
            x, w = P._element_gauss_points(e)
        elif dom.ecls[e] == CUT:
            x, w = sl.octree(e)
        else:
            continue
        if x.shape[0] == 0:
            continue
        funcs, act, _, dPhi = P._element_tables(e, x)
        C = C_fn(x)
        L = sum((dPhi[d] * (w * C[:, d, ee])) @ dPhi[ee].T for d in range(3) for ee in range(3))
        ok = act >= 0
        for ia in range(len(funcs)):
            if act[ia] < 0:
                continue
            posn = P._csr_pos(row_ptr, cols, act[ia], act[ok])
            K[posn] += L[ia, ok]
    return K
