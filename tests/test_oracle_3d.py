"""Pins of the oracle's 3D layer (assembly, classification, splits, octree, adjoint).

Reference values come from outside the oracle: Kronecker products of exact 1D Gram
matrices, closed-form integrals of B-splines, analytic volumes, counts that follow
from the plane's arithmetic, brute-force dense sums, separability, and linearity of
the loss in kappa.
"""
import itertools
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle.assemble import Problem, kappa_numpy
from oracle.domain import CUT, IN, OUT, classify_box, octree_points, phi
from oracle.spline import bspline, gauss_legendre

ONE = lambda x: np.ones(len(x))  # noqa: E731
BALL = W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.4)
PLANE = W.LevelSet(W.LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6)
TORUS = W.LevelSet(W.LS_TORUS, c=(0.5, 0.5, 0.5), r0=0.3, r1=0.12)


def dense(P, vals):
    """CSR values -> dense (n_active x n_active)."""
    rp = P.row_ptr()
    cols = P.csr_cols()
    A = np.zeros((P.dom.n_active, P.dom.n_active))
    for r in range(P.dom.n_active):
        A[r, cols[rp[r]:rp[r + 1]]] = vals[rp[r]:rp[r + 1]]
    return A


def gram_1d(line, a, npts=12):
    xi, w = gauss_legendre(npts)
    t = line.knot_coord(line.tk)
    x = np.concatenate([line.lo + (e + (1 + xi) / 2) * line.h for e in range(line.nel)])
    wx = np.tile(w * line.h / 2, line.nel)
    B = np.array([bspline(t, line.p, i, x, a) for i in range(line.n)])
    return (B * wx) @ B.T


def box_halfspace_volume(lo, hi, n, r):
    """Volume of {x in box : n.x < r} for n > 0 (inclusion-exclusion over vertices)."""
    n = np.asarray(n, dtype=float)
    v = 0.0
    for b in itertools.product((0, 1), repeat=3):
        corner = np.where(b, hi, lo)
        v += (-1) ** sum(b) * max(0.0, r - float(n @ corner)) ** 3
    return v / (6.0 * n.prod())


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("nel,p", [(3, 2), (2, 3), (4, 1)])
def test_uncut_kappa1_kronecker(nel, p):
    """kappa = 1, no cut: M = M1 x M1 x M1, K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1."""
    P = Problem(W.custom(nel, p))
    M, K = P.assemble_full_wq(ONE)
    M1 = gram_1d(P.lines[0], 0)
    K1 = gram_1d(P.lines[0], 1)
    Mr = np.kron(np.kron(M1, M1), M1)
    Kr = np.kron(np.kron(K1, M1), M1) + np.kron(np.kron(M1, K1), M1) + np.kron(np.kron(M1, M1), K1)
    assert np.abs(dense(P, M) - Mr).max() <= 1e-14 * np.abs(Mr).max()
    assert np.abs(dense(P, K) - Kr).max() <= 1e-13 * np.abs(Kr).max()


def test_row_sums_and_total_uncut():
    """sum_J M_IJ = int B_I = prod_d (t_{I_d+p+1} - t_{I_d})/(p+1); sum M = 1; sum_J K_IJ = 0."""
    p = 3
    P = Problem(W.custom(5, p))
    M, K = P.assemble_full_wq(ONE)
    rp = P.row_ptr()
    rs = np.add.reduceat(M, rp[:-1])
    line = P.lines[0]
    t = line.knot_coord(line.tk)
    for r, k in enumerate(P.dom.active_lex):
        I = P.dom.unlex(k)
        ref = np.prod([(t[I[d] + p + 1] - t[I[d]]) / (p + 1) for d in range(3)])
        assert abs(rs[r] - ref) <= 1e-15
    assert abs(M.sum() - 1.0) < 1e-13
    kap = kappa_numpy(W.custom(5, p, kappa="rf", seed=7))
    M, K = P.assemble_full_wq(kap)
    ks = np.add.reduceat(K, rp[:-1])
    assert np.abs(ks).max() <= 1e-13 * np.abs(K).max()


@pytest.mark.parametrize("ls", [BALL, PLANE, TORUS], ids=["ball", "plane", "torus"])
@pytest.mark.parametrize("p", [2, 3])
def test_wq_equals_gauss_kappa1_cut(ls, p):
    """kappa = 1: every WQ / DWQ part is exact, so the WQ matrix equals the Gauss one."""
    P = Problem(W.custom(5, p, ls))
    M, K = P.assemble_full_wq(ONE)
    Mg, Kg = P.assemble_full_gauss(ONE)
    assert np.abs(M - Mg).max() <= 1e-13 * np.abs(Mg).max()
    assert np.abs(K - Kg).max() <= 1e-13 * np.abs(Kg).max()
    # the conventional matrices are symmetric
    D = dense(P, Mg)
    assert np.abs(D - D.T).max() <= 1e-15 * np.abs(D).max()
    rp = P.row_ptr()
    assert np.abs(np.add.reduceat(K, rp[:-1])).max() <= 1e-13 * np.abs(K).max()
    if ls is PLANE:
        vol = 1.6 ** 3 / 6 - 3 * 0.6 ** 3 / 6
        assert abs(M.sum() - vol) < 2e-3


def test_separable_kappa_uncut():
    """kappa = f1(x) f2(y) f3(z): the 3D WQ matrices are Kronecker products of 1D WQ sums."""
    fs = [lambda x: 1 + 0.3 * np.sin(3 * x), lambda y: np.exp(y), lambda z: 2 - z * z]
    kap = W.kappa_separable(fs)
    nel, p = 4, 2
    P = Problem(W.custom(nel, p))
    M, K = P.assemble_full_wq(kap)
    line = P.lines[0]
    t = line.knot_coord(line.tk)
    A = [np.zeros((line.n, line.n)) for _ in range(3)]       # 00 rule with f_d
    D = [np.zeros((line.n, line.n)) for _ in range(3)]       # 11 rule with f_d
    for d in range(3):
        for i in range(line.n):
            Q0, w0 = P.rules[d].rule[0][i]
            Q1, w1 = P.rules[d].rule[1][i]
            x0, x1 = line.coord(Q0), line.coord(Q1)
            for j in range(line.n):
                A[d][i, j] = np.sum(w0 * fs[d](x0) * bspline(t, p, j, x0))
                D[d][i, j] = np.sum(w1 * fs[d](x1) * bspline(t, p, j, x1, 1))
    Mr = np.kron(np.kron(A[0], A[1]), A[2])
    Kr = np.kron(np.kron(D[0], A[1]), A[2]) + np.kron(np.kron(A[0], D[1]), A[2]) + np.kron(np.kron(A[0], A[1]), D[2])
    assert np.abs(dense(P, M) - Mr).max() <= 1e-14 * np.abs(Mr).max()
    assert np.abs(dense(P, K) - Kr).max() <= 1e-13 * np.abs(Kr).max()


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_bruteforce_2cube(p):
    """2^3 elements: windowed row sums == dense full-grid sums; kappa=1 == 12-point Gauss."""
    wl = W.custom(2, p, kappa="rf", seed=11)
    kap = kappa_numpy(wl)
    P = Problem(wl)
    M, K = P.assemble_full_wq(kap)
    Md, Kd = dense(P, M), dense(P, K)
    line = P.lines[0]
    t = line.knot_coord(line.tk)
    X = line.Xcoord
    nx = len(X)
    # zero-padded 1D weights over the whole point list
    Wp = np.zeros((2, line.n, nx))
    for a in (0, 1):
        for i in range(line.n):
            Q, w = P.rules[0].rule[a][i]
            Wp[a, i, [line.xidx[q] for q in Q]] = w
    B = np.array([bspline(t, p, j, X) for j in range(line.n)])
    dB = np.array([bspline(t, p, j, X, 1) for j in range(line.n)])
    grid = np.stack(np.meshgrid(X, X, X, indexing="ij"), -1).reshape(-1, 3)
    kg = kap(grid).reshape(nx, nx, nx)
    n = line.n
    for I in itertools.product(range(n), repeat=3):
        r = P.dom.lex_to_active[P.dom.lex(I)]
        WM = np.einsum("a,b,c->abc", Wp[0, I[0]], Wp[0, I[1]], Wp[0, I[2]]) * kg
        WK = [np.einsum("a,b,c->abc", *[Wp[1 if d == k else 0, I[d]] for d in range(3)]) * kg for k in range(3)]
        for J in itertools.product(range(n), repeat=3):
            c = P.dom.lex_to_active[P.dom.lex(J)]
            BJ = np.einsum("a,b,c->abc", B[J[0]], B[J[1]], B[J[2]])
            m = np.sum(WM * BJ)
            kk = sum(np.sum(WK[k] * np.einsum("a,b,c->abc", *[dB[J[d]] if d == k else B[J[d]] for d in range(3)]))
                     for k in range(3))
            assert abs(Md[r, c] - m) <= 1e-15 * np.abs(Md).max() + 1e-15
            assert abs(Kd[r, c] - kk) <= 1e-14 * np.abs(Kd).max()
    # kappa = 1 against a 12-point Gauss tensor rule
    M1, _ = P.assemble_full_wq(ONE)
    Mg = np.kron(np.kron(gram_1d(line, 0), gram_1d(line, 0)), gram_1d(line, 0))
    assert np.abs(dense(P, M1) - Mg).max() <= 1e-14 * np.abs(Mg).max()


# ------------------------------------------------------------------------------------------
def test_plane_classification_counts_48():
    """x+y+z < 1.6 on 48^3: element (i,j,k) is interior iff i+j+k+3 <= 76.8, exterior iff
    i+j+k >= 76.8; a function's support spans elements max(I-p,0)..min(I,47)."""
    wl = W.workload("plane48_p4")
    P = Problem(wl)
    s = np.indices((48, 48, 48)).sum(0)
    assert np.array_equal(P.dom.ecls == IN, s + 3 <= 76)
    assert np.array_equal(P.dom.ecls == OUT, s >= 77)
    I = np.indices((52, 52, 52))
    smax = np.minimum(I, 47).sum(0)
    smin = np.maximum(I - 4, 0).sum(0)
    assert np.array_equal(P.dom.fcls == IN, smax + 3 <= 76)
    assert np.array_equal(P.dom.fcls == OUT, smin >= 77)
    assert (P.dom.ecls == IN).sum() == 60472 and (P.dom.ecls == CUT).sum() == 5122
    assert (P.dom.fcls == IN).sum() == 65008 and (P.dom.fcls == CUT).sum() == 28550
    assert P.row_ptr()[-1] == 58302298


def test_pattern_counts_bruteforce():
    P = Problem(W.custom(6, 2, BALL))
    rp = P.row_ptr()
    for r, k in enumerate(P.dom.active_lex):
        I = P.dom.unlex(k)
        cnt = 0
        for J in itertools.product(*[range(max(I[d] - 2, 0), min(I[d] + 2, P.dom.nfun[d] - 1) + 1) for d in range(3)]):
            sup = P.dom.ecls[tuple(slice(max(J[d] - 2, 0), min(J[d], 5) + 1) for d in range(3))]
            cnt += int(np.any(sup != OUT))
        assert rp[r + 1] - rp[r] == cnt


def test_ball_box_classification_sampled():
    """Exact ball test never contradicts dense point sampling of the box."""
    rng = np.random.default_rng(5)
    for _ in range(300):
        lo = rng.uniform(0, 0.9, 3)
        hi = lo + rng.uniform(0.01, 0.3, 3)
        c = classify_box(BALL, lo, hi)
        pts = lo + (hi - lo) * rng.uniform(0, 1, (2000, 3))
        ph = phi(BALL, pts)
        if c == IN:
            assert np.all(ph <= 0)
        elif c == OUT:
            assert np.all(ph >= 0)
        for ls in (TORUS,):
            ct = classify_box(ls, lo, hi)
            pt = phi(ls, pts)
            if ct == IN:
                assert np.all(pt <= 0)
            if ct == OUT:
                assert np.all(pt >= 0)


def test_split_is_valid_and_maximal():
    P = Problem(W.custom(8, 3, BALL))
    dom = P.dom
    n_box = 0
    for I in zip(*np.nonzero(dom.fcls == CUT)):
        I = tuple(int(v) for v in I)
        sp = dom.split(I)
        rng = [dom.support_range(I, d) for d in range(3)]
        best = 0
        for d in range(3):
            for s in range(rng[d][0] + 1, rng[d][1] + 1):
                for box_d in ((s, rng[d][1]), (rng[d][0], s - 1)):
                    box = list(rng)
                    box[d] = box_d
                    sub = dom.ecls[tuple(slice(a, b + 1) for a, b in box)]
                    if np.all(sub == IN):
                        best = max(best, sub.size)
        if sp is None:
            assert best == 0
            continue
        n_box += 1
        d, s, high, box = sp
        sub = dom.ecls[tuple(slice(a, b + 1) for a, b in box)]
        assert np.all(sub == IN) and sub.size == best
        assert box[d] == ((s, rng[d][1]) if high else (rng[d][0], s - 1))
    assert n_box > 0


def test_split_tie_break():
    """Reading of the split search (Section 2.2 step 2 and the 3D paragraph after Fig. 3):
    among valid boxes with the most elements the first in the order d ascending, s
    ascending, high side before low wins.  Two hand-built element patterns inside the
    3 x 3 x 3 support of a p = 2 function produce ties."""
    P = Problem(W.custom(6, 2))
    dom = P.dom
    I = (3, 3, 3)
    rng = [dom.support_range(I, d) for d in range(3)]
    assert rng == [(1, 3)] * 3

    def run(cut_elems):
        dom.ecls[...] = IN
        for e in cut_elems:
            dom.ecls[e] = CUT
        dom._split = {}
        return dom.split(I)

    # an edge column (first two offsets 0) is cut: d = 0 and d = 1 (s = 2, high side)
    # both keep 18 elements; d = 0 comes first
    sp = run([(1, 1, c) for c in range(1, 4)])
    assert sp[:3] == (0, 2, True) and sp[3] == ((2, 3), (1, 3), (1, 3))
    # the middle slab in direction 0 is cut: (s = 2, low) and (s = 3, high) both keep 9
    # elements; s = 2 comes first
    sp = run([(2, b, c) for b in range(1, 4) for c in range(1, 4)])
    assert sp[:3] == (0, 2, False) and sp[3] == ((1, 1), (1, 3), (1, 3))
    # the far corner slab in direction 1 is cut: (d = 1, s = 2, low) keeps 9 elements,
    # (d = 1, s = 3, low) keeps 18 and wins over the smaller valid boxes
    sp = run([(a, 3, c) for a in range(1, 4) for c in range(1, 4)])
    assert sp[:3] == (1, 3, False) and sp[3] == ((1, 3), (1, 2), (1, 3))


# ------------------------------------------------------------------------------------------
def test_octree_plane_volume_converges():
    """Octree weights of a cut element -> exact volume of the element below the plane."""
    wl = W.custom(6, 2, PLANE)
    P = Problem(wl)
    h = 1 / 6
    errs = {1: [], 2: [], 3: []}
    for e in P.dom.cut_elements()[:12]:
        lo = np.array(e) * h
        exact = box_halfspace_volume(lo, lo + h, (1, 1, 1), 1.6)
        for L in (1, 2, 3):
            x, w = octree_points(P.lines, PLANE, e, L)
            errs[L].append(abs(w.sum() - exact) / h ** 3)
            assert np.all(w >= 0)
    assert np.mean(errs[3]) < np.mean(errs[2]) < np.mean(errs[1])
    assert max(errs[3]) < 0.02


def test_octree_interior_cells_exact():
    """An octree of a cut element integrates polynomials of degree <= 2p+1 exactly on the
    part of the element covered by interior cells; with no cut the cells cover the box."""
    wl = W.custom(4, 3, BALL)
    P = Problem(wl)
    e = P.dom.cut_elements()[0]
    x, w = octree_points(P.lines, W.LevelSet(), e, 3)       # kind 0: the whole element
    h = 0.25
    lo = np.array(e) * h
    assert abs(w.sum() - h ** 3) < 1e-17
    f = (x[:, 0] - lo[0]) ** 7 * (x[:, 1] - lo[1]) ** 3
    assert abs(np.sum(w * f) - h ** 8 / 8 * h ** 4 / 4 * h) < 1e-15 * h ** 13 * 1e3


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("ls", [BALL, TORUS], ids=["ball", "torus"])
def test_adjoint_linearity_identity(ls):
    """L = sum_IJ G_IJ A_IJ(kappa) is linear in kappa, so sum_slots kappa * dL/dkappa = L."""
    wl = W.custom(5, 2, ls, kappa="rf", seed=3)
    kap = kappa_numpy(wl)
    P = Problem(wl)
    M, K = P.assemble_full_wq(kap)
    GM = W.random_values(1, len(M))
    GK = W.random_values(2, len(K))
    dk = P.adjoint(GM, GK)
    sl = P.slots()
    ks = kap(sl.coords())
    L = GM @ M + GK @ K
    assert abs(ks @ dk - L) <= 1e-12 * (np.abs(GM * M).sum() + np.abs(GK * K).sum())


def test_adjoint_rank1_octree_closed_form():
    """G = u v^T on the pattern: at an octree slot, dL/dkappa = w_g u_h(x_g) v_h(x_g)."""
    wl = W.custom(4, 2, BALL)
    P = Problem(wl)
    u, v = W.uv_vectors(4, P.dom.n_active)
    rp, cols = P.row_ptr(), P.csr_cols()
    rows = np.repeat(np.arange(P.dom.n_active), np.diff(rp))
    G = u[rows] * v[cols]
    dk = P.adjoint(G, None)
    sl = P.slots()
    line = P.lines[0]
    t = line.knot_coord(line.tk)
    for e in P.dom.cut_elements()[:6]:
        x, w = sl.octree(e)
        base = sl.oct_base[e]
        uh = np.zeros(len(w)); vh = np.zeros(len(w))
        for a in itertools.product(*[range(e[d], e[d] + 3) for d in range(3)]):
            r = P.dom.lex_to_active[P.dom.lex(a)]
            if r < 0:
                continue
            Ba = np.prod([bspline(t, 2, a[d], x[:, d]) for d in range(3)], axis=0)
            uh += u[r] * Ba
            vh += v[r] * Ba
        assert np.allclose(dk[base:base + len(w)], w * uh * vh, atol=1e-15 * np.abs(w).max())


def test_rowwise_equals_elementwise():
    """Row-by-row direct sums (every part of a row) == element-grouped whole matrices."""
    wl = W.custom(5, 2, BALL, kappa="sin3")
    kap = kappa_numpy(wl)
    P = Problem(wl)
    M, K = P.assemble_full_wq(kap)
    rp = P.row_ptr()
    rows = W.sample_indices(9, P.dom.n_active, 25)
    for r, (pat, m, k) in zip(rows, P.assemble_rows(rows, kap)):
        assert np.abs(M[rp[r]:rp[r + 1]] - m).max() <= 1e-14 * np.abs(m).max()
        assert np.abs(K[rp[r]:rp[r + 1]] - k).max() <= 1e-14 * np.abs(k).max()
    GM = W.random_values(1, len(M))
    dk = P.adjoint(GM, None)
    dkr = P.adjoint_rows(range(P.dom.n_active), [GM[rp[r]:rp[r + 1]] for r in range(P.dom.n_active)],
                         [np.zeros(rp[r + 1] - rp[r]) for r in range(P.dom.n_active)])
    assert np.abs(dk - dkr).max() <= 1e-14 * np.abs(dk).max()


@pytest.mark.parametrize("ls", [PLANE, BALL], ids=["plane", "ball"])
def test_hybrid_gauss_scheme(ls):
    """Hybrid Gauss scheme (Section 3.1, compared schemes): with no DWQ boxes a cut row is
    integrated exactly as in the conventional element-by-element Gauss assembly (element Gauss
    on its interior elements, octree on its cut elements), for any kappa; interior rows are
    the WQ rows of the DWQ scheme."""
    wl = W.custom(6, 3, ls, kappa="rf", seed=3)
    kap = kappa_numpy(wl)
    Ph = Problem(wl, hybrid_gauss=True)
    Pd = Problem(wl)
    assert all(Ph.dom.split(Ph.dom.unlex(k)) is None for k in Ph.dom.active_lex)
    Mh, Kh = Ph.assemble_full_wq(kap)
    Md, Kd = Pd.assemble_full_wq(kap)
    Mg, Kg = Pd.assemble_full_gauss(kap)
    rp = Pd.row_ptr()
    fc = Pd.dom.fcls.ravel()[Pd.dom.active_lex]
    ent_cut = np.repeat(fc == CUT, np.diff(rp))
    for h, d, g in ((Mh, Md, Mg), (Kh, Kd, Kg)):
        assert np.array_equal(h[~ent_cut], d[~ent_cut])
        assert np.abs(h[ent_cut] - g[ent_cut]).max() <= 1e-13 * np.abs(g).max()
    # the schemes differ on the cut rows that DWQ gives a box (variable kappa)
    boxed = [r for r in range(Pd.dom.n_active)
             if fc[r] == CUT and Pd.dom.split(Pd.dom.unlex(Pd.dom.active_lex[r])) is not None]
    assert boxed or ls is not PLANE
    for r in boxed[:1]:
        assert np.abs(Mh[rp[r]:rp[r + 1]] - Md[rp[r]:rp[r + 1]]).max() > 1e-10 * np.abs(Md[rp[r]:rp[r + 1]]).max()
