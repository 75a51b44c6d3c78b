"""CPU pins of the L2-projection oracle (Section 3.1 test setting, Section 3.2 accuracy).

Each pin rests on something other than the oracle's own code: hand-computed Lagrange
values, the closed form of a B-spline's integral, Marsden's identity (the B-spline
coefficients of x are the Greville abscissae), partition of unity, polynomial
reproduction of Lagrange extrapolation, brute-force searches on small meshes, and the
optimal convergence order p+1 of an L2 projection.
"""
import itertools
import math

import numpy as np
import pytest

import oracle_pool
import workloads as W
from oracle.assemble import Problem
from oracle.domain import IN
from oracle.projection import Projection, lagrange_weights
from oracle.spline import bspline, gauss_legendre

BALL8_P2 = W.custom(8, 2, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.3))
BALL10_P3 = W.custom(10, 3, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.28))
UNCUT4_P2 = W.custom(4, 2)


def _proj(wl):
    return Projection(Problem(wl))


def test_lagrange_weights_hand_values():
    # nodes 0, 1, 2: L0(3) = (3-1)(3-2)/2 = 1, L1(3) = 3(3-2)/(-1) = -3, L2(3) = 3*2/2 = 3
    assert np.allclose(lagrange_weights(2, 3.0), [1.0, -3.0, 3.0], rtol=0, atol=1e-15)
    assert np.allclose(lagrange_weights(2, -1.0), [3.0, -3.0, 1.0], rtol=0, atol=1e-15)
    # at a node: the unit vector
    assert np.array_equal(lagrange_weights(4, 3.0), [0.0, 0.0, 0.0, 1.0, 0.0])


def test_inner_functions_ball():
    """Ball r=0.3 on 8^3, p=2: the interior elements are exactly {3,4}^3 (the corner of
    element 2 nearest to no axis is 0.306 from the centre), so the inner functions are
    the j in [3,6]^3 whose support [j-2, j] meets {3,4}."""
    pr = _proj(BALL8_P2)
    dom = pr.dom
    assert sorted(zip(*np.nonzero(dom.ecls == IN))) == list(itertools.product((3, 4), repeat=3))
    inner = pr.inner_mask()
    got = sorted(dom.unlex(k) for k in dom.active_lex[inner])
    assert got == list(itertools.product(range(3, 7), repeat=3))


def test_extension_is_identity_without_cut():
    pr = _proj(UNCUT4_P2)
    assert pr.inner_mask().all()
    assert np.array_equal(pr.extension(), np.eye(pr.dom.n_active))


@pytest.mark.parametrize("wl", [BALL8_P2, W.paper_plane(4, 2), W.paper_plane(4, 3)],
                         ids=["ball8_p2", "paper4_p2", "paper4_p3"])
def test_arrays_brute_force(wl):
    """Every outer function's array is all inner and no all-inner array is nearer
    (first in lexicographic order among the nearest), by a plain search over every base."""
    pr = _proj(wl)
    dom, p = pr.dom, pr.p
    inner_set = {dom.unlex(k) for k in dom.active_lex[pr.inner_mask()]}
    bases = []
    for l in itertools.product(*[range(n - p) for n in dom.nfun]):
        if all(tuple(l[d] + a[d] for d in range(3)) in inner_set
               for a in itertools.product(range(p + 1), repeat=3)):
            bases.append(l)
    assert bases
    arrays = pr.arrays()
    outer = [r for r in range(dom.n_active) if not pr.inner_mask()[r]]
    assert sorted(arrays) == outer
    for r in outer:
        j = dom.unlex(dom.active_lex[r])
        best, best_d = None, None
        for l in bases:
            dd = sum((l[d] + p / 2.0 - j[d]) ** 2 for d in range(3))
            if best_d is None or dd < best_d:
                best, best_d = l, dd
        assert arrays[r] == best, (j, arrays[r], best)


@pytest.mark.parametrize("wl", [BALL8_P2, W.paper_plane(4, 2), W.paper_plane(4, 3)],
                         ids=["ball8_p2", "paper4_p2", "paper4_p3"])
def test_extension_reproduces_index_polynomials(wl):
    """Lagrange extrapolation of degree p is exact for polynomials of degree <= p in each
    index: E applied to Q(inner indices) gives Q at every active index."""
    pr = _proj(wl)
    dom, p = pr.dom, pr.p
    rng = np.random.default_rng(7)
    C = rng.standard_normal((p + 1, p + 1, p + 1))
    J = np.array([dom.unlex(k) for k in dom.active_lex], dtype=np.float64)
    V = [np.stack([J[:, d] ** a for a in range(p + 1)], axis=1) for d in range(3)]
    Q = np.einsum("abc,na,nb,nc->n", C, V[0], V[1], V[2])
    E = pr.extension()
    got = E @ Q[pr.inner_mask()]
    assert np.allclose(got, Q, rtol=0, atol=1e-9 * np.abs(Q).max())


def _spline_integral(line, tk, i, g):
    """int B_i(x) g(x) dx by 12-point Gauss on every element of the support."""
    xg, wg = gauss_legendre(12)
    tot = 0.0
    t = line.knot_coord(tk)
    for e in range(max(i - line.p, 0), min(i, line.nel - 1) + 1):
        a, b = line.lo + e * line.h, line.lo + (e + 1) * line.h
        x = (a + b) / 2 + (b - a) / 2 * xg
        tot += float(np.sum(wg * (b - a) / 2 * bspline(t, line.p, i, x) * g(x)))
    return tot


def test_load_vector_closed_form_uncut():
    """f = 1: b_I is the integral of B_I, prod_d (t_{i+p+1} - t_i) h / (p+1), and the
    entries sum to the volume."""
    pr = _proj(UNCUT4_P2)
    b = pr.load_vector(lambda x: np.ones(len(x)))
    p = pr.p
    lines = pr.P.lines
    for r, k in enumerate(pr.dom.active_lex):
        I = pr.dom.unlex(k)
        want = 1.0
        for d in range(3):
            tk = lines[d].tk
            want *= (tk[I[d] + p + 1] - tk[I[d]]) * lines[d].h / (p + 1)
        assert abs(b[r] - want) <= 1e-14
    assert abs(b.sum() - 1.0) <= 1e-13


def test_load_vector_interior_rows_exact():
    """Interior rows integrate B_I f exactly when f lies in the spline space (poly2_f is a
    sum of four separable terms of degree <= 2 per variable)."""
    wl = W.paper_plane(8, 2)
    pr = _proj(wl)
    b = oracle_pool.load_vector(wl, "poly2_f", pr.dom.n_active)
    terms = [(0.5, (lambda x: np.ones_like(x),) * 3),
             (1.0, (lambda x: x * x, lambda x: x, lambda x: np.ones_like(x))),
             (-3.0, (lambda x: np.ones_like(x), lambda x: x * x, lambda x: x)),
             (0.25, (lambda x: x, lambda x: np.ones_like(x), lambda x: x))]
    lines = pr.P.lines
    n_checked = 0
    for r, k in enumerate(pr.dom.active_lex):
        I = pr.dom.unlex(k)
        if pr.dom.fcls[I] != IN:
            continue
        want = sum(c * math.prod(_spline_integral(lines[d], lines[d].tk, I[d], g[d]) for d in range(3))
                   for c, g in terms)
        assert abs(b[r] - want) <= 1e-14, (I, b[r], want)
        n_checked += 1
    assert n_checked >= 50


def test_load_vector_is_mass_row_sum():
    """f = 1: the active functions of a row sum to one at each of its quadrature points
    (partition of unity; every function that is nonzero there is active and in the row's
    pattern), so b equals the row sums of the mass matrix with kappa = 1."""
    wl = BALL8_P2
    pr = _proj(wl)
    M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
    rp = pr.P.row_ptr()
    rows = np.add.reduceat(M, rp[:-1])
    b = pr.load_vector(lambda x: np.ones(len(x)))
    assert np.allclose(b, rows, rtol=0, atol=1e-14)


def test_l2_error_closed_forms():
    """Uncut unit cube: ||f||^2 = 1 for f = 1; u = Greville abscissae is the spline x
    (Marsden's identity), so the error of f(x) = x vanishes."""
    pr = _proj(UNCUT4_P2)
    dom, p = pr.dom, pr.p
    u0 = np.zeros(dom.n_active)
    e2, f2 = pr.l2_error(u0, lambda x: np.ones(len(x)))
    assert abs(f2 - 1.0) <= 1e-14 and abs(e2 - 1.0) <= 1e-14
    line = pr.P.lines[0]
    t = line.knot_coord(line.tk)
    gre = np.array([np.mean(t[i + 1:i + p + 1]) for i in range(line.n)])
    u = np.array([gre[dom.unlex(k)[0]] for k in dom.active_lex])
    e2, f2 = pr.l2_error(u, lambda x: x[:, 0])
    assert abs(f2 - 1.0 / 3.0) <= 1e-14 and e2 <= 1e-28


def test_l2_error_ball_volume():
    """f = 1, u = 0 on the ball: ||f||^2 is the octree + Gauss volume of the ball."""
    pr = _proj(BALL8_P2)
    _, f2 = pr.l2_error(np.zeros(pr.dom.n_active), lambda x: np.ones(len(x)))
    assert abs(f2 - 4.0 / 3.0 * math.pi * 0.3 ** 3) <= 0.01 * f2


@pytest.mark.parametrize("wl", [BALL8_P2, BALL10_P3], ids=["ball8_p2", "ball10_p3"])
def test_projection_exact_in_extended_space(wl):
    """poly2_f has index-polynomial coefficients on every active function here (the ball
    stays inside the region of uniform knots), so it lies in the extended space and its
    projection is exact to rounding."""
    pr = _proj(wl)
    M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
    b = oracle_pool.load_vector(wl, "poly2_f", pr.dom.n_active)
    u = pr.solve(M, b)
    e2, f2 = pr.l2_error(u, W.poly2_f)
    assert math.sqrt(e2 / f2) <= 1e-12


def test_projection_rate_paper_geometry():
    """Section 3.2: optimal order p+1 of the relative L2 error; at p=2 halving h divides
    it by about 8 (9.3 on h = 4 -> 8); ||f|| agrees across meshes."""
    errs, norms = [], []
    for h in (4, 8):
        wl = W.paper_plane(h, 2)
        pr = _proj(wl)
        M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
        b = oracle_pool.load_vector(wl, "target_f", pr.dom.n_active)
        e2, f2 = pr.l2_error(pr.solve(M, b), W.target_f)
        errs.append(math.sqrt(e2 / f2))
        norms.append(f2)
    assert 6.0 <= errs[0] / errs[1] <= 12.0, errs
    assert abs(norms[0] - norms[1]) <= 1e-3 * norms[1]
