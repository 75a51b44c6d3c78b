"""CPU pins of the L2-projection oracle (Section 3.1 test setting, Section 3.2 accuracy).

Each pin rests on something other than the oracle's own code: hand-computed Lagrange
values (the extension on uniform knots), the closed form of a B-spline's integral, Marsden's
identity (the B-spline coefficients of x are the Greville abscissae), partition of unity,
polynomial reproduction of the extension checked against coefficients from interpolation at
the Greville points, brute-force searches on small meshes, exact projection of a polynomial
of the spline degree, and the optimal convergence order p+1 of an L2 projection.
"""
import itertools
import math

import numpy as np
import pytest

import oracle_pool
import workloads as W
from oracle.assemble import Problem
from oracle.domain import IN
from oracle.projection import Projection, dual_coefficient
from oracle.spline import Line, bspline, gauss_legendre

BALL8_P2 = W.custom(8, 2, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.3))
BALL10_P3 = W.custom(10, 3, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.28))
UNCUT4_P2 = W.custom(4, 2)


def _proj(wl):
    return Projection(Problem(wl))


def lagrange(p, x):
    """Lagrange polynomials on the integer nodes 0..p at x."""
    return np.array([math.prod((x - m) / (a - m) for m in range(p + 1) if m != a) for a in range(p + 1)])


def test_lagrange_hand_values():
    # nodes 0, 1, 2: L0(3) = (3-1)(3-2)/2 = 1, L1(3) = 3(3-2)/(-1) = -3, L2(3) = 3*2/2 = 3
    assert np.allclose(lagrange(2, 3.0), [1.0, -3.0, 3.0], rtol=0, atol=1e-15)
    assert np.allclose(lagrange(2, -1.0), [3.0, -3.0, 1.0], rtol=0, atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4])
def test_dual_coefficients_uniform_are_lagrange(p):
    """Where every knot involved is uniform, lambda_j(P_m) is a polynomial of degree p in j
    that is 1 at j = m and 0 at the other functions of the root element: the Lagrange
    extrapolation weight in the index."""
    line = Line(4 * p + 4, p)
    l = p + 1
    for j in (l - 2, l - 1, l + p + 1, l + p + 2):
        want = lagrange(p, j - l)
        got = [dual_coefficient(line, l, l + a, j) for a in range(p + 1)]
        assert np.allclose(got, want, rtol=0, atol=1e-15 * np.abs(want).max()), (j, got, want)
    # at a function of the root element itself: the unit vector
    got = [dual_coefficient(line, l, l + a, l + 1) for a in range(p + 1)]
    assert np.array_equal(got, np.eye(p + 1)[1])


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
    """Every outer function's root element is interior, every function supported on it is
    inner, and no interior element is nearer (first in lexicographic order among the
    nearest), by a plain search over every element."""
    pr = _proj(wl)
    dom, p = pr.dom, pr.p
    inner_set = {dom.unlex(k) for k in dom.active_lex[pr.inner_mask()]}
    interior = [e for e in itertools.product(*[range(n) for n in dom.nel]) if dom.ecls[e] == IN]
    assert interior
    for e in interior:
        assert all(tuple(e[d] + a[d] for d in range(3)) in inner_set
                   for a in itertools.product(range(p + 1), repeat=3))
    arrays = pr.arrays()
    outer = [r for r in range(dom.n_active) if not pr.inner_mask()[r]]
    assert sorted(arrays) == outer
    for r in outer:
        j = dom.unlex(dom.active_lex[r])
        best, best_d = None, None
        for l in interior:
            dd = sum((l[d] + p / 2.0 - j[d]) ** 2 for d in range(3))
            if best_d is None or dd < best_d:
                best, best_d = l, dd
        assert arrays[r] == best, (j, arrays[r], best)


def test_extension_uniform_knots_is_lagrange():
    """On the ball mesh every knot the extension touches is uniform, so E holds the products
    of Lagrange weights prod_d L_{i_d - l_d}(j_d - l_d)."""
    pr = _proj(BALL8_P2)
    dom, p = pr.dom, pr.p
    E = pr.extension()
    inner = pr.inner_mask()
    inner_idx = np.cumsum(inner) - 1
    for r, l in pr.arrays().items():
        j = dom.unlex(dom.active_lex[r])
        lam = [lagrange(p, j[d] - l[d]) for d in range(3)]
        want = np.zeros(E.shape[1])
        for a in itertools.product(range(p + 1), repeat=3):
            ri = dom.lex_to_active[dom.lex(tuple(l[d] + a[d] for d in range(3)))]
            want[inner_idx[ri]] = lam[0][a[0]] * lam[1][a[1]] * lam[2][a[2]]
        assert np.allclose(E[r], want, rtol=0, atol=1e-10 * np.abs(want).max())


def _greville_coefficients(pr, q):
    """B-spline coefficients (active functions) of a polynomial q by tensor interpolation at
    the Greville abscissae (Schoenberg-Whitney: the 1D collocation matrices are regular)."""
    A, g = [], []
    for line in pr.P.lines:
        t = line.knot_coord(line.tk)
        gr = np.array([np.mean(t[k + 1:k + line.p + 1]) for k in range(line.n)])
        g.append(gr)
        A.append(np.stack([bspline(t, line.p, k, gr) for k in range(line.n)], axis=1))
    X = np.stack(np.meshgrid(*g, indexing="ij"), -1).reshape(-1, 3)
    Q = q(X).reshape(len(g[0]), len(g[1]), len(g[2]))
    C = np.einsum("ai,bj,ck,ijk->abc", *[np.linalg.inv(a) for a in A], Q)
    return np.array([C[pr.dom.unlex(k)] for k in pr.dom.active_lex])


@pytest.mark.parametrize("wl", [BALL8_P2, W.paper_plane(4, 2), W.paper_plane(4, 3), W.paper_plane(5, 4)],
                         ids=["ball8_p2", "paper4_p2", "paper4_p3", "paper5_p4"])
def test_extension_reproduces_polynomials(wl):
    """A polynomial of degree <= p in each variable has B-spline coefficients c (found by
    interpolation, independently of the extension); E c[inner] gives c on every active
    function, boundary knots included."""
    pr = _proj(wl)
    p = pr.p
    C = np.random.default_rng(7).standard_normal((p + 1, p + 1, p + 1))

    def q(x):
        V = [np.stack([x[:, d] ** a for a in range(p + 1)], axis=1) for d in range(3)]
        return np.einsum("abc,na,nb,nc->n", C, V[0], V[1], V[2])

    c = _greville_coefficients(pr, q)
    got = pr.extension() @ c[pr.inner_mask()]
    assert np.allclose(got, c, rtol=0, atol=1e-9 * np.abs(c).max())


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
    """The active functions of a row sum to one at each of its quadrature points (partition
    of unity; every function that is nonzero there is active and in the row's pattern), so b
    equals the row sums of the mass matrix assembled with kappa = f: f = 1 on the ball, the
    target function on the paper's geometry."""
    wl = BALL8_P2
    pr = _proj(wl)
    M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
    rp = pr.P.row_ptr()
    rows = np.add.reduceat(M, rp[:-1])
    b = pr.load_vector(lambda x: np.ones(len(x)))
    assert np.allclose(b, rows, rtol=0, atol=1e-14)
    wl = W.paper_plane(4, 2)
    pr = _proj(wl)
    Mf, _ = pr.P.assemble_full_wq(W.target_f)
    rows = np.add.reduceat(Mf, pr.P.row_ptr()[:-1])
    b = pr.load_vector(W.target_f)
    assert np.abs(b - rows).max() <= 1e-14 * np.abs(b).max()


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


@pytest.mark.parametrize("wl", [BALL8_P2, BALL10_P3, W.paper_plane(4, 2), W.paper_plane(4, 3)],
                         ids=["ball8_p2", "ball10_p3", "paper4_p2", "paper4_p3"])
def test_projection_exact_in_extended_space(wl):
    """poly2_f has degree <= 2 in each variable, so it lies in the extended space (which
    reproduces polynomials of degree p) and its projection is exact to rounding."""
    pr = _proj(wl)
    M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
    b = oracle_pool.load_vector(wl, "poly2_f", pr.dom.n_active)
    u = pr.solve(M, b)
    e2, f2 = pr.l2_error(u, W.poly2_f)
    assert math.sqrt(e2 / f2) <= 1e-12


def test_projection_rate_paper_geometry():
    """Section 3.2: optimal order p+1 of the relative L2 error; at p=2 halving h divides
    it by about 8 (12.9 on these coarse meshes, h = 4 -> 8); ||f|| agrees across meshes."""
    errs, norms = [], []
    for h in (4, 8):
        wl = W.paper_plane(h, 2)
        pr = _proj(wl)
        M, _ = oracle_pool.full_wq(wl, n_active=pr.dom.n_active)
        b = oracle_pool.load_vector(wl, "target_f", pr.dom.n_active)
        e2, f2 = pr.l2_error(pr.solve(M, b), W.target_f)
        errs.append(math.sqrt(e2 / f2))
        norms.append(f2)
    assert 6.0 <= errs[0] / errs[1] <= 20.0, errs
    assert abs(norms[0] - norms[1]) <= 1e-3 * norms[1]
