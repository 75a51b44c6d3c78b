"""CPU pins of the fitted cut-element rule (a cheaper cut-element integration): NK^3 =
(2p+1)^3 tensor Gauss points per cut element whose weights reproduce the octree rule on every
polynomial of degree <= 2p in each variable.

Pins: integrals of random polynomials in the monomial basis (the weights are fitted in the
Legendre basis) against the octree rule; with kappa = 1 the matrices equal the octree's (every
product B_a B_b and grad B_a . grad B_b lies in that space); a variable kappa changes them only
by a quadrature error far below the entries.
"""
import itertools

import numpy as np
import pytest

import workloads as W
from oracle.assemble import Problem, kappa_numpy
from oracle.domain import fitted_rule, octree_points
from oracle.spline import Line

BALL = W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.4)
PLANE = W.LevelSet(W.LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("ls", [BALL, PLANE], ids=["ball", "plane"])
def test_fitted_rule_reproduces_octree_polynomials(p, ls):
    nel = 5
    lines = [Line(nel, p)] * 3
    P = Problem(W.custom(nel, p, ls))
    rng = np.random.default_rng(p)
    checked = 0
    for e in P.dom.cut_elements()[:6]:
        pts, w = octree_points(lines, ls, e, 3)
        xf, wf = fitted_rule(lines, e, pts, w)
        assert xf.shape == ((2 * p + 1) ** 3, 3)
        C = rng.standard_normal((2 * p + 1,) * 3)

        def q(x):
            V = [np.stack([x[:, d] ** a for a in range(2 * p + 1)], axis=1) for d in range(3)]
            return np.einsum("abc,na,nb,nc->n", C, V[0], V[1], V[2])

        ref = float(np.sum(w * q(pts)))
        got = float(np.sum(wf * q(xf)))
        scale = float(np.sum(np.abs(w * q(pts)))) + 1e-300
        assert abs(got - ref) <= 1e-11 * scale, (e, got, ref)
        checked += 1
    assert checked > 0


@pytest.mark.parametrize("name,wl", [("ball5_p2", W.custom(5, 2, BALL)), ("plane6_p3", W.custom(6, 3, PLANE)),
                                     ("ball4_p4", W.custom(4, 4, BALL))])
def test_fitted_kappa_one_equals_octree(name, wl):
    wf = W.with_cut_rule(wl, "fit")
    Mo, Ko = Problem(wl).assemble_full_wq(kappa_numpy(wl))
    Mf, Kf = Problem(wf).assemble_full_wq(kappa_numpy(wf))
    assert np.abs(Mf - Mo).max() <= 1e-12 * np.abs(Mo).max()
    assert np.abs(Kf - Ko).max() <= 1e-12 * np.abs(Ko).max()


def test_fitted_slots_and_variable_kappa():
    wl = W.custom(5, 2, BALL, kappa="sin3")
    wf = W.with_cut_rule(wl, "fit")
    Po, Pf = Problem(wl), Problem(wf)
    so, sf = Po.slots(), Pf.slots()
    nk3 = 5 ** 3
    assert sf.n_slots - sf.base_oct == len(Pf.dom.cut_elements()) * nk3
    assert so.n_slots - so.base_oct > 10 * (sf.n_slots - sf.base_oct)
    Mo, Ko = Po.assemble_full_wq(kappa_numpy(wl))
    Mf, Kf = Pf.assemble_full_wq(kappa_numpy(wf))
    assert np.abs(Mf - Mo).max() <= 1e-3 * np.abs(Mo).max()
    assert np.abs(Kf - Ko).max() <= 1e-3 * np.abs(Ko).max()
