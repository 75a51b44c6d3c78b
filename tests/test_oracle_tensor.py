"""Pins of the oracle's full-coefficient-tensor stiffness (identity map lifted, Section 2):
mixed 1D rules against their exactness conditions integrated by an independent Gauss rule,
the isotropic tensor against the scalar stiffness, a constant tensor against the conventional
element loop (weighted quadrature is exact for constant coefficients), and zero row sums
for a variable tensor (the trial functions sum to one)."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import tensor as OT
from oracle.assemble import Problem, kappa_numpy
from oracle.spline import Line, bspline, dwq_rule, gauss_legendre, support

PLANE = W.LevelSet(W.LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6)
CUT_P3 = W.custom(6, 3, PLANE, kappa="sin3", cut_rule="fit")


@functools.lru_cache(maxsize=None)
def _problem(wl):
    return Problem(wl)


def _const(C0):
    return lambda x: np.broadcast_to(C0, (x.shape[0], 3, 3))


def _integral(line, tk, i, at, j, ac):
    """int B_i^(at) B_j^(ac) (same degree, same knots) by p+3 Gauss points per element."""
    p = line.p
    t = line.knot_coord(tk)
    xi, gw = gauss_legendre(p + 3)
    s = 0.0
    for e in range(line.nel):
        x = line.lo + (e + (1.0 + xi) / 2.0) * line.h
        s += float(np.sum(gw * line.h / 2.0 * bspline(t, p, i, x, at) * bspline(t, p, j, x, ac)))
    return s


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mixed_rules_exact(p):
    """sum_q w_q B_j^(ac)(x_q) = int B_i^(at) B_j^(ac) for every j of the row window, for the
    standard rules of every function and the one-sided rules of a few breaks."""
    line = Line(3 * p + 3, p)
    t = line.knot_coord(line.tk)
    from oracle.spline import Rules1D
    R = Rules1D(line)
    for fam in ((1, 0), (0, 1)):
        at, ac = fam
        for i in range(line.n):
            Q, w = R.family(fam, i)
            x = line.coord(Q)
            for j in range(max(0, i - p), min(line.n, i + p + 1)):
                got = float(np.sum(w * bspline(t, p, j, x, ac)))
                assert abs(got - _integral(line, line.tk, i, at, j, ac)) <= 1e-13, (fam, i, j)
        i = p + 2                                     # one-sided rules at every interior break
        sa, sb = support(line.tk, p, i)
        for s in range(sa + 1, sb):
            for high in (True, False):
                Q, w = dwq_rule(line, i, s, high, fam)
                x = line.coord(Q)
                lo, hi = (s, sb) if high else (sa, s)
                for j in range(i - p, i + p + 1):
                    # exact over the kept side: integral of the test function restricted there
                    xi, gw = gauss_legendre(p + 3)
                    ref = 0.0
                    for e in range(lo, hi):
                        xx = line.lo + (e + (1.0 + xi) / 2.0) * line.h
                        ref += float(np.sum(gw * line.h / 2.0 * bspline(t, p, i, xx, at) * bspline(t, p, j, xx, ac)))
                    got = float(np.sum(w * bspline(t, p, j, x, ac)))
                    assert abs(got - ref) <= 1e-13, (fam, s, high, j)


def test_family_of_terms():
    """Term (d, e) uses (1, 1) in direction d = e, (1, 0) in d and (0, 1) in e otherwise,
    (0, 0) in the remaining directions."""
    assert [OT.family(x, 1, 1) for x in range(3)] == [0, 1, 0]
    assert [OT.family(x, 0, 2) for x in range(3)] == [(1, 0), 0, (0, 1)]
    assert [OT.family(x, 2, 0) for x in range(3)] == [(0, 1), 0, (1, 0)]


def test_isotropic_tensor_is_the_scalar_stiffness():
    """C = kappa I gives the scalar stiffness of the same kappa (box rows, remainder and the
    fitted cut rule included)."""
    P = _problem(CUT_P3)
    kap = kappa_numpy(CUT_P3)
    _, Ks = P.assemble_full_wq(kap)
    Kt = OT.assemble(P, lambda x: kap(x)[:, None, None] * np.eye(3)[None])
    assert np.abs(Kt - Ks).max() <= 1e-13 * np.abs(Ks).max()


@pytest.mark.parametrize("name", ["uncut5_p2", "uncut4_p4", "cut6_p3"])
def test_constant_tensor_matches_element_loop(name):
    """With a constant tensor every quadrature of the path is exact, so the weighted-quadrature
    matrix equals the conventional element loop (on cut elements both use the same rule)."""
    wl = {"uncut5_p2": W.custom(5, 2), "uncut4_p4": W.custom((4, 5, 4), 4), "cut6_p3": CUT_P3}[name]
    P = _problem(wl)
    C0 = W.constant_tensor(1)
    K = OT.assemble(P, _const(C0))
    Kg = OT.assemble_gauss(P, _const(C0))
    assert np.abs(K - Kg).max() <= 1e-13 * np.abs(Kg).max()
    if name == "cut6_p3":
        sp = [P.dom.split(tuple(int(v) for v in I)) for I in zip(*np.nonzero(P.dom.fcls == 2))]
        assert sum(s is not None for s in sp) > 0          # DWQ box rows take part


def test_variable_tensor_row_sums_vanish():
    """sum_J d_e B_J = 0 at every point, so every row of the stiffness sums to zero for any
    coefficient tensor (here the pull-back of the smooth map)."""
    P = _problem(CUT_P3)
    K = OT.assemble(P, W.map_tensor)
    rp = P.row_ptr()
    for r in range(len(rp) - 1):
        row = K[rp[r]:rp[r + 1]]
        assert abs(row.sum()) <= 1e-12 * np.abs(row).max()
