"""GPU parity of the L2 projection (Section 3.1 test setting, Section 3.2 accuracy): load
vector, extension operator, PCG solve and relative L2 error through the C ABI against the
FP64 oracle on the same inputs.

Bars: integer outputs of the extension (inner flags, array bases, column indices) exact;
E values, load vector and error sums within 1e-12 relative (FP64 sums in another order); the
PCG solution (relative residual 1e-13) leaves a residual below 1e-11 relative in the oracle's
system E^T M E c = E^T b, and its coefficients lie within cond(E^T M E) * 1e-11 of the
oracle's direct solve.
"""
import math

import numpy as np
import pytest
import torch

import oracle_pool
import workloads as W
from oracle.assemble import Problem
from oracle.projection import Projection

pytestmark = pytest.mark.gpu

BALL8_P2 = W.custom(8, 2, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.3))
CASES = {
    "ball8_p2": BALL8_P2,
    "paper4_p2": W.paper_plane(4, 2),
    "paper4_p3": W.paper_plane(4, 3),
    "paper8_p2": W.paper_plane(8, 2),
    "paper6_p4": W.paper_plane(6, 4),
    "paper6_p5": W.paper_plane(6, 5),
    "paper6_p6": W.paper_plane(6, 6),
}
F_OF = {"ball8_p2": "poly2_f"}


def _rules(wl):
    from paper_2211_06427_amd import Rules
    return Rules.from_workload(wl)


def _f_inputs(rules, f_name):
    f = W.FUNCTIONS[f_name]
    return f(rules.gauss_coords()), f(rules.kappa_xyz())


def _oracle(wl):
    P = Problem(wl)
    return P, Projection(P)


def _dense_E(ext, n_active):
    ptr = ext.e_ptr().cpu().numpy()
    col = ext.e_col().cpu().numpy()
    val = ext.e_val().cpu().numpy()
    E = np.zeros((n_active, ext.n_inner))
    for r in range(n_active):
        E[r, col[ptr[r]:ptr[r + 1]]] = val[ptr[r]:ptr[r + 1]]
    return E, ptr, col


@pytest.mark.parametrize("name", list(CASES))
def test_extension_matches_oracle(name):
    wl = CASES[name]
    rules = _rules(wl)
    ext = rules.extension()
    _, pr = _oracle(wl)
    inner = pr.inner_mask()
    got_inner = ext.inner_of_active().cpu().numpy()
    assert np.array_equal(got_inner >= 0, inner)
    assert np.array_equal(got_inner[inner], np.arange(int(inner.sum())))
    arrays = pr.arrays()
    outer = ext.outer_rows().cpu().numpy()
    assert list(outer) == sorted(arrays)
    base = ext.outer_base().cpu().numpy()
    assert [tuple(int(v) for v in b) for b in base] == [arrays[int(r)] for r in outer]
    E, ptr, col = _dense_E(ext, rules.n_active)
    Eo = pr.extension()
    for r in range(rules.n_active):                     # columns exact, ascending
        want = np.nonzero(Eo[r])[0] if inner[r] else None
        if want is not None:
            assert list(col[ptr[r]:ptr[r + 1]]) == list(want)
    assert np.abs(E - Eo).max() <= 1e-12 * max(1.0, np.abs(Eo).max())


@pytest.mark.parametrize("name", ["ball8_p2", "paper4_p3", "paper8_p2", "paper6_p4", "paper6_p5", "paper6_p6"])
def test_load_vector_matches_oracle(name):
    """Every row for p <= 4; at p = 5, 6 (the oracle's octree rows are slow) 24 cut rows and
    8 interior rows drawn with a fixed seed."""
    wl = CASES[name]
    f_name = F_OF.get(name, "target_f")
    rules = _rules(wl)
    _, f = _f_inputs(rules, f_name)
    b = rules.load_vector(f).cpu().numpy()
    if wl.degree <= 4:
        pick = np.arange(rules.n_active)
        bo = oracle_pool.load_vector(wl, f_name, rules.n_active)
    else:
        cut = set(int(v) for v in rules.cut_rows().cpu().numpy())
        rows_int = [r for r in range(rules.n_active) if r not in cut]
        rng = np.random.default_rng(wl.degree)
        pick = np.array(sorted(set(rng.choice(sorted(cut), 24, replace=False).tolist()
                                   + rng.choice(rows_int, 8, replace=False).tolist())))
        bo = oracle_pool.load_vector(wl, f_name, rows=pick)
    assert np.abs(b[pick] - bo[pick]).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("name", ["ball8_p2", "paper6_p5", "paper4_p6"])
def test_l2_error_matches_oracle(name):
    """Error sums of one seeded coefficient vector on both sides (every degree's kernel)."""
    wl = CASES.get(name) or W.paper_plane(4, 6)
    f_name = F_OF.get(name, "target_f")
    rules = _rules(wl)
    fg, f = _f_inputs(rules, f_name)
    u = W.random_values(17, rules.n_active)
    e2, f2 = rules.l2_error(torch.as_tensor(u, device=rules.device), fg, f)
    _, pr = _oracle(wl)
    e2o, f2o = pr.l2_error(u, W.FUNCTIONS[f_name])
    assert abs(f2 - f2o) <= 1e-12 * f2o
    assert abs(e2 - e2o) <= 1e-12 * e2o


@pytest.mark.parametrize("name", ["ball8_p2", "paper4_p2", "paper8_p2", "paper6_p4"])
def test_projection_and_error_match_oracle(name):
    wl = CASES[name]
    f_name = F_OF.get(name, "target_f")
    f_fn = W.FUNCTIONS[f_name]
    rules = _rules(wl)
    fg, f = _f_inputs(rules, f_name)
    M, _ = rules.assemble(torch.ones(rules.n_kappa, dtype=torch.float64, device=rules.device), which=1)
    ext = rules.extension()
    u, iters, rel = rules.project(ext, M, rules.load_vector(f), tol=1e-13, max_iter=20000)
    assert rel <= 1e-13 and iters > 0
    _, pr = _oracle(wl)
    Mo, _ = oracle_pool.full_wq(wl, n_active=rules.n_active)
    bo = oracle_pool.load_vector(wl, f_name, rules.n_active)
    uo = pr.solve(Mo, bo)
    ug = u.cpu().numpy()
    # the GPU solution solves the oracle's system to the PCG tolerance plus the 1e-12 parity of
    # M and b; its coefficients then sit within cond(E^T M E) times that of the direct solve
    E = pr.extension()
    Md = pr.dense_mass(Mo)
    A = E.T @ Md @ E
    rhs = E.T @ bo
    assert np.linalg.norm(E.T @ (Md @ ug - bo)) <= 1e-11 * np.linalg.norm(rhs)
    assert np.abs(ug - uo).max() <= np.linalg.cond(A) * 1e-11 * np.abs(uo).max()
    # error sums of one coefficient vector (the oracle's) on both sides
    e2, f2 = rules.l2_error(torch.as_tensor(uo, device=rules.device), fg, f)
    e2o, f2o = pr.l2_error(uo, f_fn)
    assert abs(f2 - f2o) <= 1e-12 * f2o
    assert abs(e2 - e2o) <= 1e-12 * f2o
    # end to end
    e2g, f2g = rules.l2_error(u, fg, f)
    assert abs(math.sqrt(e2g / f2g) - math.sqrt(e2o / f2o)) <= 1e-6 * math.sqrt(e2o / f2o) + 1e-13


@pytest.mark.parametrize("name", ["ball8_p2", "paper4_p2", "paper6_p4"])
def test_projection_exact_in_extended_space(name):
    """poly2_f has degree <= 2 in each variable and the extended space reproduces polynomials
    of degree p, so the projection returns it to rounding."""
    rules = _rules(CASES[name])
    fg, f = _f_inputs(rules, "poly2_f")
    M, _ = rules.assemble(torch.ones(rules.n_kappa, dtype=torch.float64, device=rules.device), which=1)
    u, _, _ = rules.project(rules.extension(), M, rules.load_vector(f), tol=1e-14, max_iter=20000)
    e2, f2 = rules.l2_error(u, fg, f)
    assert math.sqrt(e2 / f2) <= 1e-11


def test_projection_rate_on_gpu():
    """Order p+1 at p=3 on the paper's geometry: halving h from 1/4 to 1/8 of the box side
    divides the relative error by about 16."""
    errs = []
    for h in (8, 16):
        rules = _rules(W.paper_plane(h, 3))
        fg, f = _f_inputs(rules, "target_f")
        M, _ = rules.assemble(torch.ones(rules.n_kappa, dtype=torch.float64, device=rules.device), which=1)
        u, _, _ = rules.project(rules.extension(), M, rules.load_vector(f), tol=1e-12)
        e2, f2 = rules.l2_error(u, fg, f)
        errs.append(math.sqrt(e2 / f2))
    assert 8.0 <= errs[0] / errs[1] <= 32.0, errs


def test_paper32_p4_sampled():
    """The paper's geometry at h = 32, p = 4: array bases of every outer function exact against
    the oracle; sampled load-vector rows (interior and cut) within 1e-12; the solve converges."""
    wl = W.paper_plane(32, 4)
    rules = _rules(wl)
    ext = rules.extension()
    _, pr = _oracle(wl)
    arrays = pr.arrays()
    outer = ext.outer_rows().cpu().numpy()
    assert list(outer) == sorted(arrays)
    base = ext.outer_base().cpu().numpy()
    assert [tuple(int(v) for v in b) for b in base] == [arrays[int(r)] for r in outer]
    fg, f = _f_inputs(rules, "target_f")
    b = rules.load_vector(f).cpu().numpy()
    cut = set(int(v) for v in rules.cut_rows().cpu().numpy())
    rows_cut = sorted(cut)
    rows_int = [r for r in range(rules.n_active) if r not in cut]
    rng = np.random.default_rng(11)
    pick = sorted(set(rng.choice(rows_cut, 48, replace=False).tolist() + rng.choice(rows_int, 16, replace=False).tolist()))
    bo = oracle_pool.load_vector(wl, "target_f", rows=pick)
    scale = np.abs(b).max()
    assert np.abs(b[pick] - bo[pick]).max() <= 1e-12 * scale
    M, _ = rules.assemble(torch.ones(rules.n_kappa, dtype=torch.float64, device=rules.device), which=1)
    u, iters, rel = rules.project(ext, M, torch.as_tensor(b, device=rules.device), tol=1e-12)
    assert rel <= 1e-12
    e2, f2 = rules.l2_error(u, fg, f)
    assert math.sqrt(e2 / f2) < 1e-4


def test_projection_errors():
    from paper_2211_06427_amd import _lib as L
    # no interior element at all: no array for the outer functions
    rules = _rules(W.custom(4, 2, W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.2)))
    with pytest.raises(L.WqError) as ex:
        rules.extension()
    assert ex.value.code == -1 and "too coarse" in str(ex.value)
    # an extension of another handle
    r1, r2 = _rules(BALL8_P2), _rules(BALL8_P2)
    ext = r1.extension()
    M = torch.zeros(r2.nnz, dtype=torch.float64, device=r2.device)
    b = torch.zeros(r2.n_active, dtype=torch.float64, device=r2.device)
    with pytest.raises(L.WqError) as ex:
        r2.project(ext, M, b)
    assert ex.value.code == -1 and "another rules handle" in str(ex.value)
    with pytest.raises(L.WqError):
        r1.project(ext, M, b, tol=0.0)
