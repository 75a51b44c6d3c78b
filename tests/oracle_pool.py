"""Runs the oracle's whole-matrix loops in worker processes (test helper).

The oracle's `assemble_full_wq` and `adjoint` take a share (k, n) of their row and element
loops; the shares sum to the whole result.  Workers are started with the "spawn" method, so
they hold no GPU state of the parent and run the oracle on the CPU only.  The pool size is
capped at 16 processes, each with single-threaded BLAS (the oracle's products are small).
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_CACHE = {}


_THREAD_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _workers(n_items: int) -> int:
    return max(1, min(16, os.cpu_count() or 1, n_items))


def _map(fn, jobs):
    """pool.map over spawned workers whose BLAS runs one thread each."""
    saved = {v: os.environ.get(v) for v in _THREAD_VARS}
    for v in _THREAD_VARS:
        os.environ[v] = "1"
    try:
        with mp.get_context("spawn").Pool(len(jobs)) as pool:
            return pool.map(fn, jobs)
    finally:
        for v, old in saved.items():
            if old is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = old


def _full_share(args):
    wl, hybrid, k, n = args
    from oracle.assemble import Problem, kappa_numpy
    return Problem(wl, hybrid_gauss=hybrid).assemble_full_wq(kappa_numpy(wl), share=(k, n))


def _adj_share(args):
    wl, hybrid, GM, GK, k, n = args
    from oracle.assemble import Problem
    return Problem(wl, hybrid_gauss=hybrid).adjoint(GM, GK, share=(k, n))


def full_wq(wl, hybrid=False, n_active=None):
    """(M, K) of the oracle for workload wl, computed over worker processes."""
    key = ("full", wl, hybrid)
    if key not in _CACHE:
        n = _workers(n_active or 64)
        if n == 1:
            _CACHE[key] = _full_share((wl, hybrid, 0, 1))
        else:
            parts = _map(_full_share, [(wl, hybrid, k, n) for k in range(n)])
            _CACHE[key] = (sum(p[0] for p in parts), sum(p[1] for p in parts))
    return _CACHE[key]


def adjoint(wl, GM, GK, hybrid=False):
    """dL/dkappa of the oracle for cotangents GM, GK, computed over worker processes."""
    n = _workers(64)
    if n == 1:
        return _adj_share((wl, hybrid, GM, GK, 0, 1))
    parts = _map(_adj_share, [(wl, hybrid, GM, GK, k, n) for k in range(n)])
    return np.sum(parts, axis=0)


def _rows_share(args):
    wl, hybrid, rows = args
    from oracle.assemble import Problem, kappa_numpy
    return Problem(wl, hybrid_gauss=hybrid).assemble_rows(rows, kappa_numpy(wl))


def rows(wl, rows_active, hybrid=False):
    """The oracle's rows (list of (pattern, M row, K row)) in the given order, computed over
    worker processes (each builds the workload's Problem once)."""
    rows_active = [int(r) for r in rows_active]
    n = _workers(max(1, len(rows_active) // 8))
    if n == 1:
        return _rows_share((wl, hybrid, rows_active))
    chunks = [rows_active[k::n] for k in range(n)]
    parts = _map(_rows_share, [(wl, hybrid, c) for c in chunks])
    out = [None] * len(rows_active)
    for k, part in enumerate(parts):
        for j, res in enumerate(part):
            out[k + j * n] = res
    return out


def _load_share(args):
    wl, f_name, k, n, rows = args
    from oracle.assemble import Problem
    from oracle.projection import Projection
    import workloads
    return Projection(Problem(wl)).load_vector(workloads.FUNCTIONS[f_name], share=(k, n), rows=rows)


def load_vector(wl, f_name, n_active=None, rows=None):
    """The oracle's load vector b for workload wl and the named function of
    workloads.FUNCTIONS, computed over worker processes (rows: only these active rows, the
    other entries zero)."""
    key = ("load", wl, f_name, None if rows is None else tuple(int(r) for r in rows))
    if key not in _CACHE:
        n_items = len(rows) if rows is not None else (n_active or 64)
        n = _workers(max(1, n_items // 32))
        if n == 1:
            _CACHE[key] = _load_share((wl, f_name, 0, 1, rows))
        else:
            _CACHE[key] = np.sum(_map(_load_share, [(wl, f_name, k, n, rows) for k in range(n)]), axis=0)
    return _CACHE[key]


def _tensor_share(args):
    wl, field, mag, k, n = args
    import numpy as np

    import workloads as W
    from oracle import tensor as OT
    from oracle.assemble import Problem
    from oracle.domain import octree_points
    from oracle.spline import gauss_legendre
    P = Problem(wl)
    C_fn = W.TENSOR_FIELDS[field] if isinstance(field, str) else (lambda x, C0=np.asarray(field): np.broadcast_to(C0, (x.shape[0], 3, 3)))
    if mag:
        # rounding scale of a fitted cut rule: |w_g| + vol_e W_g / |e| on the cut elements, |C|
        sl = P.slots(with_octree=False)
        if sl.fit:
            nk = 2 * wl.degree + 1
            _, gw = gauss_legendre(nk)
            gw3 = np.einsum("a,b,c->abc", gw, gw, gw).ravel() / 8.0
            for e in sl.cut:
                xf, wf = sl.octree(e)
                vol = np.abs(octree_points(P.lines, P.dom.ls, e, sl.levels)[1]).sum()
                sl._oct[e] = (xf, np.abs(wf) + vol * gw3)
        base = C_fn
        C_fn = lambda x: np.abs(base(x))
    return OT.assemble(P, C_fn, share=(k, n))


def tensor(wl, field, n_active=None, mag=False):
    """Oracle stiffness with a coefficient tensor: field is a name of workloads.TENSOR_FIELDS
    or a constant 3x3 tensor (as a tuple of tuples).  mag=True: the same sums with |C| and,
    for a fitted cut rule, the weights |w| + vol_e W_g / |e| (the rounding scale)."""
    key = ("tensor", wl, field, mag)
    if key not in _CACHE:
        n = _workers(n_active or 64)
        if n == 1:
            _CACHE[key] = _tensor_share((wl, field, mag, 0, 1))
        else:
            _CACHE[key] = sum(_map(_tensor_share, [(wl, field, mag, k, n) for k in range(n)]))
    return _CACHE[key]
