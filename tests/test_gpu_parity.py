"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same inputs.

Integer outputs (classification, pattern, splits, slot layout) must match exactly; values
use the row-scaled error max_I max_J |A_IJ - R_IJ| / max_J |R_IJ| and the Frobenius ratio,
with tolerances 1e-12 (FP64) and 2e-6 (FP32).
"""
import itertools

import numpy as np
import pytest
import torch

import oracle_pool
import workloads as W
from oracle.assemble import Problem, kappa_numpy
from oracle.domain import octree_points
from oracle.spline import gauss_legendre

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-12, torch.float32: 2e-6}
BALL = W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.4)
PLANE = W.LevelSet(W.LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6)
TORUS = W.LevelSet(W.LS_TORUS, c=(0.5, 0.5, 0.5), r0=0.3, r1=0.12)

SMALL = {
    "uncut4_p1": W.custom(4, 1, kappa="rf", seed=1),
    "uncut5_p3": W.custom((5, 4, 6), 3, kappa="rf", seed=2),
    "ball6_p2": W.custom(6, 2, BALL, kappa="sin3"),
    "plane6_p3": W.custom(6, 3, PLANE, kappa="rf", seed=3),
    "torus8_p2": W.custom(8, 2, TORUS, kappa="rf", seed=4),
    "ball5_p4": W.custom(5, 4, BALL, kappa="rf", seed=5),
}
# degrees 5 and 6 (general cut-element and row kernels)
HIGH = {
    "ball4_p5": W.custom(4, 5, BALL, kappa="rf", seed=6),
    "ball4_p6": W.custom(4, 6, BALL, kappa="rf", seed=6),
}


def rules_for(wl):
    from paper_2211_06427_amd import Rules
    return Rules.from_workload(wl)


def kappa_slots(rules, wl, dtype):
    """kappa at the library's slot coordinates (evaluated on the device by the input module)."""
    return W.kappa_at(wl, rules.kappa_xyz()).to(dtype=dtype)


def row_errors(got, ref, row_ptr):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    e_row = 0.0
    for r in range(len(row_ptr) - 1):
        s, t = row_ptr[r], row_ptr[r + 1]
        if t == s:
            continue
        scale = np.abs(ref[s:t]).max()
        if scale == 0.0:
            assert np.abs(got[s:t]).max() == 0.0
            continue
        e_row = max(e_row, np.abs(got[s:t] - ref[s:t]).max() / scale)
    e_f = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)
    return e_row, e_f


_ORACLE = {}


def oracle_full(name, wl):
    if name not in _ORACLE:
        P = Problem(wl)
        M, K = P.assemble_full_wq(kappa_numpy(wl))
        _ORACLE[name] = (P, M, K)
    return _ORACLE[name]


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(SMALL) + ["uncut8_p2", "ball16_p3"])
def test_structure_matches_oracle(name):
    wl = SMALL.get(name) or W.workload(name)
    print("case", name, flush=True)
    P = Problem(wl)
    R = rules_for(wl)
    dom = P.dom
    assert R.n_active == dom.n_active
    assert np.array_equal(R.elem_class().cpu().numpy(), dom.ecls.ravel())
    assert np.array_equal(R.fun_class().cpu().numpy(), dom.fcls.ravel())
    assert np.array_equal(R.active_to_lex().cpu().numpy(), dom.active_lex)
    assert np.array_equal(R.row_ptr().cpu().numpy(), P.row_ptr())
    assert np.array_equal(R.col_idx().cpu().numpy(), P.csr_cols())
    cut = np.nonzero(dom.fcls.ravel()[dom.active_lex] == 2)[0]
    assert np.array_equal(R.cut_rows().cpu().numpy(), cut)
    sp = R.split().cpu().numpy()
    n_split = 0
    for c, r in enumerate(cut):
        ref = dom.split(dom.unlex(dom.active_lex[r]))
        if ref is None:
            assert sp[c, 0] == -1
        else:
            n_split += 1
            assert (sp[c, 0], sp[c, 1], sp[c, 2]) == (ref[0], ref[1], int(ref[2]))
    assert R.n_rows_split == n_split
    assert R.n_rem_pairs == sum(len(P.remainder_elements(dom.unlex(dom.active_lex[r]))) for r in cut)
    sl = P.slots()
    assert R.n_grid == sl.n_grid
    assert np.array_equal(R.block_elems().cpu().numpy(),
                          np.array([(e[0] * dom.nel[1] + e[1]) * dom.nel[2] + e[2] for e in sl.Eg], dtype=np.int32))
    assert R.n_kappa == sl.n_slots
    xyz = R.kappa_xyz().cpu().numpy()
    assert np.abs(xyz - sl.coords()).max() <= 1e-15
    ow = R.octree_w().cpu().numpy()
    ref_w = np.concatenate([sl.octree(e)[1] for e in sl.cut]) if sl.cut else np.zeros(0)
    assert ow.shape == ref_w.shape
    assert np.abs(ow - ref_w).max(initial=0.0) <= 8e-15 * max(np.abs(ref_w).max(initial=0.0), 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", list(SMALL) + ["uncut8_p2", "ball16_p3"] + list(HIGH))
def test_forward_full_matrices(name, dtype):
    wl = SMALL.get(name) or HIGH.get(name) or W.workload(name)
    print("case", name, dtype, flush=True)
    P, Mr, Kr = oracle_full(name, wl)
    R = rules_for(wl)
    kap = kappa_slots(R, wl, dtype)
    vm, vk = R.assemble(kap)
    torch.cuda.synchronize()
    rp = P.row_ptr()
    em = row_errors(vm.cpu().numpy(), Mr, rp)
    ek = row_errors(vk.cpu().numpy(), Kr, rp)
    print(f"{name} {dtype}: mass e_row={em[0]:.2e} e_F={em[1]:.2e}  stiff e_row={ek[0]:.2e} e_F={ek[1]:.2e}")
    assert em[0] <= TOL[dtype] and ek[0] <= TOL[dtype]


@pytest.mark.parametrize("name", ["ball6_p2", "uncut5_p3"])
def test_which_subsets_and_determinism(name):
    """MASS-only / STIFF-only launches agree with the combined launch; the row kernels (no
    atomics) are bitwise deterministic, the cut part (atomics) agrees to rounding."""
    wl = SMALL[name]
    R = rules_for(wl)
    kap = kappa_slots(R, wl, torch.float64)
    vm, vk = R.assemble(kap)
    vm1, _ = R.assemble(kap, which=1)
    _, vk2 = R.assemble(kap, which=2)
    rm = [torch.empty_like(vm) for _ in range(2)]
    rk = [torch.empty_like(vk) for _ in range(2)]
    for i in range(2):
        R.assemble_rows(kap, rm[i], rk[i])
    torch.cuda.synchronize()
    assert torch.equal(rm[0], rm[1]) and torch.equal(rk[0], rk[1])
    # the whole assembly sums in a fixed order for p <= 4 (no atomics): bitwise repeatable
    if wl.degree <= 4:
        vm2, vk2 = R.assemble(kap)
        torch.cuda.synchronize()
        assert torch.equal(vm, vm2) and torch.equal(vk, vk2)
    assert float((vm - vm1).abs().max()) <= 1e-14 * float(vm.abs().max())
    assert float((vk - vk2).abs().max()) <= 1e-14 * float(vk.abs().max())
    # the cut part split into its remainder and octree calls equals the combined call
    from paper_2211_06427_amd._lib import WQ_CUT_OCTREE, WQ_CUT_REMAINDER
    pm, pk = torch.empty_like(vm), torch.empty_like(vk)
    R.assemble_rows(kap, pm, pk)
    R.cut_assemble(kap, pm, pk, parts=WQ_CUT_REMAINDER)
    R.cut_assemble(kap, pm, pk, parts=WQ_CUT_OCTREE)
    torch.cuda.synchronize()
    assert float((vm - pm).abs().max()) <= 1e-14 * float(vm.abs().max())
    assert float((vk - pk).abs().max()) <= 1e-14 * float(vk.abs().max())


_GAUSS = {}


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
@pytest.mark.parametrize("name", ["uncut4_p1", "ball6_p2", "plane6_p3", "torus8_p2", "ball5_p4", "ball4_p5"])
def test_gauss_assemble_matches_oracle(name, dtype):
    """Conventional element-by-element Gauss assembly against the oracle's element loop."""
    wl = SMALL.get(name) or HIGH[name]
    print("case gauss", name, dtype, flush=True)
    if name not in _GAUSS:
        P = Problem(wl)
        _GAUSS[name] = (P, P.assemble_full_gauss(kappa_numpy(wl)))
    P, (M, K) = _GAUSS[name]
    R = rules_for(wl)
    xg = R.gauss_coords()
    assert xg.shape == (R.n_gauss_elems * (wl.degree + 1) ** 3, 3)
    kg = W.kappa_at(wl, xg).to(dtype)
    vm, vk = R.gauss_assemble(kg, kappa_slots(R, wl, dtype))
    torch.cuda.synchronize()
    rp = P.row_ptr()
    em = row_errors(vm.cpu().numpy(), M, rp)
    ek = row_errors(vk.cpu().numpy(), K, rp)
    print(f"gauss {name} {dtype}: mass e_row={em[0]:.2e} stiff e_row={ek[0]:.2e}")
    assert em[0] <= TOL[dtype] and ek[0] <= TOL[dtype]


def test_gauss_equals_wq_for_unit_kappa():
    """kappa = 1: WQ is exact, so the WQ matrices equal the Gauss ones (uncut and cut, up to
    degree 6)."""
    for name in ("uncut5_p3", "ball6_p2", "ball4_p5", "ball4_p6"):
        wl = SMALL.get(name) or HIGH[name]
        R = rules_for(wl)
        one = torch.ones(R.n_kappa, dtype=torch.float64, device=R.device)
        og = torch.ones(R.n_gauss_elems * (wl.degree + 1) ** 3, dtype=torch.float64, device=R.device)
        vm, vk = R.assemble(one)
        gm, gk = R.gauss_assemble(og, one)
        torch.cuda.synchronize()
        assert float((vm - gm).abs().max()) <= 1e-12 * float(gm.abs().max())
        assert float((vk - gk).abs().max()) <= 1e-12 * float(gk.abs().max())


def _row_err(got, ref):
    """max |got - ref| / max |ref| over one row; a row that is zero in the reference (a cut
    row whose octree points all lie outside the domain) must be zero in both."""
    scale = np.abs(ref).max()
    if scale == 0.0:
        return 0.0 if np.abs(got).max() == 0.0 else np.inf
    return np.abs(got - ref).max() / scale


def _stratified_rows_check(R, wl, rows, tag):
    """The listed rows of the GPU matrices (FP64 and FP32) against the oracle row by row."""
    res = oracle_pool.rows(wl, rows)
    rp = R.row_ptr().cpu().numpy()
    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        torch.cuda.synchronize()
        vmh = vm.cpu().numpy(); vkh = vk.cpu().numpy()
        worst = 0.0
        for r, (pat, m, k) in zip(rows, res):
            s, t = rp[r], rp[r + 1]
            assert t - s == len(m)
            em = _row_err(vmh[s:t], m)
            ek = _row_err(vkh[s:t], k)
            worst = max(worst, em, ek)
            assert em <= TOL[dtype] and ek <= TOL[dtype], (tag, dtype, int(r), em, ek)
        print(f"  {tag} {dtype}: {len(rows)} rows, worst row-scaled error {worst:.2e}", flush=True)
        del vm, vk


def _line_rows(R, fc, lines):
    """Active indices of the interior rows along direction 1 at the given (i2, i3): whole
    runs, so every position of the interior kernel's line blocks (and both halves of an
    FP64 block) is covered."""
    n1, n2, n3 = R.nfun
    a2l = R.active_to_lex().cpu().numpy()
    lex2act = -np.ones(n1 * n2 * n3, dtype=np.int64)
    lex2act[a2l] = np.arange(len(a2l))
    out = []
    for i2, i3 in lines:
        for i1 in range(n1):
            a = lex2act[(i1 * n2 + i2) * n3 + i3]
            if a >= 0 and fc[a] == 1:
                out.append(int(a))
    return np.array(out, dtype=np.int64)


def _box_class_rows(R, cut, seed, per_class):
    """Cut rows with a DWQ box, up to per_class from every (direction, side) class present,
    and the rows without a box."""
    sp = R.split().cpu().numpy()
    picks = []
    classes = sorted({(int(d), int(h)) for d, _, h, _ in sp if d >= 0})
    for j, (d, h) in enumerate(classes):
        idx = np.nonzero((sp[:, 0] == d) & (sp[:, 2] == h))[0]
        picks.append(cut[idx[W.sample_indices(seed + j, len(idx), per_class)]])
    unboxed = np.nonzero(sp[:, 0] < 0)[0]
    picks.append(cut[unboxed[W.sample_indices(seed + 99, len(unboxed), per_class)]])
    return np.concatenate(picks), classes


def test_plane48_stratified_rows():
    """Full-size 48^3 p=4 plane cut: whole interior line runs (boundary and interior
    windows), 40 box rows of every (direction, side) class and 40 rows without a box,
    FP64 and FP32, against the oracle row by row."""
    wl = W.workload("plane48_p4")
    print("case plane48_p4 stratified", flush=True)
    R = rules_for(wl)
    assert R.n_active == 93558 and R.nnz == 58302298
    fc = R.fun_class().long()[R.active_to_lex().long()].cpu().numpy()
    cut = R.cut_rows().cpu().numpy()
    lines = _line_rows(R, fc, [(0, 0), (3, 7), (20, 10), (10, 30)])
    boxed, classes = _box_class_rows(R, cut, 32, 40)
    assert len(classes) == 3
    rows = np.concatenate([lines, boxed])
    assert len(rows) >= 300
    _stratified_rows_check(R, wl, rows, "plane48_p4")


def test_torus32_stratified_rows():
    """Full-size 32^3 p=3 torus: every interior row, 40 box rows of each of the six
    (direction, side) classes and 40 rows without a box, FP64 and FP32, against the oracle."""
    wl = W.workload("torus32_p3")
    print("case torus32_p3 stratified", flush=True)
    R = rules_for(wl)
    fc = R.fun_class().long()[R.active_to_lex().long()].cpu().numpy()
    cut = R.cut_rows().cpu().numpy()
    interior = np.nonzero(fc == 1)[0]
    boxed, classes = _box_class_rows(R, cut, 72, 40)
    assert len(classes) == 6
    rows = np.concatenate([interior, boxed])
    assert len(rows) >= 300
    _stratified_rows_check(R, wl, rows, "torus32_p3")


# Plane cuts whose DWQ box rows cover every (direction, side) class at every degree: with
# the normal (1, -1, 1) the domain lies on the low side of a break in directions 0 and 2 and
# on the high side in direction 1; with (-1, 1, -1) the reverse.  At p = 6 the octree stops
# at depth 2 to bound the oracle's time (depth 3 at p = 6 is covered by ball4_p6).
def _boxed_plane(p, sign):
    return W.custom(6, p, W.LevelSet(W.LS_PLANE, n=(sign, -sign, sign), r0=0.5 * sign), kappa="rf", seed=20 + p,
                    octree_levels=3 if p < 6 else 2)


BOXED = {f"plane6_p{p}_{'a' if s > 0 else 'b'}": (_boxed_plane(p, s), s) for p in range(1, 7) for s in (1.0, -1.0)}


@pytest.mark.parametrize("name", list(BOXED))
def test_box_rows_all_degrees(name):
    """Structure, whole matrices (FP64, FP32) and the adjoint (FP64) against the oracle on
    meshes whose box rows hold three (direction, side) classes each."""
    wl, sign = BOXED[name]
    print("case boxed", name, flush=True)
    R = rules_for(wl)
    P = Problem(wl)
    dom = P.dom
    assert R.n_rows_split > 0
    sp = R.split().cpu().numpy()
    want = {(0, 0), (1, 1), (2, 0)} if sign > 0 else {(0, 1), (1, 0), (2, 1)}
    assert {(int(d), int(h)) for d, _, h, _ in sp if d >= 0} == want
    assert np.array_equal(R.row_ptr().cpu().numpy(), P.row_ptr())
    assert np.array_equal(R.col_idx().cpu().numpy(), P.csr_cols())
    cut = R.cut_rows().cpu().numpy()
    for c, r in enumerate(cut):
        ref = dom.split(dom.unlex(dom.active_lex[r]))
        if ref is None:
            assert sp[c, 0] == -1
        else:
            assert tuple(int(v) for v in sp[c, :3]) == (ref[0], ref[1], int(ref[2])), (c, ref)
    M, K = oracle_pool.full_wq(wl, n_active=R.n_active)
    rp = R.row_ptr().cpu().numpy()
    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        torch.cuda.synchronize()
        em = row_errors(vm.cpu().numpy(), M, rp)
        ek = row_errors(vk.cpu().numpy(), K, rp)
        print(f"  {name} {dtype}: mass e_row={em[0]:.2e} stiff e_row={ek[0]:.2e}", flush=True)
        assert em[0] <= TOL[dtype] and ek[0] <= TOL[dtype]
    GM = W.random_values(131, R.nnz)
    GK = W.random_values(132, R.nnz)
    ref = oracle_pool.adjoint(wl, GM, GK)
    got = R.adjoint(torch.tensor(GM, device=R.device), torch.tensor(GK, device=R.device)).cpu().numpy()
    assert got.shape == ref.shape
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"  {name} adjoint: {err:.2e}", flush=True)
    assert err <= 1e-12


# Uncut meshes large enough for whole line blocks at degrees 5 and 6 (every row interior);
# the oracle's full assembly is too slow there, so rows are sampled across the line blocks.
BLOCKS = {
    "uncut_p5_blocks": W.custom((8, 9, 7), 5, kappa="rf", seed=9),
    "uncut_p6_blocks": W.custom((9, 8, 10), 6, kappa="rf", seed=8),
}


def _sampled_rows_check(R, P, rows, kap_fn, wl):
    res = P.assemble_rows(rows, kap_fn)
    rp = R.row_ptr().cpu().numpy()
    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        torch.cuda.synchronize()
        vmh = vm.cpu().numpy(); vkh = vk.cpu().numpy()
        for r, (pat, m, k) in zip(rows, res):
            s, t = rp[r], rp[r + 1]
            assert t - s == len(m)
            em = np.abs(vmh[s:t] - m).max() / np.abs(m).max()
            ek = np.abs(vkh[s:t] - k).max() / np.abs(k).max()
            assert em <= TOL[dtype] and ek <= TOL[dtype], (dtype, r, em, ek)
    return res


@pytest.mark.parametrize("name", list(BLOCKS))
def test_line_blocks_high_degree(name):
    """Degrees 5 and 6 with full line blocks: sampled rows (forward, FP64 and FP32) and the
    adjoint of a cotangent supported on those rows, against the oracle row by row."""
    wl = BLOCKS[name]
    print("case blocks", name, flush=True)
    R = rules_for(wl)
    P = Problem(wl)
    assert R.n_active == P.dom.n_active and R.n_rows_cut == 0
    n1, n2, n3 = R.nfun
    # first, last and middle rows of line blocks plus seeded picks
    lex = [(0, 0, 0), (n1 - 1, n2 - 1, n3 - 1), (n1 // 2, n2 // 2, n3 // 2), (n1 - 1, 0, n3 // 2),
           (wl.degree, n2 // 3, 1), (n1 // 2 + 1, n2 - 2, n3 - 1)]
    a2l = {int(v): i for i, v in enumerate(R.active_to_lex().cpu().numpy())}
    rows = [a2l[(i * n2 + j) * n3 + k] for i, j, k in lex]
    rows = np.unique(np.concatenate([rows, W.sample_indices(41, R.n_active, 8)]))
    kap_fn = kappa_numpy(wl)
    res = _sampled_rows_check(R, P, rows, kap_fn, wl)
    # adjoint restricted to the sampled rows
    rp = R.row_ptr().cpu().numpy()
    GM = np.zeros(R.nnz); GK = np.zeros(R.nnz)
    gm_rows, gk_rows = [], []
    for j, (r, (pat, m, k)) in enumerate(zip(rows, res)):
        g1 = W.random_values(200 + j, len(m)); g2 = W.random_values(300 + j, len(m))
        GM[rp[r]:rp[r + 1]] = g1; GK[rp[r]:rp[r + 1]] = g2
        gm_rows.append(g1); gk_rows.append(g2)
    ref = P.adjoint_rows(rows, gm_rows, gk_rows)
    dev = R.device
    got = R.adjoint(torch.tensor(GM, device=dev), torch.tensor(GK, device=dev)).cpu().numpy()
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), np.abs(got - ref).max() / np.abs(ref).max()


def test_ball64_p6_sampled_rows():
    """Full-size 64^3 p=6 ball: sampled rows of every class against the oracle row by row."""
    wl = W.workload("ball64_p6")
    print("case ball64_p6 sampled", flush=True)
    R = rules_for(wl)
    P = Problem(wl)
    dom = P.dom
    assert R.n_active == dom.n_active
    fc = dom.fcls.ravel()[dom.active_lex]
    cut = np.nonzero(fc == 2)[0]
    sp = R.split().cpu().numpy()
    interior = W.sample_indices(51, dom.n_active, 4000)
    interior = interior[fc[interior] == 1][:6]
    boxed = cut[sp[:, 0] >= 0][W.sample_indices(52, int((sp[:, 0] >= 0).sum()), 4)]
    unboxed = cut[sp[:, 0] < 0][W.sample_indices(53, int((sp[:, 0] < 0).sum()), 3)]
    _sampled_rows_check(R, P, np.concatenate([interior, boxed, unboxed]), kappa_numpy(wl), wl)
    # every row: FP32 against FP64 wherever FP32 can carry the row (row maximum at least
    # 2^-100, 26 bits above FP32's smallest normal; thinner slivers of the ball underflow)
    v64 = R.assemble(kappa_slots(R, wl, torch.float64))
    v32 = R.assemble(kappa_slots(R, wl, torch.float32))
    rp = R.row_ptr()
    rows = torch.repeat_interleave(torch.arange(R.n_active, device=rp.device), torch.diff(rp))
    for a, b in zip(v32, v64):
        d = torch.zeros(R.n_active, dtype=torch.float64, device=a.device)
        m = torch.zeros_like(d)
        d.scatter_reduce_(0, rows, (a.double() - b).abs(), "amax")
        m.scatter_reduce_(0, rows, b.abs(), "amax")
        ok = m >= 2.0 ** -100
        assert int(ok.sum()) >= 0.95 * R.n_active
        assert float((d[ok] / m[ok]).max()) <= TOL[torch.float32]


# ------------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["ball6_p2", "torus8_p2", "plane6_p3", "uncut5_p3", "ball5_p4", "ball4_p5", "ball4_p6"])
def test_adjoint_matches_oracle(name):
    wl = SMALL.get(name) or HIGH[name]
    print("case adjoint", name, flush=True)
    P = Problem(wl)
    R = rules_for(wl)
    nnz = R.nnz
    GM = W.random_values(101, nnz)
    GK = W.random_values(102, nnz)
    ref = P.adjoint(GM, GK)
    dev = R.device
    dk = R.adjoint(torch.tensor(GM, device=dev), torch.tensor(GK, device=dev))
    got = dk.cpu().numpy()
    scale = np.abs(ref).max()
    assert got.shape == ref.shape
    tol = 1e-12
    assert np.abs(got - ref).max() <= tol * scale, np.abs(got - ref).max() / scale
    # the same through autograd
    kap = kappa_slots(R, wl, torch.float64).requires_grad_(True)
    from paper_2211_06427_amd import WQAssemble
    vm, vk = WQAssemble.apply(kap, R)
    L = (vm * torch.tensor(GM, device=dev)).sum() + (vk * torch.tensor(GK, device=dev)).sum()
    L.backward()
    assert np.abs(kap.grad.cpu().numpy() - ref).max() <= tol * scale
    # linearity: <kappa, dL/dkappa> = L
    assert abs(float((kap.detach() * kap.grad).sum()) - float(L.detach())) <= 1e-11 * float(torch.abs(vm).sum() + torch.abs(vk).sum())


def test_ball64_p6_adjoint_directional():
    """Full size, 64^3 p=6: the adjoint at seeded grid, block and octree slots equals the
    exact directional derivative <G, A(e_s)> (A is linear in kappa), FP64."""
    wl = W.workload("ball64_p6")
    print("case ball64_p6 adjoint", flush=True)
    R = rules_for(wl)
    dev = R.device
    G = torch.tensor(W.random_values(61, R.nnz), device=dev)
    dk = R.adjoint(G, G).cpu().numpy()
    rng = np.random.default_rng(62)
    picks = np.concatenate([rng.choice(R.n_grid, 3, replace=False), R.n_grid + rng.choice(R.n_block, 3, replace=False),
                            R.n_grid + R.n_block + rng.choice(R.n_octree, 6, replace=False)])
    ks = torch.zeros(R.n_kappa, dtype=torch.float64, device=dev)
    for s in picks:
        ks.zero_()
        ks[int(s)] = 1.0
        ms, kss = R.assemble(ks)
        val = float((ms * G).sum() + (kss * G).sum())
        scale = float((ms.abs() * G.abs()).sum() + (kss.abs() * G.abs()).sum())
        assert abs(val - dk[s]) <= 1e-12 * scale + 1e-300, (s, val, dk[s], scale)
        del ms, kss


def test_adjoint_torus32_fd():
    """Torus 32^3 p=3, L = u^T A(kappa) v: finite differences at 50 seeded slots (steps 1e-6 and
    1e-2) and the exact directional derivative along each slot's unit vector."""
    wl = W.workload("torus32_p3")
    print("case torus32 fd", flush=True)
    R = rules_for(wl)
    dev = R.device
    u, v = W.uv_vectors(4, R.n_active)
    rp = R.row_ptr().cpu().numpy()
    cols = R.col_idx().cpu().numpy()
    rows = np.repeat(np.arange(R.n_active), np.diff(rp))
    G = torch.tensor(u[rows] * v[cols], device=dev)
    kap = kappa_slots(R, wl, torch.float64)
    dk = R.adjoint(G, G)
    torch.cuda.synchronize()

    def mats(k):
        return R.assemble(k)

    # stratified slots: grid, blocks, octree (only slots that carry weight)
    ow = R.octree_w().cpu().numpy()
    rng = np.random.default_rng(44)
    grid_used = np.nonzero(dk[:R.n_grid].cpu().numpy())[0]
    blk_used = R.n_grid + np.nonzero(dk[R.n_grid:R.n_grid + R.n_block].cpu().numpy())[0]
    oct_used = R.n_grid + R.n_block + np.nonzero(ow)[0]
    picks = np.concatenate([rng.choice(grid_used, 17, replace=False), rng.choice(blk_used, 17, replace=False),
                            rng.choice(oct_used, 16, replace=False)])
    dkh = dk.cpu().numpy()
    m0, k0 = mats(kap)
    # run-to-run noise of <G, A(kappa)> (the cut part adds with atomics)
    noise = 0.0
    for _ in range(3):
        m1, k1 = mats(kap)
        noise = max(noise, abs(float(((m1 - m0) * G).sum() + ((k1 - k0) * G).sum())))
    u_fp64 = np.finfo(np.float64).eps / 2
    for step, rel in ((1e-6, 1e-4), (1e-2, 1e-9)):
        for s in picks:
            kp = kap.clone(); kp[s] += step
            km = kap.clone(); km[s] -= step
            mp, kp_ = mats(kp)
            mm, km_ = mats(km)
            # L is linear in kappa: difference the matrices first, then contract with G.  With
            # no truncation error, the FD error is the rounding of the entries that the
            # perturbation changes (a few u of their magnitude each) over 2*step.
            fd = float(((mp - mm) * G).sum() + ((kp_ - km_) * G).sum()) / (2 * step)
            chg = (mp != mm) | (kp_ != km_)
            mag = float((G.abs() * (mp.abs() + mm.abs() + kp_.abs() + km_.abs()))[chg].sum())
            tol = rel * abs(dkh[s]) + (4 * u_fp64 * mag + 10 * noise) / (2 * step) + 1e-15 * np.abs(dkh).max()
            assert abs(fd - dkh[s]) <= tol, (step, s, fd, dkh[s], noise, mag)
    # exact directional derivative: A is linear in kappa, so A(e_s) (kappa = 1 at slot s,
    # 0 elsewhere) is dA/dkappa_s and <G, A(e_s)> must equal the adjoint at s
    for s in picks:
        ks = torch.zeros_like(kap)
        ks[s] = 1.0
        ms, kss = mats(ks)
        val = float((ms * G).sum() + (kss * G).sum())
        scale = float((ms.abs() * G.abs()).sum() + (kss.abs() * G.abs()).sum())
        assert abs(val - dkh[s]) <= 1e-12 * scale + 1e-300, (s, val, dkh[s], scale)


def _row_scaled(a, b, rp, rows_sel=None):
    """max over rows of max |a - b| / max |b| (b the reference), on the device."""
    n = len(rp) - 1
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device), torch.diff(rp))
    d = torch.zeros(n, dtype=torch.float64, device=a.device)
    m = torch.zeros_like(d)
    d.scatter_reduce_(0, rows, (a.double() - b.double()).abs(), "amax")
    m.scatter_reduce_(0, rows, b.double().abs(), "amax")
    ok = m >= 2.0 ** -100
    if rows_sel is not None:
        ok &= rows_sel
    return float((d[ok] / m[ok]).max())


FIT = {
    "ball6_p2_fit": W.with_cut_rule(SMALL["ball6_p2"], "fit"),
    "plane6_p3_fit": W.with_cut_rule(SMALL["plane6_p3"], "fit"),
    "ball5_p4_fit": W.with_cut_rule(SMALL["ball5_p4"], "fit"),
    "ball4_p5_fit": W.with_cut_rule(HIGH["ball4_p5"], "fit"),
}


@pytest.mark.parametrize("name", list(FIT))
def test_fitted_cut_rule_matches_oracle(name):
    """WQ_OPT_MOMENT_FIT: slot layout (NK^3 points per cut element), weights, matrices (FP64 and
    FP32) and the adjoint against the oracle's fitted rule."""
    wl = FIT[name]
    print("case fit", name, flush=True)
    R = rules_for(wl)
    P = Problem(wl)
    nk3 = (2 * wl.degree + 1) ** 3
    assert R.n_octree == R.n_cut_elems * nk3
    sl = P.slots()
    assert R.n_kappa == sl.n_slots
    assert np.abs(R.kappa_xyz().cpu().numpy() - sl.coords()).max() <= 1e-14
    # weights per cut element within 1e-13 of the element's octree weight sum (the Legendre
    # moments are sums of positive terms bounded by it)
    wg = R.octree_w().cpu().numpy().reshape(-1, nk3)
    for c, e in enumerate(sl.cut):
        vol = np.abs(octree_points(P.lines, P.dom.ls, e, sl.levels)[1]).sum()
        assert np.abs(wg[c] - sl.octree(e)[1]).max() <= 1e-13 * vol, (e, vol)
    M, K = oracle_pool.full_wq(wl, n_active=R.n_active)
    rp = P.row_ptr()
    # Rounding model of the fitted rule (the bar's scale).  (i) Its weights have both signs, so an
    # entry is a sum of terms that can be much larger than itself: scale |w| |kappa|.  (ii) A
    # weight is a linear map of the element's Legendre moments, which are sums of positive octree
    # weights; it is fixed to rounding relative to the element's Omega-volume vol_e spread over
    # the points like the Gauss weights: scale vol_e W_g / |e| |kappa|.  The row scale is the
    # largest of the row's maximum and the row maximum of the matrices with the weights
    # |w_g| + vol_e W_g / |e| on the cut elements and |kappa|.  (A perturbation of the weights by
    # 1e-16 vol_e alone moves row-scaled entries by up to 5e-9 on plane6_p3, by 4e-14 against
    # this scale.)
    Pa = Problem(wl)
    sla = Pa.slots(with_octree=False)
    nk = 2 * wl.degree + 1
    _, gwk = gauss_legendre(nk)
    gw3 = np.einsum("a,b,c->abc", gwk, gwk, gwk).ravel() / 8.0
    for e in sla.cut:
        xf, wf = sla.octree(e)
        vol = np.abs(octree_points(Pa.lines, Pa.dom.ls, e, sla.levels)[1]).sum()
        sla._oct[e] = (xf, np.abs(wf) + vol * gw3)
    kap_abs = kappa_numpy(wl)
    Ma, Ka = Pa.assemble_full_wq(lambda x: np.abs(kap_abs(x)))

    def scaled_err(got, ref, ref_abs):
        e = 0.0
        for r in range(len(rp) - 1):
            a, b = rp[r], rp[r + 1]
            if b > a:
                sc = max(np.abs(ref[a:b]).max(), np.abs(ref_abs[a:b]).max())
                if sc > 0:
                    e = max(e, np.abs(got[a:b] - ref[a:b]).max() / sc)
        return e

    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        em = scaled_err(vm.cpu().numpy(), M, Ma)
        ek = scaled_err(vk.cpu().numpy(), K, Ka)
        assert em <= TOL[dtype] and ek <= TOL[dtype], (dtype, em, ek)
        assert row_errors(vm.cpu().numpy(), M, rp)[1] <= TOL[dtype]
    GM = W.random_values(111, R.nnz)
    GK = W.random_values(112, R.nnz)
    ref = oracle_pool.adjoint(wl, GM, GK)
    got = R.adjoint(torch.tensor(GM, device=R.device), torch.tensor(GK, device=R.device)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_fitted_cut_rule_plane48():
    """48^3 p=4: with kappa = 1 the fitted rule gives the octree's matrices; with the random
    field the two differ only by the fitted rule's quadrature error on the cut elements."""
    wl = W.workload("plane48_p4")
    print("case fit plane48", flush=True)
    Ro = rules_for(wl)
    Rf = rules_for(W.with_cut_rule(wl, "fit"))
    assert Rf.n_octree == Rf.n_cut_elems * 9 ** 3 and Rf.n_octree * 10 < Ro.n_octree
    rp = Ro.row_ptr()
    one_o = torch.ones(Ro.n_kappa, dtype=torch.float64, device=Ro.device)
    one_f = torch.ones(Rf.n_kappa, dtype=torch.float64, device=Rf.device)
    # entrywise against the matrix maximum: a fitted weight is fixed only to rounding relative to
    # its element's Omega-volume, so rows that see a sliver of Omega carry errors large against
    # their own maximum (the small cases bound them against the rounding scale of the rule)
    for a, b in zip(Rf.assemble(one_f), Ro.assemble(one_o)):
        assert float((a - b).abs().max()) <= 1e-12 * float(b.abs().max())
        assert float((a - b).norm() / b.norm()) <= 1e-13
    fo = Ro.assemble(kappa_slots(Ro, wl, torch.float64))
    ff = Rf.assemble(kappa_slots(Rf, wl, torch.float64))
    for a, b in zip(ff, fo):
        assert float((a - b).norm() / b.norm()) <= 1e-3


@pytest.mark.parametrize("name", ["plane6_p3", "ball5_p4", "ball4_p6", "plane48_p4", "ball4_p2_o4", "plane6_p3_rows"])
def test_fused_assembly_bitwise(name):
    """wq_assemble (rows, remainder and the cut elements' element work on three streams, then
    the gather) equals wq_assemble_rows followed by cut_assemble, bitwise; also where it falls
    back to the two calls (octree depth 4) and with every row on the cut path (Gauss rows)."""
    print("case fused", name, flush=True)
    from paper_2211_06427_amd import Rules
    if name == "ball4_p2_o4":
        wl = W.custom(4, 2, BALL, kappa="rf", seed=7, octree_levels=4)
        R = rules_for(wl)
    elif name == "plane6_p3_rows":
        wl = SMALL["plane6_p3"]
        R = Rules.from_workload(wl, gauss_rows=True)
    else:
        wl = SMALL.get(name) or HIGH.get(name) or W.workload(name)
        R = rules_for(wl)
    for dtype in (torch.float64, torch.float32):
        k = kappa_slots(R, wl, dtype)
        a = [torch.full((R.nnz,), float("nan"), dtype=dtype, device=R.device) for _ in range(2)]
        b = [torch.empty(R.nnz, dtype=dtype, device=R.device) for _ in range(2)]
        R.assemble_fused(k, *a)
        R.assemble_rows(k, *b)
        R.cut_assemble(k, *b)
        m1 = torch.full((R.nnz,), float("nan"), dtype=dtype, device=R.device)
        R.assemble_fused(k, m1, None)                   # one matrix
        torch.cuda.synchronize()
        if name == "ball4_p2_o4":
            # deeper octrees add their leaves with atomics (order varies between calls)
            rp = R.row_ptr().cpu().numpy()
            for x, y in ((a[0], b[0]), (a[1], b[1]), (m1, b[0])):
                assert row_errors(x.cpu().numpy(), y.cpu().numpy(), rp)[0] <= TOL[dtype], dtype
        else:
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]), dtype
            assert torch.equal(m1, b[0])
        del a, b, m1


@pytest.mark.parametrize("name", ["plane6_p3", "ball4_p6", "plane48_p4"])
def test_cut_parts_in_one_call(name):
    """cut_assemble with both parts in one call (the remainder beside the octree moments and
    local rows on a second stream) equals the two parts called in turn, bitwise."""
    wl = SMALL.get(name) or HIGH.get(name) or W.workload(name)
    print("case cut one call", name, flush=True)
    from paper_2211_06427_amd._lib import WQ_CUT_OCTREE, WQ_CUT_REMAINDER
    R = rules_for(wl)
    for dtype in (torch.float64, torch.float32):
        k = kappa_slots(R, wl, dtype)
        a = [torch.empty(R.nnz, dtype=dtype, device=R.device) for _ in range(2)]
        b = [torch.empty(R.nnz, dtype=dtype, device=R.device) for _ in range(2)]
        R.assemble_rows(k, *a)
        R.cut_assemble(k, *a)
        R.assemble_rows(k, *b)
        R.cut_assemble(k, *b, parts=WQ_CUT_REMAINDER)
        R.cut_assemble(k, *b, parts=WQ_CUT_OCTREE)
        torch.cuda.synchronize()
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        del a, b


@pytest.mark.parametrize("name", ["ball6_p2", "plane6_p3", "ball5_p4", "ball4_p5", "plane48_p4"])
def test_gauss_rows_equal_conventional(name):
    """WQ_OPT_GAUSS_ROWS: every row by element Gauss with sum factorization (row-owned, no
    atomics, no weighted quadrature) gives the conventional element-by-element Gauss matrices
    (the same integrals summed in another order)."""
    wl = SMALL.get(name) or HIGH.get(name) or W.workload(name)
    print("case gauss_rows", name, flush=True)
    from paper_2211_06427_amd import Rules
    Rg = Rules.from_workload(wl, gauss_rows=True)
    Rc = rules_for(wl)
    assert Rg.n_rows_interior == 0 and Rg.n_line_blocks == 0 and Rg.n_rows_split == 0
    assert Rg.nnz == Rc.nnz and torch.equal(Rg.row_ptr(), Rc.row_ptr())
    rp = Rc.row_ptr()
    dtypes = (torch.float32,) if name == "plane48_p4" else (torch.float64, torch.float32)
    for dtype in dtypes:
        vm, vk = Rg.assemble(kappa_slots(Rg, wl, dtype))
        gm, gk = Rc.gauss_assemble(W.kappa_at(wl, Rc.gauss_coords()).to(dtype), kappa_slots(Rc, wl, dtype))
        torch.cuda.synchronize()
        assert _row_scaled(vm, gm, rp) <= TOL[dtype] and _row_scaled(vk, gk, rp) <= TOL[dtype]
        del vm, vk, gm, gk


# BF16x3 split products (hi*hi + hi*lo + lo*hi): each product within 3 * 2^-16 (4.6e-5) of
# the exact one relative to |a||b| (two 8-bit roundings per operand, the lo*lo term dropped);
# a row entry sums <= 4p such products, so the error relative to the row maximum stays near
# that figure unless the row cancels.  The experiment is reported (measured ~1e-5), not held
# to the FP32 bar; 1e-4 leaves a factor ~2 for cancellation in the stiffness rows.
BF3_TOL = 1e-4


@pytest.mark.parametrize("name", ["uncut5_p3", "plane6_p3", "ball5_p4", "uncut_p5_blocks", "uncut_p6_blocks"])
def test_bf16x3_rows(name):
    """BF16x3 experiment: interior rows against the FP64 oracle; cut rows and the cut part
    identical to the FP32 path (the split applies to the interior rows only)."""
    wl = SMALL.get(name) or BLOCKS[name]
    print("case bf16x3", name, flush=True)
    R = rules_for(wl)
    k32 = kappa_slots(R, wl, torch.float32)
    b3 = R.assemble(k32, bf16x3=True)
    f32 = R.assemble(k32)
    f64 = R.assemble(kappa_slots(R, wl, torch.float64))
    torch.cuda.synchronize()
    rp = R.row_ptr()
    fc = R.fun_class().long()[R.active_to_lex().long()]
    interior = fc == 1
    for a, f, r in zip(b3, f32, f64):
        if bool(interior.any()):
            e = _row_scaled(a, r, rp, interior)
            print(f"  bf16x3 interior row-scaled error vs FP64: {e:.3e}", flush=True)
            assert e <= BF3_TOL
        rows = torch.repeat_interleave(torch.arange(R.n_active, device=rp.device), torch.diff(rp))
        cut_entries = ~interior[rows]
        assert torch.equal(a[cut_entries], f[cut_entries])
    if name in SMALL:
        P, M, K = oracle_full(name, wl)
        rph = rp.cpu().numpy()
        for a, ref in zip(b3, (M, K)):
            e_row, _ = row_errors(a.cpu().numpy(), ref, rph)
            assert e_row <= BF3_TOL


def test_bf16x3_plane48():
    """BF16x3 experiment at 48^3 p=4: every interior row against FP64 (reported error)."""
    wl = W.workload("plane48_p4")
    print("case bf16x3 plane48_p4", flush=True)
    R = rules_for(wl)
    k64 = kappa_slots(R, wl, torch.float64)
    b3 = R.assemble(k64.float(), bf16x3=True)
    f64 = R.assemble(k64)
    rp = R.row_ptr()
    fc = R.fun_class().long()[R.active_to_lex().long()]
    for a, r in zip(b3, f64):
        e = _row_scaled(a, r, rp, fc == 1)
        print(f"  bf16x3 interior row-scaled error vs FP64: {e:.3e}", flush=True)
        assert e <= BF3_TOL


# ------------------------------------------------------------------------------------------
# Hybrid Gauss scheme (no DWQ boxes)
@pytest.mark.parametrize("name", ["ball6_p2", "plane6_p3", "torus8_p2", "ball5_p4"])
def test_hybrid_gauss_matches_oracle(name):
    wl = SMALL[name]
    print("case hybrid", name, flush=True)
    from paper_2211_06427_amd import Rules
    R = Rules.from_workload(wl, hybrid_gauss=True)
    P = Problem(wl, hybrid_gauss=True)
    assert R.n_rows_split == 0 and R.n_dwq_rules == 0
    assert np.array_equal(R.row_ptr().cpu().numpy(), P.row_ptr())
    assert R.n_rem_pairs == sum(len(P.remainder_elements(P.dom.unlex(k)))
                                for k in P.dom.active_lex if P.dom.fcls.ravel()[k] == 2)
    M, K = P.assemble_full_wq(kappa_numpy(wl))
    rp = R.row_ptr().cpu().numpy()
    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        torch.cuda.synchronize()
        for got, ref in ((vm, M), (vk, K)):
            e_row, e_f = row_errors(got.cpu().numpy(), ref, rp)
            assert e_row <= TOL[dtype] and e_f <= TOL[dtype], (dtype, e_row, e_f)
    GM = W.random_values(111, R.nnz)
    GK = W.random_values(112, R.nnz)
    ref = P.adjoint(GM, GK)
    got = R.adjoint(torch.tensor(GM, device=R.device), torch.tensor(GK, device=R.device)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_hybrid_gauss_plane48():
    """Full size, 48^3 p=4: Hybrid Gauss cut rows equal the conventional Gauss assembly's rows
    (the same integrals, element by element) and its interior rows equal the DWQ run's."""
    wl = W.workload("plane48_p4")
    print("case hybrid plane48_p4", flush=True)
    from paper_2211_06427_amd import Rules
    Rh = Rules.from_workload(wl, hybrid_gauss=True)
    Rd = rules_for(wl)
    assert Rh.n_rows_split == 0 and Rh.nnz == Rd.nnz and Rh.n_kappa == Rd.n_kappa
    rp = Rd.row_ptr()
    assert torch.equal(rp, Rh.row_ptr())
    k64 = kappa_slots(Rd, wl, torch.float64)
    assert torch.equal(Rh.kappa_xyz(), Rd.kappa_xyz())
    h = Rh.assemble(k64)
    d = Rd.assemble(k64)
    g = Rd.gauss_assemble(W.kappa_at(wl, Rd.gauss_coords()), k64)
    torch.cuda.synchronize()
    fc = Rd.fun_class().long()[Rd.active_to_lex().long()]
    rows = torch.repeat_interleave(torch.arange(Rd.n_active, device=rp.device), torch.diff(rp))
    cut_ent = (fc == 2)[rows]
    for a, b, c in zip(h, d, g):
        assert torch.equal(a[~cut_ent], b[~cut_ent])
        assert _row_scaled(a, c, rp, fc == 2) <= 1e-12
    del h, d, g


# ------------------------------------------------------------------------------------------
# octree depths other than 3: the moment form covers depths 0-3, deeper octrees take the
# direct per-point cut-element kernels (forward and adjoint)
DEPTHS = {
    "ball5_p2_L0": W.custom(5, 2, BALL, kappa="sin3", octree_levels=0),
    "ball5_p2_L1": W.custom(5, 2, BALL, kappa="sin3", octree_levels=1),
    "ball5_p2_L2": W.custom(5, 2, BALL, kappa="sin3", octree_levels=2),
    "ball5_p2_L4": W.custom(5, 2, BALL, kappa="sin3", octree_levels=4),
    "ball4_p4_L4": W.custom(4, 4, BALL, kappa="rf", seed=7, octree_levels=4),
    "ball4_p3_L5": W.custom(4, 3, BALL, kappa="rf", seed=7, octree_levels=5),
}


@pytest.mark.parametrize("name", list(DEPTHS))
def test_octree_depths_match_oracle(name):
    wl = DEPTHS[name]
    print("case depth", name, flush=True)
    R = rules_for(wl)
    P = Problem(wl)
    assert R.n_kappa == P.slots().n_slots
    ow = R.octree_w().cpu().numpy()
    sl = P.slots()
    ref_w = np.concatenate([sl.octree(e)[1] for e in sl.cut]) if sl.cut else np.zeros(0)
    assert np.abs(ow - ref_w).max(initial=0.0) <= 8e-15 * max(np.abs(ref_w).max(initial=0.0), 1e-300)
    M, K = P.assemble_full_wq(kappa_numpy(wl))
    rp = R.row_ptr().cpu().numpy()
    for dtype in (torch.float64, torch.float32):
        vm, vk = R.assemble(kappa_slots(R, wl, dtype))
        torch.cuda.synchronize()
        for got, ref in ((vm, M), (vk, K)):
            e_row, e_f = row_errors(got.cpu().numpy(), ref, rp)
            assert e_row <= TOL[dtype] and e_f <= TOL[dtype], (dtype, e_row, e_f)
    GM = W.random_values(121, R.nnz)
    GK = W.random_values(122, R.nnz)
    ref = P.adjoint(GM, GK)
    got = R.adjoint(torch.tensor(GM, device=R.device), torch.tensor(GK, device=R.device)).cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_errors_are_reported():
    from paper_2211_06427_amd import Rules, WqError
    with pytest.raises(WqError):
        Rules(4, 0)
    with pytest.raises(WqError):
        Rules(4, 7)
    R = Rules(3, 2)
    with pytest.raises(ValueError):
        R.assemble(torch.zeros(5, dtype=torch.float64, device=R.device))
    # the BF16x3 split is a forward-only experiment: the adjoint refuses it
    from paper_2211_06427_amd import _lib as L
    g = torch.zeros(R.nnz, dtype=torch.float32, device=R.device)
    dk = torch.zeros(R.n_kappa, dtype=torch.float32, device=R.device)
    st = L.load().wq_assemble_adjoint(R._h, L.WQ_BF16X3, L.WQ_MASS, g.data_ptr(), None, dk.data_ptr(), None)
    assert st == -5 and b"forward rows only" in L.load().wq_last_error()
