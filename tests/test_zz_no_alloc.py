"""The allocation-free cut assembly (fixed device scratch) against cut_assemble, through the
C ABI: two calls in a row, the second on a smaller mesh, FP64 at 1e-12 and FP32 at 2e-6 of
each matrix's largest entry (batches of cut elements add into a row in more than one pass,
so the summation order differs from the single-pass call)."""
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu

BALL = W.LevelSet(W.LS_BALL, c=(0.5, 0.5, 0.5), r0=0.4)
PLANE = W.LevelSet(W.LS_PLANE, n=(1.0, 1.0, 1.0), r0=1.6)


def _check(wl, dtype):
    from paper_2211_06427_amd import Rules
    R = Rules.from_workload(wl)
    print("case no-alloc", wl.name, wl.degree, dtype, R.n_cut_elems, "cut elements", flush=True)
    kap = W.kappa_at(wl, R.kappa_xyz()).to(dtype)
    ref_m = torch.empty(R.nnz, dtype=dtype, device=R.device)
    ref_k = torch.empty_like(ref_m)
    R.assemble_rows(kap, ref_m, ref_k)
    got_m, got_k = ref_m.clone(), ref_k.clone()
    R.cut_assemble(kap, ref_m, ref_k)
    R.cut_assemble_noalloc(kap, got_m, got_k)
    torch.cuda.synchronize()
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    for a, b in ((got_m, ref_m), (got_k, ref_k)):
        scale = float(b.abs().max())
        assert float((a - b).abs().max()) <= tol * scale
    return R


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32], ids=["f64", "f32"])
def test_noalloc_matches_cut_assemble(dtype):
    # a mesh large enough to need several batches of the fixed scratch, then a smaller one
    big = W.workload("plane48_p4")
    R = _check(big, dtype)
    per = (2 * 4 + 1) ** 3 + 5 * 2 * 25 * 125
    assert R.n_cut_elems * per * (8 if dtype == torch.float64 else 4) > (64 << 20)
    _check(W.custom(8, 3, BALL, kappa="rf", seed=3), dtype)


def test_noalloc_high_degree_and_repeat():
    _check(W.custom(6, 6, BALL, kappa="rf", seed=4), torch.float64)
    _check(W.custom(5, 5, PLANE, kappa="rf", seed=5), torch.float64)
