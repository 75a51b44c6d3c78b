"""Python face of libwqfd: rules handles, assembly calls and the autograd function.

PyTorch supplies device memory and the current stream; all computation happens in the HIP
library behind the C ABI of include/wqfd.h.
"""
from __future__ import annotations

import ctypes as C
import sys

import torch

from . import _lib as L

_DT = {torch.float64: L.WQ_F64, torch.float32: L.WQ_F32}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, n, dtype, device, name):
    if t is None:
        return
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and t.numel() == n and t.device == device):
        raise ValueError(f"{name}: expected a contiguous {dtype} tensor of {n} elements on {device}, "
                         f"got {tuple(t.shape)} {t.dtype} on {t.device}")


class Rules:
    """Kappa-independent data of one mesh + domain (built on the GPU, FP64)."""

    def __init__(self, nel, degree, levelset=None, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0), octree_levels=3,
                 device=None, hybrid_gauss=False, gauss_rows=False, cut_rule="octree", tensor=False):
        """hybrid_gauss=True: the Hybrid Gauss scheme (no DWQ boxes; the regular support of
        every cut row goes through element Gauss with sum factorization).  gauss_rows=True: no
        weighted quadrature; every row by element Gauss with sum factorization (the
        conventional Gauss matrices, row-owned and atomic-free; for comparison).  cut_rule="fit":
        cut elements by the rule fitted to the octree on (2p+1)^3 Gauss points per element.
        tensor=True: also build the mixed rule families of assemble_tensor (p <= 4)."""
        if cut_rule not in ("octree", "fit"):
            raise ValueError(f"cut_rule must be 'octree' or 'fit', got {cut_rule!r}")
        lib = L.load()
        if isinstance(nel, int):
            nel = (nel, nel, nel)
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        mesh = L.WqMesh((C.c_int32 * 3)(*nel), int(degree), (C.c_double * 3)(*lo), (C.c_double * 3)(*hi))
        ls = L.WqLevelset()
        if levelset is not None:
            ls.kind = int(levelset.kind)
            ls.c = (C.c_double * 3)(*levelset.c)
            ls.n = (C.c_double * 3)(*levelset.n)
            ls.r0, ls.r1 = float(levelset.r0), float(levelset.r1)
        opts = L.WqOptions(int(octree_levels), (L.WQ_OPT_HYBRID_GAUSS if hybrid_gauss else 0) |
                           (L.WQ_OPT_GAUSS_ROWS if gauss_rows else 0) |
                           (L.WQ_OPT_MOMENT_FIT if cut_rule == "fit" else 0) |
                           (L.WQ_OPT_TENSOR if tensor else 0))
        self.cut_rule = cut_rule
        self.hybrid_gauss = bool(hybrid_gauss)
        self.gauss_rows = bool(gauss_rows)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.wq_build_rules(C.byref(mesh), C.byref(ls), C.byref(opts),
                                       C.c_void_p(_stream_handle(self.device)), C.byref(h)))
        self._h = h
        self.degree = int(degree)
        self.nel = tuple(nel)
        info = L.WqRulesInfo()
        L.check(lib.wq_rules_info_get(h, C.byref(info)))
        self._info = info
        for k in ("n_active", "nnz", "n_rows_interior", "n_rows_cut", "n_rows_split", "n_dwq_rules", "n_kappa",
                  "n_grid", "n_block", "n_octree", "n_block_elems", "n_cut_elems", "n_cells", "n_line_blocks",
                  "n_oct_xgroups", "n_oct_columns", "n_rem_pairs", "n_gauss_elems"):
            setattr(self, k, int(getattr(info, k)))
        self.grid_dims = tuple(info.grid_dims)
        self.nfun = tuple(info.nfun)

    @classmethod
    def from_workload(cls, wl, device=None, hybrid_gauss=False, gauss_rows=False, tensor=False):
        return cls(wl.nel, wl.degree, wl.levelset, wl.lo, wl.hi, wl.octree_levels, device, hybrid_gauss, gauss_rows,
                   getattr(wl, "cut_rule", "octree"), tensor)

    def __del__(self):
        h = getattr(self, "_h", None)
        if sys.is_finalizing():
            return
        if h is not None and h.value:
            L.load().wq_rules_free(h)
            self._h = None

    # --- read-only views (copied into torch tensors) ---------------------------------
    def _view(self, field, n, dtype, shape=None, info=None):
        out = torch.empty(n, dtype=dtype, device=self.device)
        ptr = getattr(self._info if info is None else info, field)
        if n > 0:
            hip = L.hip_runtime()
            with torch.cuda.device(self.device):
                rc = hip.hipMemcpyAsync(C.c_void_p(out.data_ptr()), C.c_void_p(ptr), out.numel() * out.element_size(),
                                        3, C.c_void_p(_stream_handle(self.device)))
            if rc != 0:
                raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
        return out if shape is None else out.view(*shape)

    def row_ptr(self):
        return self._view("row_ptr", self.n_active + 1, torch.int64)

    def col_idx(self):
        return self._view("col_idx", self.nnz, torch.int32)

    def active_to_lex(self):
        return self._view("active_to_lex", self.n_active, torch.int32)

    def kappa_xyz(self):
        return self._view("kappa_xyz", 3 * self.n_kappa, torch.float64, (self.n_kappa, 3))

    def octree_w(self):
        return self._view("octree_w", self.n_octree, torch.float64)

    def block_elems(self):
        return self._view("block_elems", self.n_block_elems, torch.int32)

    def fun_class(self):
        return self._view("fun_class", self.nfun[0] * self.nfun[1] * self.nfun[2], torch.int8)

    def elem_class(self):
        return self._view("elem_class", self.nel[0] * self.nel[1] * self.nel[2], torch.int8)

    def split(self):
        return self._view("split", 4 * self.n_rows_cut, torch.int32, (self.n_rows_cut, 4))

    def cut_rows(self):
        return self._view("cut_rows", self.n_rows_cut, torch.int32)

    # --- assembly -----------------------------------------------------------------------
    def _call(self, fn, kappa, vm, vk, which, bf16x3=False):
        dtype = kappa.dtype
        if dtype not in _DT:
            raise ValueError(f"unsupported dtype {dtype}")
        if bf16x3 and dtype != torch.float32:
            raise ValueError("the BF16x3 split takes float32 kappa and values")
        _need(kappa, self.n_kappa, dtype, self.device, "kappa")
        _need(vm, self.nnz, dtype, self.device, "vals_mass")
        _need(vk, self.nnz, dtype, self.device, "vals_stiff")
        code = L.WQ_BF16X3 if bf16x3 else _DT[dtype]
        L.check(fn(self._h, code, int(which), _ptr(kappa), _ptr(vm), _ptr(vk),
                   C.c_void_p(_stream_handle(self.device))))

    def assemble_rows(self, kappa, vals_mass=None, vals_stiff=None, which=None, bf16x3=False):
        """Overwrites the values.  bf16x3=True (float32 only): the interior rows' direction-1
        contraction runs on matrix cores with bf16 hi/lo split operands (an experiment)."""
        which = which if which is not None else (L.WQ_MASS if vals_mass is not None else 0) | \
            (L.WQ_STIFF if vals_stiff is not None else 0)
        self._call(L.load().wq_assemble_rows, kappa, vals_mass, vals_stiff, which, bf16x3)

    def cut_assemble(self, kappa, vals_mass=None, vals_stiff=None, which=None, parts=0):
        """Accumulates the cut part; parts = WQ_CUT_REMAINDER and/or WQ_CUT_OCTREE (0: both)."""
        which = which if which is not None else (L.WQ_MASS if vals_mass is not None else 0) | \
            (L.WQ_STIFF if vals_stiff is not None else 0)
        self._call(L.load().cut_assemble, kappa, vals_mass, vals_stiff, which | parts)

    def cut_assemble_noalloc(self, kappa, vals_mass=None, vals_stiff=None, which=None, parts=0):
        """cut_assemble through the allocation-free entry point (fixed device scratch)."""
        which = which if which is not None else (L.WQ_MASS if vals_mass is not None else 0) | \
            (L.WQ_STIFF if vals_stiff is not None else 0)
        self._call(L.load().cut_assemble_noalloc, kappa, vals_mass, vals_stiff, which | parts)

    def assemble_fused(self, kappa, vals_mass=None, vals_stiff=None, which=None):
        """Rows and both cut parts in one call over three streams (wq_assemble); overwrites the
        values, bitwise equal to assemble_rows followed by cut_assemble."""
        which = which if which is not None else (L.WQ_MASS if vals_mass is not None else 0) | \
            (L.WQ_STIFF if vals_stiff is not None else 0)
        self._call(L.load().wq_assemble, kappa, vals_mass, vals_stiff, which)

    def assemble(self, kappa, which=L.WQ_MASS | L.WQ_STIFF, bf16x3=False):
        """Whole matrices: rows, then the cut part. Returns (M values or None, K values or None)."""
        vm = torch.empty(self.nnz, dtype=kappa.dtype, device=self.device) if which & L.WQ_MASS else None
        vk = torch.empty(self.nnz, dtype=kappa.dtype, device=self.device) if which & L.WQ_STIFF else None
        self.assemble_rows(kappa, vm, vk, which, bf16x3)
        self.cut_assemble(kappa, vm, vk, which)
        return vm, vk

    def assemble_tensor(self, coef, out=None):
        """Stiffness values with a full symmetric coefficient tensor: coef (6, n_kappa) components
        C11, C22, C33, C12, C13, C23 at the slots (float64 or float32)."""
        if coef.dim() != 2 or coef.shape[0] != 6 or coef.shape[1] != self.n_kappa or not coef.is_contiguous() or \
                coef.device != self.device or coef.dtype not in (torch.float64, torch.float32):
            raise ValueError(f"assemble_tensor: expected a contiguous (6, {self.n_kappa}) float tensor on {self.device}, "
                             f"got {tuple(coef.shape)} {coef.dtype} on {coef.device}")
        vk = torch.empty(self.nnz, dtype=coef.dtype, device=self.device) if out is None else out
        _need(vk, self.nnz, coef.dtype, self.device, "vals_stiff")
        L.check(L.load().wq_assemble_tensor(self._h, _DT[coef.dtype], _ptr(coef), _ptr(vk),
                                            C.c_void_p(_stream_handle(self.device))))
        return vk

    def gauss_coords(self):
        """(n_gauss_elems * (p+1)^3, 3) coordinates of the interior elements' Gauss points."""
        n = self.n_gauss_elems * (self.degree + 1) ** 3
        out = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if n > 0:
            with torch.cuda.device(self.device):
                L.check(L.load().wq_gauss_coords(self._h, C.c_void_p(out.data_ptr()),
                                                 C.c_void_p(_stream_handle(self.device))))
        return out

    def gauss_assemble(self, kappa_gauss, kappa, which=L.WQ_MASS | L.WQ_STIFF):
        """Conventional element-by-element Gauss assembly of the same matrices (comparison)."""
        dtype = kappa.dtype
        _need(kappa_gauss, self.n_gauss_elems * (self.degree + 1) ** 3, dtype, self.device, "kappa_gauss")
        _need(kappa, self.n_kappa, dtype, self.device, "kappa")
        vm = torch.empty(self.nnz, dtype=dtype, device=self.device) if which & L.WQ_MASS else None
        vk = torch.empty(self.nnz, dtype=dtype, device=self.device) if which & L.WQ_STIFF else None
        L.check(L.load().gauss_assemble(self._h, _DT[dtype], int(which), _ptr(kappa_gauss), _ptr(kappa), _ptr(vm),
                                        _ptr(vk), C.c_void_p(_stream_handle(self.device))))
        return vm, vk

    def adjoint(self, g_mass=None, g_stiff=None, out=None):
        """dL/dkappa over all slots for L = <G_mass, M> + <G_stiff, K>."""
        ref = g_mass if g_mass is not None else g_stiff
        which = (L.WQ_MASS if g_mass is not None else 0) | (L.WQ_STIFF if g_stiff is not None else 0)
        dk = torch.empty(self.n_kappa, dtype=ref.dtype, device=self.device) if out is None else out
        _need(dk, self.n_kappa, ref.dtype, self.device, "dkappa")
        _need(g_mass, self.nnz, ref.dtype, self.device, "G_mass")
        _need(g_stiff, self.nnz, ref.dtype, self.device, "G_stiff")
        L.check(L.load().wq_assemble_adjoint(self._h, _DT[ref.dtype], which, _ptr(g_mass), _ptr(g_stiff), _ptr(dk),
                                             C.c_void_p(_stream_handle(self.device))))
        return dk


    # --- L2 projection (FP64) --------------------------------------------------------------
    def load_vector(self, f):
        """b_I = sum_q W_I(q) f(x_q) over the mass row's points; f: (n_kappa) float64 slot values."""
        _need(f, self.n_kappa, torch.float64, self.device, "f")
        b = torch.empty(self.n_active, dtype=torch.float64, device=self.device)
        L.check(L.load().wq_load_vector(self._h, _ptr(f), _ptr(b), C.c_void_p(_stream_handle(self.device))))
        return b

    def extension(self):
        """The extended B-spline operator of this mesh and domain."""
        return Extension(self)

    def project(self, ext, vals_mass, b, tol=1e-12, max_iter=5000):
        """u = E c with E^T M E c = E^T b (Jacobi PCG). Returns (u, iterations, relative residual)."""
        _need(vals_mass, self.nnz, torch.float64, self.device, "vals_mass")
        _need(b, self.n_active, torch.float64, self.device, "b")
        u = torch.empty(self.n_active, dtype=torch.float64, device=self.device)
        it, rel = C.c_int32(0), C.c_double(0.0)
        L.check(L.load().wq_project(self._h, ext._h, _ptr(vals_mass), _ptr(b), _ptr(u), float(tol), int(max_iter),
                                    C.byref(it), C.byref(rel), C.c_void_p(_stream_handle(self.device))))
        return u, int(it.value), float(rel.value)

    def l2_error(self, u, f_gauss, f):
        """(sum w (u_h - f)^2, sum w f^2) over Omega: Gauss points of interior elements (f_gauss at
        gauss_coords()) and octree points of cut elements (f: slot values)."""
        _need(u, self.n_active, torch.float64, self.device, "u")
        _need(f, self.n_kappa, torch.float64, self.device, "f")
        if self.n_gauss_elems > 0:
            _need(f_gauss, self.n_gauss_elems * (self.degree + 1) ** 3, torch.float64, self.device, "f_gauss")
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        L.check(L.load().wq_l2_error(self._h, _ptr(u), _ptr(f_gauss), _ptr(f), _ptr(out),
                                     C.c_void_p(_stream_handle(self.device))))
        return float(out[0]), float(out[1])


class Extension:
    """Extended B-spline operator E of a Rules handle (device buffers owned by the library)."""

    def __init__(self, rules: Rules):
        lib = L.load()
        h = C.c_void_p()
        with torch.cuda.device(rules.device):
            L.check(lib.wq_extension_build(rules._h, C.c_void_p(_stream_handle(rules.device)), C.byref(h)))
        self._h = h
        self.rules = rules          # keeps the rules handle alive
        info = L.WqExtensionInfo()
        L.check(lib.wq_extension_info_get(h, C.byref(info)))
        self._info = info
        self.n_inner, self.n_outer, self.nnz_e = int(info.n_inner), int(info.n_outer), int(info.nnz_e)

    def __del__(self):
        h = getattr(self, "_h", None)
        if sys.is_finalizing():
            return
        if h is not None and h.value:
            L.load().wq_extension_free(h)
            self._h = None

    def _view(self, field, n, dtype, shape=None):
        return Rules._view(self.rules, field, n, dtype, shape, info=self._info)

    def inner_of_active(self):
        return self._view("inner_of_active", self.rules.n_active, torch.int32)

    def outer_rows(self):
        return self._view("outer_rows", self.n_outer, torch.int32)

    def outer_base(self):
        return self._view("outer_base", 3 * self.n_outer, torch.int32, (self.n_outer, 3))

    def e_ptr(self):
        return self._view("e_ptr", self.rules.n_active + 1, torch.int64)

    def e_col(self):
        return self._view("e_col", self.nnz_e, torch.int32)

    def e_val(self):
        return self._view("e_val", self.nnz_e, torch.float64)


class WQAssemble(torch.autograd.Function):
    """(M, K) = assembly(kappa); backward returns dL/dkappa through the adjoint kernels."""

    @staticmethod
    def forward(ctx, kappa, rules: Rules):
        vm, vk = rules.assemble(kappa.contiguous(), L.WQ_MASS | L.WQ_STIFF)
        ctx.rules = rules
        return vm, vk

    @staticmethod
    def backward(ctx, gm, gk):
        rules = ctx.rules
        gm = gm.contiguous() if gm is not None else None
        gk = gk.contiguous() if gk is not None else None
        return rules.adjoint(gm, gk), None
