"""ctypes binding of libwqfd.so (argument marshalling only; every step runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwqfd.so")

WQ_F64, WQ_F32, WQ_BF16X3 = 0, 1, 2
WQ_OPT_HYBRID_GAUSS, WQ_OPT_GAUSS_ROWS, WQ_OPT_MOMENT_FIT, WQ_OPT_TENSOR = 1, 2, 4, 8
WQ_MASS, WQ_STIFF = 1, 2
WQ_CUT_REMAINDER, WQ_CUT_OCTREE = 4, 8
STATUS = {0: "WQ_OK", -1: "WQ_EINVAL", -2: "WQ_ENOMEM", -3: "WQ_EHIP", -4: "WQ_ESINGULAR", -5: "WQ_EUNSUPPORTED"}

EXPORTS = ["wq_build_rules", "wq_rules_info_get", "wq_assemble_rows", "cut_assemble", "wq_assemble_adjoint",
           "wq_rules_free", "wq_last_error", "gauss_assemble", "wq_gauss_coords", "cut_assemble_noalloc",
           "wq_load_vector", "wq_extension_build", "wq_extension_info_get", "wq_extension_free", "wq_project",
           "wq_l2_error", "wq_assemble_tensor", "wq_assemble"]


class WqMesh(C.Structure):
    _fields_ = [("nel", C.c_int32 * 3), ("degree", C.c_int32), ("lo", C.c_double * 3), ("hi", C.c_double * 3)]


class WqLevelset(C.Structure):
    _fields_ = [("kind", C.c_int32), ("c", C.c_double * 3), ("n", C.c_double * 3), ("r0", C.c_double),
                ("r1", C.c_double)]


class WqOptions(C.Structure):
    _fields_ = [("octree_levels", C.c_int32), ("flags", C.c_int32)]


class WqRulesInfo(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n_active", "nnz", "n_rows_interior", "n_rows_cut", "n_rows_split",
                                         "n_dwq_rules", "n_kappa", "n_grid", "n_block", "n_octree",
                                         "n_block_elems", "n_cut_elems", "n_cells", "n_line_blocks",
                                         "n_oct_xgroups", "n_oct_columns", "n_rem_pairs", "n_gauss_elems")] + [
        ("grid_dims", C.c_int32 * 3), ("nfun", C.c_int32 * 3),
        ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("active_to_lex", C.c_void_p),
        ("kappa_xyz", C.c_void_p), ("octree_w", C.c_void_p), ("block_elems", C.c_void_p),
        ("fun_class", C.c_void_p), ("elem_class", C.c_void_p), ("split", C.c_void_p), ("cut_rows", C.c_void_p)]


class WqExtensionInfo(C.Structure):
    _fields_ = [("n_inner", C.c_int64), ("n_outer", C.c_int64), ("nnz_e", C.c_int64),
                ("inner_of_active", C.c_void_p), ("outer_rows", C.c_void_p), ("outer_base", C.c_void_p),
                ("e_ptr", C.c_void_p), ("e_col", C.c_void_p), ("e_val", C.c_void_p)]


class WqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libwqfd.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libwqfd.so not found at {path}; build it with paper_2211_06427_amd/build.py")
    lib = C.CDLL(path)
    vp, i32, u32 = C.c_void_p, C.c_int, C.c_uint32
    lib.wq_build_rules.argtypes = [C.POINTER(WqMesh), C.POINTER(WqLevelset), C.POINTER(WqOptions), vp, C.POINTER(vp)]
    lib.wq_rules_info_get.argtypes = [vp, C.POINTER(WqRulesInfo)]
    for f in (lib.wq_assemble_rows, lib.cut_assemble, lib.cut_assemble_noalloc, lib.wq_assemble):
        f.argtypes = [vp, i32, u32, vp, vp, vp, vp]
    lib.wq_assemble_adjoint.argtypes = [vp, i32, u32, vp, vp, vp, vp]
    lib.gauss_assemble.argtypes = [vp, i32, u32, vp, vp, vp, vp, vp]
    lib.wq_gauss_coords.argtypes = [vp, vp, vp]
    lib.wq_assemble_tensor.argtypes = [vp, i32, vp, vp, vp]
    lib.wq_load_vector.argtypes = [vp, vp, vp, vp]
    lib.wq_extension_build.argtypes = [vp, vp, C.POINTER(vp)]
    lib.wq_extension_info_get.argtypes = [vp, C.POINTER(WqExtensionInfo)]
    lib.wq_extension_free.argtypes = [vp]
    lib.wq_extension_free.restype = None
    lib.wq_project.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_int32),
                               C.POINTER(C.c_double), vp]
    lib.wq_l2_error.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.wq_rules_free.argtypes = [vp]
    lib.wq_rules_free.restype = None
    lib.wq_last_error.restype = C.c_char_p
    for name in ("wq_build_rules", "wq_rules_info_get", "wq_assemble_rows", "cut_assemble", "wq_assemble_adjoint",
                 "cut_assemble_noalloc", "gauss_assemble", "wq_gauss_coords", "wq_load_vector", "wq_extension_build",
                 "wq_extension_info_get", "wq_project", "wq_l2_error", "wq_assemble_tensor", "wq_assemble"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def check(code: int):
    if code != 0:
        raise WqError(code, _lib.wq_last_error().decode())


_hip = None


def hip_runtime():
    """libamdhip64 (already loaded by torch on ROCm) for device-to-device copies of views."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
        _hip.hipMemcpyAsync.restype = C.c_int
    return _hip
