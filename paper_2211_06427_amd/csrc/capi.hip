// C ABI of libwqfd: argument validation, dispatch by dtype, error reporting.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "rows.h"

static thread_local char g_err[1024] = "";

int wq_set_error(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

static int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wq_set_error(WQ_EHIP, "%s: kernel launch failed: %s", what, hipGetErrorString(e));
    return WQ_OK;
}

static int check_values(const wq_rules* r, int dtype, uint32_t which, const void* kappa, const void* a,
                        const void* b, const char* what, uint32_t extra_bits = 0) {
    if (!r) return wq_set_error(WQ_EINVAL, "%s: rules handle is NULL", what);
    if (dtype != WQ_F64 && dtype != WQ_F32 && dtype != WQ_BF16X3)
        return wq_set_error(WQ_EINVAL, "%s: unknown dtype %d", what, dtype);
    if ((which & 3u) == 0 || (which & ~(3u | extra_bits)))
        return wq_set_error(WQ_EINVAL, "%s: which must hold a non-empty subset of MASS|STIFF%s", what,
                            extra_bits ? " (plus optional part bits)" : "");
    if (!kappa) return wq_set_error(WQ_EINVAL, "%s: kappa is NULL", what);
    if ((which & WQ_MASS) && !a) return wq_set_error(WQ_EINVAL, "%s: mass output requested but pointer is NULL", what);
    if ((which & WQ_STIFF) && !b) return wq_set_error(WQ_EINVAL, "%s: stiffness output requested but pointer is NULL", what);
    return WQ_OK;
}

// Device scratch of the allocation-free cut assembly: a fixed array, one copy on every device
// the library runs on (held until the process ends).  Host code never uses the array's name
// as an address: the device address comes from hipGetSymbolAddress, once per device, with
// that device current.
static constexpr size_t WQ_NOALLOC_SCRATCH_BYTES = (size_t)64 << 20;
static constexpr int WQ_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[WQ_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[WQ_MAX_DEVICES] = {};

static int scratch_address(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return wq_set_error(WQ_EHIP, "cut_assemble_noalloc: hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= WQ_MAX_DEVICES)
        return wq_set_error(WQ_EUNSUPPORTED, "cut_assemble_noalloc: device %d beyond the supported %d", dev,
                            WQ_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return wq_set_error(WQ_EHIP, "cut_assemble_noalloc: device address of the scratch array: %s",
                                hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WQ_OK;
}

// rows + both cut parts over three streams (see wq_assemble in the header)
template <typename T>
static int assemble_fused(const wq_rules* r, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const size_t bytes = cut_fused_scratch_bytes<T>(r);
    if (bytes == 0 || !r->side || !r->side2 || !r->ev_join2) {
        launch_rows<T>(r, which, kappa, vm, vk, s);
        return launch_cut<T>(r, which, WQ_CUT_REMAINDER | WQ_CUT_OCTREE, kappa, vm, vk, s);
    }
    void* scratch = nullptr;
    hipError_t err = r->scratch_alloc(&scratch, bytes, s);
    if (err != hipSuccess)
        return wq_set_error(WQ_ENOMEM, "wq_assemble: scratch allocation failed: %s", hipGetErrorString(err));
    int st = WQ_OK;
    {
        std::lock_guard<std::mutex> lock(*r->side_mu);
        const bool forked = hipEventRecord(r->ev_fork, s) == hipSuccess &&
                            hipStreamWaitEvent(r->side, r->ev_fork, 0) == hipSuccess &&
                            hipStreamWaitEvent(r->side2, r->ev_fork, 0) == hipSuccess;
        if (!forked) {
            (void)hipGetLastError();
            launch_rows_split<T>(r, which, kappa, vm, vk, s, s);
            st = launch_cut_prep<T>(r, which, kappa, vm, vk, s, s, scratch);
        } else {
            // interior rows on s; cut rows then the remainder on side; moments and local rows on side2
            launch_rows_split<T>(r, which, kappa, vm, vk, s, r->side);
            st = launch_cut_prep<T>(r, which, kappa, vm, vk, r->side, r->side2, scratch);
            if (hipEventRecord(r->ev_join, r->side) != hipSuccess || hipEventRecord(r->ev_join2, r->side2) != hipSuccess ||
                hipStreamWaitEvent(s, r->ev_join, 0) != hipSuccess || hipStreamWaitEvent(s, r->ev_join2, 0) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipStreamSynchronize(r->side);     // the join failed: finish the side streams' work here
                (void)hipStreamSynchronize(r->side2);
            }
        }
    }
    if (st == WQ_OK) launch_cut_finish<T>(r, which, scratch, vm, vk, s);
    err = hipFreeAsync(scratch, s);
    if (st) return st;
    if (err != hipSuccess) return wq_set_error(WQ_EHIP, "wq_assemble: scratch release failed: %s", hipGetErrorString(err));
    return WQ_OK;
}

extern "C" {

const char* wq_last_error(void) { return g_err; }

int wq_build_rules(const wq_mesh* mesh, const wq_levelset* ls, const wq_options* opts, void* stream, wq_rules** out) {
    if (!mesh || !ls || !out) return wq_set_error(WQ_EINVAL, "wq_build_rules: mesh, levelset and out must be non-NULL");
    *out = nullptr;
    if (mesh->degree < 1) return wq_set_error(WQ_EINVAL, "wq_build_rules: degree must be >= 1 (got %d)", mesh->degree);
    if (mesh->degree > WQ_PMAX)
        return wq_set_error(WQ_EUNSUPPORTED, "wq_build_rules: degree %d exceeds the supported maximum %d", mesh->degree, WQ_PMAX);
    int64_t nf = 1, ne = 1;
    for (int d = 0; d < 3; ++d) {
        if (mesh->nel[d] < 1) return wq_set_error(WQ_EINVAL, "wq_build_rules: nel[%d] must be >= 1", d);
        if (!(std::isfinite(mesh->lo[d]) && std::isfinite(mesh->hi[d]) && mesh->lo[d] < mesh->hi[d]))
            return wq_set_error(WQ_EINVAL, "wq_build_rules: need finite lo[%d] < hi[%d]", d, d);
        ne *= mesh->nel[d];
        nf *= mesh->nel[d] + mesh->degree;
    }
    if (nf >= ((int64_t)1 << 31) || ne >= ((int64_t)1 << 31))
        return wq_set_error(WQ_EUNSUPPORTED, "wq_build_rules: mesh too large for 32-bit function indices");
    if (ls->kind < 0 || ls->kind > 3) return wq_set_error(WQ_EINVAL, "wq_build_rules: unknown level-set kind %d", ls->kind);
    if (ls->kind == 1 && !(ls->n[0] != 0 || ls->n[1] != 0 || ls->n[2] != 0))
        return wq_set_error(WQ_EINVAL, "wq_build_rules: plane normal is zero");
    if (ls->kind == 2 && !(ls->r0 > 0)) return wq_set_error(WQ_EINVAL, "wq_build_rules: ball radius must be > 0");
    if (ls->kind == 3 && !(ls->r1 > 0 && ls->r0 > 0)) return wq_set_error(WQ_EINVAL, "wq_build_rules: torus radii must be > 0");
    wq_options o = {3, 0};
    if (opts) o = *opts;
    if (o.octree_levels < 0 || o.octree_levels > 5)
        return wq_set_error(WQ_EINVAL, "wq_build_rules: octree_levels must be in 0..5 (got %d)", o.octree_levels);
    if (o.flags & ~(WQ_OPT_HYBRID_GAUSS | WQ_OPT_GAUSS_ROWS | WQ_OPT_MOMENT_FIT | WQ_OPT_TENSOR))
        return wq_set_error(WQ_EINVAL, "wq_build_rules: unknown option flags 0x%x", o.flags);
    if ((o.flags & WQ_OPT_TENSOR) && mesh->degree > 4)
        return wq_set_error(WQ_EUNSUPPORTED, "wq_build_rules: the coefficient-tensor stiffness supports degrees 1..4 (got %d)",
                            mesh->degree);
    if ((o.flags & WQ_OPT_MOMENT_FIT) && o.octree_levels > 3)
        return wq_set_error(WQ_EUNSUPPORTED, "wq_build_rules: the fitted cut rule needs octree_levels <= 3 (got %d)",
                            o.octree_levels);
    return build_rules(mesh, ls, &o, (hipStream_t)stream, out);
}

int wq_rules_info_get(const wq_rules* r, wq_rules_info* out) {
    if (!r || !out) return wq_set_error(WQ_EINVAL, "wq_rules_info_get: NULL argument");
    memset(out, 0, sizeof(*out));
    const DevRules& R = r->R;
    out->n_active = r->n_active;
    out->nnz = r->nnz;
    out->n_rows_interior = r->n_interior_rows;
    out->n_rows_cut = r->n_cut;
    out->n_rows_split = r->n_split;
    out->n_dwq_rules = r->n_dwq;
    out->n_kappa = R.n_kappa;
    out->n_grid = R.n_grid;
    out->n_block = R.n_block;
    out->n_octree = r->n_oct;
    out->n_block_elems = r->n_block_elems;
    out->n_cut_elems = R.n_cut_elems;
    out->n_cells = R.n_cells;
    out->n_line_blocks = R.n_lblocks;
    out->n_oct_xgroups = r->n_oct_xgroups;
    out->n_oct_columns = r->n_oct_columns;
    out->n_rem_pairs = r->n_rem_pairs;
    out->n_gauss_elems = r->n_int_elems;
    for (int d = 0; d < 3; ++d) { out->grid_dims[d] = R.nx[d]; out->nfun[d] = R.nfun[d]; }
    out->row_ptr = R.row_ptr;
    out->col_idx = R.col_idx;
    out->active_to_lex = R.act2lex;
    out->kappa_xyz = r->kappa_xyz;
    out->octree_w = R.oct_w;
    out->block_elems = r->block_elems;
    out->fun_class = R.fcls;
    out->elem_class = R.ecls;
    out->split = (const int32_t*)R.split;
    out->cut_rows = R.cut_rows;
    return WQ_OK;
}

int wq_assemble_rows(const wq_rules* r, int dtype, uint32_t which, const void* kappa, void* vm, void* vk, void* stream) {
    int st = check_values(r, dtype, which, kappa, vm, vk, "wq_assemble_rows");
    if (st) return st;
    if (r->nnz == 0) return WQ_OK;
    if (dtype == WQ_F64)
        launch_rows<double>(r, which, (const double*)kappa, (double*)vm, (double*)vk, (hipStream_t)stream);
    else if (dtype == WQ_BF16X3)
        launch_rows_bf16x3(r, which, (const float*)kappa, (float*)vm, (float*)vk, (hipStream_t)stream);
    else
        launch_rows<float>(r, which, (const float*)kappa, (float*)vm, (float*)vk, (hipStream_t)stream);
    return check_launch("wq_assemble_rows");
}

int cut_assemble(const wq_rules* r, int dtype, uint32_t which, const void* kappa, void* vm, void* vk, void* stream) {
    int st = check_values(r, dtype, which, kappa, vm, vk, "cut_assemble", WQ_CUT_REMAINDER | WQ_CUT_OCTREE);
    if (st) return st;
    if (r->nnz == 0) return WQ_OK;
    uint32_t parts = which & (WQ_CUT_REMAINDER | WQ_CUT_OCTREE);
    if (parts == 0) parts = WQ_CUT_REMAINDER | WQ_CUT_OCTREE;
    if (dtype == WQ_F64)
        st = launch_cut<double>(r, which & 3u, parts, (const double*)kappa, (double*)vm, (double*)vk, (hipStream_t)stream);
    else
        st = launch_cut<float>(r, which & 3u, parts, (const float*)kappa, (float*)vm, (float*)vk, (hipStream_t)stream);
    if (st) return st;
    return check_launch("cut_assemble");
}

int cut_assemble_noalloc(const wq_rules* r, int dtype, uint32_t which, const void* kappa, void* vm, void* vk,
                         void* stream) {
    int st = check_values(r, dtype, which, kappa, vm, vk, "cut_assemble_noalloc", WQ_CUT_REMAINDER | WQ_CUT_OCTREE);
    if (st) return st;
    if (r->nnz == 0) return WQ_OK;
    void* buf = nullptr;
    st = scratch_address(&buf);
    if (st) return st;
    uint32_t parts = which & (WQ_CUT_REMAINDER | WQ_CUT_OCTREE);
    if (parts == 0) parts = WQ_CUT_REMAINDER | WQ_CUT_OCTREE;
    if (dtype == WQ_F64)
        st = launch_cut<double>(r, which & 3u, parts, (const double*)kappa, (double*)vm, (double*)vk, (hipStream_t)stream,
                                buf, WQ_NOALLOC_SCRATCH_BYTES);
    else
        st = launch_cut<float>(r, which & 3u, parts, (const float*)kappa, (float*)vm, (float*)vk, (hipStream_t)stream,
                               buf, WQ_NOALLOC_SCRATCH_BYTES);
    if (st) return st;
    return check_launch("cut_assemble_noalloc");
}

int wq_assemble_adjoint(const wq_rules* r, int dtype, uint32_t which, const void* gm, const void* gk, void* dk,
                        void* stream) {
    int st = check_values(r, dtype, which, dk, gm, gk, "wq_assemble_adjoint");
    if (st) return st;
    if (dtype == WQ_BF16X3)
        return wq_set_error(WQ_EUNSUPPORTED, "wq_assemble_adjoint: the BF16x3 split covers the forward rows only");
    if (dtype == WQ_F64)
        st = launch_adjoint<double>(r, which, (const double*)gm, (const double*)gk, (double*)dk, (hipStream_t)stream);
    else
        st = launch_adjoint<float>(r, which, (const float*)gm, (const float*)gk, (float*)dk, (hipStream_t)stream);
    if (st) return st;
    return check_launch("wq_assemble_adjoint");
}

int wq_assemble(const wq_rules* r, int dtype, uint32_t which, const void* kappa, void* vm, void* vk, void* stream) {
    int st = check_values(r, dtype, which, kappa, vm, vk, "wq_assemble");
    if (st) return st;
    if (dtype == WQ_BF16X3) return wq_set_error(WQ_EUNSUPPORTED, "wq_assemble: dtype must be F64 or F32");
    if (r->nnz == 0) return WQ_OK;
    st = dtype == WQ_F64 ? assemble_fused<double>(r, which, (const double*)kappa, (double*)vm, (double*)vk, (hipStream_t)stream)
                         : assemble_fused<float>(r, which, (const float*)kappa, (float*)vm, (float*)vk, (hipStream_t)stream);
    if (st) return st;
    return check_launch("wq_assemble");
}

int wq_assemble_tensor(const wq_rules* r, int dtype, const void* C, void* vals_stiff, void* stream) {
    if (!r) return wq_set_error(WQ_EINVAL, "wq_assemble_tensor: rules handle is NULL");
    if (dtype != WQ_F64 && dtype != WQ_F32) return wq_set_error(WQ_EINVAL, "wq_assemble_tensor: dtype must be F64 or F32");
    if (!C || !vals_stiff) return wq_set_error(WQ_EINVAL, "wq_assemble_tensor: NULL argument");
    if (!r->R.tensor)
        return wq_set_error(WQ_EINVAL, "wq_assemble_tensor: the rules were built without WQ_OPT_TENSOR");
    if (r->nnz == 0) return WQ_OK;
    int st = dtype == WQ_F64 ? launch_tensor<double>(r, (const double*)C, (double*)vals_stiff, (hipStream_t)stream)
                             : launch_tensor<float>(r, (const float*)C, (float*)vals_stiff, (hipStream_t)stream);
    if (st == WQ_EUNSUPPORTED) return wq_set_error(st, "wq_assemble_tensor: unsupported degree %d", r->R.p);
    if (st) return st;                                  // the message is set where the error arose
    return check_launch("wq_assemble_tensor");
}

int wq_gauss_coords(const wq_rules* r, double* xyz, void* stream) {
    if (!r || !xyz) return wq_set_error(WQ_EINVAL, "wq_gauss_coords: NULL argument");
    launch_gauss_coords(r, xyz, (hipStream_t)stream);
    return check_launch("wq_gauss_coords");
}

int gauss_assemble(const wq_rules* r, int dtype, uint32_t which, const void* kappa_gauss, const void* kappa, void* vm,
                   void* vk, void* stream) {
    int st = check_values(r, dtype, which, kappa, vm, vk, "gauss_assemble");
    if (st) return st;
    if (dtype == WQ_BF16X3)
        return wq_set_error(WQ_EUNSUPPORTED, "gauss_assemble: the BF16x3 split covers the forward rows only");
    if (!kappa_gauss && r->n_int_elems > 0) return wq_set_error(WQ_EINVAL, "gauss_assemble: kappa_gauss is NULL");
    if (r->nnz == 0) return WQ_OK;
    if (dtype == WQ_F64)
        st = launch_gauss<double>(r, which, (const double*)kappa_gauss, (const double*)kappa, (double*)vm, (double*)vk,
                                  (hipStream_t)stream);
    else
        st = launch_gauss<float>(r, which, (const float*)kappa_gauss, (const float*)kappa, (float*)vm, (float*)vk,
                                 (hipStream_t)stream);
    if (st) return st;
    return check_launch("gauss_assemble");
}

int wq_load_vector(const wq_rules* r, const double* f, double* b, void* stream) {
    if (!r || !f || !b) return wq_set_error(WQ_EINVAL, "wq_load_vector: NULL argument");
    int st = projection_load_vector(r, f, b, (hipStream_t)stream);
    if (st) return st;
    return check_launch("wq_load_vector");
}

int wq_extension_build(const wq_rules* r, void* stream, wq_extension** out) {
    if (!r || !out) return wq_set_error(WQ_EINVAL, "wq_extension_build: NULL argument");
    *out = nullptr;
    return projection_build_extension(r, (hipStream_t)stream, out);
}

int wq_extension_info_get(const wq_extension* x, wq_extension_info* out) {
    if (!x || !out) return wq_set_error(WQ_EINVAL, "wq_extension_info_get: NULL argument");
    return projection_info(x, out);
}

void wq_extension_free(wq_extension* x) {
    if (!x) return;
    (void)hipDeviceSynchronize();
    projection_free(x);
}

int wq_project(const wq_rules* r, const wq_extension* x, const double* vm, const double* b, double* u, double tol,
               int32_t max_iter, int32_t* iters, double* relres, void* stream) {
    if (!r || !x || !vm || !b || !u) return wq_set_error(WQ_EINVAL, "wq_project: NULL argument");
    if (projection_owner(x) != r) return wq_set_error(WQ_EINVAL, "wq_project: the extension belongs to another rules handle");
    if (!(tol > 0.0) || max_iter < 1) return wq_set_error(WQ_EINVAL, "wq_project: need tol > 0 and max_iter >= 1");
    return projection_solve(r, x, vm, b, u, tol, max_iter, iters, relres, (hipStream_t)stream);
}

int wq_l2_error(const wq_rules* r, const double* u, const double* fg, const double* f, double* out, void* stream) {
    if (!r || !u || !f || !out) return wq_set_error(WQ_EINVAL, "wq_l2_error: NULL argument");
    if (!fg && r->n_int_elems > 0) return wq_set_error(WQ_EINVAL, "wq_l2_error: f_gauss is NULL");
    int st = projection_error(r, u, fg, f, out, (hipStream_t)stream);
    if (st) return st;
    return check_launch("wq_l2_error");
}

void wq_rules_free(wq_rules* r) {
    if (!r) return;
    (void)hipDeviceSynchronize();
    delete r;
}

}  // extern "C"
