// Host-side rules handle and build helpers.
#pragma once

#include <cstdarg>
#include <mutex>
#include <vector>

#include "common.h"

// Rows per interior line block of the row kernel (limited by the LDS slab of stage 2).
inline int row_block_rows(int p) { return p <= 4 ? 16 : 8; }

struct wq_rules {
    DevRules R;
    wq_mesh mesh;
    std::vector<void*> allocs;          // device buffers owned by the handle
    double* gxi = nullptr;              // Gauss nodes / weights on [-1,1] (device)
    double* gw = nullptr;
    int64_t n_active = 0, nnz = 0, n_interior_rows = 0, n_cut = 0, n_dwq = 0;
    int64_t n_block_elems = 0, n_cells = 0, n_oct = 0;
    int64_t n_oct_xgroups = 0, n_oct_columns = 0;    // octree leaf groups of the cut kernels
    int64_t n_rem_pairs = 0;                         // (cut row, remainder element) pairs
    int32_t* int_elems = nullptr;                    // interior elements, lexicographic
    int64_t n_int_elems = 0;
    int row_block = 16;
    int32_t* act2cut = nullptr;         // active row -> cut row or -1
    int32_t* box = nullptr;             // [cut row][6] DWQ box (inclusive element ranges)
    int32_t* block_elems = nullptr;
    int8_t* cell_cut = nullptr;         // octree leaf is a cut cell (indicator applies)
    int32_t* cell_elem = nullptr;       // octree leaf -> cut element
    double* kappa_xyz = nullptr;
    int64_t n_split = 0;
    // host copies for batching the cut elements: direction-1 element index of every cut
    // element and direction-1 function index of every cut row (both non-decreasing)
    std::vector<int32_t> h_cut_elem_e1, h_cut_row_i1;
    hipMemPool_t pool = nullptr;        // stream-ordered scratch of the assembly calls (may be null)
    // second stream of the row assembly: the cut rows run on it beside the interior rows
    // (forked from and joined back into the caller's stream with the two events); the
    // mutex keeps one call's record / wait sequence from interleaving with another's
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // third stream of the fused assembly (wq_assemble): the cut elements' moments and local
    // rows run on it beside the rows and the remainder
    hipStream_t side2 = nullptr;
    hipEvent_t ev_join2 = nullptr;
    std::mutex* side_mu = nullptr;
    ~wq_rules() {
        if (side) (void)hipStreamDestroy(side);
        if (side2) (void)hipStreamDestroy(side2);
        if (ev_join2) (void)hipEventDestroy(ev_join2);
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        delete side_mu;
        for (void* p : allocs) (void)hipFree(p);
        if (pool) (void)hipMemPoolDestroy(pool);
    }
    // stream-ordered scratch: from the handle's pool (kept across calls), else the default pool
    hipError_t scratch_alloc(void** p, size_t n, hipStream_t s) const {
        return pool ? hipMallocFromPoolAsync(p, n, pool, s) : hipMallocAsync(p, n, s);
    }
};

// Allocation / error bookkeeping while a handle is being built.
struct Builder {
    wq_rules* H;
    hipStream_t stream;
    int status = 0;
    std::vector<void*> tmps;
    Builder(wq_rules* h, hipStream_t s) : H(h), stream(s) {}
    ~Builder() {
        if (!tmps.empty()) {
            (void)hipStreamSynchronize(stream);
            for (void* p : tmps) (void)hipFree(p);
        }
    }
    int check(hipError_t e) {
        if (e != hipSuccess) {
            status = wq_set_error(WQ_EHIP, "HIP error during rule build: %s", hipGetErrorString(e));
            return status;
        }
        return 0;
    }
    template <typename T> T* alloc(int64_t n, bool keep_it) {
        void* p = nullptr;
        if (n < 1) n = 1;
        if (hipMalloc(&p, sizeof(T) * (size_t)n) != hipSuccess) {
            (void)hipGetLastError();
            status = wq_set_error(WQ_ENOMEM, "device allocation of %lld bytes failed", (long long)(sizeof(T) * n));
            return nullptr;
        }
        (keep_it ? H->allocs : tmps).push_back(p);
        return (T*)p;
    }
    template <typename T> T* keep(int64_t n) { return alloc<T>(n, true); }
    template <typename T> T* tmp(int64_t n) { return alloc<T>(n, false); }
    void release_tmp() {
        (void)hipStreamSynchronize(stream);
        for (void* p : tmps) (void)hipFree(p);
        tmps.clear();
    }
    int fail() {
        int s = status ? status : wq_set_error(WQ_EHIP, "rule build failed");
        release_tmp();
        delete H;
        H = nullptr;
        return s;
    }
    int fail_msg(int code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        status = wq_set_error(code, "%s", buf);
        return fail();
    }
};

int build_rules(const wq_mesh* mesh, const wq_levelset* ls, const wq_options* opts, hipStream_t stream,
                wq_rules** out);

// octree moments of every cut element with an FP64 kappa in the basis whose interval values
// table holds (layout of the Bernstein interval table; cut.hip).  The rule build fits the cut
// rule from Legendre moments.
int launch_octree_moments_f64(const wq_rules* H, const double* table, const double* kappa, double* mom, hipStream_t s);
