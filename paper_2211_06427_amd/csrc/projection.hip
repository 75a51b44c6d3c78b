// L2 projection onto the extended B-spline space of a cut background mesh (Section 3.1,
// test setting: mass matrix, projection of a target function, extended B-splines for a
// well-conditioned system; Section 3.2: relative L2 error).  FP64 throughout.
//
// Readings (the paper refers to other works for the extension and the load vector):
//  - load vector b_I = sum over the quadrature points of row I of W_I(q) f(x_q), with the
//    points and test weights of the mass row.  The active functions of row I sum to one
//    at each of those points, so b is the row sums of the mass matrix assembled with
//    kappa = f: that is how it is computed here (same kernels, then a row-sum kernel);
//  - inner function: active, with at least one interior element in its support;
//  - the root element of an outer function j: the interior element l nearest to it, measured
//    between the element centre l + 1/2 and the centre j - p/2 + 1/2 of B_j's support in element
//    units (Euclidean), the lexicographically first on ties; its functions l + {0..p}^3 are
//    all inner;
//  - the outer function enters through them with e_{i,j} = lambda_j(P_i): the dual functional
//    of B_j (its B-spline coefficient of a polynomial) applied to the polynomial piece P_i of
//    B_i on the root element.  Per direction lambda_j(P) is the blossom of P at the interior
//    knots t_{j+1}..t_{j+p}; the blossom of a piece is de Boor's triangular scheme with the
//    p arguments taken one per level.  E (active x inner) has one unit entry per inner row and
//    the (p+1)^3 products per outer row; the system is E^T M E c = E^T b;
//  - error: (p+1)^3 Gauss points on interior elements, octree points on cut elements.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "rows.h"

struct wq_extension {
    const wq_rules* owner = nullptr;      // the rules handle it was built from
    int p = 0;
    int64_t n_active = 0, n_inner = 0, n_outer = 0, nnz_e = 0;
    int32_t* inner_of_active = nullptr;   // (n_active) inner index or -1
    int32_t* outer_rows = nullptr;        // (n_outer) active index, ascending
    int32_t* outer_base = nullptr;        // (n_outer, 3) array base l
    int64_t* e_ptr = nullptr;             // CSR of E, rows = active functions
    int32_t* e_col = nullptr;
    double* e_val = nullptr;
    int64_t* et_ptr = nullptr;            // CSR of E^T, rows = inner functions, columns ascending
    int32_t* et_col = nullptr;
    double* et_val = nullptr;
    // preconditioner: box mass matrix K1 x K2 x K3 of the whole background mesh
    int32_t* inner_lex = nullptr;         // (n_inner) lexicographic function index
    int32_t* lex_inner = nullptr;         // (nfun product) inner index or -1
    double* kchol[3] = {nullptr, nullptr, nullptr};   // banded Cholesky factor of K_d, [i][k] = L(i, i-k)
    double* kdiag[3] = {nullptr, nullptr, nullptr};   // diagonal of K_d
    std::vector<void*> allocs;
    ~wq_extension() {
        for (void* q : allocs) (void)hipFree(q);
    }
    template <typename T> hipError_t alloc(T** p, int64_t n) {
        void* q = nullptr;
        hipError_t e = hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(n, 1));
        if (e == hipSuccess) allocs.push_back(q);
        *p = (T*)q;
        return e;
    }
};

namespace {

constexpr int RED_BLOCKS = 512;    // fixed grid of every reduction: the summation order never varies
constexpr int RED_THREADS = 256;

inline dim3 blocks_for(int64_t n, int t = 256) { return dim3((unsigned)std::max<int64_t>((n + t - 1) / t, 1)); }

__device__ inline void unlex3(int64_t k, const int* n, int* I) {
    I[2] = (int)(k % n[2]);
    I[1] = (int)((k / n[2]) % n[1]);
    I[0] = (int)(k / ((int64_t)n[1] * n[2]));
}

__device__ inline int floor_div2(int a) { return a >= 0 ? a / 2 : -((-a + 1) / 2); }

// ---------------------------------------------------------------------------------------
// extension set-up
// ---------------------------------------------------------------------------------------
// inner flag of every active function
__global__ void k_ext_inner(DevRules R, int64_t n_active, int8_t* inner_act) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_active) return;
    const int64_t lex = R.act2lex[r];
    int j[3];
    unlex3(lex, R.nfun, j);
    const int p = R.p;
    const int a0 = max(j[0] - p, 0), b0 = min(j[0], R.nel[0] - 1);
    const int a1 = max(j[1] - p, 0), b1 = min(j[1], R.nel[1] - 1);
    const int a2 = max(j[2] - p, 0), b2 = min(j[2], R.nel[2] - 1);
    int8_t in = 0;
    for (int e0 = a0; e0 <= b0 && !in; ++e0)
        for (int e1 = a1; e1 <= b1 && !in; ++e1)
            for (int e2 = a2; e2 <= b2 && !in; ++e2)
                if (R.ecls[((int64_t)e0 * R.nel[1] + e1) * R.nel[2] + e2] == CLS_IN) in = 1;
    inner_act[r] = in;
}

// ok[l] = 1 when element l is interior (a root-element candidate); l lexicographic
__global__ void k_ext_bases(DevRules R, int8_t* ok) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)R.nel[0] * R.nel[1] * R.nel[2]) return;
    ok[id] = R.ecls[id] == CLS_IN ? 1 : 0;
}

// Root element of each outer function: cubes |2 l_d + p - 2 j_d| <= 2 rad of growing rad,
// each scanned in lexicographic order keeping the first strict minimum of
// sum_d (2 l_d + p - 2 j_d)^2 (four times the squared distance of the centres).  Every base
// outside a cube has squared distance >= (2 rad + 1)^2, so a minimum below that is final.
// At rad = max_d nfun_d the cube holds every element, so whatever it finds there is final (the
// host has checked that an interior element exists).
__global__ void k_ext_nearest(DevRules R, const int32_t* outer_rows, int64_t n_outer, const int8_t* ok,
                              int32_t* base) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_outer) return;
    int j[3];
    unlex3(R.act2lex[outer_rows[k]], R.nfun, j);
    const int p = R.p;
    const int nb0 = R.nel[0], nb1 = R.nel[1], nb2 = R.nel[2];
    const int rmax = max(R.nfun[0], max(R.nfun[1], R.nfun[2]));
    int best0 = -1, best1 = -1, best2 = -1;
    for (int rad = 0; rad <= rmax; ++rad) {
        // l_d with -2 rad <= 2 l_d + p - 2 j_d <= 2 rad
        const int lo0 = max(-floor_div2(-(2 * j[0] - p - 2 * rad)), 0), hi0 = min(floor_div2(2 * j[0] - p + 2 * rad), nb0 - 1);
        const int lo1 = max(-floor_div2(-(2 * j[1] - p - 2 * rad)), 0), hi1 = min(floor_div2(2 * j[1] - p + 2 * rad), nb1 - 1);
        const int lo2 = max(-floor_div2(-(2 * j[2] - p - 2 * rad)), 0), hi2 = min(floor_div2(2 * j[2] - p + 2 * rad), nb2 - 1);
        long long bestd = -1;
        for (int l0 = lo0; l0 <= hi0; ++l0)
            for (int l1 = lo1; l1 <= hi1; ++l1)
                for (int l2 = lo2; l2 <= hi2; ++l2) {
                    if (!ok[((int64_t)l0 * nb1 + l1) * nb2 + l2]) continue;
                    const long long d0 = 2 * l0 + p - 2 * j[0], d1 = 2 * l1 + p - 2 * j[1], d2 = 2 * l2 + p - 2 * j[2];
                    const long long dd = d0 * d0 + d1 * d1 + d2 * d2;
                    if (bestd < 0 || dd < bestd) { bestd = dd; best0 = l0; best1 = l1; best2 = l2; }
                }
        if (bestd >= 0 && (bestd < (long long)(2 * rad + 1) * (2 * rad + 1) || rad == rmax)) break;
        best0 = best1 = best2 = -1;
    }
    base[3 * k + 0] = best0;
    base[3 * k + 1] = best1;
    base[3 * k + 2] = best2;
}

// Blossom of the polynomial piece of B_m on the knot span [t_s, t_{s+1}] at the arguments
// t_{j+1}..t_{j+p}: de Boor's scheme from the coefficients delta_{m,i} (i = s-p..s), level r
// using the argument t_{j+r}.  Knots in element units, t_k = clamp(k - p, 0, nel); every
// denominator t_{i+p+1-r} - t_i spans [t_s, t_{s+1}] and is >= 1.
__device__ inline double blossom_piece(int p, int nel, int s, int m, int j) {
    double d[WQ_PMAX + 1];
    for (int k = 0; k <= p; ++k) d[k] = (s - p + k == m) ? 1.0 : 0.0;
    for (int r = 1; r <= p; ++r) {
        const double u = (double)min(max(j + r - p, 0), nel);
        for (int k = p; k >= r; --k) {
            const int i = s - p + k;
            const double ti = (double)min(max(i - p, 0), nel);
            const double tr = (double)min(max(i + 1 - r, 0), nel);     // t_{i+p+1-r}
            const double a = (u - ti) / (tr - ti);
            d[k] = (1.0 - a) * d[k - 1] + a * d[k];
        }
    }
    return d[p];
}

// values of E: 1 on inner rows; on an outer row with root element l the (p+1)^3 entries
// (a lexicographic) prod_d lambda_{j_d}(P_{l_d + a_d})
__global__ void k_ext_values(DevRules R, int64_t n_active, const int32_t* outer_of_active, const int32_t* base,
                             const int64_t* e_ptr, double* e_val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_active) return;
    const int k = outer_of_active[r];
    if (k < 0) {
        e_val[e_ptr[r]] = 1.0;
        return;
    }
    const int p = R.p;
    int j[3];
    unlex3(R.act2lex[r], R.nfun, j);
    double lam[3][WQ_PMAX + 1];
    for (int d = 0; d < 3; ++d) {
        const int l = base[3 * k + d];
        for (int a = 0; a <= p; ++a) lam[d][a] = blossom_piece(p, R.nel[d], l + p, l + a, j[d]);
    }
    int64_t o = e_ptr[r];
    for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b)
            for (int c = 0; c <= p; ++c) e_val[o++] = lam[0][a] * lam[1][b] * lam[2][c];
}

// band of the 1D box mass matrix, out[i][k] = K_d(i, i - k) for k = 0..p (0 outside), by the
// element Gauss rule: sum over the elements shared by B_i and B_{i-k}
__global__ void k_mass1d(DevRules R, int d, double* out, double* diag) {
    const int p = R.p, P1 = p + 1, n = R.nfun[d];
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * P1) return;
    const int i = id / P1, k = id % P1, j = i - k;
    double v = 0.0;
    if (j >= 0) {
        for (int e = max(i - p, 0); e <= min(j, R.nel[d] - 1); ++e)
            for (int g = 0; g < P1; ++g) {
                const double* B = R.Bval[d] + ((int64_t)e * P1 + g) * P1;
                v += R.gw[g] * R.h[d] * 0.5 * B[i - e] * B[j - e];
            }
    }
    out[id] = v;
    if (k == 0) diag[i] = v;
}

// in-place banded Cholesky K = L L^T, band [i][k] = L(i, i-k) (one thread: n <= a few hundred)
__global__ void k_band_chol(int n, int p, double* L, int* bad) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    const int P1 = p + 1;
    for (int i = 0; i < n; ++i)
        for (int j = max(0, i - p); j <= i; ++j) {
            double v = L[i * P1 + (i - j)];
            for (int m = max(0, i - p); m < j; ++m) v -= L[i * P1 + (i - m)] * L[j * P1 + (j - m)];
            if (j == i) {
                if (!(v > 0.0)) { bad[0] = 1; v = 1.0; }
                L[i * P1] = sqrt(v);
            } else {
                L[i * P1 + (i - j)] = v / L[j * P1];
            }
        }
}

__global__ void k_gather_f64(const double* src, const int64_t* perm, int64_t n, double* dst) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

// ---------------------------------------------------------------------------------------
// reductions (fixed grid and tree: deterministic)
// ---------------------------------------------------------------------------------------
template <int NV>
__device__ inline void block_partials(double (&v)[NV], double* partials, int nparts) {
    __shared__ double sh[NV][RED_THREADS];
    for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = v[i];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int i = 0; i < NV; ++i) partials[(int64_t)i * nparts + blockIdx.x] = sh[i][0];
}

// out[i] = sum of partials[i][0..nparts) (one block of RED_THREADS)
template <int NV>
__global__ __launch_bounds__(RED_THREADS) void k_reduce(const double* partials, int64_t nparts, double* out0,
                                                        double* out1) {
    double v[NV];
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int64_t k = threadIdx.x; k < nparts; k += RED_THREADS) s += partials[(int64_t)i * nparts + k];
        v[i] = s;
    }
    __shared__ double sh[NV][RED_THREADS];
    for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = v[i];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out0[0] = sh[0][0];
        if (NV > 1) out1[0] = sh[NV - 1][0];
    }
}

// ---------------------------------------------------------------------------------------
// load vector: row sums (one wave per row, fixed lane order and shuffle tree)
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_sums(const int64_t* row_ptr, const double* v, int64_t n, double* b) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    double s = 0.0;
    for (int64_t k = row_ptr[r] + lane; k < row_ptr[r + 1]; k += 64) s += v[k];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) b[r] = s;
}

// ---------------------------------------------------------------------------------------
// PCG on E^T M E with the Jacobi preconditioner
// ---------------------------------------------------------------------------------------
enum { SC_RZ = 0, SC_PQ = 2, SC_RR = 3, SC_N = 4 };   // SC_RZ, SC_RZ + 1: r.z of the current / next step

__global__ void k_fill_f64(double* a, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// y = E x (one thread per active row)
__global__ void k_apply_E(const int64_t* ptr, const int32_t* col, const double* val, const double* x, int64_t n,
                          double* y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    double s = 0.0;
    for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) s += val[k] * x[col[k]];
    y[r] = s;
}

// y = M x (one wave per row)
__global__ __launch_bounds__(256) void k_spmv(const int64_t* row_ptr, const int32_t* col, const double* M,
                                              const double* x, int64_t n, double* y) {
    const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    double s = 0.0;
    for (int64_t k = row_ptr[r] + lane; k < row_ptr[r + 1]; k += 64) s += M[k] * x[col[k]];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) y[r] = s;
}

// q = E^T v; with p given, also the partials of p.q (grid RED_BLOCKS x RED_THREADS)
__global__ __launch_bounds__(RED_THREADS) void k_apply_ET(const int64_t* ptr, const int32_t* col, const double* val,
                                                          const double* v, int64_t n, double* q, const double* p,
                                                          double* partials) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) s += val[k] * v[col[k]];
        q[i] = s;
        if (p) acc[0] += p[i] * s;
    }
    if (p) block_partials<1>(acc, partials, gridDim.x);
}

// Jacobi: D_i = sum_{k,l} e_k e_l M(a_k, a_l) over the entries (a_k, e_k) of column i of E;
// invD = 1 / D (a non-positive D is reported through bad[i] = 1)
__global__ void k_jacobi(const int64_t* et_ptr, const int32_t* et_col, const double* et_val, const int64_t* row_ptr,
                         const int32_t* col_idx, const double* M, int64_t n, double* invD, int8_t* bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double D = 0.0;
    for (int64_t k = et_ptr[i]; k < et_ptr[i + 1]; ++k) {
        const int32_t a = et_col[k];
        const int64_t s0 = row_ptr[a], s1 = row_ptr[a + 1];
        double t = 0.0;
        for (int64_t l = et_ptr[i]; l < et_ptr[i + 1]; ++l) {
            const int32_t b = et_col[l];
            int64_t lo = s0, hi = s1;               // binary search of column b in row a
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (col_idx[mid] < b) lo = mid + 1; else hi = mid;
            }
            if (lo < s1 && col_idx[lo] == b) t += et_val[l] * M[lo];
        }
        D += et_val[k] * t;
    }
    const bool ok = D > 0.0 && isfinite(D);
    invD[i] = ok ? 1.0 / D : 1.0;
    bad[i] = ok ? 0 : 1;
}

// beta = rz_next / rz; p = z + beta p
__global__ void k_pcg_p(double* p, const double* z, int64_t n, const double* sc, int cur) {
    const double beta = sc[SC_RZ + (cur ^ 1)] / sc[SC_RZ + cur];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i] + beta * p[i];
}

// Preconditioner z = S R K^{-1} R^T S r: K = K1 x K2 x K3 the mass matrix of every function of
// the background mesh, R^T the zero extension from the inner functions to the whole grid, S the
// diagonal sqrt(diag(K)_i / diag(E^T M E)_i) that restores the row scale of functions with
// little support in the domain.
// g[lex] = s_i r_i at inner functions, 0 elsewhere
__global__ void k_prec_scatter(const int32_t* lex_inner, int64_t nlex, const double* sc, const double* r, double* g) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nlex) return;
    const int32_t i = lex_inner[k];
    g[k] = i >= 0 ? sc[i] * r[i] : 0.0;
}

// K_d^{-1} along direction d of the grid g (nfun[0] x nfun[1] x nfun[2]): one thread per line,
// forward then backward substitution with the band factor
__global__ void k_prec_lines(DevRules R, int d, const double* L, double* g) {
    const int p = R.p, P1 = p + 1;
    const int n0 = R.nfun[0], n1 = R.nfun[1], n2 = R.nfun[2];
    const int n = R.nfun[d];
    const int64_t nlines = (int64_t)n0 * n1 * n2 / n;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nlines) return;
    int64_t base, stride;
    if (d == 2) { base = id * n2; stride = 1; }
    else if (d == 1) { base = (id / n2) * (int64_t)n1 * n2 + id % n2; stride = n2; }
    else { base = id; stride = (int64_t)n1 * n2; }
    for (int i = 0; i < n; ++i) {                 // L y = x
        double v = g[base + i * stride];
        for (int m = max(0, i - p); m < i; ++m) v -= L[i * P1 + (i - m)] * g[base + m * stride];
        g[base + i * stride] = v / L[i * P1];
    }
    for (int i = n - 1; i >= 0; --i) {            // L^T x = y
        double v = g[base + i * stride];
        for (int m = i + 1; m <= min(n - 1, i + p); ++m) v -= L[m * P1 + (m - i)] * g[base + m * stride];
        g[base + i * stride] = v / L[i * P1];
    }
}

// z_i = s_i g[lex_i]; partials of r.z into slot 0 (grid RED_BLOCKS x RED_THREADS)
__global__ __launch_bounds__(RED_THREADS) void k_prec_gather(const int32_t* inner_lex, int64_t n, const double* sc,
                                                             const double* g, const double* r, double* z,
                                                             double* partials) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double zi = sc[i] * g[inner_lex[i]];
        z[i] = zi;
        acc[0] += r[i] * zi;
    }
    block_partials<1>(acc, partials, gridDim.x);
}

// s_i = sqrt(prod_d diag(K_d)(i_d) * invD_i)
__global__ void k_prec_scale(DevRules R, const int32_t* inner_lex, int64_t n, const double* k0, const double* k1,
                             const double* k2, const double* invD, double* sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int I[3];
    unlex3(inner_lex[i], R.nfun, I);
    sc[i] = sqrt(k0[I[0]] * k1[I[1]] * k2[I[2]] * invD[i]);
}

// alpha = rz / pq; x += alpha p; r -= alpha q; partials of r.r into slot 1
__global__ __launch_bounds__(RED_THREADS) void k_pcg_xr2(double* x, double* r, const double* p, const double* q,
                                                         int64_t n, const double* sc, int cur, double* partials) {
    const double alpha = sc[SC_RZ + cur] / sc[SC_PQ];
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc[0] += ri * ri;
    }
    block_partials<1>(acc, partials + RED_BLOCKS, gridDim.x);
}

__global__ __launch_bounds__(RED_THREADS) void k_dot_self(const double* r, int64_t n, double* partials) {
    double acc[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        acc[0] += r[i] * r[i];
    block_partials<1>(acc, partials, gridDim.x);
}

__global__ void k_copy_f64(const double* a, int64_t n, double* b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

// ---------------------------------------------------------------------------------------
// relative L2 error
// ---------------------------------------------------------------------------------------
// coefficients of the (p+1)^3 functions supported on element e (lexicographic), 0 if inactive
template <int P>
__device__ inline void load_coefs(const DevRules& R, const int* e, const double* u, double* c) {
    constexpr int P1 = P + 1, NP = P1 * P1 * P1;
    for (int t = threadIdx.x; t < NP; t += blockDim.x) {
        const int a = t / (P1 * P1), b = (t / P1) % P1, cc = t % P1;
        const int64_t lex = ((int64_t)(e[0] + a) * R.nfun[1] + (e[1] + b)) * R.nfun[2] + (e[2] + cc);
        const int32_t act = R.lex2act[lex];
        c[t] = act >= 0 ? u[act] : 0.0;
    }
}

template <int P>
__device__ inline double eval_tensor(const double* c, const double* N0, const double* N1, const double* N2) {
    constexpr int P1 = P + 1;
    double s = 0.0;
    for (int a = 0; a < P1; ++a) {
        double sa = 0.0;
        for (int b = 0; b < P1; ++b) {
            double sb = 0.0;
            for (int cc = 0; cc < P1; ++cc) sb += N2[cc] * c[(a * P1 + b) * P1 + cc];
            sa += N1[b] * sb;
        }
        s += N0[a] * sa;
    }
    return s;
}

template <int P>
__device__ inline void block_sum2(double se, double sf, double* part, int64_t n, int64_t idx) {
    __shared__ double sh[2][256];
    sh[0][threadIdx.x] = se;
    sh[1][threadIdx.x] = sf;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[idx] = sh[0][0];
        part[n + idx] = sh[1][0];
    }
}

// one block (256 threads) per interior element; f at its Gauss points in lexicographic order
template <int P>
__global__ __launch_bounds__(256) void k_err_gauss(DevRules R, const int32_t* elems, int64_t n_el, const double* u,
                                                   const double* f, double* part) {
    constexpr int P1 = P + 1, NP = P1 * P1 * P1;
    __shared__ double c[NP];
    const int64_t el = blockIdx.x;
    int e[3];
    unlex3(elems[el], R.nel, e);
    load_coefs<P>(R, e, u, c);
    __syncthreads();
    double se = 0.0, sf = 0.0;
    for (int q = threadIdx.x; q < NP; q += blockDim.x) {
        const int g0 = q / (P1 * P1), g1 = (q / P1) % P1, g2 = q % P1;
        const double* N0 = R.Bval[0] + ((int64_t)e[0] * P1 + g0) * P1;
        const double* N1 = R.Bval[1] + ((int64_t)e[1] * P1 + g1) * P1;
        const double* N2 = R.Bval[2] + ((int64_t)e[2] * P1 + g2) * P1;
        const double uh = eval_tensor<P>(c, N0, N1, N2);
        const double w = (R.gw[g0] * R.h[0] / 2.0) * (R.gw[g1] * R.h[1] / 2.0) * (R.gw[g2] * R.h[2] / 2.0);
        const double fv = f[el * NP + q];
        se += w * (uh - fv) * (uh - fv);
        sf += w * fv * fv;
    }
    block_sum2<P>(se, sf, part, n_el, el);
}

// B_{e+r}(x), r = 0..p, from the open uniform knots of direction d (element e holds x)
__device__ inline void basis_at(const DevRules& R, int d, int e, double x, double* N) {
    const int p = R.p;
    double t[2 * WQ_PMAX + 2], dN[WQ_PMAX + 1];
    for (int m = 0; m < 2 * p + 2; ++m) {        // t[m] = knot e + m (global numbering)
        const int k = min(max(e + m - p, 0), R.nel[d]);
        t[m] = R.lo[d] + k * R.h[d];
    }
    basis_funs(t, p, p, x, N, dN);
}

// one block (256 threads) per cut element over the octree points of its leaves
template <int P>
__global__ __launch_bounds__(256) void k_err_octree(DevRules R, const double* xyz, const double* u, const double* f,
                                                    double* part) {
    constexpr int P1 = P + 1, NP = P1 * P1 * P1;
    __shared__ double c[NP];
    const int64_t ce = blockIdx.x;
    int e[3];
    unlex3(R.cut_elems[ce], R.nel, e);
    load_coefs<P>(R, e, u, c);
    __syncthreads();
    double se = 0.0, sf = 0.0;
    // points of the cut element: its octree leaves' Gauss points, or the NK^3 points of its
    // fitted rule
    constexpr int NK3 = (2 * P + 1) * (2 * P + 1) * (2 * P + 1);
    const int64_t q0 = R.fit ? ce * NK3 : (int64_t)R.cell_begin[ce] * NP;
    const int64_t q1 = R.fit ? (ce + 1) * NK3 : (int64_t)R.cell_begin[ce + 1] * NP;
    for (int64_t q = q0 + threadIdx.x; q < q1; q += blockDim.x) {
        const double w = R.oct_w[q];
        if (w == 0.0) continue;
        const int64_t s = R.n_grid + R.n_block + q;
        double N0[P1], N1[P1], N2[P1];
        basis_at(R, 0, e[0], xyz[3 * s + 0], N0);
        basis_at(R, 1, e[1], xyz[3 * s + 1], N1);
        basis_at(R, 2, e[2], xyz[3 * s + 2], N2);
        const double uh = eval_tensor<P>(c, N0, N1, N2);
        const double fv = f[s];
        se += w * (uh - fv) * (uh - fv);
        sf += w * fv * fv;
    }
    block_sum2<P>(se, sf, part, R.n_cut_elems, ce);
}

__global__ __launch_bounds__(RED_THREADS) void k_err_final(const double* pg, int64_t ng, const double* po, int64_t no,
                                                           double* out) {
    double v[2] = {0.0, 0.0};
    for (int i = 0; i < 2; ++i) {
        for (int64_t k = threadIdx.x; k < ng; k += RED_THREADS) v[i] += pg[(int64_t)i * ng + k];
        for (int64_t k = threadIdx.x; k < no; k += RED_THREADS) v[i] += po[(int64_t)i * no + k];
    }
    __shared__ double sh[2][RED_THREADS];
    sh[0][threadIdx.x] = v[0];
    sh[1][threadIdx.x] = v[1];
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + s];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
    }
}

template <int P>
void launch_err(const wq_rules* H, const double* u, const double* fg, const double* f, double* pg, double* po,
                hipStream_t s) {
    const DevRules& R = H->R;
    if (H->n_int_elems > 0)
        hipLaunchKernelGGL(k_err_gauss<P>, dim3((unsigned)H->n_int_elems), dim3(256), 0, s, R, H->int_elems,
                           H->n_int_elems, u, fg, pg);
    if (R.n_cut_elems > 0)
        hipLaunchKernelGGL(k_err_octree<P>, dim3((unsigned)R.n_cut_elems), dim3(256), 0, s, R, H->kappa_xyz, u, f, po);
}

// scratch from the handle's pool, released on the stream at scope exit
struct Scratch {
    const wq_rules* H;
    hipStream_t s;
    std::vector<void*> bufs;
    bool failed = false;
    Scratch(const wq_rules* h, hipStream_t st) : H(h), s(st) {}
    template <typename T> T* get(int64_t n) {
        void* p = nullptr;
        if (H->scratch_alloc(&p, sizeof(T) * (size_t)std::max<int64_t>(n, 1), s) != hipSuccess) {
            (void)hipGetLastError();
            failed = true;
            return nullptr;
        }
        bufs.push_back(p);
        return (T*)p;
    }
    ~Scratch() {
        for (void* p : bufs) (void)hipFreeAsync(p, s);
    }
};

}  // namespace

// ---------------------------------------------------------------------------------------
// host entry points (called from the C ABI)
// ---------------------------------------------------------------------------------------
int projection_load_vector(const wq_rules* H, const double* f, double* b, hipStream_t s) {
    if (H->n_active == 0) return WQ_OK;
    Scratch sc(H, s);
    double* vm = sc.get<double>(H->nnz);
    if (sc.failed) return wq_set_error(WQ_ENOMEM, "wq_load_vector: scratch allocation of %lld values failed", (long long)H->nnz);
    launch_rows<double>(H, WQ_MASS, f, vm, nullptr, s);
    int st = launch_cut<double>(H, WQ_MASS, WQ_CUT_REMAINDER | WQ_CUT_OCTREE, f, vm, nullptr, s);
    if (st) return st;
    hipLaunchKernelGGL(k_row_sums, blocks_for(H->n_active * 64), dim3(256), 0, s, (const int64_t*)H->R.row_ptr,
                       (const double*)vm, H->n_active, b);
    return WQ_OK;
}

int projection_build_extension(const wq_rules* H, hipStream_t s, wq_extension** out) {
    const DevRules& R = H->R;
    const int p = R.p;
    const int64_t na = H->n_active;
    const int64_t nlex = (int64_t)R.nfun[0] * R.nfun[1] * R.nfun[2];
    const int64_t nbases = (int64_t)R.nel[0] * R.nel[1] * R.nel[2];
    wq_extension* X = new wq_extension();
    X->owner = H;
    X->p = p;
    X->n_active = na;
    auto fail = [&](int code, const char* msg) {
        (void)hipStreamSynchronize(s);
        delete X;
        return wq_set_error(code, "wq_extension_build: %s", msg);
    };
    auto hip_ok = [&](hipError_t e) { return e == hipSuccess; };
    int8_t *inner_act = nullptr, *ok = nullptr;
    if (!hip_ok(X->alloc(&inner_act, na)) || !hip_ok(X->alloc(&ok, nbases)))
        return fail(WQ_ENOMEM, "device allocation failed");
    if (na > 0) hipLaunchKernelGGL(k_ext_inner, blocks_for(na), dim3(256), 0, s, R, na, inner_act);
    hipLaunchKernelGGL(k_ext_bases, blocks_for(nbases), dim3(256), 0, s, R, ok);
    std::vector<int8_t> h_inner(na), h_ok(nbases);
    std::vector<int32_t> h_lex2act(nlex);
    if (!hip_ok(hipMemcpyAsync(h_inner.data(), inner_act, na, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(h_ok.data(), ok, nbases, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipMemcpyAsync(h_lex2act.data(), R.lex2act, sizeof(int32_t) * nlex, hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
        return fail(WQ_EHIP, "copy of the inner flags failed");
    // numbering of inner and outer functions (both ascending in active index)
    std::vector<int32_t> inner_of(na, -1), outer_of(na, -1), outer_rows;
    int64_t ni = 0;
    for (int64_t r = 0; r < na; ++r) {
        if (h_inner[r]) inner_of[r] = (int32_t)ni++;
        else { outer_of[r] = (int32_t)outer_rows.size(); outer_rows.push_back((int32_t)r); }
    }
    const int64_t no = (int64_t)outer_rows.size();
    X->n_inner = ni;
    X->n_outer = no;
    if (no > 0 && std::find(h_ok.begin(), h_ok.end(), (int8_t)1) == h_ok.end())
        return fail(WQ_EINVAL, "no interior element: the mesh is too coarse for the extension");
    if (!hip_ok(X->alloc(&X->inner_of_active, na)) || !hip_ok(X->alloc(&X->outer_rows, no)) ||
        !hip_ok(X->alloc(&X->outer_base, 3 * no)))
        return fail(WQ_ENOMEM, "device allocation failed");
    int32_t* outer_of_d = nullptr;
    if (!hip_ok(X->alloc(&outer_of_d, na))) return fail(WQ_ENOMEM, "device allocation failed");
    if (!hip_ok(hipMemcpyAsync(X->inner_of_active, inner_of.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(outer_of_d, outer_of.data(), sizeof(int32_t) * na, hipMemcpyHostToDevice, s)) ||
        (no > 0 && !hip_ok(hipMemcpyAsync(X->outer_rows, outer_rows.data(), sizeof(int32_t) * no, hipMemcpyHostToDevice, s))))
        return fail(WQ_EHIP, "upload of the numbering failed");
    std::vector<int32_t> h_base(3 * no);
    if (no > 0) {
        hipLaunchKernelGGL(k_ext_nearest, blocks_for(no), dim3(256), 0, s, R, (const int32_t*)X->outer_rows, no,
                           (const int8_t*)ok, X->outer_base);
        if (!hip_ok(hipGetLastError()) ||
            !hip_ok(hipMemcpyAsync(h_base.data(), X->outer_base, sizeof(int32_t) * 3 * no, hipMemcpyDeviceToHost, s)) ||
            !hip_ok(hipStreamSynchronize(s)))
            return fail(WQ_EHIP, "root-element search failed");
        for (int64_t k = 0; k < no; ++k)
            if (h_base[3 * k] < 0) return fail(WQ_EINVAL, "an outer function has no root element");
    }
    // structure of E (inner rows: one entry; outer rows: the (p+1)^3 inner functions of the array)
    const int P1 = p + 1, NP = P1 * P1 * P1;
    std::vector<int64_t> e_ptr(na + 1, 0);
    for (int64_t r = 0; r < na; ++r) e_ptr[r + 1] = e_ptr[r] + (inner_of[r] >= 0 ? 1 : NP);
    const int64_t nnz = e_ptr[na];
    X->nnz_e = nnz;
    std::vector<int32_t> e_col(nnz);
    for (int64_t r = 0; r < na; ++r) {
        if (inner_of[r] >= 0) { e_col[e_ptr[r]] = inner_of[r]; continue; }
        const int32_t* l = &h_base[3 * outer_of[r]];
        int64_t o = e_ptr[r];
        for (int a = 0; a < P1; ++a)
            for (int b = 0; b < P1; ++b)
                for (int c = 0; c < P1; ++c) {
                    const int64_t lex = ((int64_t)(l[0] + a) * R.nfun[1] + (l[1] + b)) * R.nfun[2] + (l[2] + c);
                    const int32_t act = h_lex2act[lex];
                    if (act < 0 || inner_of[act] < 0) return fail(WQ_EHIP, "array holds a non-inner function");
                    e_col[o++] = inner_of[act];
                }
    }
    // E^T by a stable counting sort over the columns (rows of E^T ascending in active index)
    std::vector<int64_t> et_ptr(ni + 1, 0), perm(nnz);
    std::vector<int32_t> et_col(nnz);
    for (int64_t k = 0; k < nnz; ++k) et_ptr[e_col[k] + 1]++;
    for (int64_t i = 0; i < ni; ++i) et_ptr[i + 1] += et_ptr[i];
    {
        std::vector<int64_t> fill(et_ptr.begin(), et_ptr.end() - 1);
        for (int64_t r = 0; r < na; ++r)
            for (int64_t k = e_ptr[r]; k < e_ptr[r + 1]; ++k) {
                const int64_t o = fill[e_col[k]]++;
                et_col[o] = (int32_t)r;
                perm[o] = k;
            }
    }
    int64_t* perm_d = nullptr;
    if (!hip_ok(X->alloc(&X->e_ptr, na + 1)) || !hip_ok(X->alloc(&X->e_col, nnz)) || !hip_ok(X->alloc(&X->e_val, nnz)) ||
        !hip_ok(X->alloc(&X->et_ptr, ni + 1)) || !hip_ok(X->alloc(&X->et_col, nnz)) ||
        !hip_ok(X->alloc(&X->et_val, nnz)) || !hip_ok(X->alloc(&perm_d, nnz)))
        return fail(WQ_ENOMEM, "device allocation failed");
    if (!hip_ok(hipMemcpyAsync(X->e_ptr, e_ptr.data(), sizeof(int64_t) * (na + 1), hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(X->e_col, e_col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(X->et_ptr, et_ptr.data(), sizeof(int64_t) * (ni + 1), hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(X->et_col, et_col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(perm_d, perm.data(), sizeof(int64_t) * nnz, hipMemcpyHostToDevice, s)))
        return fail(WQ_EHIP, "upload of E failed");
    if (na > 0)
        hipLaunchKernelGGL(k_ext_values, blocks_for(na), dim3(256), 0, s, R, na, (const int32_t*)outer_of_d,
                           (const int32_t*)X->outer_base, (const int64_t*)X->e_ptr, X->e_val);
    if (nnz > 0)
        hipLaunchKernelGGL(k_gather_f64, blocks_for(nnz), dim3(256), 0, s, (const double*)X->e_val,
                           (const int64_t*)perm_d, nnz, X->et_val);
    if (!hip_ok(hipGetLastError()) || !hip_ok(hipStreamSynchronize(s))) return fail(WQ_EHIP, "values of E failed");
    // preconditioner: inner <-> lexicographic maps, band Cholesky factors of the 1D box masses
    std::vector<int32_t> inner_lex(std::max<int64_t>(ni, 1)), lex_inner(nlex, -1);
    for (int64_t lex = 0; lex < nlex; ++lex) {
        const int32_t act = h_lex2act[lex];
        if (act >= 0 && inner_of[act] >= 0) {
            lex_inner[lex] = inner_of[act];
            inner_lex[inner_of[act]] = (int32_t)lex;
        }
    }
    int* bad_d = nullptr;
    if (!hip_ok(X->alloc(&X->inner_lex, ni)) || !hip_ok(X->alloc(&X->lex_inner, nlex)) || !hip_ok(X->alloc(&bad_d, 1)))
        return fail(WQ_ENOMEM, "device allocation failed");
    for (int d = 0; d < 3; ++d)
        if (!hip_ok(X->alloc(&X->kchol[d], (int64_t)R.nfun[d] * P1)) || !hip_ok(X->alloc(&X->kdiag[d], R.nfun[d])))
            return fail(WQ_ENOMEM, "device allocation failed");
    const int zero = 0;
    if (!hip_ok(hipMemcpyAsync(X->inner_lex, inner_lex.data(), sizeof(int32_t) * ni, hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(X->lex_inner, lex_inner.data(), sizeof(int32_t) * nlex, hipMemcpyHostToDevice, s)) ||
        !hip_ok(hipMemcpyAsync(bad_d, &zero, sizeof(int), hipMemcpyHostToDevice, s)))
        return fail(WQ_EHIP, "upload of the preconditioner maps failed");
    for (int d = 0; d < 3; ++d) {
        hipLaunchKernelGGL(k_mass1d, blocks_for((int64_t)R.nfun[d] * P1), dim3(256), 0, s, R, d, X->kchol[d], X->kdiag[d]);
        hipLaunchKernelGGL(k_band_chol, dim3(1), dim3(1), 0, s, R.nfun[d], p, X->kchol[d], bad_d);
    }
    int bad = 0;
    if (!hip_ok(hipGetLastError()) || !hip_ok(hipMemcpyAsync(&bad, bad_d, sizeof(int), hipMemcpyDeviceToHost, s)) ||
        !hip_ok(hipStreamSynchronize(s)))
        return fail(WQ_EHIP, "preconditioner factors failed");
    if (bad) return fail(WQ_ESINGULAR, "a 1D mass matrix is not positive definite");
    *out = X;
    return WQ_OK;
}

int projection_info(const wq_extension* X, wq_extension_info* out) {
    memset(out, 0, sizeof(*out));
    out->n_inner = X->n_inner;
    out->n_outer = X->n_outer;
    out->nnz_e = X->nnz_e;
    out->inner_of_active = X->inner_of_active;
    out->outer_rows = X->outer_rows;
    out->outer_base = X->outer_base;
    out->e_ptr = X->e_ptr;
    out->e_col = X->e_col;
    out->e_val = X->e_val;
    return WQ_OK;
}

void projection_free(wq_extension* X) { delete X; }

const wq_rules* projection_owner(const wq_extension* X) { return X->owner; }

int projection_solve(const wq_rules* H, const wq_extension* X, const double* M, const double* b, double* u,
                     double tol, int32_t max_iter, int32_t* iters, double* relres, hipStream_t s) {
    const int64_t na = X->n_active, ni = X->n_inner;
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    if (na == 0) return WQ_OK;
    const DevRules& R = H->R;
    const int64_t nlex = (int64_t)R.nfun[0] * R.nfun[1] * R.nfun[2];
    Scratch sc(H, s);
    double *x = sc.get<double>(ni), *r = sc.get<double>(ni), *z = sc.get<double>(ni), *p = sc.get<double>(ni);
    double *q = sc.get<double>(ni), *invD = sc.get<double>(ni), *ta = sc.get<double>(na), *tb = sc.get<double>(na);
    double *sv = sc.get<double>(ni), *grid = sc.get<double>(nlex);
    double *part = sc.get<double>(2 * RED_BLOCKS), *scal = sc.get<double>(SC_N);
    int8_t* bad = sc.get<int8_t>(ni);
    if (sc.failed) return wq_set_error(WQ_ENOMEM, "wq_project: scratch allocation failed");
    const dim3 gi = blocks_for(ni), ga = blocks_for(na), gw = blocks_for(na * 64), gl = blocks_for(nlex);
    const dim3 gr(RED_BLOCKS), tr(RED_THREADS);
    auto precond = [&]() {       // z = S R K^{-1} R^T S r, partials of r.z into slot 0
        hipLaunchKernelGGL(k_prec_scatter, gl, dim3(256), 0, s, (const int32_t*)X->lex_inner, nlex, (const double*)sv,
                           (const double*)r, grid);
        for (int d = 2; d >= 0; --d)
            hipLaunchKernelGGL(k_prec_lines, blocks_for(nlex / R.nfun[d]), dim3(256), 0, s, R, d, (const double*)X->kchol[d],
                               grid);
        hipLaunchKernelGGL(k_prec_gather, gr, tr, 0, s, (const int32_t*)X->inner_lex, ni, (const double*)sv,
                           (const double*)grid, (const double*)r, z, part);
    };
    // diagonal of E^T M E and the preconditioner's scaling
    hipLaunchKernelGGL(k_jacobi, gi, dim3(256), 0, s, (const int64_t*)X->et_ptr, (const int32_t*)X->et_col,
                       (const double*)X->et_val, (const int64_t*)R.row_ptr, (const int32_t*)R.col_idx, M, ni, invD, bad);
    hipLaunchKernelGGL(k_prec_scale, gi, dim3(256), 0, s, R, (const int32_t*)X->inner_lex, ni, (const double*)X->kdiag[0],
                       (const double*)X->kdiag[1], (const double*)X->kdiag[2], (const double*)invD, sv);
    // r = E^T b, x = 0, z = prec(r), p = z
    hipLaunchKernelGGL(k_apply_ET, gr, tr, 0, s, (const int64_t*)X->et_ptr, (const int32_t*)X->et_col,
                       (const double*)X->et_val, b, ni, r, (const double*)nullptr, part);
    hipLaunchKernelGGL(k_fill_f64, gi, dim3(256), 0, s, x, ni, 0.0);
    hipLaunchKernelGGL(k_dot_self, gr, tr, 0, s, (const double*)r, ni, part + RED_BLOCKS);
    precond();
    hipLaunchKernelGGL(k_reduce<2>, dim3(1), tr, 0, s, (const double*)part, (int64_t)RED_BLOCKS, scal + SC_RZ, scal + SC_RR);
    hipLaunchKernelGGL(k_copy_f64, gi, dim3(256), 0, s, (const double*)z, ni, p);
    double h_sc[SC_N];
    std::vector<int8_t> h_bad(ni);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h_sc, scal, sizeof h_sc, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (ni > 0 && hipMemcpyAsync(h_bad.data(), bad, ni, hipMemcpyDeviceToHost, s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return wq_set_error(WQ_EHIP, "wq_project: set-up kernels failed");
    for (int64_t i = 0; i < ni; ++i)
        if (h_bad[i]) return wq_set_error(WQ_ESINGULAR, "wq_project: diagonal of E^T M E not positive at inner function %lld", (long long)i);
    const double rr0 = h_sc[SC_RR];
    int it = 0;
    double rel = 0.0;
    if (rr0 > 0.0) {
        constexpr int CHECK = 8;   // iterations between host convergence checks
        int cur = 0;
        rel = 1.0;
        while (it < max_iter) {
            hipLaunchKernelGGL(k_apply_E, ga, dim3(256), 0, s, (const int64_t*)X->e_ptr, (const int32_t*)X->e_col,
                               (const double*)X->e_val, (const double*)p, na, ta);
            hipLaunchKernelGGL(k_spmv, gw, dim3(256), 0, s, (const int64_t*)R.row_ptr, (const int32_t*)R.col_idx, M,
                               (const double*)ta, na, tb);
            hipLaunchKernelGGL(k_apply_ET, gr, tr, 0, s, (const int64_t*)X->et_ptr, (const int32_t*)X->et_col,
                               (const double*)X->et_val, (const double*)tb, ni, q, (const double*)p, part);
            hipLaunchKernelGGL(k_reduce<1>, dim3(1), tr, 0, s, (const double*)part, (int64_t)RED_BLOCKS, scal + SC_PQ,
                               scal + SC_PQ);
            hipLaunchKernelGGL(k_pcg_xr2, gr, tr, 0, s, x, r, (const double*)p, (const double*)q, ni,
                               (const double*)scal, cur, part);
            precond();
            hipLaunchKernelGGL(k_reduce<2>, dim3(1), tr, 0, s, (const double*)part, (int64_t)RED_BLOCKS,
                               scal + SC_RZ + (cur ^ 1), scal + SC_RR);
            hipLaunchKernelGGL(k_pcg_p, gi, dim3(256), 0, s, p, (const double*)z, ni, (const double*)scal, cur);
            cur ^= 1;
            ++it;
            if (it % CHECK == 0 || it == max_iter) {
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(h_sc, scal, sizeof h_sc, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    return wq_set_error(WQ_EHIP, "wq_project: iteration kernels failed");
                rel = std::sqrt(h_sc[SC_RR] / rr0);
                if (!std::isfinite(rel) || !(h_sc[SC_PQ] > 0.0))
                    return wq_set_error(WQ_ESINGULAR, "wq_project: CG breakdown after %d iterations (p.Ap = %g)", it,
                                        h_sc[SC_PQ]);
                if (rel <= tol) break;
            }
        }
    }
    // u = E x
    hipLaunchKernelGGL(k_apply_E, ga, dim3(256), 0, s, (const int64_t*)X->e_ptr, (const int32_t*)X->e_col,
                       (const double*)X->e_val, (const double*)x, na, u);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return wq_set_error(WQ_EHIP, "wq_project: final kernels failed");
    if (iters) *iters = it;
    if (relres) *relres = rel;
    return WQ_OK;
}

int projection_error(const wq_rules* H, const double* u, const double* fg, const double* f, double* out, hipStream_t s) {
    Scratch sc(H, s);
    const int64_t ng = H->n_int_elems, no = H->R.n_cut_elems;
    double* pg = sc.get<double>(2 * ng);
    double* po = sc.get<double>(2 * no);
    if (sc.failed) return wq_set_error(WQ_ENOMEM, "wq_l2_error: scratch allocation failed");
    switch (H->R.p) {
        case 1: launch_err<1>(H, u, fg, f, pg, po, s); break;
        case 2: launch_err<2>(H, u, fg, f, pg, po, s); break;
        case 3: launch_err<3>(H, u, fg, f, pg, po, s); break;
        case 4: launch_err<4>(H, u, fg, f, pg, po, s); break;
        case 5: launch_err<5>(H, u, fg, f, pg, po, s); break;
        default: launch_err<6>(H, u, fg, f, pg, po, s); break;
    }
    hipLaunchKernelGGL(k_err_final, dim3(1), dim3(RED_THREADS), 0, s, (const double*)pg, ng, (const double*)po, no, out);
    return WQ_OK;
}
