// Shared device-side definitions for libwqfd (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wqfd.h"

#define WQ_PMAX 6                       // highest supported degree
#define WQ_MMAX (2 * WQ_PMAX + 1)       // trial indices per direction in a row window
#define WQ_NWMAX (4 * WQ_PMAX)          // points of a standard 1D WQ rule (both boundary elements in one support: 4p)
#define WQ_NDQMAX (WQ_PMAX * (WQ_PMAX + 1))  // points of a one-sided DWQ rule
#define WQ_NQREF ((WQ_PMAX + 1) * (WQ_PMAX + 1))  // points of a refined-function rule

// Device view of a rules handle; passed by value to kernels.
struct DevRules {
    int p, m, nw, ndq;                  // degree, 2p+1, 4p (weight-table stride), p(p+1)
    int nel[3], nfun[3], nx[3], ny[3];
    double lo[3], h[3];
    int levels;
    wq_levelset ls;
    const double* gxi;                  // Gauss-Legendre nodes / weights on [-1, 1], p+1 each
    const double* gw;
    // per direction
    const double* ycoord[3];            // Gauss point coordinates, y = e*(p+1)+g
    const int32_t* y2x[3];              // X index of a Gauss point or -1
    const int32_t* x2y[3];
    const int32_t* xs[3];               // first X index of the window of function i
    const int32_t* nwin[3];             // window size of function i
    const double* Wt64[3];              // [i][a][jj][q], n x 2 x m x nw
    const float* Wt32[3];
    int tensor;                         // WQ_OPT_TENSOR: mixed families built
    const double* Wtx64[3];             // [i][f][jj][q]: f = 0 family (1, 0) times B_j, f = 1 family (0, 1) times B_j'
    const float* Wtx32[3];
    const int8_t* qlo[3];               // [i][jj]: nonzero q range of W[i][.][jj][.]
    const int8_t* qhi[3];
    const double* Bval[3];              // [y][k]: B_{e+k}(y), k = 0..p (e = element of y)
    const double* dBval[3];
    // classification / pattern
    const int8_t* ecls;                 // elements, lexicographic
    const int8_t* fcls;                 // functions, lexicographic
    const int32_t* lex2act;
    const int32_t* act2lex;
    const int64_t* row_ptr;
    const int32_t* col_idx;
    // interior line blocks: (i1 start, i2, i3, count)
    const int4* lblocks;
    int64_t n_lblocks;
    const int4* fblocks;                // the same runs cut into blocks of at most 8 rows (FP32 rows, p <= 4)
    int64_t n_fblocks;
    // cut rows
    const int32_t* cut_rows;            // active index
    const int4* split;                  // d, s, high, dwq rule (-1: none)
    const int32_t* pos_map;             // [cut row][m^3]: offset in row or -1
    int64_t n_cut;
    const int32_t* box_rows;            // cut-row indices with a DWQ box, ascending
    int64_t n_box;
    // DWQ rules
    const int32_t* dwq_np;
    const int32_t* dwq_y;               // [r][ndq]
    const double* dwq_Wt64;             // [r][a][jj][ndq]
    const float* dwq_Wt32;
    const double* dwq_Wtx64;            // [r][f][jj][ndq], mixed families as Wtx64
    const float* dwq_Wtx32;
    // element Gauss blocks
    const int32_t* elem_block;          // element -> block or -1
    const int32_t* blk_slot;            // [block][(p+1)^3] canonical kappa slot of each Gauss point
    const int32_t* rem_ptr;             // [cut row + 1] offsets into rem_list
    const int2* rem_list;               // remainder elements: (I_d - e_d packed 4 bits/direction, block)
    const int32_t* rcut_ptr;            // [cut row + 1] offsets into rcut_list
    const int2* rcut_list;              // cut elements of a cut row: (cut element, I_d - e_d packed 4 bits/direction)
    const double* rem_w64[3];           // per direction: [e][kI][a][k][g] element-Gauss test x trial weights
    const float* rem_w32[3];
    // octree
    const int32_t* cut_elems;           // lexicographic element index of each cut element
    const int32_t* cell_begin;          // (n_cut_elems + 1)
    const double* cell_lo;              // [cell][3]
    const int8_t* cell_depth;
    const int32_t* cell_key;            // depth | offx << 3 | offy << 9 | offz << 15
    const int32_t* cell_perm;           // per cut element, leaves sorted by (depth, offx, offy, offz)
    const double* oct_pp64[3];          // per direction: [element][interval][v][a b][g] basis products
    const float* oct_pp32[3];
    const double* oct_w;                // [cell * (p+1)^3 + point]
    const float* oct_w32;               // the same rounded once to FP32
    const double* bern_q64[3];          // per direction [e][v][a][b][k]: Bernstein coefficients of basis products
    const float* bern_q32[3];
    const double* bern_qx64[3];         // WQ_OPT_TENSOR: per direction [e][a][b][k], phi_a' phi_b
    const float* bern_qx32[3];
    const double* bern_i64;             // [interval][k][g]: degree-2p Bernstein values at octree Gauss points
    const float* bern_i32;
    // fitted cut-element rule (WQ_OPT_MOMENT_FIT): the NK^3 tensor Gauss points of every cut
    // element replace its octree points in the slot layout; oct_w then holds their weights
    int fit;
    const double* fit_V64;              // [k][g]: degree-2p Bernstein polynomial k at fitted node g
    const float* fit_V32;
    int64_t n_cut_elems, n_cells;
    // slots
    int64_t n_grid, n_block, n_kappa;
};

// ----------------------------------------------------------------------------------------
// B-spline evaluation (local triangular scheme of the Cox-de Boor recursion)
// ----------------------------------------------------------------------------------------
// Knot span s with t[s] <= x < t[s+1] (non-empty), searched in [p, nt-p-2].
// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD b mod 8).
// Returns a logical index such that consecutive logical indices run on the same XCD, so
// workgroups that share data also share that XCD's L2.  A bijection of [0, n).
__device__ __host__ inline int xcd_logical(int b, int n) {
    constexpr int NX = 8;
    const int x = b % NX, q = n / NX, r = n % NX;
    return x * q + (x < r ? x : r) + b / NX;
}

// a * b + c with one rounding, for float and double
__device__ inline float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __host__ inline int find_span(const double* t, int nt, int p, double x) {
    int lo = p, hi = nt - p - 2;
    if (x >= t[hi + 1]) {
        while (hi > lo && t[hi] == t[hi + 1]) --hi;
        return hi;
    }
    while (lo < hi) {                      // largest s in [lo,hi] with t[s] <= x
        int mid = (lo + hi + 1) >> 1;
        if (t[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// N[r] = B_{s-p+r}(x), dN[r] = B'_{s-p+r}(x), r = 0..p.
__device__ __host__ inline void basis_funs(const double* t, int p, int s, double x, double* N, double* dN) {
    double left[WQ_PMAX + 1], right[WQ_PMAX + 1], Nm[WQ_PMAX + 1];
    N[0] = 1.0;
    for (int j = 1; j <= p; ++j) {
        left[j] = x - t[s + 1 - j];
        right[j] = t[s + j] - x;
        double saved = 0.0;
        for (int r = 0; r < j; ++r) {
            double tmp = N[r] / (right[r + 1] + left[j - r]);
            N[r] = saved + right[r + 1] * tmp;
            saved = left[j - r] * tmp;
        }
        N[j] = saved;
        if (j == p - 1)
            for (int r = 0; r <= j; ++r) Nm[r] = N[r];
    }
    if (p == 0) { dN[0] = 0.0; return; }
    if (p == 1) Nm[0] = 1.0;
    // B'_{i,p} = p/(t_{i+p}-t_i) B_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) B_{i+1,p-1}, i = s-p+r;
    // the degree p-1 functions at x are Nm[k] = B_{s-p+1+k,p-1}.
    for (int r = 0; r <= p; ++r) {
        int i = s - p + r;
        double v = 0.0;
        if (r >= 1) {
            double den = t[i + p] - t[i];
            if (den != 0.0) v += p * Nm[r - 1] / den;
        }
        if (r <= p - 1) {
            double den = t[i + p + 1] - t[i + 1];
            if (den != 0.0) v -= p * Nm[r] / den;
        }
        dN[r] = v;
    }
}

// ----------------------------------------------------------------------------------------
// Level set and box test
// ----------------------------------------------------------------------------------------
enum { CLS_OUT = 0, CLS_IN = 1, CLS_CUT = 2 };

__device__ __host__ inline double ls_phi(const wq_levelset& ls, double x, double y, double z) {
    if (ls.kind == 1) {
        double nn = sqrt(ls.n[0] * ls.n[0] + ls.n[1] * ls.n[1] + ls.n[2] * ls.n[2]);
        return (x * ls.n[0] + y * ls.n[1] + z * ls.n[2] - ls.r0) / nn;
    }
    if (ls.kind == 2) {
        double dx = x - ls.c[0], dy = y - ls.c[1], dz = z - ls.c[2];
        return sqrt(dx * dx + dy * dy + dz * dz) - ls.r0;
    }
    if (ls.kind == 3) {
        double rho = hypot(x - ls.c[0], y - ls.c[1]);
        return hypot(rho - ls.r0, z - ls.c[2]) - ls.r1;
    }
    return -1.0;
}

// Interior if max phi <= 0 on the box, exterior if min phi >= 0, cut otherwise.  Plane and
// ball use the exact extrema over the box, the torus the 1-Lipschitz bound at the centre.
__device__ __host__ inline int classify_box(const wq_levelset& ls, const double* lo, const double* hi) {
    if (ls.kind == 0) return CLS_IN;
    double vmin, vmax;
    if (ls.kind == 1) {
        vmin = 1e300; vmax = -1e300;
        for (int b = 0; b < 8; ++b) {
            double v = ls_phi(ls, (b & 4) ? hi[0] : lo[0], (b & 2) ? hi[1] : lo[1], (b & 1) ? hi[2] : lo[2]);
            vmin = fmin(vmin, v); vmax = fmax(vmax, v);
        }
    } else if (ls.kind == 2) {
        double dn = 0.0, df = 0.0;
        for (int d = 0; d < 3; ++d) {
            double c = ls.c[d];
            double nearest = fmin(fmax(c, lo[d]), hi[d]);
            double far = (fabs(lo[d] - c) > fabs(hi[d] - c)) ? lo[d] : hi[d];
            dn += (nearest - c) * (nearest - c);
            df += (far - c) * (far - c);
        }
        vmin = sqrt(dn) - ls.r0;
        vmax = sqrt(df) - ls.r0;
    } else {
        double m0 = 0.5 * (lo[0] + hi[0]), m1 = 0.5 * (lo[1] + hi[1]), m2 = 0.5 * (lo[2] + hi[2]);
        double d0 = hi[0] - lo[0], d1 = hi[1] - lo[1], d2 = hi[2] - lo[2];
        double hd = 0.5 * sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        double v = ls_phi(ls, m0, m1, m2);
        vmin = v - hd; vmax = v + hd;
    }
    if (vmax <= 0.0) return CLS_IN;
    if (vmin >= 0.0) return CLS_OUT;
    return CLS_CUT;
}

// ----------------------------------------------------------------------------------------
// Slot of a Gauss point (y1, y2, y3): the WQ grid when all three are WQ points, else the
// element's Gauss block.
// ----------------------------------------------------------------------------------------
// value along direction d of a triple given in the order (A, B, C) of directions (dA, dB,
// the remaining one): selects rather than an indexed array, so nothing goes to scratch
__device__ inline int pick3(int d, int dA, int dB, int a, int b, int c) { return d == dA ? a : (d == dB ? b : c); }

__device__ inline int64_t slot_of(const DevRules& R, int y1, int y2, int y3) {
    int x1 = R.y2x[0][y1], x2 = R.y2x[1][y2], x3 = R.y2x[2][y3];
    if (x1 >= 0 && x2 >= 0 && x3 >= 0) return ((int64_t)x1 * R.nx[1] + x2) * R.nx[2] + x3;
    int p1 = R.p + 1;
    int e1 = y1 / p1, e2 = y2 / p1, e3 = y3 / p1;
    int b = R.elem_block[((int64_t)e1 * R.nel[1] + e2) * R.nel[2] + e3];
    return R.n_grid + (int64_t)b * p1 * p1 * p1 + ((y1 % p1) * p1 + (y2 % p1)) * p1 + (y3 % p1);
}

// host-side error plumbing (defined in capi.cpp)
int wq_set_error(int code, const char* fmt, ...);
