// wq_build_rules: everything that does not depend on kappa, computed on the GPU in FP64.
//
// Gauss-Legendre rule (Newton on the three-term recurrence), WQ point layout and 1D WQ
// rules (Section 1 WQ ingredient, Section 2.2 step 1 and its last paragraph), function
// types (Section 2.1), CSR pattern, DWQ splits and one-sided rules (Section 2.2 steps 2-6),
// element Gauss blocks, octree cells for cut elements and the kappa slot layout.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rules.h"

// ----------------------------------------------------------------------------------------
// small device-wide exclusive scan (int32 counts -> int64 offsets)
// ----------------------------------------------------------------------------------------
static constexpr int SCAN_BLOCK = 256, SCAN_ITEMS = 4, SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

template <typename TIn>
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_tile(const TIn* in, int64_t* out, int64_t* tile_sum, int64_t n) {
    __shared__ int64_t s[SCAN_BLOCK];
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
    int64_t v[SCAN_ITEMS];
    int64_t acc = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        v[k] = (base + k < n) ? (int64_t)in[base + k] : 0;
        acc += v[k];
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < SCAN_BLOCK; off <<= 1) {
        int64_t t = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = s[threadIdx.x] - acc;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == SCAN_BLOCK - 1) tile_sum[blockIdx.x] = s[SCAN_BLOCK - 1];
}

__global__ void k_scan_add(int64_t* out, const int64_t* tile_off, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / SCAN_TILE];
}

// total = exclusive offset of the last tile + that tile's sum
__global__ void k_scan_total(const int64_t* tile_off, const int64_t* tile_sum, int64_t ntiles, int64_t* total) {
    *total = tile_off[ntiles - 1] + tile_sum[ntiles - 1];
}

// out[0..n) = exclusive prefix sums, out[n] = total; returns the total on the host.
template <typename TIn>
static int scan_exclusive(Builder& B, const TIn* in, int64_t* out, int64_t n, int64_t* total_host) {
    if (n == 0) {
        if (B.check(hipMemsetAsync(out, 0, sizeof(int64_t), B.stream))) return B.status;
        if (B.check(hipStreamSynchronize(B.stream))) return B.status;
        *total_host = 0;
        return 0;
    }
    int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int64_t* tsum = B.tmp<int64_t>(ntiles);
    int64_t* toff = B.tmp<int64_t>(ntiles + 1);
    if (!tsum || !toff) return B.status;
    hipLaunchKernelGGL(k_scan_tile<TIn>, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, B.stream, in, out, tsum, n);
    if (ntiles > 1) {
        int64_t dummy;
        if (scan_exclusive<int64_t>(B, tsum, toff, ntiles, &dummy)) return B.status;
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, B.stream, out, toff, n);
    } else {
        if (B.check(hipMemsetAsync(toff, 0, sizeof(int64_t), B.stream))) return B.status;
    }
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, B.stream, toff, tsum, ntiles, out + n);
    if (B.check(hipGetLastError())) return B.status;
    if (B.check(hipMemcpyAsync(total_host, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, B.stream))) return B.status;
    if (B.check(hipStreamSynchronize(B.stream))) return B.status;
    return 0;
}

// ----------------------------------------------------------------------------------------
// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n, evaluated by the
// three-term recurrence; P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1).
// ----------------------------------------------------------------------------------------
__global__ void k_gauss(int n, double* xi, double* w) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double x = cos(pi * (i + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            if (n == 1) { p1 = x; p0 = 1.0; }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
            double dx = p1 / dp;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        {   // final derivative at the converged node
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (x * p1 - p0) / (x * x - 1.0);
        }
        double wi = 2.0 / ((1.0 - x * x) * dp * dp);
        // ascending order: the largest node goes last
        xi[n - 1 - i] = x;  w[n - 1 - i] = wi;
        xi[i] = -x;         w[i] = wi;
    }
    if (n % 2 == 1) xi[n / 2] = 0.0;
}

// ----------------------------------------------------------------------------------------
// per-direction tables: Gauss points, basis values there, WQ point layout
// ----------------------------------------------------------------------------------------
__device__ inline double knot_at(int k, int p, int nel, double lo, double h) {
    int kk = k - p;
    kk = kk < 0 ? 0 : (kk > nel ? nel : kk);
    return lo + (double)kk * h;
}

// Element e keeps all p+1 Gauss points when it is a boundary element or p == 1, else the
// symmetric pair nearest its midpoint (excluding a node at the midpoint).
__device__ inline bool kept_point(int e, int g, int p, int nel) {
    if (e == 0 || e == nel - 1 || p == 1) return true;
    if (p % 2 == 0) return g == p / 2 - 1 || g == p / 2 + 1;
    return g == (p - 1) / 2 || g == (p + 1) / 2;
}

__global__ void k_dir_tables(DevRules R, int d, const double* gxi, double* ycoord, double* Bval, double* dBval,
                             int32_t* y2x, int32_t* x2y) {
    int y = blockIdx.x * blockDim.x + threadIdx.x;
    int p = R.p, p1 = p + 1, nel = R.nel[d];
    if (y >= nel * p1) return;
    int e = y / p1, g = y % p1;
    double x = R.lo[d] + (e + (1.0 + gxi[g]) / 2.0) * R.h[d];
    ycoord[y] = x;
    // knots of the direction (open uniform)
    double t[2 * WQ_PMAX + 2];
    // local window of knots: span of element e is knot index e + p
    int s = e + p;
    for (int k = 0; k < 2 * p + 2; ++k) t[k] = knot_at(s - p + k, p, nel, R.lo[d], R.h[d]);
    double N[WQ_PMAX + 1], dN[WQ_PMAX + 1];
    basis_funs(t, p, p, x, N, dN);        // span index p inside the local window
    for (int k = 0; k <= p; ++k) {
        Bval[(int64_t)y * p1 + k] = N[k];
        dBval[(int64_t)y * p1 + k] = dN[k];
    }
    // X index: kept points of the elements before e plus the rank inside e
    int before;
    if (e == 0) before = 0;
    else if (p == 1) before = 2 * e;
    else before = p1 + 2 * (e - 1);
    int rank = 0;
    bool kept = kept_point(e, g, p, nel);
    for (int gg = 0; gg < g; ++gg) rank += kept_point(e, gg, p, nel) ? 1 : 0;
    if (kept) {
        y2x[y] = before + rank;
        x2y[before + rank] = y;
    } else {
        y2x[y] = -1;
    }
}

// ----------------------------------------------------------------------------------------
// weighted-quadrature weights of one test function over a local knot vector
// ----------------------------------------------------------------------------------------
// T[0..nT): knots (non-decreasing); test function l (local index) of degree p, derivative
// order a; points xq[0..nq) inside supp B_l with their Gauss weights gq (physical).
// shortcut: use w_q = gq * B_l^(a)(x_q) (every element of the support keeps all its Gauss
// points).  Otherwise the minimum-norm solution of the exactness conditions
//   sum_q w_q B_j^(a)(x_q) = int B_l^(a) B_j^(a),  j overlapping l,
// by Householder QR of the transposed system with every condition scaled to unit norm
// (the solution does not depend on that scaling).  For a = 1 the conditions are posed on
// the degree p-1 B-splines N_k over the same knots that are nonzero on supp B_l: the B_j'
// are combinations of them and span the same space there (less one dimension, since they
// sum to zero), so sum_q w_q N_k(x_q) = int B_l' N_k fixes the same weights without a
// redundant condition.  Returns 0, or WQ_ESINGULAR when a pivot vanishes.
//
// Families of a full coefficient tensor (at = test derivative order, ac = trial derivative
// order): (0, 0) and (1, 1) above, and the mixed (1, 0) (conditions on the B_j, right-hand
// sides int B_l' B_j) and (0, 1) (conditions on the N_k, right-hand sides int B_l N_k).
__device__ int wq_local_rule(const double* T, int nT, int p, int l, int at, int ac, const double* xq, const double* gq,
                             int nq, bool shortcut, const double* gxi, const double* gw, double* w) {
    double N[WQ_PMAX + 1], dN[WQ_PMAX + 1];
    if (shortcut) {
        for (int q = 0; q < nq; ++q) {
            int s = find_span(T, nT, p, xq[q]);
            basis_funs(T, p, s, xq[q], N, dN);
            int r = l - (s - p);
            double b = (r >= 0 && r <= p) ? (at ? dN[r] : N[r]) : 0.0;
            w[q] = gq[q] * b;
        }
        return 0;
    }
    // condition functions: degree pc = p - ac over T, indices clo..chi (nonzero and
    // overlapping supp B_l)
    const int pc = p - ac;
    const int nfc = nT - pc - 1;
    double tl = T[l], tr = T[l + p + 1];
    int clo = -1, chi = -1;
    for (int j = 0; j < nfc; ++j) {
        if (T[j] == T[j + pc + 1]) continue;
        double a0 = fmax(tl, T[j]), b0 = fmin(tr, T[j + pc + 1]);
        if (a0 < b0) { if (clo < 0) clo = j; chi = j; }
    }
    int mc = chi - clo + 1;
    if (clo < 0 || mc > WQ_MMAX || nq < mc) return WQ_ESINGULAR;
    double At[WQ_NQREF][WQ_MMAX];
    double b[WQ_MMAX], beta[WQ_MMAX], diag[WQ_MMAX];
    double Nc[WQ_PMAX + 1], dNc[WQ_PMAX + 1];
    for (int q = 0; q < nq; ++q) {
        int s = find_span(T, nT, p, xq[q]);
        basis_funs(T, pc, s, xq[q], Nc, dNc);     // Nc[r] = N_{s-pc+r}
        for (int c = 0; c < mc; ++c) {
            int r = clo + c - (s - pc);
            At[q][c] = (r >= 0 && r <= pc) ? Nc[r] : 0.0;
        }
    }
    for (int c = 0; c < mc; ++c) b[c] = 0.0;
    for (int k = l; k <= l + p; ++k) {          // spans of supp B_l
        double t0 = T[k], t1 = T[k + 1];
        if (!(t0 < t1)) continue;
        for (int g = 0; g <= p; ++g) {
            double x = t0 + (1.0 + gxi[g]) / 2.0 * (t1 - t0);
            double wg = gw[g] * (t1 - t0) / 2.0;
            basis_funs(T, p, k, x, N, dN);
            double bl = at ? dN[l - (k - p)] : N[l - (k - p)];
            basis_funs(T, pc, k, x, Nc, dNc);
            for (int c = 0; c < mc; ++c) {
                int r = clo + c - (k - pc);
                if (r >= 0 && r <= pc) b[c] += wg * bl * Nc[r];
            }
        }
    }
    // unit-norm conditions
    for (int c = 0; c < mc; ++c) {
        double nrm = 0.0;
        for (int q = 0; q < nq; ++q) nrm += At[q][c] * At[q][c];
        if (!(nrm > 0.0)) return WQ_ESINGULAR;
        const double sc = 1.0 / sqrt(nrm);
        for (int q = 0; q < nq; ++q) At[q][c] *= sc;
        b[c] *= sc;
    }
    // Householder QR of At (nq x mc)
    double dmax = 0.0;
    for (int c = 0; c < mc; ++c) {
        double nrm = 0.0;
        for (int q = c; q < nq; ++q) nrm += At[q][c] * At[q][c];
        nrm = sqrt(nrm);
        double alpha = At[c][c] > 0 ? -nrm : nrm;
        At[c][c] -= alpha;
        double vn = 0.0;
        for (int q = c; q < nq; ++q) vn += At[q][c] * At[q][c];
        beta[c] = vn > 0.0 ? 2.0 / vn : 0.0;
        diag[c] = alpha;
        dmax = fmax(dmax, fabs(alpha));
        for (int c2 = c + 1; c2 < mc; ++c2) {
            double dot = 0.0;
            for (int q = c; q < nq; ++q) dot += At[q][c] * At[q][c2];
            dot *= beta[c];
            for (int q = c; q < nq; ++q) At[q][c2] -= dot * At[q][c];
        }
    }
    for (int c = 0; c < mc; ++c)
        if (!(fabs(diag[c]) > 1e-13 * dmax)) return WQ_ESINGULAR;
    // R^T y = b (R[c][c2] = At[c][c2] for c2 > c, diagonal diag[c])
    double y[WQ_MMAX];
    for (int c = 0; c < mc; ++c) {
        double s = b[c];
        for (int c0 = 0; c0 < c; ++c0) s -= At[c0][c] * y[c0];
        y[c] = s / diag[c];
    }
    for (int q = 0; q < nq; ++q) w[q] = q < mc ? y[q] : 0.0;
    for (int c = mc - 1; c >= 0; --c) {
        double dot = 0.0;
        for (int q = c; q < nq; ++q) dot += At[q][c] * w[q];
        dot *= beta[c];
        for (int q = c; q < nq; ++q) w[q] -= dot * At[q][c];
    }
    return 0;
}

// local knot window of function i: knots t_{i-p} .. t_{i+2p+1} (clamped), 3p+2 values;
// local function index of i is p.
__device__ inline void local_knots(const DevRules& R, int d, int i, double* T) {
    int p = R.p;
    for (int k = 0; k < 3 * p + 2; ++k) T[k] = knot_at(i - p + k, p, R.nel[d], R.lo[d], R.h[d]);
}

// ----------------------------------------------------------------------------------------
// standard 1D WQ rules: one thread per (direction, function, derivative order)
// ----------------------------------------------------------------------------------------
// nfam = 2: families (0, 0), (1, 1) into Wt; nfam = 4 adds (1, 0), (0, 1) into Wtx.
__global__ void k_std_rules(DevRules R, int d, int nfam, const double* gxi, const double* gw, int32_t* xs, int32_t* nwin,
                            double* Wt, double* Wtx, int8_t* qlo, int8_t* qhi, int* err) {
    int tid = blockIdx.x * blockDim.x + threadIdx.x;
    int n = R.nfun[d], p = R.p, p1 = p + 1, m = R.m, NW = R.nw, nel = R.nel[d];
    if (tid >= nfam * n) return;
    const int i = tid / nfam, f = tid % nfam;
    const int at = f == 0 || f == 3 ? 0 : 1, ac = f == 0 || f == 2 ? 0 : 1;
    const int a = f;                                   // a < 2: the (a, a) family
    int elo = i - p < 0 ? 0 : i - p, ehi = i < nel - 1 ? i : nel - 1;   // inclusive
    // points: X points of elements elo..ehi (contiguous X range)
    int x0 = -1, cnt = 0;
    bool all_gauss = true;
    double xq[WQ_NWMAX], gq[WQ_NWMAX];
    int yq[WQ_NWMAX];
    for (int e = elo; e <= ehi; ++e) {
        bool full = (e == 0 || e == nel - 1 || p == 1);
        all_gauss = all_gauss && full;
        for (int g = 0; g <= p; ++g) {
            int y = e * p1 + g;
            int x = R.y2x[d][y];
            if (x < 0) continue;
            if (x0 < 0) x0 = x;
            if (cnt < WQ_NWMAX) { xq[cnt] = R.ycoord[d][y]; gq[cnt] = gw[g] * R.h[d] / 2.0; yq[cnt] = y; }
            ++cnt;
        }
    }
    if (cnt > NW) { atomicExch(err, WQ_ESINGULAR); return; }
    if (a == 0) { xs[i] = x0; nwin[i] = cnt; }
    double T[3 * WQ_PMAX + 2];
    local_knots(R, d, i, T);
    double w[WQ_NQREF];
    int st = wq_local_rule(T, 3 * p + 2, p, p, at, ac, xq, gq, cnt, all_gauss, gxi, gw, w);
    if (st) { atomicExch(err, st); return; }
    // premultiply with the trial functions j = i-p+jj: W[jj][q] = w_q B_j^(ac)(x_q)
    double* out = f < 2 ? Wt + (((int64_t)i * 2 + f) * m) * NW : Wtx + (((int64_t)i * 2 + f - 2) * m) * NW;
    for (int jj = 0; jj < m; ++jj) {
        int j = i - p + jj;
        int lo = -1, hi = -1;
        for (int q = 0; q < NW; ++q) {
            double v = 0.0;
            if (q < cnt) {
                int y = yq[q], e = y / p1;
                int k = j - e;          // functions on element e are e..e+p
                if (k >= 0 && k <= p) {
                    double bj = ac ? R.dBval[d][(int64_t)y * p1 + k] : R.Bval[d][(int64_t)y * p1 + k];
                    v = w[q] * bj;
                    if (lo < 0) lo = q;
                    hi = q + 1;
                }
            }
            out[jj * NW + q] = v;
        }
        if (a == 0) {
            qlo[i * m + jj] = (int8_t)(lo < 0 ? 0 : lo);
            qhi[i * m + jj] = (int8_t)(lo < 0 ? 0 : hi);
        }
    }
}

// ----------------------------------------------------------------------------------------
// classification, active numbering, CSR pattern
// ----------------------------------------------------------------------------------------
__global__ void k_elem_class(DevRules R, int8_t* ecls) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ne = (int64_t)R.nel[0] * R.nel[1] * R.nel[2];
    if (id >= ne) return;
    int e3 = id % R.nel[2], e2 = (id / R.nel[2]) % R.nel[1], e1 = id / ((int64_t)R.nel[1] * R.nel[2]);
    int e[3] = {e1, e2, e3};
    double lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = R.lo[d] + e[d] * R.h[d];
        hi[d] = R.lo[d] + (e[d] + 1) * R.h[d];
    }
    ecls[id] = (int8_t)classify_box(R.ls, lo, hi);
}

__device__ inline void fun_support(const DevRules& R, const int* I, int* elo, int* ehi) {
    for (int d = 0; d < 3; ++d) {
        elo[d] = I[d] - R.p < 0 ? 0 : I[d] - R.p;
        ehi[d] = I[d] < R.nel[d] - 1 ? I[d] : R.nel[d] - 1;
    }
}

__device__ inline void unlex3(int64_t k, const int* n, int* I) {
    I[2] = (int)(k % n[2]);
    I[1] = (int)((k / n[2]) % n[1]);
    I[0] = (int)(k / ((int64_t)n[1] * n[2]));
}

__global__ void k_fun_class(DevRules R, const int8_t* ecls, int8_t* fcls, int32_t* active_flag) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nf = (int64_t)R.nfun[0] * R.nfun[1] * R.nfun[2];
    if (id >= nf) return;
    int I[3], lo[3], hi[3];
    unlex3(id, R.nfun, I);
    fun_support(R, I, lo, hi);
    int nin = 0, nout = 0, tot = 0;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int c = lo[2]; c <= hi[2]; ++c) {
                int8_t v = ecls[((int64_t)a * R.nel[1] + b) * R.nel[2] + c];
                nin += v == CLS_IN; nout += v == CLS_OUT; ++tot;
            }
    int8_t cl = nout == tot ? CLS_OUT : (nin == tot ? CLS_IN : CLS_CUT);
    fcls[id] = cl;
    active_flag[id] = cl != CLS_OUT;
}

__global__ void k_active_index(int64_t nf, const int32_t* flag, const int64_t* off, int32_t* lex2act, int32_t* act2lex) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nf) return;
    if (flag[id]) { lex2act[id] = (int32_t)off[id]; act2lex[off[id]] = (int32_t)id; }
    else lex2act[id] = -1;
}

__global__ void k_row_count(DevRules R, int64_t na, const int32_t* act2lex, const int8_t* fcls, int32_t* cnt,
                            int32_t* cut_flag, int all_rows) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    int I[3];
    unlex3(act2lex[r], R.nfun, I);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = I[d] - R.p < 0 ? 0 : I[d] - R.p;
        hi[d] = I[d] + R.p > R.nfun[d] - 1 ? R.nfun[d] - 1 : I[d] + R.p;
    }
    int c = 0;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int k = lo[2]; k <= hi[2]; ++k)
                c += fcls[((int64_t)a * R.nfun[1] + b) * R.nfun[2] + k] != CLS_OUT;
    cnt[r] = c;
    cut_flag[r] = all_rows || fcls[act2lex[r]] == CLS_CUT;      // all_rows: every row takes the cut-row path
}

__global__ void k_col_fill(DevRules R, int64_t na, const int32_t* act2lex, const int32_t* lex2act,
                           const int64_t* row_ptr, int32_t* col) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    int I[3];
    unlex3(act2lex[r], R.nfun, I);
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
        lo[d] = I[d] - R.p < 0 ? 0 : I[d] - R.p;
        hi[d] = I[d] + R.p > R.nfun[d] - 1 ? R.nfun[d] - 1 : I[d] + R.p;
    }
    int64_t k = row_ptr[r];
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int c = lo[2]; c <= hi[2]; ++c) {
                int32_t v = lex2act[((int64_t)a * R.nfun[1] + b) * R.nfun[2] + c];
                if (v >= 0) col[k++] = v;
            }
}

__global__ void k_cut_list(int64_t na, const int32_t* flag, const int64_t* off, int32_t* cut_rows, int32_t* act2cut) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= na) return;
    if (flag[r]) { cut_rows[off[r]] = (int32_t)r; act2cut[r] = (int32_t)off[r]; }
    else act2cut[r] = -1;
}

// ----------------------------------------------------------------------------------------
// DWQ split search (Section 2.2 step 2): the valid one-sided box with most elements,
// first strict maximum in the order d, s ascending, high side before low.
// ----------------------------------------------------------------------------------------
__device__ inline int dwq_key(const DevRules& R, int d, int i, int s, int high, int nmax) {
    int o = s - (i - R.p) - 1;        // 0..p-1
    return (((d * nmax) + i) * R.p + o) * 2 + (high ? 0 : 1);
}

// hybrid: no search, every cut row keeps its whole support for the element Gauss part.
__global__ void k_split(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex, const int8_t* ecls,
                        int4* split, int32_t* box, int32_t* key_used, int nmax, int hybrid) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int I[3], lo[3], hi[3];
    unlex3(act2lex[cut_rows[c]], R.nfun, I);
    fun_support(R, I, lo, hi);
    int best = 0, bd = -1, bs = 0, bh = 0;
    for (int d = 0; d < (hybrid ? 0 : 3); ++d) {
        for (int s = lo[d] + 1; s <= hi[d]; ++s) {
            for (int side = 0; side < 2; ++side) {
                int blo[3] = {lo[0], lo[1], lo[2]}, bhi[3] = {hi[0], hi[1], hi[2]};
                if (side == 0) blo[d] = s; else bhi[d] = s - 1;
                int cnt = (bhi[0] - blo[0] + 1) * (bhi[1] - blo[1] + 1) * (bhi[2] - blo[2] + 1);
                if (cnt <= best) continue;
                bool ok = true;
                for (int a = blo[0]; a <= bhi[0] && ok; ++a)
                    for (int b = blo[1]; b <= bhi[1] && ok; ++b)
                        for (int k = blo[2]; k <= bhi[2] && ok; ++k)
                            ok = ecls[((int64_t)a * R.nel[1] + b) * R.nel[2] + k] == CLS_IN;
                if (ok) { best = cnt; bd = d; bs = s; bh = side == 0; }
            }
        }
    }
    int4 sp;
    sp.x = bd; sp.y = bs; sp.z = bh; sp.w = -1;
    split[c] = sp;
    for (int d = 0; d < 3; ++d) {
        int blo = lo[d], bhi = hi[d];
        if (d == bd) { if (bh) blo = bs; else bhi = bs - 1; }
        box[c * 6 + 2 * d] = blo;
        box[c * 6 + 2 * d + 1] = bhi;
    }
    if (bd >= 0) key_used[dwq_key(R, bd, I[bd], bs, bh, nmax)] = 1;
}

__global__ void k_split_flag(int64_t ncut, const int4* split, int32_t* flag) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncut) flag[c] = split[c].x >= 0;
}

__global__ void k_split_rule(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex, int4* split,
                             const int64_t* key_off, int nmax) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int4 sp = split[c];
    if (sp.x < 0) return;
    int I[3];
    unlex3(act2lex[cut_rows[c]], R.nfun, I);
    sp.w = (int)key_off[dwq_key(R, sp.x, I[sp.x], sp.y, sp.z, nmax)];
    split[c] = sp;
}

// ----------------------------------------------------------------------------------------
// one-sided DWQ rules (Section 2.2 steps 3-6): one thread per distinct (d, i, s, side)
// ----------------------------------------------------------------------------------------
__global__ void k_dwq_rules(DevRules R, int nkeys, const int32_t* key_used, const int64_t* key_off, int nmax, int nfam,
                            const double* gxi, const double* gw, int32_t* np_out, int32_t* y_out, double* Wt, double* Wtx,
                            int* err) {
    int key = blockIdx.x * blockDim.x + threadIdx.x;
    if (key >= nkeys || !key_used[key]) return;
    int p = R.p, p1 = p + 1, m = R.m, NDQ = R.ndq;
    int high = (key & 1) == 0;
    int rest = key >> 1;
    int o = rest % p; rest /= p;
    int i = rest % nmax; int d = rest / nmax;
    int s = i - p + 1 + o;
    int nel = R.nel[d];
    int r = (int)key_off[key];
    // step 3: local knots of B_i with s inserted to multiplicity p+1, and S (Boehm)
    double T[4 * WQ_PMAX + 2];
    int nT = 3 * p + 2;
    local_knots(R, d, i, T);
    double S[3 * WQ_PMAX + 1];
    int nf = nT - p - 1;                      // 2p+1 local functions, B_i is local p
    for (int l = 0; l < nf; ++l) S[l] = (l == p) ? 1.0 : 0.0;
    double xi_s = R.lo[d] + (double)s * R.h[d];
    for (int ins = 0; ins < p; ++ins) {
        int k = 0;                            // last index with T[k] <= xi_s
        for (int q = 0; q < nT; ++q) if (T[q] <= xi_s) k = q;
        double Sn[3 * WQ_PMAX + 2];
        for (int l = 0; l <= nf; ++l) {
            if (l <= k - p) Sn[l] = S[l];
            else if (l >= k + 1) Sn[l] = S[l - 1];
            else {
                double al = (xi_s - T[l]) / (T[l + p] - T[l]);
                Sn[l] = al * S[l] + (1.0 - al) * S[l - 1];
            }
        }
        for (int q = nT; q > k + 1; --q) T[q] = T[q - 1];
        T[k + 1] = xi_s;
        ++nT; ++nf;
        for (int l = 0; l < nf; ++l) S[l] = Sn[l];
    }
    // step 4: points of the kept side inside supp B_i; nested points = all Gauss points of
    // the element next to the break on that side
    int elo = i - p < 0 ? 0 : i - p, ehi = i < nel - 1 ? i : nel - 1;
    int slo = high ? s : elo, shi = high ? ehi : s - 1;
    int estar = high ? s : s - 1;
    double xq[WQ_NDQMAX], gq[WQ_NDQMAX];
    int yq[WQ_NDQMAX], eq[WQ_NDQMAX];
    int nq = 0;
    for (int e = slo; e <= shi; ++e) {
        bool full = (e == estar) || e == 0 || e == nel - 1 || p == 1;
        for (int g = 0; g <= p; ++g) {
            int y = e * p1 + g;
            if (!full && R.y2x[d][y] < 0) continue;
            if (nq >= NDQ) { atomicExch(err, WQ_ESINGULAR); return; }
            xq[nq] = R.ycoord[d][y]; gq[nq] = gw[g] * R.h[d] / 2.0; yq[nq] = y; eq[nq] = e;
            ++nq;
        }
    }
    np_out[r] = nq;
    for (int q = 0; q < NDQ; ++q) y_out[(int64_t)r * NDQ + q] = q < nq ? yq[q] : yq[0];
    double wacc[4][WQ_NDQMAX];
    for (int a = 0; a < nfam; ++a)
        for (int q = 0; q < nq; ++q) wacc[a][q] = 0.0;
    double side_lo = R.lo[d] + (double)slo * R.h[d], side_hi = R.lo[d] + (double)(shi + 1) * R.h[d];
    // step 5: WQ weights of every refined function on the kept side inside supp B_i
    for (int l = 0; l < nf; ++l) {
        double tl = T[l], tr = T[l + p + 1];
        if (!(tl < tr) || tl < side_lo || tr > side_hi) continue;
        double xl[WQ_NQREF], gl[WQ_NQREF];
        int map[WQ_NQREF];
        int nl = 0;
        bool all_gauss = true;
        for (int q = 0; q < nq; ++q) {
            if (xq[q] > tl && xq[q] < tr) { xl[nl] = xq[q]; gl[nl] = gq[q]; map[nl] = q; ++nl; }
        }
        // refined layout: full Gauss in e*, the boundary elements, or everywhere when p = 1
        for (int e = slo; e <= shi; ++e) {
            double e0 = R.lo[d] + (double)e * R.h[d], e1 = R.lo[d] + (double)(e + 1) * R.h[d];
            if (e0 >= tl && e1 <= tr) {
                bool full = (e == estar) || e == 0 || e == nel - 1 || p == 1;
                all_gauss = all_gauss && full;
            }
        }
        for (int a = 0; a < nfam; ++a) {
            double wl[WQ_NQREF];
            const int at = a == 0 || a == 3 ? 0 : 1, ac = a == 0 || a == 2 ? 0 : 1;
            int st = wq_local_rule(T, nT, p, l, at, ac, xl, gl, nl, all_gauss, gxi, gw, wl);
            if (st) { atomicExch(err, st); return; }
            // step 6: w = sum_l S_il wtilde_l
            for (int q = 0; q < nl; ++q) wacc[a][map[q]] += S[l] * wl[q];
        }
    }
    // premultiply with the original trial functions j = i-p+jj
    for (int a = 0; a < nfam; ++a) {
        const int ac = a == 0 || a == 2 ? 0 : 1;
        double* out = a < 2 ? Wt + (((int64_t)r * 2 + a) * m) * NDQ : Wtx + (((int64_t)r * 2 + a - 2) * m) * NDQ;
        for (int jj = 0; jj < m; ++jj) {
            int j = i - p + jj;
            for (int q = 0; q < NDQ; ++q) {
                double v = 0.0;
                if (q < nq) {
                    int k = j - eq[q];
                    if (k >= 0 && k <= p) {
                        int y = yq[q];
                        v = wacc[a][q] * (ac ? R.dBval[d][(int64_t)y * p1 + k] : R.Bval[d][(int64_t)y * p1 + k]);
                    }
                }
                out[jj * NDQ + q] = v;
            }
        }
    }
}

// position of each pattern entry of a cut row in a dense (2p+1)^3 window
__global__ void k_pos_map(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex,
                          const int64_t* row_ptr, const int32_t* col, int32_t* pos) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int m = R.m, m3 = m * m * m;
    int32_t* P = pos + c * (int64_t)m3;
    for (int k = 0; k < m3; ++k) P[k] = -1;
    int r = cut_rows[c];
    int I[3];
    unlex3(act2lex[r], R.nfun, I);
    for (int64_t k = row_ptr[r]; k < row_ptr[r + 1]; ++k) {
        int J[3];
        unlex3(act2lex[col[k]], R.nfun, J);
        int jj = ((J[0] - I[0] + R.p) * m + (J[1] - I[1] + R.p)) * m + (J[2] - I[2] + R.p);
        P[jj] = (int32_t)(k - row_ptr[r]);
    }
}

// ----------------------------------------------------------------------------------------
// interior row line blocks: runs of interior functions along direction 1
// ----------------------------------------------------------------------------------------
__global__ void k_line_count(DevRules R, const int8_t* fcls, int rb, int32_t* cnt) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
    if (id >= nl) return;
    int c = 0, run = 0;
    for (int i1 = 0; i1 <= R.nfun[0]; ++i1) {
        bool in = i1 < R.nfun[0] && fcls[(int64_t)i1 * nl + id] == CLS_IN;
        if (in) ++run;
        else { c += (run + rb - 1) / rb; run = 0; }
    }
    cnt[id] = c;
}

__global__ void k_line_fill(DevRules R, const int8_t* fcls, int rb, const int64_t* off, int4* blocks) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
    if (id >= nl) return;
    int i2 = (int)(id / R.nfun[2]), i3 = (int)(id % R.nfun[2]);
    int64_t k = off[id];
    int run = 0;
    for (int i1 = 0; i1 <= R.nfun[0]; ++i1) {
        bool in = i1 < R.nfun[0] && fcls[(int64_t)i1 * nl + id] == CLS_IN;
        if (in) { ++run; continue; }
        int start = i1 - run;
        while (run > 0) {
            int c = run < rb ? run : rb;
            blocks[k++] = make_int4(start, i2, i3, c);
            start += c; run -= c;
        }
    }
}

// ----------------------------------------------------------------------------------------
// element Gauss blocks: interior elements in the support of a cut function
// ----------------------------------------------------------------------------------------
__global__ void k_mark_blocks(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex,
                              const int8_t* ecls, int32_t* flag) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int I[3], lo[3], hi[3];
    unlex3(act2lex[cut_rows[c]], R.nfun, I);
    fun_support(R, I, lo, hi);
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                int64_t e = ((int64_t)a * R.nel[1] + b) * R.nel[2] + k;
                if (ecls[e] == CLS_IN) flag[e] = 1;
            }
}

// Remainder elements of each cut row: interior elements of its support outside its DWQ box,
// lexicographic.  Entry = (offsets I_d - e_d packed 4 bits each, element's block index).
template <bool FILL>
__global__ void k_rem_list(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex, const int8_t* ecls,
                           const int32_t* box, const int32_t* eblock, int32_t* cnt, const int64_t* off, int2* list) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int I[3], lo[3], hi[3];
    unlex3(act2lex[cut_rows[c]], R.nfun, I);
    fun_support(R, I, lo, hi);
    const int* bx = box + c * 6;
    const bool has_box = R.split[c].x >= 0;
    int32_t n = 0;
    int64_t o = FILL ? off[c] : 0;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                const int64_t e = ((int64_t)a * R.nel[1] + b) * R.nel[2] + k;
                const bool inbox = has_box && a >= bx[0] && a <= bx[1] && b >= bx[2] && b <= bx[3] && k >= bx[4] &&
                                   k <= bx[5];
                if (ecls[e] != CLS_IN || inbox) continue;
                if (FILL) list[o + n] = make_int2((I[0] - a) | (I[1] - b) << 4 | (I[2] - k) << 8, eblock[e]);
                ++n;
            }
    if (!FILL) cnt[c] = n;
}

// Cut elements of each cut row's support, lexicographic.  Entry = (cut element index, offsets
// I_d - e_d packed 4 bits each).
template <bool FILL>
__global__ void k_rowcut_list(DevRules R, int64_t ncut, const int32_t* cut_rows, const int32_t* act2lex, const int8_t* ecls,
                              const int32_t* ceidx, int32_t* cnt, const int64_t* off, int2* list) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncut) return;
    int I[3], lo[3], hi[3];
    unlex3(act2lex[cut_rows[c]], R.nfun, I);
    fun_support(R, I, lo, hi);
    int32_t n = 0;
    const int64_t o = FILL ? off[c] : 0;
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b)
            for (int k = lo[2]; k <= hi[2]; ++k) {
                const int64_t e = ((int64_t)a * R.nel[1] + b) * R.nel[2] + k;
                if (ecls[e] != CLS_CUT) continue;
                if (FILL) list[o + n] = make_int2(ceidx[e], (I[0] - a) | (I[1] - b) << 4 | (I[2] - k) << 8);
                ++n;
            }
    if (!FILL) cnt[c] = n;
}

__global__ void k_flag_index(int64_t n, const int32_t* flag, const int64_t* off, int32_t* idx, int32_t* list) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    if (flag[e]) { idx[e] = (int32_t)off[e]; list[off[e]] = (int32_t)e; }
    else idx[e] = -1;
}

__global__ void k_flag_eq(int64_t n, const int8_t* v, int8_t want, int32_t* flag) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) flag[e] = v[e] == want;
}

// ----------------------------------------------------------------------------------------
// octree of a cut element: depth-first, children in lexicographic order (first offset
// bit slowest); leaves are interior cells at any depth and cut cells at depth L.
// ----------------------------------------------------------------------------------------
// cell key: depth | offx << 3 | offy << 9 | offz << 15 (offsets in units of h / 2^depth)
template <bool FILL>
__global__ void k_octree(DevRules R, int64_t nce, const int32_t* cut_elems, int32_t* cnt, const int64_t* begin,
                         double* cell_lo, int8_t* cell_depth, int8_t* cell_cut, int32_t* cell_elem, int32_t* cell_key) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nce) return;
    int64_t eid = cut_elems[c];
    int e[3];
    e[2] = (int)(eid % R.nel[2]); e[1] = (int)((eid / R.nel[2]) % R.nel[1]);
    e[0] = (int)(eid / ((int64_t)R.nel[1] * R.nel[2]));
    int L = R.levels;
    // stack of (depth, off0, off1, off2)
    int sd[8 * 6 + 1], so[8 * 6 + 1][3];
    int top = 0;
    sd[0] = 0; so[0][0] = so[0][1] = so[0][2] = 0; top = 1;
    int64_t k = FILL ? begin[c] : 0;
    int n = 0;
    while (top > 0) {
        --top;
        int dep = sd[top];
        int off[3] = {so[top][0], so[top][1], so[top][2]};
        int scale = 1 << dep;
        double lo[3], hi[3], size[3];
        for (int d = 0; d < 3; ++d) {
            size[d] = R.h[d] / scale;
            lo[d] = R.lo[d] + ((double)e[d] * scale + off[d]) * (R.h[d] / scale);
            hi[d] = lo[d] + size[d];
        }
        int cls = dep > 0 ? classify_box(R.ls, lo, hi) : CLS_CUT;
        if (cls == CLS_OUT) continue;
        if (cls == CLS_IN || dep == L) {
            if (FILL) {
                for (int d = 0; d < 3; ++d) cell_lo[k * 3 + d] = lo[d];
                cell_depth[k] = (int8_t)dep;
                cell_cut[k] = (int8_t)(cls != CLS_IN);
                cell_elem[k] = (int32_t)c;
                cell_key[k] = dep | (off[0] << 3) | (off[1] << 9) | (off[2] << 15);
                ++k;
            }
            ++n;
            continue;
        }
        for (int b = 7; b >= 0; --b) {        // push in reverse so child 0 is visited first
            sd[top] = dep + 1;
            so[top][0] = 2 * off[0] + ((b >> 2) & 1);
            so[top][1] = 2 * off[1] + ((b >> 1) & 1);
            so[top][2] = 2 * off[2] + (b & 1);
            ++top;
        }
    }
    if (!FILL) cnt[c] = n;
}

// Per cut element: leaves ordered by key, so that leaves sharing an x-interval (same depth
// and x offset) are contiguous and, inside, leaves sharing an (x, y) column are contiguous.
__global__ void k_octree_sort(int64_t nce, const int64_t* begin, const int32_t* cell_key, int32_t* perm) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nce) return;
    const int64_t b = begin[c], e = begin[c + 1];
    for (int64_t k = b; k < e; ++k) {          // insertion sort by (depth, offx, offy, offz)
        const int32_t v = (int32_t)k;
        const int32_t key = cell_key[k];
        const int32_t kk = (key & 7) << 18 | ((key >> 3) & 63) << 12 | ((key >> 9) & 63) << 6 | ((key >> 15) & 63);
        int64_t j = k - 1;
        while (j >= b) {
            const int32_t o = cell_key[perm[j]];
            const int32_t ok = (o & 7) << 18 | ((o >> 3) & 63) << 12 | ((o >> 9) & 63) << 6 | ((o >> 15) & 63);
            if (ok <= kk) break;
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

// Counts of x-groups (leaves sharing depth and x offset) and columns (sharing depth, x and y
// offsets) over all cut elements, from the sorted leaf order.
__global__ void k_octree_groups(int64_t nce, const int64_t* begin, const int32_t* cell_key, const int32_t* perm,
                                unsigned long long* counts) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nce) return;
    unsigned long long nx = 0, ncol = 0;
    int32_t prev = -1;
    for (int64_t k = begin[c]; k < begin[c + 1]; ++k) {
        const int32_t key = cell_key[perm[k]];
        if (prev < 0 || (key & 511) != (prev & 511)) ++nx;
        if (prev < 0 || (key & 32767) != (prev & 32767)) ++ncol;
        prev = key;
    }
    atomicAdd(&counts[0], nx);
    atomicAdd(&counts[1], ncol);
}

// 1D basis products of element e's functions at the Gauss points of each octree interval
// (depth l, offset o; index 2^l - 1 + o) in direction d:
// pp[((e * NI + iv) * 2 + v) * P1^2 + a * P1 + b][g] = phi_a phi_b (v = 0) or phi_a' phi_b' (v = 1),
// with the leaf coordinates formed exactly as for the octree weights.
__global__ void k_oct_basis(DevRules R, int d, const double* gxi, double* pp) {
    const int p = R.p, p1 = p + 1, p2 = p1 * p1;
    const int ni = (2 << R.levels) - 1;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)R.nel[d] * ni * p1) return;
    const int g = (int)(id % p1);
    const int iv = (int)((id / p1) % ni);
    const int e = (int)(id / ((int64_t)p1 * ni));
    int dep = 0;
    while ((2 << dep) - 1 <= iv) ++dep;
    const int off = iv - ((1 << dep) - 1);
    const int scale = 1 << dep;
    const double size = R.h[d] / scale;
    const double lo = R.lo[d] + ((double)e * scale + off) * (R.h[d] / scale);
    const double x = lo + (1.0 + gxi[g]) / 2.0 * size;
    double kn[2 * WQ_PMAX + 2];
    for (int j = 0; j < 2 * p + 2; ++j) kn[j] = knot_at(e + j, p, R.nel[d], R.lo[d], R.h[d]);
    double N[WQ_PMAX + 1], dN[WQ_PMAX + 1];
    basis_funs(kn, p, p, x, N, dN);
    double* out = pp + ((int64_t)e * ni + iv) * 2 * p2 * p1;
    for (int a = 0; a < p1; ++a)
        for (int b = 0; b < p1; ++b) {
            out[(a * p1 + b) * p1 + g] = N[a] * N[b];
            out[p2 * p1 + (a * p1 + b) * p1 + g] = dN[a] * dN[b];
        }
}

// Bernstein form of the cut-element integrand.  On element e of direction d the local
// functions phi_a (a = 0..p, phi_a = B_{e+a}) are degree-p polynomials; their products are
// degree 2p.  Q[((e * 2 + v) * P1^2 + a * P1 + b) * (2p+1) + k] holds the degree-2p
// Bernstein coefficients (in the element's local coordinate t in [0, 1]) of
// phi_a phi_b (v = 0) and of phi_a' phi_b' (v = 1, physical derivatives).
__device__ inline double binom(int n, int k) {
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

__device__ inline double bernstein(int n, int k, double t) {
    double r = binom(n, k);
    for (int i = 0; i < k; ++i) r *= t;
    for (int i = 0; i < n - k; ++i) r *= 1.0 - t;
    return r;
}

// Bernstein coefficients cb[a][i] of phi_a (degree p) and db[a][i] of phi_a' (degree p - 1) on
// element e of direction d.
__device__ void elem_bernstein(const DevRules& R, int d, int e, double cb[][WQ_PMAX + 1], double db[][WQ_PMAX + 1]) {
    const int p = R.p;
    const double h = R.h[d];
    double kn[2 * WQ_PMAX + 2];
    for (int j = 0; j < 2 * p + 2; ++j) kn[j] = knot_at(e + j, p, R.nel[d], R.lo[d], h);
    for (int a = 0; a <= p; ++a)
        for (int i = 0; i <= p; ++i) {
            double dv[WQ_PMAX + 1];
            for (int j = 0; j <= p; ++j) dv[j] = j == a ? 1.0 : 0.0;
            for (int rr = 1; rr <= p; ++rr) {
                const double u = rr <= p - i ? kn[p] : kn[p + 1];
                for (int j = p; j >= rr; --j) {
                    const double al = (u - kn[j]) / (kn[j + 1 + p - rr] - kn[j]);
                    dv[j] = (1.0 - al) * dv[j - 1] + al * dv[j];
                }
            }
            cb[a][i] = dv[p];
        }
    for (int a = 0; a <= p; ++a)
        for (int i = 0; i < p; ++i) db[a][i] = p * (cb[a][i + 1] - cb[a][i]) / h;
}

// Qx[((e * P1 + a) * P1 + b) * (2p+1) + k]: degree-2p Bernstein coefficients of phi_a' phi_b
// (degree 2p - 1 raised once), the mixed products of the coefficient-tensor stiffness.
__global__ void k_bern_mixed(DevRules R, int d, double* Qx) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R.nel[d]) return;
    const int p = R.p, p1 = p + 1, nk = 2 * p + 1;
    double cb[WQ_PMAX + 1][WQ_PMAX + 1], db[WQ_PMAX + 1][WQ_PMAX + 1];
    elem_bernstein(R, d, e, cb, db);
    const int n = 2 * p - 1;
    for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) {
            double r[2 * WQ_PMAX + 1];
            for (int k = 0; k <= n; ++k) {
                double s = 0.0;
                for (int i = 0; i < p; ++i) {
                    const int j = k - i;
                    if (j < 0 || j > p) continue;
                    s += db[a][i] * cb[b][j] * binom(p - 1, i) * binom(p, j);
                }
                r[k] = s / binom(n, k);
            }
            double* q = Qx + (((int64_t)e * p1 + a) * p1 + b) * nk;
            for (int k = 0; k <= n + 1; ++k) {              // degree n -> n + 1
                const double lo = k > 0 ? r[k - 1] : 0.0, hi = k <= n ? r[k] : 0.0;
                q[k] = (double)k / (n + 1) * lo + (1.0 - (double)k / (n + 1)) * hi;
            }
        }
}

__global__ void k_bern_products(DevRules R, int d, double* Q) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= R.nel[d]) return;
    const int p = R.p, p1 = p + 1, nk = 2 * p + 1;
    const double h = R.h[d];
    double kn[2 * WQ_PMAX + 2];
    for (int j = 0; j < 2 * p + 2; ++j) kn[j] = knot_at(e + j, p, R.nel[d], R.lo[d], h);
    // Bernstein coefficients of phi_a on the element: the blossom of the polynomial piece at
    // (left end repeated p-i times, right end repeated i times), evaluated by de Boor's
    // algorithm on the unit control vector of phi_a.  Every step is a convex combination, so
    // coefficients are accurate relative to themselves and structural zeros stay exact.
    double cb[WQ_PMAX + 1][WQ_PMAX + 1];               // cb[a][i]: Bernstein coefficients of phi_a
    for (int a = 0; a <= p; ++a)
        for (int i = 0; i <= p; ++i) {
            double dv[WQ_PMAX + 1];
            for (int j = 0; j <= p; ++j) dv[j] = j == a ? 1.0 : 0.0;
            for (int rr = 1; rr <= p; ++rr) {
                const double u = rr <= p - i ? kn[p] : kn[p + 1];
                for (int j = p; j >= rr; --j) {
                    const double al = (u - kn[j]) / (kn[j + 1 + p - rr] - kn[j]);
                    dv[j] = (1.0 - al) * dv[j - 1] + al * dv[j];
                }
            }
            cb[a][i] = dv[p];
        }
    // derivative: degree p-1 coefficients p (c_{i+1} - c_i) / h
    double db[WQ_PMAX + 1][WQ_PMAX + 1];
    for (int a = 0; a <= p; ++a)
        for (int i = 0; i < p; ++i) db[a][i] = p * (cb[a][i + 1] - cb[a][i]) / h;
    for (int a = 0; a <= p; ++a)
        for (int b = 0; b <= p; ++b) {
            double* q0 = Q + (((int64_t)e * 2 + 0) * p1 * p1 + a * p1 + b) * nk;
            double* q1 = Q + (((int64_t)e * 2 + 1) * p1 * p1 + a * p1 + b) * nk;
            for (int k = 0; k < nk; ++k) {
                double s = 0.0;
                for (int i = 0; i <= p; ++i) {
                    const int j = k - i;
                    if (j < 0 || j > p) continue;
                    s += cb[a][i] * cb[b][j] * binom(p, i) * binom(p, j);
                }
                q0[k] = s / binom(2 * p, k);
            }
            // derivative product: degree 2p-2, then raised twice to degree 2p
            double r[2 * WQ_PMAX + 1], r2[2 * WQ_PMAX + 1];
            const int n = 2 * p - 2;
            for (int k = 0; k <= n; ++k) {
                double s = 0.0;
                for (int i = 0; i < p; ++i) {
                    const int j = k - i;
                    if (j < 0 || j > p - 1) continue;
                    s += db[a][i] * db[b][j] * binom(p - 1, i) * binom(p - 1, j);
                }
                r[k] = s / binom(n, k);
            }
            for (int m = n; m < 2 * p; ++m) {          // degree m -> m + 1
                for (int k = 0; k <= m + 1; ++k) {
                    const double lo = k > 0 ? r[k - 1] : 0.0, hi = k <= m ? r[k] : 0.0;
                    r2[k] = (double)k / (m + 1) * lo + (1.0 - (double)k / (m + 1)) * hi;
                }
                for (int k = 0; k <= m + 1; ++k) r[k] = r2[k];
            }
            for (int k = 0; k < nk; ++k) q1[k] = r[k];
        }
}

// B[(iv * (2p+1) + k) * P1 + g]: degree-2p Bernstein polynomial k at the g-th Gauss point of
// octree interval iv (depth l, offset o: iv = 2^l - 1 + o), in the element's local coordinate.
__global__ void k_bern_intervals(DevRules R, const double* gxi, double* B) {
    const int p = R.p, p1 = p + 1, nk = 2 * p + 1;
    const int ni = (2 << R.levels) - 1;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ni * nk * p1) return;
    const int g = id % p1, k = (id / p1) % nk, iv = id / (p1 * nk);
    int dep = 0;
    while ((2 << dep) - 1 <= iv) ++dep;
    const int off = iv - ((1 << dep) - 1);
    const double t = (off + (1.0 + gxi[g]) / 2.0) / (double)(1 << dep);
    B[id] = bernstein(2 * p, k, t);
}

__global__ void k_octree_weights(DevRules R, const double* gxi, const double* gw, const double* cell_lo,
                                 const int8_t* cell_depth, const int8_t* cell_cut, double* w, double* xyz) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int p1 = R.p + 1, npc = p1 * p1 * p1;
    if (id >= R.n_cells * npc) return;
    int64_t cell = id / npc;
    int pt = (int)(id % npc);
    int g[3] = {pt / (p1 * p1), (pt / p1) % p1, pt % p1};
    int scale = 1 << cell_depth[cell];
    double x[3], wt = 1.0;
    for (int d = 0; d < 3; ++d) {
        double size = R.h[d] / scale;
        x[d] = cell_lo[cell * 3 + d] + (1.0 + gxi[g[d]]) / 2.0 * size;
        wt *= gw[g[d]] * size / 2.0;
    }
    if (cell_cut[cell] && !(ls_phi(R.ls, x[0], x[1], x[2]) < 0.0)) wt = 0.0;
    w[id] = wt;
    int64_t s = R.n_grid + R.n_block + id;
    xyz[s * 3 + 0] = x[0]; xyz[s * 3 + 1] = x[1]; xyz[s * 3 + 2] = x[2];
}

// Legendre polynomial L_k(x), k <= 2p, by the three-term recurrence
__device__ inline double legendre(int k, double x) {
    double l0 = 1.0, l1 = x;
    if (k == 0) return l0;
    for (int n = 1; n < k; ++n) {
        const double l2 = ((2 * n + 1) * x * l1 - n * l0) / (n + 1);
        l0 = l1; l1 = l2;
    }
    return l1;
}

// L[(iv * (2p+1) + k) * P1 + g]: L_k(2t - 1) at the g-th Gauss point t of octree interval iv
// (the layout of k_bern_intervals); the fitted rule's moments are taken in this basis.
__global__ void k_leg_intervals(DevRules R, const double* gxi, double* L) {
    const int p = R.p, p1 = p + 1, nk = 2 * p + 1;
    const int ni = (2 << R.levels) - 1;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= ni * nk * p1) return;
    const int g = id % p1, k = (id / p1) % nk, iv = id / (p1 * nk);
    int dep = 0;
    while ((2 << dep) - 1 <= iv) ++dep;
    const int off = iv - ((1 << dep) - 1);
    const double t = (off + (1.0 + gxi[g]) / 2.0) / (double)(1 << dep);
    L[id] = legendre(k, 2.0 * t - 1.0);
}

// Fitted cut rule tables.  V[k][g] = B_k(tau_g), the degree-2p Bernstein polynomials at the NK
// Gauss nodes tau_g = (1 + xi_g) / 2 of the element (the assembly forms Bernstein moments on the
// fitted points with it).  Ainv[g][k] = W_g (2k + 1) / 2 L_k(xi_g) is the inverse of the Legendre
// matrix [k][g] = L_k(xi_g): the NK-point Gauss rule integrates L_k L_j (degree <= 4p < 2 NK)
// exactly, so sum_g L_k(xi_g) Ainv[g][j] is the orthogonality relation.  The fitted weights are
// Ainv applied to the Legendre moments in each direction; Legendre moments of a positive rule are
// bounded by its total weight and Ainv's entries by (2p + 1) / 2 * W_g, so nothing cancels
// beyond the final sums (an inverse Bernstein matrix grows with the degree).
__global__ void k_fit_tables(int p, const double* xi, const double* wg, double* V, double* Ainv) {
    const int nk = 2 * p + 1;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nk * nk) return;
    const int a = id / nk, b = id % nk;
    V[id] = bernstein(2 * p, a, 0.5 * (1.0 + xi[b]));              // [k = a][g = b]
    Ainv[id] = wg[a] * (2 * b + 1) * 0.5 * legendre(b, xi[a]);      // [g = a][k = b]
}

// fitted weights of one cut element: w[g1 g2 g3] = sum_k Ainv[g1][k1] Ainv[g2][k2] Ainv[g3][k3] m[k],
// m the Legendre moments of the element's octree rule (kappa = 1); one workgroup per element
__global__ void __launch_bounds__(256) k_fit_weights(int p, const double* Ainv, const double* m, double* w) {
    const int nk = 2 * p + 1, nk2 = nk * nk, nk3 = nk2 * nk;
    __shared__ double s_a[WQ_MMAX * WQ_MMAX * WQ_MMAX], s_b[WQ_MMAX * WQ_MMAX * WQ_MMAX];
    __shared__ double s_ai[WQ_MMAX * WQ_MMAX];
    const int64_t ce = blockIdx.x;
    for (int i = threadIdx.x; i < nk2; i += blockDim.x) s_ai[i] = Ainv[i];
    for (int i = threadIdx.x; i < nk3; i += blockDim.x) s_a[i] = m[ce * nk3 + i];
    __syncthreads();
    for (int i = threadIdx.x; i < nk3; i += blockDim.x) {      // [k1 k2][g3]
        const int k12 = i / nk, g3 = i % nk;
        double v = 0.0;
        for (int k3 = 0; k3 < nk; ++k3) v += s_ai[g3 * nk + k3] * s_a[k12 * nk + k3];
        s_b[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nk3; i += blockDim.x) {      // [k1][g2 g3]
        const int k1 = i / nk2, g2 = (i / nk) % nk, g3 = i % nk;
        double v = 0.0;
        for (int k2 = 0; k2 < nk; ++k2) v += s_ai[g2 * nk + k2] * s_b[(k1 * nk + k2) * nk + g3];
        s_a[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nk3; i += blockDim.x) {      // [g1][g2 g3]
        const int g1 = i / nk2, g23 = i % nk2;
        double v = 0.0;
        for (int k1 = 0; k1 < nk; ++k1) v += s_ai[g1 * nk + k1] * s_a[k1 * nk2 + g23];
        w[ce * nk3 + i] = v;
    }
}

// coordinates of the fitted points: slot n_grid + n_block + ce * NK^3 + g, g lexicographic
__global__ void k_fit_xyz(DevRules R, int64_t nce, const int32_t* cut_elems, const double* xi, int64_t base,
                          double* xyz) {
    const int nk = 2 * R.p + 1, nk3 = nk * nk * nk;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nce * nk3) return;
    const int64_t ce = id / nk3;
    const int g = (int)(id % nk3), g1 = g / (nk * nk), g2 = (g / nk) % nk, g3 = g % nk;
    const int64_t eid = cut_elems[ce];
    const int e3 = (int)(eid % R.nel[2]), e2 = (int)((eid / R.nel[2]) % R.nel[1]);
    const int e1 = (int)(eid / ((int64_t)R.nel[1] * R.nel[2]));
    const int64_t sl = base + id;
    xyz[sl * 3 + 0] = R.lo[0] + (e1 + 0.5 * (1.0 + xi[g1])) * R.h[0];
    xyz[sl * 3 + 1] = R.lo[1] + (e2 + 0.5 * (1.0 + xi[g2])) * R.h[1];
    xyz[sl * 3 + 2] = R.lo[2] + (e3 + 0.5 * (1.0 + xi[g3])) * R.h[2];
}

__global__ void k_fill_f64(double* a, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// canonical slot of every Gauss point of every block element (grid slot when the point is a
// WQ grid point, else the block entry)
__global__ void k_blk_slot(DevRules R, const int32_t* block_elems, int64_t nb, int32_t* out) {
    const int p1 = R.p + 1, npe = p1 * p1 * p1;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= nb * npe) return;
    const int64_t eid = block_elems[id / npe];
    const int pt = (int)(id % npe);
    const int e3 = (int)(eid % R.nel[2]), e2 = (int)((eid / R.nel[2]) % R.nel[1]);
    const int e1 = (int)(eid / ((int64_t)R.nel[1] * R.nel[2]));
    out[id] = (int32_t)slot_of(R, e1 * p1 + pt / (p1 * p1), e2 * p1 + (pt / p1) % p1, e3 * p1 + pt % p1);
}

// Element-Gauss test x trial weights of one direction:
// W[((e * P1 + kI) * 2 + a) * P1^2 + k * P1 + g] = omega_g (h/2) B^(a)_{e+kI}(y) B^(a)_{e+k}(y), y the g-th
// Gauss point of element e (kI: the test function's offset on the element).
__global__ void k_rem_w(DevRules R, int d, const double* gw, double* W) {
    const int p1 = R.p + 1;
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (int64_t)R.nel[d] * p1 * 2 * p1 * p1) return;
    const int g = (int)(id % p1), k = (int)((id / p1) % p1), a = (int)((id / (p1 * p1)) % 2);
    const int kI = (int)((id / (2 * p1 * p1)) % p1);
    const int64_t e = id / (2 * p1 * p1 * p1);
    const int64_t y = e * p1 + g;
    const double* tab = a ? R.dBval[d] : R.Bval[d];
    W[id] = gw[g] * R.h[d] * 0.5 * tab[y * p1 + kI] * tab[y * p1 + k];
}

// grid and block slot coordinates
__global__ void k_slot_xyz(DevRules R, const int32_t* block_elems, double* xyz) {
    int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= R.n_grid + R.n_block) return;
    double x[3];
    if (id < R.n_grid) {
        int x3 = (int)(id % R.nx[2]), x2 = (int)((id / R.nx[2]) % R.nx[1]);
        int x1 = (int)(id / ((int64_t)R.nx[1] * R.nx[2]));
        x[0] = R.ycoord[0][R.x2y[0][x1]]; x[1] = R.ycoord[1][R.x2y[1][x2]]; x[2] = R.ycoord[2][R.x2y[2][x3]];
    } else {
        int p1 = R.p + 1, npe = p1 * p1 * p1;
        int64_t k = id - R.n_grid;
        int64_t eid = block_elems[k / npe];
        int pt = (int)(k % npe);
        int e3 = (int)(eid % R.nel[2]), e2 = (int)((eid / R.nel[2]) % R.nel[1]);
        int e1 = (int)(eid / ((int64_t)R.nel[1] * R.nel[2]));
        x[0] = R.ycoord[0][e1 * p1 + pt / (p1 * p1)];
        x[1] = R.ycoord[1][e2 * p1 + (pt / p1) % p1];
        x[2] = R.ycoord[2][e3 * p1 + pt % p1];
    }
    xyz[id * 3 + 0] = x[0]; xyz[id * 3 + 1] = x[1]; xyz[id * 3 + 2] = x[2];
}

__global__ void k_i64_to_i32(const int64_t* in, int32_t* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

template <typename TO>
__global__ void k_convert(const double* in, TO* out, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (TO)in[i];
}

static inline dim3 grid_for(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// ----------------------------------------------------------------------------------------
// host orchestration
// ----------------------------------------------------------------------------------------
int build_rules(const wq_mesh* mesh, const wq_levelset* ls, const wq_options* opts, hipStream_t stream,
                wq_rules** out) {
    wq_rules* H = new wq_rules();
    Builder B(H, stream);
    DevRules& R = H->R;
    memset(&R, 0, sizeof(R));
    int p = mesh->degree;
    R.p = p; R.m = 2 * p + 1; R.nw = 4 * p; R.ndq = p * (p + 1);
    R.levels = opts ? opts->octree_levels : 3;
    R.ls = *ls;
    H->mesh = *mesh;
    const bool tensor = opts && (opts->flags & WQ_OPT_TENSOR);
    R.tensor = tensor ? 1 : 0;
    int p1 = p + 1;
    int nmax = 0;
    for (int d = 0; d < 3; ++d) {
        R.nel[d] = mesh->nel[d];
        R.nfun[d] = mesh->nel[d] + p;
        R.lo[d] = mesh->lo[d];
        R.h[d] = (mesh->hi[d] - mesh->lo[d]) / mesh->nel[d];
        R.ny[d] = R.nel[d] * p1;
        R.nx[d] = (p == 1 || R.nel[d] == 1) ? R.nel[d] * p1 : 2 * p1 + 2 * (R.nel[d] - 2);
        nmax = R.nfun[d] > nmax ? R.nfun[d] : nmax;
    }
    int* d_err = B.tmp<int>(1);
    double* gxi = B.keep<double>(p1);
    double* gw = B.keep<double>(p1);
    if (!d_err || !gxi || !gw) return B.fail();
    if (B.check(hipMemsetAsync(d_err, 0, sizeof(int), stream))) return B.fail();
    H->gxi = gxi; H->gw = gw;
    R.gxi = gxi; R.gw = gw;
    hipLaunchKernelGGL(k_gauss, dim3(1), dim3(1), 0, stream, p1, gxi, gw);

    // per-direction tables
    for (int d = 0; d < 3; ++d) {
        double* yc = B.keep<double>(R.ny[d]);
        double* bv = B.keep<double>((int64_t)R.ny[d] * p1);
        double* dbv = B.keep<double>((int64_t)R.ny[d] * p1);
        int32_t* y2x = B.keep<int32_t>(R.ny[d]);
        int32_t* x2y = B.keep<int32_t>(R.nx[d]);
        if (!yc || !bv || !dbv || !y2x || !x2y) return B.fail();
        R.ycoord[d] = yc; R.Bval[d] = bv; R.dBval[d] = dbv; R.y2x[d] = y2x; R.x2y[d] = x2y;
        hipLaunchKernelGGL(k_dir_tables, grid_for(R.ny[d]), dim3(256), 0, stream, R, d, gxi, yc, bv, dbv, y2x, x2y);
    }
    for (int d = 0; d < 3; ++d) {
        int n = R.nfun[d];
        int32_t* xs = B.keep<int32_t>(n);
        int32_t* nw = B.keep<int32_t>(n);
        int64_t nwt = (int64_t)n * 2 * R.m * R.nw;
        double* wt = B.keep<double>(nwt);
        float* wt32 = B.keep<float>(nwt);
        int8_t* qlo = B.keep<int8_t>((int64_t)n * R.m);
        int8_t* qhi = B.keep<int8_t>((int64_t)n * R.m);
        if (!xs || !nw || !wt || !wt32 || !qlo || !qhi) return B.fail();
        R.xs[d] = xs; R.nwin[d] = nw; R.Wt64[d] = wt; R.Wt32[d] = wt32; R.qlo[d] = qlo; R.qhi[d] = qhi;
        double* wtx = nullptr;
        float* wtx32 = nullptr;
        if (tensor) {
            wtx = B.keep<double>(nwt);
            wtx32 = B.keep<float>(nwt);
            if (!wtx || !wtx32) return B.fail();
        }
        R.Wtx64[d] = wtx; R.Wtx32[d] = wtx32;
        const int nfam = tensor ? 4 : 2;
        hipLaunchKernelGGL(k_std_rules, grid_for(nfam * n, 64), dim3(64), 0, stream, R, d, nfam, gxi, gw, xs, nw, wt, wtx,
                           qlo, qhi, d_err);
        hipLaunchKernelGGL(k_convert<float>, grid_for(nwt), dim3(256), 0, stream, wt, wt32, nwt);
        if (tensor) hipLaunchKernelGGL(k_convert<float>, grid_for(nwt), dim3(256), 0, stream, wtx, wtx32, nwt);
    }
    if (B.check(hipGetLastError())) return B.fail();

    // classification
    int64_t ne = (int64_t)R.nel[0] * R.nel[1] * R.nel[2];
    int64_t nf = (int64_t)R.nfun[0] * R.nfun[1] * R.nfun[2];
    int8_t* ecls = B.keep<int8_t>(ne);
    int8_t* fcls = B.keep<int8_t>(nf);
    int32_t* aflag = B.tmp<int32_t>(nf);
    int64_t* aoff = B.tmp<int64_t>(nf + 1);
    int32_t* lex2act = B.keep<int32_t>(nf);
    if (!ecls || !fcls || !aflag || !aoff || !lex2act) return B.fail();
    R.ecls = ecls; R.fcls = fcls; R.lex2act = lex2act;
    hipLaunchKernelGGL(k_elem_class, grid_for(ne), dim3(256), 0, stream, R, ecls);
    hipLaunchKernelGGL(k_fun_class, grid_for(nf), dim3(256), 0, stream, R, ecls, fcls, aflag);
    int64_t na = 0;
    if (scan_exclusive(B, aflag, aoff, nf, &na)) return B.fail();
    H->n_active = na;
    int32_t* act2lex = B.keep<int32_t>(na > 0 ? na : 1);
    if (!act2lex) return B.fail();
    R.act2lex = act2lex;
    hipLaunchKernelGGL(k_active_index, grid_for(nf), dim3(256), 0, stream, nf, aflag, aoff, lex2act, act2lex);

    // pattern
    int32_t* rcnt = B.tmp<int32_t>(na + 1);
    int32_t* cflag = B.tmp<int32_t>(na + 1);
    int64_t* row_ptr = B.keep<int64_t>(na + 1);
    if (!rcnt || !cflag || !row_ptr) return B.fail();
    R.row_ptr = row_ptr;
    const bool gauss_rows = opts && (opts->flags & WQ_OPT_GAUSS_ROWS);
    const bool fit_rule = opts && (opts->flags & WQ_OPT_MOMENT_FIT);
    if (na > 0)
        hipLaunchKernelGGL(k_row_count, grid_for(na), dim3(256), 0, stream, R, na, act2lex, fcls, rcnt, cflag,
                           gauss_rows ? 1 : 0);
    int64_t nnz = 0;
    if (scan_exclusive(B, rcnt, row_ptr, na, &nnz)) return B.fail();
    H->nnz = nnz;
    int32_t* col = B.keep<int32_t>(nnz > 0 ? nnz : 1);
    if (!col) return B.fail();
    R.col_idx = col;
    if (na > 0) hipLaunchKernelGGL(k_col_fill, grid_for(na), dim3(256), 0, stream, R, na, act2lex, lex2act, row_ptr, col);

    // cut rows and splits
    int64_t* coff = B.tmp<int64_t>(na + 1);
    if (!coff) return B.fail();
    int64_t ncut = 0;
    if (scan_exclusive(B, cflag, coff, na, &ncut)) return B.fail();
    H->n_cut = ncut;
    H->n_interior_rows = na - ncut;
    int32_t* cut_rows = B.keep<int32_t>(ncut > 0 ? ncut : 1);
    int32_t* act2cut = B.keep<int32_t>(na > 0 ? na : 1);
    int4* split = B.keep<int4>(ncut > 0 ? ncut : 1);
    int32_t* box = B.keep<int32_t>(6 * (ncut > 0 ? ncut : 1));
    int nkeys = 3 * nmax * p * 2;
    int32_t* key_used = B.tmp<int32_t>(nkeys);
    int64_t* key_off = B.tmp<int64_t>(nkeys + 1);
    if (!cut_rows || !act2cut || !split || !box || !key_used || !key_off) return B.fail();
    R.cut_rows = cut_rows; R.split = split; R.n_cut = ncut;
    H->act2cut = act2cut; H->box = box;
    if (B.check(hipMemsetAsync(key_used, 0, sizeof(int32_t) * nkeys, stream))) return B.fail();
    if (na > 0) hipLaunchKernelGGL(k_cut_list, grid_for(na), dim3(256), 0, stream, na, cflag, coff, cut_rows, act2cut);
    if (ncut > 0)
        hipLaunchKernelGGL(k_split, grid_for(ncut, 64), dim3(64), 0, stream, R, ncut, cut_rows, act2lex, ecls, split, box,
                           key_used, nmax, (opts && (opts->flags & (WQ_OPT_HYBRID_GAUSS | WQ_OPT_GAUSS_ROWS))) ? 1 : 0);
    {
        int32_t* sflag = B.tmp<int32_t>(ncut + 1);
        int64_t* soff = B.tmp<int64_t>(ncut + 1);
        if (!sflag || !soff) return B.fail();
        if (ncut > 0) hipLaunchKernelGGL(k_split_flag, grid_for(ncut), dim3(256), 0, stream, ncut, split, sflag);
        if (scan_exclusive(B, sflag, soff, ncut, &H->n_split)) return B.fail();
        int32_t* sidx = B.tmp<int32_t>(ncut + 1);
        int32_t* box_rows = B.keep<int32_t>(H->n_split > 0 ? H->n_split : 1);
        if (!sidx || !box_rows) return B.fail();
        if (ncut > 0) hipLaunchKernelGGL(k_flag_index, grid_for(ncut), dim3(256), 0, stream, ncut, sflag, soff, sidx, box_rows);
        R.box_rows = box_rows; R.n_box = H->n_split;
    }
    int64_t ndwq = 0;
    if (scan_exclusive(B, key_used, key_off, nkeys, &ndwq)) return B.fail();
    H->n_dwq = ndwq;
    if (ncut > 0)
        hipLaunchKernelGGL(k_split_rule, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, split, key_off, nmax);
    {
        int64_t nr = ndwq > 0 ? ndwq : 1;
        int32_t* dnp = B.keep<int32_t>(nr);
        int32_t* dy = B.keep<int32_t>(nr * R.ndq);
        int64_t nwt = nr * 2 * R.m * R.ndq;
        double* dwt = B.keep<double>(nwt);
        float* dwt32 = B.keep<float>(nwt);
        double* dwtx = tensor ? B.keep<double>(nwt) : nullptr;
        float* dwtx32 = tensor ? B.keep<float>(nwt) : nullptr;
        if (!dnp || !dy || !dwt || !dwt32 || (tensor && (!dwtx || !dwtx32))) return B.fail();
        R.dwq_np = dnp; R.dwq_y = dy; R.dwq_Wt64 = dwt; R.dwq_Wt32 = dwt32;
        R.dwq_Wtx64 = dwtx; R.dwq_Wtx32 = dwtx32;
        if (ndwq > 0) {
            hipLaunchKernelGGL(k_dwq_rules, grid_for(nkeys, 64), dim3(64), 0, stream, R, nkeys, key_used, key_off, nmax,
                               tensor ? 4 : 2, gxi, gw, dnp, dy, dwt, dwtx, d_err);
            hipLaunchKernelGGL(k_convert<float>, grid_for(nwt), dim3(256), 0, stream, dwt, dwt32, nwt);
            if (tensor) hipLaunchKernelGGL(k_convert<float>, grid_for(nwt), dim3(256), 0, stream, dwtx, dwtx32, nwt);
        }
    }
    {
        int64_t m3 = (int64_t)R.m * R.m * R.m;
        int32_t* pos = B.keep<int32_t>((ncut > 0 ? ncut : 1) * m3);
        if (!pos) return B.fail();
        R.pos_map = pos;
        if (ncut > 0)
            hipLaunchKernelGGL(k_pos_map, grid_for(ncut, 64), dim3(64), 0, stream, R, ncut, cut_rows, act2lex, row_ptr, col, pos);
    }

    // interior line blocks
    {
        int rb = row_block_rows(p);
        H->row_block = rb;
        int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
        int32_t* lc = B.tmp<int32_t>(nl);
        int64_t* loff = B.tmp<int64_t>(nl + 1);
        if (!lc || !loff) return B.fail();
        hipLaunchKernelGGL(k_line_count, grid_for(nl), dim3(256), 0, stream, R, fcls, rb, lc);
        int64_t nb = 0;
        if (scan_exclusive(B, lc, loff, nl, &nb)) return B.fail();
        if (gauss_rows) nb = 0;                  // every row is on the cut-row path
        int4* blocks = B.keep<int4>(nb > 0 ? nb : 1);
        if (!blocks) return B.fail();
        R.lblocks = blocks; R.n_lblocks = nb;
        if (nb > 0) hipLaunchKernelGGL(k_line_fill, grid_for(nl), dim3(256), 0, stream, R, fcls, rb, loff, blocks);
        // blocks of at most 8 rows for the FP32 row kernel (p <= 4)
        R.fblocks = nullptr; R.n_fblocks = 0;
        if (p <= 4 && !gauss_rows) {
            hipLaunchKernelGGL(k_line_count, grid_for(nl), dim3(256), 0, stream, R, fcls, 8, lc);
            int64_t nf = 0;
            if (scan_exclusive(B, lc, loff, nl, &nf)) return B.fail();
            int4* fb = B.keep<int4>(nf > 0 ? nf : 1);
            if (!fb) return B.fail();
            R.fblocks = fb; R.n_fblocks = nf;
            hipLaunchKernelGGL(k_line_fill, grid_for(nl), dim3(256), 0, stream, R, fcls, 8, loff, fb);
        }
    }

    // element Gauss blocks
    {
        int32_t* bflag = B.tmp<int32_t>(ne);
        int64_t* boff = B.tmp<int64_t>(ne + 1);
        int32_t* eblock = B.keep<int32_t>(ne);
        if (!bflag || !boff || !eblock) return B.fail();
        if (B.check(hipMemsetAsync(bflag, 0, sizeof(int32_t) * ne, stream))) return B.fail();
        if (ncut > 0)
            hipLaunchKernelGGL(k_mark_blocks, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, ecls, bflag);
        int64_t nbe = 0;
        if (scan_exclusive(B, bflag, boff, ne, &nbe)) return B.fail();
        int32_t* blist = B.keep<int32_t>(nbe > 0 ? nbe : 1);
        if (!blist) return B.fail();
        hipLaunchKernelGGL(k_flag_index, grid_for(ne), dim3(256), 0, stream, ne, bflag, boff, eblock, blist);
        R.elem_block = eblock;
        H->block_elems = blist;
        H->n_block_elems = nbe;
        // per cut row remainder element lists
        int32_t* rcnt2 = B.tmp<int32_t>(ncut + 1);
        int64_t* roff = B.tmp<int64_t>(ncut + 1);
        int32_t* rptr = B.keep<int32_t>(ncut + 1);
        if (!rcnt2 || !roff || !rptr) return B.fail();
        if (ncut > 0)
            hipLaunchKernelGGL(k_rem_list<false>, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, ecls, box,
                               eblock, rcnt2, nullptr, nullptr);
        int64_t npairs = 0;
        if (scan_exclusive(B, rcnt2, roff, ncut, &npairs)) return B.fail();
        if (npairs >= ((int64_t)1 << 31)) return B.fail_msg(WQ_EUNSUPPORTED, "too many remainder pairs (%lld)", (long long)npairs);
        int2* rlist = B.keep<int2>(npairs > 0 ? npairs : 1);
        if (!rlist) return B.fail();
        if (ncut > 0)
            hipLaunchKernelGGL(k_rem_list<true>, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, ecls, box,
                               eblock, nullptr, roff, rlist);
        hipLaunchKernelGGL(k_i64_to_i32, grid_for(ncut + 1), dim3(256), 0, stream, roff, rptr, ncut + 1);
        R.rem_ptr = rptr; R.rem_list = rlist;
        H->n_rem_pairs = npairs;
    }

    // octree
    {
        int32_t* cflag2 = B.tmp<int32_t>(ne);
        int64_t* ceoff = B.tmp<int64_t>(ne + 1);
        int32_t* ceidx = B.tmp<int32_t>(ne);
        if (!cflag2 || !ceoff || !ceidx) return B.fail();
        hipLaunchKernelGGL(k_flag_eq, grid_for(ne), dim3(256), 0, stream, ne, ecls, (int8_t)CLS_CUT, cflag2);
        int64_t nce = 0;
        if (scan_exclusive(B, cflag2, ceoff, ne, &nce)) return B.fail();
        int32_t* cut_elems = B.keep<int32_t>(nce > 0 ? nce : 1);
        if (!cut_elems) return B.fail();
        hipLaunchKernelGGL(k_flag_index, grid_for(ne), dim3(256), 0, stream, ne, cflag2, ceoff, ceidx, cut_elems);
        R.cut_elems = cut_elems; R.n_cut_elems = nce;
        {   // interior elements (conventional Gauss assembly)
            int32_t* iflag = B.tmp<int32_t>(ne);
            int64_t* ioff = B.tmp<int64_t>(ne + 1);
            int32_t* iidx = B.tmp<int32_t>(ne);
            if (!iflag || !ioff || !iidx) return B.fail();
            hipLaunchKernelGGL(k_flag_eq, grid_for(ne), dim3(256), 0, stream, ne, ecls, (int8_t)CLS_IN, iflag);
            int64_t nie = 0;
            if (scan_exclusive(B, iflag, ioff, ne, &nie)) return B.fail();
            int32_t* ilist = B.keep<int32_t>(nie > 0 ? nie : 1);
            if (!ilist) return B.fail();
            hipLaunchKernelGGL(k_flag_index, grid_for(ne), dim3(256), 0, stream, ne, iflag, ioff, iidx, ilist);
            H->int_elems = ilist; H->n_int_elems = nie;
        }
        {   // per cut row: its cut elements
            int32_t* ccnt2 = B.tmp<int32_t>(ncut + 1);
            int64_t* coff2 = B.tmp<int64_t>(ncut + 1);
            int32_t* cptr = B.keep<int32_t>(ncut + 1);
            if (!ccnt2 || !coff2 || !cptr) return B.fail();
            if (ncut > 0)
                hipLaunchKernelGGL(k_rowcut_list<false>, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, ecls,
                                   ceidx, ccnt2, nullptr, nullptr);
            int64_t np2 = 0;
            if (scan_exclusive(B, ccnt2, coff2, ncut, &np2)) return B.fail();
            if (np2 >= ((int64_t)1 << 31)) return B.fail_msg(WQ_EUNSUPPORTED, "too many cut pairs (%lld)", (long long)np2);
            int2* clist = B.keep<int2>(np2 > 0 ? np2 : 1);
            if (!clist) return B.fail();
            if (ncut > 0)
                hipLaunchKernelGGL(k_rowcut_list<true>, grid_for(ncut), dim3(256), 0, stream, R, ncut, cut_rows, act2lex, ecls,
                                   ceidx, nullptr, coff2, clist);
            hipLaunchKernelGGL(k_i64_to_i32, grid_for(ncut + 1), dim3(256), 0, stream, coff2, cptr, ncut + 1);
            R.rcut_ptr = cptr; R.rcut_list = clist;
        }
        int32_t* ccnt = B.tmp<int32_t>(nce + 1);
        int64_t* cbeg = B.tmp<int64_t>(nce + 1);
        int32_t* cbeg32 = B.keep<int32_t>(nce + 1);
        if (!ccnt || !cbeg || !cbeg32) return B.fail();
        if (nce > 0)
            hipLaunchKernelGGL(k_octree<false>, grid_for(nce, 64), dim3(64), 0, stream, R, nce, cut_elems, ccnt, nullptr,
                               nullptr, nullptr, nullptr, nullptr, nullptr);
        int64_t ncell = 0;
        if (scan_exclusive(B, ccnt, cbeg, nce, &ncell)) return B.fail();
        if (ncell >= (int64_t)1 << 31) return B.fail_msg(WQ_EUNSUPPORTED, "octree has too many cells (%lld)", (long long)ncell);
        H->n_cells = ncell;
        R.n_cells = ncell;
        int64_t nc = ncell > 0 ? ncell : 1;
        double* clo = B.keep<double>(nc * 3);
        int8_t* cdep = B.keep<int8_t>(nc);
        int8_t* ccut = B.keep<int8_t>(nc);
        int32_t* celem = B.keep<int32_t>(nc);
        int32_t* ckey = B.keep<int32_t>(nc);
        int32_t* cperm = B.keep<int32_t>(nc);
        if (!clo || !cdep || !ccut || !celem || !ckey || !cperm) return B.fail();
        if (nce > 0) {
            hipLaunchKernelGGL(k_octree<true>, grid_for(nce, 64), dim3(64), 0, stream, R, nce, cut_elems, nullptr, cbeg,
                               clo, cdep, ccut, celem, ckey);
            hipLaunchKernelGGL(k_octree_sort, grid_for(nce, 64), dim3(64), 0, stream, nce, cbeg, ckey, cperm);
        }
        unsigned long long* grp = B.tmp<unsigned long long>(2);
        if (!grp) return B.fail();
        if (B.check(hipMemsetAsync(grp, 0, 2 * sizeof(unsigned long long), stream))) return B.fail();
        if (nce > 0)
            hipLaunchKernelGGL(k_octree_groups, grid_for(nce, 64), dim3(64), 0, stream, nce, cbeg, ckey, cperm, grp);
        unsigned long long hg[2] = {0, 0};
        if (B.check(hipMemcpyAsync(hg, grp, sizeof(hg), hipMemcpyDeviceToHost, stream))) return B.fail();
        if (B.check(hipStreamSynchronize(stream))) return B.fail();
        H->n_oct_xgroups = (int64_t)hg[0];
        H->n_oct_columns = (int64_t)hg[1];
        R.cell_key = ckey; R.cell_perm = cperm;
        const int ni = (2 << R.levels) - 1;
        for (int d = 0; d < 3; ++d) {
            const int64_t n = (int64_t)R.nel[d] * ni * 2 * p1 * p1 * p1;
            double* pp = B.keep<double>(n);
            float* pp32 = B.keep<float>(n);
            if (!pp || !pp32) return B.fail();
            hipLaunchKernelGGL(k_oct_basis, grid_for((int64_t)R.nel[d] * ni * p1), dim3(256), 0, stream, R, d, gxi, pp);
            hipLaunchKernelGGL(k_convert<float>, grid_for(n), dim3(256), 0, stream, pp, pp32, n);
            R.oct_pp64[d] = pp; R.oct_pp32[d] = pp32;
        }
        {   // Bernstein tables of the moment form of the cut-element integrals
            const int nk = 2 * p + 1;
            for (int d = 0; d < 3; ++d) {
                const int64_t n = (int64_t)R.nel[d] * 2 * p1 * p1 * nk;
                double* q = B.keep<double>(n);
                float* q32 = B.keep<float>(n);
                if (!q || !q32) return B.fail();
                hipLaunchKernelGGL(k_bern_products, grid_for(R.nel[d], 64), dim3(64), 0, stream, R, d, q);
                hipLaunchKernelGGL(k_convert<float>, grid_for(n), dim3(256), 0, stream, q, q32, n);
                R.bern_q64[d] = q; R.bern_q32[d] = q32;
                R.bern_qx64[d] = nullptr; R.bern_qx32[d] = nullptr;
                if (tensor) {
                    const int64_t nx = (int64_t)R.nel[d] * p1 * p1 * nk;
                    double* qx = B.keep<double>(nx);
                    float* qx32 = B.keep<float>(nx);
                    if (!qx || !qx32) return B.fail();
                    hipLaunchKernelGGL(k_bern_mixed, grid_for(R.nel[d], 64), dim3(64), 0, stream, R, d, qx);
                    hipLaunchKernelGGL(k_convert<float>, grid_for(nx), dim3(256), 0, stream, qx, qx32, nx);
                    R.bern_qx64[d] = qx; R.bern_qx32[d] = qx32;
                }
            }
            const int64_t n = (int64_t)ni * nk * p1;
            double* bi = B.keep<double>(n);
            float* bi32 = B.keep<float>(n);
            if (!bi || !bi32) return B.fail();
            hipLaunchKernelGGL(k_bern_intervals, grid_for(n), dim3(256), 0, stream, R, gxi, bi);
            hipLaunchKernelGGL(k_convert<float>, grid_for(n), dim3(256), 0, stream, bi, bi32, n);
            R.bern_i64 = bi; R.bern_i32 = bi32;
        }
        hipLaunchKernelGGL(k_i64_to_i32, grid_for(nce + 1), dim3(256), 0, stream, cbeg, cbeg32, nce + 1);
        R.cell_begin = cbeg32; R.cell_lo = clo; R.cell_depth = cdep;
        H->cell_cut = ccut; H->cell_elem = celem;
    }

    // slots
    {
        int64_t npe = (int64_t)p1 * p1 * p1;
        R.n_grid = (int64_t)R.nx[0] * R.nx[1] * R.nx[2];
        R.n_block = H->n_block_elems * npe;
        H->n_oct = R.n_cells * npe;
        R.n_kappa = R.n_grid + R.n_block + H->n_oct;
        // with the fitted rule the octree slots and weights only serve the fit below
        double* xyz = fit_rule ? B.tmp<double>(R.n_kappa * 3) : B.keep<double>(R.n_kappa * 3);
        double* ow = fit_rule ? B.tmp<double>(H->n_oct > 0 ? H->n_oct : 1) : B.keep<double>(H->n_oct > 0 ? H->n_oct : 1);
        if (!xyz || !ow) return B.fail();
        R.oct_w = ow;
        H->kappa_xyz = xyz;
        hipLaunchKernelGGL(k_slot_xyz, grid_for(R.n_grid + R.n_block), dim3(256), 0, stream, R, H->block_elems, xyz);
        if (R.n_kappa >= ((int64_t)1 << 31)) return B.fail_msg(WQ_EUNSUPPORTED, "too many kappa slots (%lld)", (long long)R.n_kappa);
        int32_t* bslot = B.keep<int32_t>(R.n_block > 0 ? R.n_block : 1);
        if (!bslot) return B.fail();
        if (R.n_block > 0)
            hipLaunchKernelGGL(k_blk_slot, grid_for(R.n_block), dim3(256), 0, stream, R, H->block_elems, H->n_block_elems, bslot);
        R.blk_slot = bslot;
        for (int d = 0; d < 3; ++d) {
            const int64_t n = (int64_t)R.nel[d] * p1 * 2 * p1 * p1;
            double* w = B.keep<double>(n);
            float* w32 = B.keep<float>(n);
            if (!w || !w32) return B.fail();
            hipLaunchKernelGGL(k_rem_w, grid_for(n), dim3(256), 0, stream, R, d, gw, w);
            hipLaunchKernelGGL(k_convert<float>, grid_for(n), dim3(256), 0, stream, w, w32, n);
            R.rem_w64[d] = w; R.rem_w32[d] = w32;
        }
        float* ow32 = fit_rule ? B.tmp<float>(H->n_oct > 0 ? H->n_oct : 1) : B.keep<float>(H->n_oct > 0 ? H->n_oct : 1);
        if (!ow32) return B.fail();
        R.oct_w32 = ow32;
        if (H->n_oct > 0) {
            hipLaunchKernelGGL(k_octree_weights, grid_for(H->n_oct), dim3(256), 0, stream, R, gxi, gw, R.cell_lo, R.cell_depth,
                               H->cell_cut, ow, xyz);
            hipLaunchKernelGGL(k_convert<float>, grid_for(H->n_oct), dim3(256), 0, stream, ow, ow32, H->n_oct);
        }
    }
    // fitted cut rule: Legendre moments of each cut element's octree rule (kappa = 1), weights
    // on the element's NK^3 tensor Gauss points, and the slot layout with those points
    R.fit = 0; R.fit_V64 = nullptr; R.fit_V32 = nullptr;
    if (fit_rule) {
        const int nk = 2 * p + 1, ni = (2 << R.levels) - 1;
        const int64_t nk3 = (int64_t)nk * nk * nk, nce = R.n_cut_elems;
        double* fxi = B.tmp<double>(nk);
        double* fw = B.tmp<double>(nk);
        double* V = B.keep<double>(nk * nk);
        float* V32 = B.keep<float>(nk * nk);
        double* Ainv = B.tmp<double>(nk * nk);
        double* leg = B.tmp<double>((int64_t)ni * nk * (p + 1));
        double* ones = B.tmp<double>(R.n_kappa);
        double* mom = B.tmp<double>(nce > 0 ? nce * nk3 : 1);
        double* wf = B.keep<double>(nce > 0 ? nce * nk3 : 1);
        float* wf32 = B.keep<float>(nce > 0 ? nce * nk3 : 1);
        const int64_t nkap = R.n_grid + R.n_block + nce * nk3;
        double* xyz2 = B.keep<double>(nkap * 3);
        if (!fxi || !fw || !V || !V32 || !Ainv || !leg || !ones || !mom || !wf || !wf32 || !xyz2) return B.fail();
        hipLaunchKernelGGL(k_gauss, dim3(1), dim3(1), 0, stream, nk, fxi, fw);
        hipLaunchKernelGGL(k_fit_tables, dim3(1), dim3(256), 0, stream, p, (const double*)fxi, (const double*)fw, V, Ainv);
        hipLaunchKernelGGL(k_convert<float>, dim3(1), dim3(256), 0, stream, V, V32, (int64_t)nk * nk);
        if (nce > 0) {
            hipLaunchKernelGGL(k_leg_intervals, grid_for((int64_t)ni * nk * (p + 1)), dim3(256), 0, stream, R, gxi, leg);
            hipLaunchKernelGGL(k_fill_f64, grid_for(R.n_kappa), dim3(256), 0, stream, ones, R.n_kappa, 1.0);
            int st = launch_octree_moments_f64(H, leg, ones, mom, stream);
            if (st) return B.fail_msg(st, "moments of the octree rule failed");
            hipLaunchKernelGGL(k_fit_weights, dim3((unsigned)nce), dim3(256), 0, stream, p, (const double*)Ainv,
                               (const double*)mom, wf);
            hipLaunchKernelGGL(k_convert<float>, grid_for(nce * nk3), dim3(256), 0, stream, wf, wf32, nce * nk3);
        }
        if (B.check(hipMemcpyAsync(xyz2, H->kappa_xyz, sizeof(double) * 3 * (R.n_grid + R.n_block), hipMemcpyDeviceToDevice,
                                   stream)))
            return B.fail();
        if (nce > 0)
            hipLaunchKernelGGL(k_fit_xyz, grid_for(nce * nk3), dim3(256), 0, stream, R, nce, R.cut_elems, (const double*)fxi,
                               R.n_grid + R.n_block, xyz2);
        H->n_oct = nce * nk3;
        R.n_kappa = nkap;
        R.oct_w = wf; R.oct_w32 = wf32;
        H->kappa_xyz = xyz2;
        R.fit = 1; R.fit_V64 = V; R.fit_V32 = V32;
    }
    if (B.check(hipGetLastError())) return B.fail();
    int herr = 0;
    if (B.check(hipMemcpyAsync(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost, stream))) return B.fail();
    if (B.check(hipStreamSynchronize(stream))) return B.fail();
    if (herr) return B.fail_msg(herr, "a weighted-quadrature exactness system is rank deficient");
    {   // host copies that bound the batches of the allocation-free cut assembly
        std::vector<int32_t> ce((size_t)R.n_cut_elems), cr((size_t)R.n_cut), a2l((size_t)H->n_active);
        if (R.n_cut_elems > 0 &&
            B.check(hipMemcpy(ce.data(), R.cut_elems, sizeof(int32_t) * ce.size(), hipMemcpyDeviceToHost)))
            return B.fail();
        if (R.n_cut > 0 && (B.check(hipMemcpy(cr.data(), R.cut_rows, sizeof(int32_t) * cr.size(), hipMemcpyDeviceToHost)) ||
                            B.check(hipMemcpy(a2l.data(), R.act2lex, sizeof(int32_t) * a2l.size(), hipMemcpyDeviceToHost))))
            return B.fail();
        const int64_t ep = (int64_t)R.nel[1] * R.nel[2], fp = (int64_t)R.nfun[1] * R.nfun[2];
        H->h_cut_elem_e1.resize(ce.size());
        for (size_t i = 0; i < ce.size(); ++i) H->h_cut_elem_e1[i] = (int32_t)(ce[i] / ep);
        H->h_cut_row_i1.resize(cr.size());
        for (size_t i = 0; i < cr.size(); ++i) H->h_cut_row_i1[i] = (int32_t)(a2l[cr[i]] / fp);
    }
    B.release_tmp();
    {   // scratch pool of the assembly calls; memory is kept between calls
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            hipMemPoolProps pp;
            memset(&pp, 0, sizeof(pp));
            pp.allocType = hipMemAllocationTypePinned;
            pp.handleTypes = hipMemHandleTypeNone;
            pp.location.type = hipMemLocationTypeDevice;
            pp.location.id = dev;
            if (hipMemPoolCreate(&H->pool, &pp) == hipSuccess) {
                uint64_t thr = UINT64_MAX;
                (void)hipMemPoolSetAttribute(H->pool, hipMemPoolAttrReleaseThreshold, &thr);
            } else {
                H->pool = nullptr;
                (void)hipGetLastError();
            }
        }
    }
    // side stream (default priority) and fork / join events of the row assembly; without
    // them the rows run on the caller's stream alone
    if (hipStreamCreateWithFlags(&H->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&H->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&H->ev_join, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (H->side) (void)hipStreamDestroy(H->side);
        if (H->ev_fork) (void)hipEventDestroy(H->ev_fork);
        if (H->ev_join) (void)hipEventDestroy(H->ev_join);
        H->side = nullptr; H->ev_fork = H->ev_join = nullptr;
    } else {
        H->side_mu = new std::mutex;
        if (hipStreamCreateWithFlags(&H->side2, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&H->ev_join2, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            if (H->side2) (void)hipStreamDestroy(H->side2);
            if (H->ev_join2) (void)hipEventDestroy(H->ev_join2);
            H->side2 = nullptr; H->ev_join2 = nullptr;
        }
    }
    *out = H;
    return WQ_OK;
}
