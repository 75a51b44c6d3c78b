// Stiffness matrix with a full symmetric coefficient tensor: K_IJ = int grad B_I . C grad B_J.
//
// Section 2 takes the map from the parameter space to the background mesh to be the identity
// and notes that no generality is lost; a geometry map F enters the Laplacian stiffness as
// the tensor C = |det DF| DF^-1 DF^-T (times a material coefficient), so the nine terms
// C_de d_d B_I d_e B_J replace the three diagonal ones of the scalar matrices.
//
// Regular part (interior rows; the DWQ box of cut rows, Section 2.2): weighted quadrature
// folds the test function into 1D weights per direction, so term (d, e) uses in direction x
// the rule family (x == d, x == e): (0, 0), (1, 1), and the mixed (1, 0) in direction d and
// (0, 1) in direction e when d != e (built by the rule build under WQ_OPT_TENSOR, each table
// already multiplied by the trial values or derivatives).  k_tensor_rows: one workgroup per
// row, sum factorization split direction first (A), then B, then C point by point: per point
// of C, stage A contracts the six tensor components over A for the nine terms, stage B over
// B, and stage C adds the point's share into per-thread accumulators of the row window; the
// row is then stored (interior rows: the clipped window in CSR order; cut rows through their
// position map; cut rows without a box are zeroed).
//
// Element parts of cut rows (Eq. (1)): k_tensor_rem (the element Gauss remainder, several
// elements in flight) or, for octrees deeper than three levels, k_tensor_elems, one workgroup
// per cut row, walks the row's remainder and cut elements and, per tensor block of points (an
// element's Gauss points, every leaf of its cut elements), forms the flux
// F_e(q) = w_q sum_d C_de(q) d_d B_I(x_q) at every point and contracts it with the trial
// derivatives direction by direction (3, 2, 1) into the row's window in LDS; the window is
// added into the values at the end (row-owned, no atomics).  Cut elements otherwise go through
// the moment form in cut.hip: moments of the six components, local rows once per element, the
// row gather of the scalar path.
#include "rows.h"

namespace {

template <typename T> __device__ inline const T* wt_tab(const DevRules& R, int d);
template <> __device__ inline const double* wt_tab<double>(const DevRules& R, int d) { return R.Wt64[d]; }
template <> __device__ inline const float* wt_tab<float>(const DevRules& R, int d) { return R.Wt32[d]; }
template <typename T> __device__ inline const T* wtx_tab(const DevRules& R, int d);
template <> __device__ inline const double* wtx_tab<double>(const DevRules& R, int d) { return R.Wtx64[d]; }
template <> __device__ inline const float* wtx_tab<float>(const DevRules& R, int d) { return R.Wtx32[d]; }
template <typename T> __device__ inline const T* dwq_tab(const DevRules& R);
template <> __device__ inline const double* dwq_tab<double>(const DevRules& R) { return R.dwq_Wt64; }
template <> __device__ inline const float* dwq_tab<float>(const DevRules& R) { return R.dwq_Wt32; }
template <typename T> __device__ inline const T* dwqx_tab(const DevRules& R);
template <> __device__ inline const double* dwqx_tab<double>(const DevRules& R) { return R.dwq_Wtx64; }
template <> __device__ inline const float* dwqx_tab<float>(const DevRules& R) { return R.dwq_Wtx32; }

// family of direction slot x in term (u, v): 0 = (0, 0), 1 = (1, 1), 2 = (1, 0), 3 = (0, 1)
__device__ inline int tfam(int x, int u, int v) { return x == u ? (x == v ? 1 : 2) : (x == v ? 3 : 0); }
// storage index of C_de: C11, C22, C33, C12, C13, C23
__device__ inline int tcomp(int d, int e) {
    if (d == e) return d;
    const int a = d < e ? d : e, b = d < e ? e : d;
    return a == 0 ? (b == 1 ? 3 : 4) : 5;
}

template <int P>
struct TenCfg {
    static constexpr int P1 = P + 1, M = 2 * P + 1, MM = M * M, M3 = MM * M;
    static constexpr int NW = 4 * P, NDQ = P * (P + 1), NA = NDQ > NW ? NDQ : NW;
    static constexpr int NN = 2 * P + 1;                // points per direction of a block (fitted rule: 2p+1)
    static constexpr int NT = 256;
    static constexpr int NACC = (M3 + NT - 1) / NT;
};

// ---------------------------------------------------------------------------------------
// regular part: one workgroup per active row
// ---------------------------------------------------------------------------------------
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_tensor_rows(DevRules R, const T* __restrict__ C, int64_t ldc, const int32_t* __restrict__ act2cut,
              const int32_t* __restrict__ rows, T* __restrict__ vk) {
    using Cf = TenCfg<P>;
    constexpr int M = Cf::M, MM = Cf::MM, M3 = Cf::M3, NW = Cf::NW, NDQ = Cf::NDQ, NA = Cf::NA, NT = Cf::NT;
    __shared__ T s_w[3][4 * M * NA];                  // [slot][family][jj][q]
    __shared__ int s_y[3][NA];
    __shared__ int s_n[3];
    __shared__ T s_c[6][NW * NA];                     // tensor components at one C point, [qB][qA]
    __shared__ T s_t1[9][NW * M];                     // [term][qB][jA]
    __shared__ T s_t2[9][MM];                         // [term][jB jA]
    const int ra = rows ? rows[blockIdx.x] : (int)blockIdx.x;   // rows: the cut rows only
    const int t = threadIdx.x;
    const int cr = act2cut[ra];
    const int4 sp = cr >= 0 ? R.split[cr] : make_int4(-1, 0, 0, -1);
    const int64_t rb = R.row_ptr[ra], re = R.row_ptr[ra + 1];
    if (cr >= 0 && sp.x < 0) {                        // cut row without a box: element parts only
        for (int64_t k = rb + t; k < re; k += NT) vk[k] = 0;
        return;
    }
    int I[3];
    {
        const int lex = R.act2lex[ra];
        I[2] = lex % R.nfun[2]; I[1] = (lex / R.nfun[2]) % R.nfun[1]; I[0] = lex / (R.nfun[1] * R.nfun[2]);
    }
    const int dA = sp.x >= 0 ? sp.x : 0, dB = dA == 0 ? 1 : 0, dC = dA == 2 ? 1 : 2;
    const int dirs[3] = {dA, dB, dC};
    for (int sl = 0; sl < 3; ++sl) {
        const int d = dirs[sl];
        if (sl == 0 && sp.x >= 0) {
            const int r = sp.w;
            const int np = R.dwq_np[r];
            const T* W0 = dwq_tab<T>(R) + (int64_t)r * 2 * M * NDQ;
            const T* W1 = dwqx_tab<T>(R) + (int64_t)r * 2 * M * NDQ;
            for (int k = t; k < 4 * M * NA; k += NT) {
                const int q = k % NA, row = k / NA;       // row = family * M + jj
                const T* W = row < 2 * M ? W0 : W1;
                const int rr = row < 2 * M ? row : row - 2 * M;
                s_w[sl][k] = q < NDQ ? W[rr * NDQ + q] : (T)0;
            }
            for (int q = t; q < NA; q += NT) s_y[sl][q] = q < np ? R.dwq_y[(int64_t)r * NDQ + q] : 0;
            if (t == 0) s_n[sl] = np;
        } else {
            const int i = I[d];
            const int xs = R.xs[d][i], nw = R.nwin[d][i];
            const T* W0 = wt_tab<T>(R, d) + (int64_t)i * 2 * M * NW;
            const T* W1 = wtx_tab<T>(R, d) + (int64_t)i * 2 * M * NW;
            for (int k = t; k < 4 * M * NA; k += NT) {
                const int q = k % NA, row = k / NA;
                const T* W = row < 2 * M ? W0 : W1;
                const int rr = row < 2 * M ? row : row - 2 * M;
                s_w[sl][k] = q < NW ? W[rr * NW + q] : (T)0;
            }
            for (int q = t; q < NA; q += NT) s_y[sl][q] = q < nw ? R.x2y[d][xs + q] : 0;
            if (t == 0) s_n[sl] = nw;
        }
    }
    __syncthreads();
    const int nA = s_n[0], nB = s_n[1], nC = s_n[2];
    T acc[Cf::NACC];
#pragma unroll
    for (int i = 0; i < Cf::NACC; ++i) acc[i] = 0;
    for (int qC = 0; qC < nC; ++qC) {
        const int yC = s_y[2][qC];
        for (int k = t; k < nB * nA; k += NT) {       // tensor components at the points (qA, qB, qC)
            const int qB = k / nA, qA = k % nA;
            const int yA = s_y[0][qA], yB = s_y[1][qB];
            const int64_t slot = slot_of(R, pick3(0, dA, dB, yA, yB, yC), pick3(1, dA, dB, yA, yB, yC),
                                         pick3(2, dA, dB, yA, yB, yC));
            T c[6];
#pragma unroll
            for (int comp = 0; comp < 6; ++comp) c[comp] = C[comp * ldc + slot];
#pragma unroll
            for (int comp = 0; comp < 6; ++comp) s_c[comp][qB * NA + qA] = c[comp];
        }
        __syncthreads();
        // stage A: T1[term][qB][jA] = sum_qA W_A^f[jA][qA] C_term(qA, qB)
        for (int it = t; it < 9 * nB * M; it += NT) {
            const int term = it / (nB * M), qB = (it / M) % nB, jA = it % M;
            const int u = term / 3, v = term % 3;
            const T* w = s_w[0] + (tfam(0, u, v) * M + jA) * NA;
            const T* c = s_c[tcomp(dirs[u], dirs[v])] + qB * NA;
            T a = 0;
            for (int qA = 0; qA < nA; ++qA) a = fmat(w[qA], c[qA], a);
            s_t1[term][qB * M + jA] = a;
        }
        __syncthreads();
        // stage B: T2[term][jB jA] = sum_qB W_B^f[jB][qB] T1[term][qB][jA]
        for (int it = t; it < 9 * MM; it += NT) {
            const int term = it / MM, jB = (it / M) % M, jA = it % M;
            const int u = term / 3, v = term % 3;
            const T* w = s_w[1] + (tfam(1, u, v) * M + jB) * NA;
            T a = 0;
            for (int qB = 0; qB < nB; ++qB) a = fmat(w[qB], s_t1[term][qB * M + jA], a);
            s_t2[term][jB * M + jA] = a;
        }
        __syncthreads();
        // stage C: acc[jC][jB jA] += sum_term W_C^f[jC][qC] T2[term][jB jA]
#pragma unroll
        for (int i = 0; i < Cf::NACC; ++i) {
            const int it = t + i * NT;
            if (it < M3) {
                const int jC = it / MM, jBA = it % MM;
                T a = acc[i];
#pragma unroll
                for (int term = 0; term < 9; ++term)
                    a = fmat(s_w[2][(tfam(2, term / 3, term % 3) * M + jC) * NA + qC], s_t2[term][jBA], a);
                acc[i] = a;
            }
        }
    }
    // store: window entry j (0..2p per direction) is function I - p + j
    int lo[3], n[3];
    for (int d = 0; d < 3; ++d) {
        const int a = I[d] - P < 0 ? 0 : I[d] - P, b = I[d] + P > R.nfun[d] - 1 ? R.nfun[d] - 1 : I[d] + P;
        lo[d] = a - (I[d] - P);
        n[d] = b - a + 1;
    }
    const int32_t* pos = cr >= 0 ? R.pos_map + (int64_t)cr * M3 : nullptr;
#pragma unroll
    for (int i = 0; i < Cf::NACC; ++i) {
        const int it = t + i * NT;
        if (it >= M3) continue;
        const int jC = it / MM, jB = (it / M) % M, jA = it % M;
        const int j0 = pick3(0, dA, dB, jA, jB, jC), j1 = pick3(1, dA, dB, jA, jB, jC), j2 = pick3(2, dA, dB, jA, jB, jC);
        if (pos) {
            const int o = pos[(j0 * M + j1) * M + j2];
            if (o >= 0) vk[rb + o] = acc[i];
        } else {
            const int a0 = j0 - lo[0], a1 = j1 - lo[1], a2 = j2 - lo[2];
            if (a0 >= 0 && a0 < n[0] && a1 >= 0 && a1 < n[1] && a2 >= 0 && a2 < n[2])
                vk[rb + ((int64_t)a0 * n[1] + a1) * n[2] + a2] = acc[i];
        }
    }
}

// ---------------------------------------------------------------------------------------
// interior rows in line blocks: one workgroup per block of up to RB consecutive interior rows
// along direction 1 (fixed i2, i3; SPLIT workgroups share a block of up to 8 rows)
// ---------------------------------------------------------------------------------------
// Directions 3 and 2 have the same rules for all rows of the block, so per term (d, e) the
// slab S[q1][j2 j3] = sum_q2 W2^f[j2][q2] sum_q3 W3^f[j3][q3] C_de(q1, q2, q3) is formed once
// over the union of the rows' direction-1 windows (stage 1: one thread per (q1, q2) with its
// C line in registers; stage 2: one thread per (q1, j2, j3)), and each row contracts it with
// its own direction-1 rule of the term's family into per-thread accumulators (stage 3).  The
// terms run one after another, so LDS holds one term's slab.
// the nine terms of a line block; QB bounds the points per direction of every window (2p+2
// for blocks of regular windows, 4p otherwise)
template <typename T, int P, int RB, int QB>
__device__ __forceinline__ void tensor_block_terms(const DevRules& R, const T* __restrict__ C, int64_t ldc, int i1s,
                                                   int nr, int xs1, int nu, int xs2, int n2, int xs3, int n3,
                                                   T* s_t1, T* s_s, T (*s_wa)[TenCfg<P>::M * TenCfg<P>::NW],
                                                   T (*s_wb)[TenCfg<P>::M * TenCfg<P>::NW],
                                                   T (*s_wc)[TenCfg<P>::M * TenCfg<P>::NW], const int* s_off,
                                                   const int* s_nw, bool own, int pr, int pj1, int lane, T* acc) {
    using Cf = TenCfg<P>;
    constexpr int M = Cf::M, MM = Cf::MM, NW = Cf::NW, NT = Cf::NT;
    constexpr int NPAIR = RB * M, L = NT / NPAIR, NJ = (MM + L - 1) / L;
    (void)NPAIR;
    const int t = threadIdx.x;
    for (int term = 0; term < 9; ++term) {
        const int d = term / 3, e = term % 3;
        const int comp = tcomp(d, e), fA = tfam(0, d, e), fB = tfam(1, d, e), fC = tfam(2, d, e);
        __syncthreads();                              // the previous term's slab and rules are no longer read
        for (int k = t; k < nr * M * NW; k += NT) {
            const int r = k / (M * NW), rr = k % (M * NW);
            const int i1 = i1s + r;
            s_wa[r][rr] = fA < 2 ? wt_tab<T>(R, 0)[((int64_t)i1 * 2 + fA) * M * NW + rr]
                                 : wtx_tab<T>(R, 0)[((int64_t)i1 * 2 + fA - 2) * M * NW + rr];
        }
        // stage 1: T1[q1][q2][j3] = sum_q3 W3^fC[j3][q3] C_comp(q1, q2, q3), the C line in registers
        const T* Ck = C + comp * ldc;
        for (int it = t; it < nu * n2; it += NT) {
            const int q1 = it / n2, q2 = it % n2;
            const int64_t base = ((int64_t)(xs1 + q1) * R.nx[1] + (xs2 + q2)) * R.nx[2] + xs3;
            T cl[QB];
#pragma unroll
            for (int q3 = 0; q3 < QB; ++q3) cl[q3] = q3 < n3 ? Ck[base + q3] : (T)0;
#pragma unroll
            for (int j3 = 0; j3 < M; ++j3) {
                const T* w = s_wc[fC] + j3 * NW;
                T a = 0;
#pragma unroll
                for (int q3 = 0; q3 < QB; ++q3) a = fmat(w[q3], cl[q3], a);
                s_t1[(q1 * NW + q2) * M + j3] = a;
            }
        }
        __syncthreads();
        // stage 2: S[q1][j2 j3] = sum_q2 W2^fB[j2][q2] T1[q1][q2][j3], one thread per (q1, j3) with
        // the T1 column in registers
        for (int it = t; it < nu * M; it += NT) {
            const int q1 = it / M, j3 = it % M;
            T col[QB];
#pragma unroll
            for (int q2 = 0; q2 < QB; ++q2) col[q2] = q2 < n2 ? s_t1[(q1 * NW + q2) * M + j3] : (T)0;
#pragma unroll
            for (int j2 = 0; j2 < M; ++j2) {
                const T* w = s_wb[fB] + j2 * NW;
                T a = 0;
#pragma unroll
                for (int q2 = 0; q2 < QB; ++q2) a = fmat(w[q2], col[q2], a);
                s_s[q1 * MM + j2 * M + j3] = a;
            }
        }
        __syncthreads();
        // stage 3: row r, acc[j1][j2 j3] += sum_q W1^fA[r][j1][q] S[off_r + q][j2 j3]
        if (own) {
            T w[QB];
            const int nw = s_nw[pr];
#pragma unroll
            for (int q = 0; q < QB; ++q) w[q] = q < nw ? s_wa[pr][pj1 * NW + q] : (T)0;
            const T* sl = s_s + s_off[pr] * MM;
#pragma unroll
            for (int i = 0; i < NJ; ++i) {
                const int j23 = lane + i * L;
                if (j23 < MM) {
                    T a = acc[i];
#pragma unroll
                    for (int q = 0; q < QB; ++q)
                        if (q < nw) a = fmat(w[q], sl[q * MM + j23], a);
                    acc[i] = a;
                }
            }
        }
    }
}

template <typename T, int P, int RB, int SPLIT>
__global__ void __launch_bounds__(256)
k_tensor_block(DevRules R, const T* __restrict__ C, int64_t ldc, T* __restrict__ vk) {
    using Cf = TenCfg<P>;
    constexpr int M = Cf::M, MM = Cf::MM, M3 = Cf::M3, NW = Cf::NW, NT = Cf::NT;
    constexpr int NU = NW + 2 * (RB - 1) + P + 1;     // bound of the union of the rows' direction-1 windows
    // stage 3: thread -> (row, j1) pair and a lane among L that share it; the lane takes the
    // columns j23 = lane, lane + L, ... with the pair's weights in registers
    constexpr int NPAIR = RB * M, L = NT / NPAIR, NJ = (MM + L - 1) / L;
    __shared__ T s_t1[NU * NW * M];                   // [q1][q2][j3]
    __shared__ T s_s[NU * MM];                        // [q1][j2 j3]
    __shared__ T s_wa[RB][M * NW];                    // the rows' direction-1 rules of the term's family
    __shared__ T s_wb[4][M * NW], s_wc[4][M * NW];    // directions 2 and 3, all four families
    __shared__ int s_off[RB], s_nw[RB];
    const int4 blk = R.fblocks[blockIdx.x / SPLIT];
    const int r0 = (blockIdx.x % SPLIT) * RB;
    const int nr = blk.w - r0 < RB ? blk.w - r0 : RB;
    if (nr <= 0) return;
    const int t = threadIdx.x;
    const int i1s = blk.x + r0, i2 = blk.y, i3 = blk.z;
    const int xs1 = R.xs[0][i1s];
    const int nu = R.xs[0][i1s + nr - 1] + R.nwin[0][i1s + nr - 1] - xs1;
    const int xs2 = R.xs[1][i2], n2 = R.nwin[1][i2], xs3 = R.xs[2][i3], n3 = R.nwin[2][i3];
    // The rows' windows cover the elements i1s - p .. i1s + nr - 1 (at most p + nr of them), two
    // points each plus p - 1 more in each of at most two boundary elements: nu <= 4p + 2 nr - 2
    // <= NW + 2 (RB - 1) < NU.  The check only guards the LDS bound.
    if (nu > NU) return;
    if (t < nr) { s_off[t] = R.xs[0][i1s + t] - xs1; s_nw[t] = R.nwin[0][i1s + t]; }
    for (int k = t; k < 4 * M * NW; k += NT) {
        const int f = k / (M * NW), r = k % (M * NW);
        s_wb[f][r] = f < 2 ? wt_tab<T>(R, 1)[((int64_t)i2 * 2 + f) * M * NW + r] : wtx_tab<T>(R, 1)[((int64_t)i2 * 2 + f - 2) * M * NW + r];
        s_wc[f][r] = f < 2 ? wt_tab<T>(R, 2)[((int64_t)i3 * 2 + f) * M * NW + r] : wtx_tab<T>(R, 2)[((int64_t)i3 * 2 + f - 2) * M * NW + r];
    }
    const int pair = t / L, lane = t % L;
    const int pr = pair / M, pj1 = pair % M;           // row and j1 of this thread's stage-3 items
    const bool own = pair < NPAIR && pr < nr;
    T acc[NJ];
#pragma unroll
    for (int i = 0; i < NJ; ++i) acc[i] = 0;
    __syncthreads();                                  // s_off / s_nw
    bool regular = n2 == 2 * P + 2 && n3 == 2 * P + 2;
    for (int r = 0; r < nr; ++r) regular = regular && s_nw[r] == 2 * P + 2;
    if (regular)
        tensor_block_terms<T, P, RB, 2 * P + 2>(R, C, ldc, i1s, nr, xs1, nu, xs2, n2, xs3, n3, s_t1, s_s, s_wa, s_wb, s_wc,
                                                s_off, s_nw, own, pr, pj1, lane, acc);
    else
        tensor_block_terms<T, P, RB, NW>(R, C, ldc, i1s, nr, xs1, nu, xs2, n2, xs3, n3, s_t1, s_s, s_wa, s_wb, s_wc, s_off,
                                         s_nw, own, pr, pj1, lane, acc);
    // store the clipped windows in CSR order
    if (!own) return;
    const int I[3] = {i1s + pr, i2, i3};
    int lo[3], n[3];
    for (int dd = 0; dd < 3; ++dd) {
        const int a = I[dd] - P < 0 ? 0 : I[dd] - P, b = I[dd] + P > R.nfun[dd] - 1 ? R.nfun[dd] - 1 : I[dd] + P;
        lo[dd] = a - (I[dd] - P);
        n[dd] = b - a + 1;
    }
    const int a0 = pj1 - lo[0];
    if (a0 < 0 || a0 >= n[0]) return;
    const int64_t rb = R.row_ptr[R.lex2act[((int64_t)I[0] * R.nfun[1] + I[1]) * R.nfun[2] + I[2]]];
#pragma unroll
    for (int i = 0; i < NJ; ++i) {
        const int j23 = lane + i * L;
        if (j23 >= MM) continue;
        const int a1 = j23 / M - lo[1], a2 = j23 % M - lo[2];
        if (a1 < 0 || a1 >= n[1] || a2 < 0 || a2 >= n[2]) continue;
        vk[rb + ((int64_t)a0 * n[1] + a1) * n[2] + a2] = acc[i];
    }
}

// ---------------------------------------------------------------------------------------
// element parts of the cut rows: one workgroup per cut row
// ---------------------------------------------------------------------------------------
// B_{e+k} and B'_{e+k}, k = 0..p, at x inside element e of direction d
__device__ inline void elem_basis(const DevRules& R, int d, int e, double x, double* N, double* dN) {
    const int p = R.p;
    double Tk[2 * WQ_PMAX + 2];
    for (int k = 0; k < 2 * p + 2; ++k) {
        int kk = e + k - p;
        kk = kk < 0 ? 0 : (kk > R.nel[d] ? R.nel[d] : kk);
        Tk[k] = R.lo[d] + (double)kk * R.h[d];
    }
    basis_funs(Tk, p, p, x, N, dN);
}

template <typename T, int P>
__global__ void __launch_bounds__(256)
k_tensor_elems(DevRules R, const T* __restrict__ C, int64_t ldc, const double* __restrict__ xyz, int with_cut,
               T* __restrict__ vk) {
    using Cf = TenCfg<P>;
    constexpr int P1 = Cf::P1, M = Cf::M, M3 = Cf::M3, NN = Cf::NN, NT = Cf::NT;
    constexpr int NN3 = NN * NN * NN;
    // FP64 throughout for both dtypes (this path sums over thousands of leaves per element;
    // the inputs are read in T and the row is rounded to T once)
    using A = double;
    __shared__ A s_acc[M3];
    __shared__ A s_f[3][NN3];                         // flux components at the block's points
    __shared__ A s_t1[3][NN * NN * P1];               // [e][g1 g2][k3]
    __shared__ A s_t2[3][NN * P1 * P1];               // [e][g1][k2 k3]
    __shared__ A s_b[3][2][P1][NN];                   // [d][value / derivative][k][g]
    const int64_t cr = blockIdx.x;
    const int t = threadIdx.x;
    const int ra = R.cut_rows[cr];
    int I[3];
    {
        const int lex = R.act2lex[ra];
        I[2] = lex % R.nfun[2]; I[1] = (lex / R.nfun[2]) % R.nfun[1]; I[0] = lex / (R.nfun[1] * R.nfun[2]);
    }
    for (int k = t; k < M3; k += NT) s_acc[k] = 0;
    const int nrem = R.rem_ptr[cr + 1] - R.rem_ptr[cr];
    const int ncut = with_cut ? R.rcut_ptr[cr + 1] - R.rcut_ptr[cr] : 0;
    const int64_t oct0 = R.n_grid + R.n_block;
    const int nkf = 2 * P + 1, nkf3 = nkf * nkf * nkf;
    for (int el = 0; el < nrem + ncut; ++el) {
        int e[3];
        int nblk, n;
        int64_t base = 0;                             // first slot of the block's points (octree / fitted)
        int2 en;
        bool rem = el < nrem;
        if (rem) {
            en = R.rem_list[R.rem_ptr[cr] + el];
            const int pk = en.x;
            e[0] = I[0] - (pk & 15); e[1] = I[1] - ((pk >> 4) & 15); e[2] = I[2] - ((pk >> 8) & 15);
            nblk = 1; n = P1;
        } else {
            en = R.rcut_list[R.rcut_ptr[cr] + el - nrem];
            const int pk = en.y;
            e[0] = I[0] - (pk & 15); e[1] = I[1] - ((pk >> 4) & 15); e[2] = I[2] - ((pk >> 8) & 15);
            if (R.fit) { nblk = 1; n = nkf; base = oct0 + (int64_t)en.x * nkf3; }
            else { nblk = R.cell_begin[en.x + 1] - R.cell_begin[en.x]; n = P1; }
        }
        const int kI[3] = {I[0] - e[0], I[1] - e[1], I[2] - e[2]};
        const int n3 = n * n * n;
        for (int blk = 0; blk < nblk; ++blk) {
            int64_t cell = -1;
            if (!rem && !R.fit) { cell = R.cell_begin[en.x] + blk; base = oct0 + cell * (P1 * P1 * P1); }
            // slot of point (g1, g2, g3) of the block
            auto slot_at = [&](int g1, int g2, int g3) -> int64_t {
                if (rem) return slot_of(R, e[0] * P1 + g1, e[1] * P1 + g2, e[2] * P1 + g3);
                return base + (g1 * n + g2) * n + g3;
            };
            __syncthreads();                          // the previous block's tables are no longer read
            // 1D basis values at the block's nodes (coordinates read from the slot layout)
            for (int k = t; k < 3 * n; k += NT) {
                const int d = k / n, g = k % n;
                const int64_t s = slot_at(d == 0 ? g : 0, d == 1 ? g : 0, d == 2 ? g : 0);
                double N[WQ_PMAX + 1], dN[WQ_PMAX + 1];
                elem_basis(R, d, e[d], xyz[s * 3 + d], N, dN);
                for (int kk = 0; kk < P1; ++kk) { s_b[d][0][kk][g] = N[kk]; s_b[d][1][kk][g] = dN[kk]; }
            }
            __syncthreads();
            // flux F_e = w sum_d C_de d_d B_I at every point
            for (int q = t; q < n3; q += NT) {
                const int g1 = q / (n * n), g2 = (q / n) % n, g3 = q % n;
                const int64_t s = slot_at(g1, g2, g3);
                A w;
                if (rem) w = R.gw[g1] * R.gw[g2] * R.gw[g3] * (R.h[0] * R.h[1] * R.h[2] / 8.0);
                else w = R.oct_w[s - oct0];
                const A v0 = s_b[0][0][kI[0]][g1], v1 = s_b[1][0][kI[1]][g2], v2 = s_b[2][0][kI[2]][g3];
                const A gt[3] = {s_b[0][1][kI[0]][g1] * v1 * v2, v0 * s_b[1][1][kI[1]][g2] * v2, v0 * v1 * s_b[2][1][kI[2]][g3]};
                A c[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) c[k] = (A)C[k * ldc + s];
#pragma unroll
                for (int ee = 0; ee < 3; ++ee) {
                    A f = c[tcomp(0, ee)] * gt[0];
                    f = fmat(c[tcomp(1, ee)], gt[1], f);
                    f = fmat(c[tcomp(2, ee)], gt[2], f);
                    s_f[ee][q] = w * f;
                }
            }
            __syncthreads();
            // stage 1: T1[e][g1 g2][k3] = sum_g3 D3^e[k3][g3] F_e
            for (int it = t; it < 3 * n * n * P1; it += NT) {
                const int ee = it / (n * n * P1), g12 = (it / P1) % (n * n), k3 = it % P1;
                const A* bz = s_b[2][ee == 2][k3];
                A a = 0;
                for (int g3 = 0; g3 < n; ++g3) a = fmat(bz[g3], s_f[ee][g12 * n + g3], a);
                s_t1[ee][g12 * P1 + k3] = a;
            }
            __syncthreads();
            // stage 2: T2[e][g1][k2 k3] = sum_g2 D2^e[k2][g2] T1[e][g1 g2][k3]
            for (int it = t; it < 3 * n * P1 * P1; it += NT) {
                const int ee = it / (n * P1 * P1), g1 = (it / (P1 * P1)) % n, k2 = (it / P1) % P1, k3 = it % P1;
                const A* by = s_b[1][ee == 1][k2];
                A a = 0;
                for (int g2 = 0; g2 < n; ++g2) a = fmat(by[g2], s_t1[ee][(g1 * n + g2) * P1 + k3], a);
                s_t2[ee][(g1 * P1 + k2) * P1 + k3] = a;
            }
            __syncthreads();
            // stage 3: window[k] += sum_e sum_g1 D1^e[k1][g1] T2[e][g1][k2 k3]
            for (int it = t; it < P1 * P1 * P1; it += NT) {
                const int k1 = it / (P1 * P1), k2 = (it / P1) % P1, k3 = it % P1;
                A a = 0;
#pragma unroll
                for (int ee = 0; ee < 3; ++ee) {
                    const A* bx = s_b[0][ee == 0][k1];
                    for (int g1 = 0; g1 < n; ++g1) a = fmat(bx[g1], s_t2[ee][(g1 * P1 + k2) * P1 + k3], a);
                }
                const int j0 = e[0] + k1 - (I[0] - P), j1 = e[1] + k2 - (I[1] - P), j2 = e[2] + k3 - (I[2] - P);
                s_acc[(j0 * M + j1) * M + j2] += a;
            }
        }
    }
    __syncthreads();
    const int64_t rb = R.row_ptr[ra];
    const int32_t* pos = R.pos_map + cr * M3;
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        if (o >= 0) vk[rb + o] += (T)s_acc[k];
    }
}

// Element Gauss remainder of the cut rows (the path when the cut elements go through the
// moment form): one workgroup per cut row, NS remainder elements in flight (one thread slot
// each, private LDS buffers and window accumulators summed in slot order at the end), the
// basis values at the element's Gauss points read from the direction tables.
template <typename T, int P, int NS>
__global__ void __launch_bounds__(256)
k_tensor_rem(DevRules R, const T* __restrict__ C, int64_t ldc, T* __restrict__ vk) {
    using Cf = TenCfg<P>;
    constexpr int P1 = Cf::P1, M = Cf::M, M3 = Cf::M3, NP = P1 * P1 * P1, NT = 256, NTS = NT / NS;
    __shared__ T s_acc[NS][M3];
    __shared__ T s_f[NS][3][NP];
    __shared__ T s_t1[NS][3][NP];                     // [e][g1 g2][k3]
    __shared__ T s_t2[NS][3][NP];                     // [e][g1][k2 k3]
    __shared__ T s_b[NS][3][2][P1][P1];               // [d][value / derivative][k][g]
    const int64_t cr = blockIdx.x;
    const int t = threadIdx.x, sl = t / NTS, u = t % NTS;
    const int ra = R.cut_rows[cr];
    int I[3];
    {
        const int lex = R.act2lex[ra];
        I[2] = lex % R.nfun[2]; I[1] = (lex / R.nfun[2]) % R.nfun[1]; I[0] = lex / (R.nfun[1] * R.nfun[2]);
    }
    const int l0 = R.rem_ptr[cr], nrem = R.rem_ptr[cr + 1] - l0;
    if (nrem == 0) return;
    for (int k = t; k < NS * M3; k += NT) s_acc[k / M3][k % M3] = 0;
    const T wscale = (T)(R.h[0] * R.h[1] * R.h[2] / 8.0);
    for (int r0 = 0; r0 < nrem; r0 += NS) {
        const int r = r0 + sl;
        const bool active = r < nrem;
        int e[3] = {0, 0, 0}, kI[3] = {0, 0, 0};
        int64_t blk = 0;
        if (active) {
            const int2 en = R.rem_list[l0 + r];
            const int pk = en.x;
            blk = en.y;
            kI[0] = pk & 15; kI[1] = (pk >> 4) & 15; kI[2] = (pk >> 8) & 15;
            for (int d = 0; d < 3; ++d) e[d] = I[d] - kI[d];
        }
        __syncthreads();                              // the previous round's buffers are no longer read
        if (active)
            for (int k = u; k < 3 * P1 * P1; k += NTS) {
                const int d = k / (P1 * P1), g = (k / P1) % P1, kk = k % P1;
                const int64_t y = (int64_t)e[d] * P1 + g;
                s_b[sl][d][0][kk][g] = (T)R.Bval[d][y * P1 + kk];
                s_b[sl][d][1][kk][g] = (T)R.dBval[d][y * P1 + kk];
            }
        __syncthreads();
        if (active)
            for (int q = u; q < NP; q += NTS) {      // flux F_e = w sum_d C_de d_d B_I
                const int g1 = q / (P1 * P1), g2 = (q / P1) % P1, g3 = q % P1;
                const int64_t s = R.blk_slot[blk * NP + q];   // canonical slot of the Gauss point
                const T w = (T)(R.gw[g1] * R.gw[g2] * R.gw[g3]) * wscale;
                const T v0 = s_b[sl][0][0][kI[0]][g1], v1 = s_b[sl][1][0][kI[1]][g2], v2 = s_b[sl][2][0][kI[2]][g3];
                const T gt[3] = {s_b[sl][0][1][kI[0]][g1] * v1 * v2, v0 * s_b[sl][1][1][kI[1]][g2] * v2,
                                 v0 * v1 * s_b[sl][2][1][kI[2]][g3]};
                T c[6];
#pragma unroll
                for (int k = 0; k < 6; ++k) c[k] = C[k * ldc + s];
#pragma unroll
                for (int ee = 0; ee < 3; ++ee) {
                    T f = c[tcomp(0, ee)] * gt[0];
                    f = fmat(c[tcomp(1, ee)], gt[1], f);
                    f = fmat(c[tcomp(2, ee)], gt[2], f);
                    s_f[sl][ee][q] = w * f;
                }
            }
        __syncthreads();
        if (active)
            for (int it = u; it < 3 * NP; it += NTS) {   // T1[e][g1 g2][k3] = sum_g3 D3^e[k3][g3] F_e
                const int ee = it / NP, g12 = (it / P1) % (P1 * P1), k3 = it % P1;
                const T* bz = s_b[sl][2][ee == 2][k3];
                T a = 0;
#pragma unroll
                for (int g3 = 0; g3 < P1; ++g3) a = fmat(bz[g3], s_f[sl][ee][g12 * P1 + g3], a);
                s_t1[sl][ee][g12 * P1 + k3] = a;
            }
        __syncthreads();
        if (active)
            for (int it = u; it < 3 * NP; it += NTS) {   // T2[e][g1][k2 k3] = sum_g2 D2^e[k2][g2] T1[e][g1 g2][k3]
                const int ee = it / NP, g1 = (it / (P1 * P1)) % P1, k2 = (it / P1) % P1, k3 = it % P1;
                const T* by = s_b[sl][1][ee == 1][k2];
                T a = 0;
#pragma unroll
                for (int g2 = 0; g2 < P1; ++g2) a = fmat(by[g2], s_t1[sl][ee][(g1 * P1 + g2) * P1 + k3], a);
                s_t2[sl][ee][(g1 * P1 + k2) * P1 + k3] = a;
            }
        __syncthreads();
        if (active)
            for (int it = u; it < NP; it += NTS) {       // window += sum_e sum_g1 D1^e[k1][g1] T2[e][g1][k2 k3]
                const int k1 = it / (P1 * P1), k2 = (it / P1) % P1, k3 = it % P1;
                T a = 0;
#pragma unroll
                for (int ee = 0; ee < 3; ++ee) {
                    const T* bx = s_b[sl][0][ee == 0][k1];
#pragma unroll
                    for (int g1 = 0; g1 < P1; ++g1) a = fmat(bx[g1], s_t2[sl][ee][(g1 * P1 + k2) * P1 + k3], a);
                }
                const int j0 = e[0] + k1 - (I[0] - P), j1 = e[1] + k2 - (I[1] - P), j2 = e[2] + k3 - (I[2] - P);
                s_acc[sl][(j0 * M + j1) * M + j2] += a;
            }
    }
    __syncthreads();
    const int64_t rb = R.row_ptr[ra];
    const int32_t* pos = R.pos_map + cr * M3;
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        if (o < 0) continue;
        T a = 0;
#pragma unroll
        for (int i = 0; i < NS; ++i) a += s_acc[i][k];
        vk[rb + o] += a;
    }
}

template <typename T, int P>
void launch_tensor_p(const wq_rules* H, const T* C, int64_t ldc, int with_cut, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    // interior rows by line blocks when every direction has p + 2 elements (the blocks' window
    // bound), the cut rows (and otherwise every row) one per workgroup
    const bool blocks = R.n_fblocks > 0 && R.nel[0] >= P + 2 && R.nel[1] >= P + 2 && R.nel[2] >= P + 2;
    if (blocks) {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((k_tensor_block<T, P, 8, 1>), dim3((unsigned)R.n_fblocks), dim3(256), 0, s, R, C, ldc, vk);
        else
            hipLaunchKernelGGL((k_tensor_block<T, P, 4, 2>), dim3((unsigned)(2 * R.n_fblocks)), dim3(256), 0, s, R, C, ldc, vk);
        if (H->n_cut > 0)
            hipLaunchKernelGGL((k_tensor_rows<T, P>), dim3((unsigned)H->n_cut), dim3(256), 0, s, R, C, ldc,
                               (const int32_t*)H->act2cut, (const int32_t*)R.cut_rows, vk);
    } else if (H->n_active > 0) {
        hipLaunchKernelGGL((k_tensor_rows<T, P>), dim3((unsigned)H->n_active), dim3(256), 0, s, R, C, ldc,
                           (const int32_t*)H->act2cut, (const int32_t*)nullptr, vk);
    }
    if (H->n_cut > 0) {
        if (with_cut)
            hipLaunchKernelGGL((k_tensor_elems<T, P>), dim3((unsigned)H->n_cut), dim3(256), 0, s, R, C, ldc,
                               (const double*)H->kappa_xyz, with_cut, vk);
        else
            hipLaunchKernelGGL((k_tensor_rem<T, P, sizeof(T) == 8 ? 2 : 4>), dim3((unsigned)H->n_cut), dim3(256), 0, s, R,
                               C, ldc, vk);
    }
}

}  // namespace

// Regular part and remainder row by row; the cut elements in moment form, element by element
// with the row gather (cut.hip), or row by row in k_tensor_elems when the octree is deeper than
// the moment form's three levels.
template <typename T>
int launch_tensor(const wq_rules* H, const T* C, T* vk, hipStream_t s) {
    const int64_t ldc = H->R.n_kappa;
    const int with_cut = H->R.levels > 3 ? 1 : 0;
    switch (H->R.p) {
        case 1: launch_tensor_p<T, 1>(H, C, ldc, with_cut, vk, s); break;
        case 2: launch_tensor_p<T, 2>(H, C, ldc, with_cut, vk, s); break;
        case 3: launch_tensor_p<T, 3>(H, C, ldc, with_cut, vk, s); break;
        case 4: launch_tensor_p<T, 4>(H, C, ldc, with_cut, vk, s); break;
        default: return WQ_EUNSUPPORTED;
    }
    if (!with_cut) return launch_tensor_cut<T>(H, C, vk, s);
    return WQ_OK;
}

#ifndef WQ_ONLY_F32
template int launch_tensor<double>(const wq_rules*, const double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template int launch_tensor<float>(const wq_rules*, const float*, float*, hipStream_t);
#endif
