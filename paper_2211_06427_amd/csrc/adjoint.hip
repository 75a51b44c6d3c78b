// Adjoint of the assembly: for L = sum_IJ (GM_IJ M_IJ + GK_IJ K_IJ), dL/dkappa at every slot.
//
// Every part of the forward is linear in kappa with a tensor-product structure, so the
// adjoint runs the same contractions transposed: the cotangent row (j1, j2, j3) is
// contracted with the direction-1 weights, then direction 2, then direction 3, and the
// result is added into dkappa at the quadrature points (atomics where several rows share a
// point).  The cotangents carry one value per pattern entry, like the matrices.
#include <mutex>

#include "rows.h"
#include "moments.h"

template <typename T> __device__ inline const T* wt_tab(const DevRules& R, int d);
template <> __device__ inline const double* wt_tab<double>(const DevRules& R, int d) { return R.Wt64[d]; }
template <> __device__ inline const float* wt_tab<float>(const DevRules& R, int d) { return R.Wt32[d]; }
template <typename T> __device__ inline const T* dwq_tab(const DevRules& R);
template <> __device__ inline const double* dwq_tab<double>(const DevRules& R) { return R.dwq_Wt64; }
template <> __device__ inline const float* dwq_tab<float>(const DevRules& R) { return R.dwq_Wt32; }

__device__ inline int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ inline void unlex3a(int64_t k, const int* n, int* I) {
    I[2] = (int)(k % n[2]);
    I[1] = (int)((k / n[2]) % n[1]);
    I[0] = (int)(k / ((int64_t)n[1] * n[2]));
}

__device__ inline void wave_sync_a() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__global__ void k_fill(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ----------------------------------------------------------------------------------------
// interior rows (line blocks), transposed stages 3 -> 2 -> 1.  Stage 3^T: the block's q1
// slab is split into NG contiguous ranges, one per thread group; a group visits every row
// whose window meets its range, one thread per (j2, j3) column, and adds only the q1 of its
// range, so every slab entry has a single owner and is updated without atomics.  Stage 1^T
// adds into dkappa with atomics (grid points are shared with neighbouring line blocks).
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH, int RB>
struct AdjCfg {
    static constexpr int M = 2 * P + 1, NW = 4 * P, MM = M * M;
    static constexpr int GT = ((MM + 63) / 64) * 64;       // threads per stage-3 group
    static constexpr int NG = GT >= 256 ? 1 : 256 / GT;    // groups, each owning a q1 range
    static constexpr int NT = NG * GT;                     // threads per block: whole groups only
    static constexpr int NQ1 = 2 * RB + 4 * P;
    static constexpr int QC = P <= 4 ? 8 : 4;             // q1 chunk of the stage-2/1 pass
    static constexpr bool STIFF = (WHICH & 2) != 0, MASS = (WHICH & 1) != 0;
};

template <typename T, int P, int WHICH, int RB>
__global__ void __launch_bounds__((AdjCfg<T, P, WHICH, RB>::NT))
k_adj_interior(DevRules R, const T* __restrict__ gm, const T* __restrict__ gk, T* __restrict__ dk) {
    using C = AdjCfg<T, P, WHICH, RB>;
    constexpr int M = C::M, NW = C::NW, MM = C::MM, QC = C::QC;
    __shared__ T s_a0[C::NQ1 * MM];
    __shared__ T s_a1[C::STIFF ? C::NQ1 * MM : 1];
    __shared__ T s_b[2][QC * NW * M];
    __shared__ T s_w2[2 * M * NW], s_w3[2 * M * NW];
    const int4 blk = R.lblocks[blockIdx.x];
    const int i1s = blk.x, i2 = blk.y, i3 = blk.z, nrows = blk.w;
    const T* W1 = wt_tab<T>(R, 0);
    const T* W2 = wt_tab<T>(R, 1) + (int64_t)i2 * 2 * M * NW;
    const T* W3 = wt_tab<T>(R, 2) + (int64_t)i3 * 2 * M * NW;
    for (int k = threadIdx.x; k < 2 * M * NW; k += C::NT) { s_w2[k] = W2[k]; s_w3[k] = W3[k]; }
    const int qbase = R.xs[0][i1s];
    const int i1e = i1s + nrows - 1;
    const int nq1 = R.xs[0][i1e] + R.nwin[0][i1e] - qbase;
    for (int k = threadIdx.x; k < nq1 * MM; k += C::NT) {
        s_a0[k] = 0;
        if (C::STIFF) s_a1[k] = 0;
    }
    const int xs2 = R.xs[1][i2], nw2 = R.nwin[1][i2];
    const int xs3 = R.xs[2][i3], nw3 = R.nwin[2][i3];
    const int nx2 = R.nx[1], nx3 = R.nx[2];
    __syncthreads();
    // stage 3^T
    const int grp = uni(threadIdx.x / C::GT);
    const int c = threadIdx.x % C::GT;
    const int jj2 = c / M, jj3 = c % M;
    const int p = P;
    const int lo2 = i2 - p < 0 ? p - i2 : 0, hi2 = i2 + p > R.nfun[1] - 1 ? R.nfun[1] - 1 - i2 + p : 2 * p;
    const int lo3 = i3 - p < 0 ? p - i3 : 0, hi3 = i3 + p > R.nfun[2] - 1 ? R.nfun[2] - 1 - i3 + p : 2 * p;
    const int m2 = hi2 - lo2 + 1, m3 = hi3 - lo3 + 1;
    const bool live = c < MM && jj2 >= lo2 && jj2 <= hi2 && jj3 >= lo3 && jj3 <= hi3;
    const int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
    const int qpart = (nq1 + C::NG - 1) / C::NG;
    const int qlo_g = grp * qpart, qhi_g = min(nq1, qlo_g + qpart);     // this group's q1 range
    for (int r = 0; r < nrows; ++r) {
        const int i1 = uni(i1s + r);
        const int off = uni(R.xs[0][i1] - qbase);
        const int nw1 = uni(R.nwin[0][i1]);
        if (off + nw1 <= qlo_g || off >= qhi_g) continue;
        const int ra = uni(R.lex2act[(int64_t)i1 * nl + (int64_t)i2 * R.nfun[2] + i3]);
        const int64_t base = R.row_ptr[ra];
        const int lo1 = i1 - p < 0 ? p - i1 : 0, hi1 = i1 + p > R.nfun[0] - 1 ? R.nfun[0] - 1 - i1 + p : 2 * p;
        T g0[M], g1[M];
#pragma unroll
        for (int jj1 = 0; jj1 < M; ++jj1) {
            g0[jj1] = 0; g1[jj1] = 0;
            if (live && jj1 >= lo1 && jj1 <= hi1) {
                const int64_t o = base + ((int64_t)(jj1 - lo1) * m2 + (jj2 - lo2)) * m3 + (jj3 - lo3);
                if (C::MASS) g0[jj1] = gm[o];
                if (C::STIFF) g1[jj1] = gk[o];
            }
        }
        const T* w10 = W1 + (int64_t)i1 * 2 * M * NW;
        const T* w11 = w10 + M * NW;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            if (q >= nw1) break;
            if (off + q < qlo_g || off + q >= qhi_g) continue;
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int jj1 = 0; jj1 < M; ++jj1) {
                const T w0 = w10[jj1 * NW + q];
                if (C::MASS) a0 += w0 * g0[jj1];
                if (C::STIFF) { a0 += w11[jj1 * NW + q] * g1[jj1]; a1 += w0 * g1[jj1]; }
            }
            if (live) {                             // column c has one owner: no atomics
                s_a0[(off + q) * MM + c] += a0;
                if (C::STIFF) s_a1[(off + q) * MM + c] += a1;
            }
        }
    }
    __syncthreads();
    // stages 2^T and 1^T by chunks of q1, one thread per output entry
    for (int q1c = 0; q1c < nq1; q1c += QC) {
        const int nqc = nq1 - q1c < QC ? nq1 - q1c : QC;
        // B_v[ql][q2][j3] = sum_j2 W2 A: items (ql, q2, j3)
        for (int it = threadIdx.x; it < nqc * nw2 * M; it += C::NT) {
            const int ql = it / (nw2 * M), q2 = (it / M) % nw2, j3 = it % M;
            const T* a0p = s_a0 + (q1c + ql) * MM + j3;
            const T* a1p = s_a1 + (C::STIFF ? (q1c + ql) * MM + j3 : 0);
            T b0 = 0, b1 = 0;
#pragma unroll
            for (int j2 = 0; j2 < M; ++j2) {
                const T a0 = a0p[j2 * M];
                const T w0 = s_w2[j2 * NW + q2];
                b0 += w0 * a0;
                if (C::STIFF) {
                    const T a1 = a1p[j2 * M];
                    b0 += s_w2[(M + j2) * NW + q2] * a1;
                    b1 += w0 * a1;
                }
            }
            s_b[0][(ql * NW + q2) * M + j3] = b0;
            if (C::STIFF) s_b[1][(ql * NW + q2) * M + j3] = b1;
        }
        __syncthreads();
        // dkappa[q1][q2][q3] += sum_j3 W3 B: items (ql, q2, q3), consecutive threads along q3
        for (int it = threadIdx.x; it < nqc * nw2 * nw3; it += C::NT) {
            const int ql = it / (nw2 * nw3), q2 = (it / nw3) % nw2, q3 = it % nw3;
            const T* b0p = s_b[0] + (ql * NW + q2) * M;
            const T* b1p = s_b[1] + (ql * NW + q2) * M;
            T v = 0;
#pragma unroll
            for (int j3 = 0; j3 < M; ++j3) {
                v += s_w3[j3 * NW + q3] * b0p[j3];
                if (C::STIFF) v += s_w3[(M + j3) * NW + q3] * b1p[j3];
            }
            atomicAdd(&dk[((int64_t)(qbase + q1c + ql) * nx2 + xs2 + q2) * nx3 + xs3 + q3], v);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------
// cut rows with a DWQ box: transposed stages C -> B -> A, kappa slots through slot_of
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_adj_cut(DevRules R, const T* __restrict__ gm, const T* __restrict__ gk, T* __restrict__ dk) {
    constexpr int M = 2 * P + 1, NW = 4 * P, NDQ = P * (P + 1), MM = M * M, M3 = M * M * M;
    constexpr int NA = NDQ > NW ? NDQ : NW;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_w[3][2 * M * NA];
    __shared__ int s_y[3][NA];
    __shared__ int s_n[3];
    __shared__ T s_g[2][M3];                      // cotangent window [v][jC][jB][jA]
    __shared__ T s_c[2][NW * MM];                 // [v][qC][jB jA]
    const int64_t cr = R.box_rows[blockIdx.x];     // cut rows with a DWQ box only
    const int4 sp = R.split[cr];
    if (sp.x < 0) return;
    const int ra = R.cut_rows[cr];
    int I[3];
    unlex3a(R.act2lex[ra], R.nfun, I);
    const int dA = sp.x, dB = dA == 0 ? 1 : 0, dC = dA == 2 ? 1 : 2;
    const int dirs[3] = {dA, dB, dC};
    for (int sl = 0; sl < 3; ++sl) {
        const int d = dirs[sl];
        if (sl == 0) {
            const int r = sp.w;
            const int np = R.dwq_np[r];
            const T* W = dwq_tab<T>(R) + (int64_t)r * 2 * M * NDQ;
            for (int k = threadIdx.x; k < 2 * M * NA; k += 256) {
                const int q = k % NA, row = k / NA;
                s_w[sl][k] = q < NDQ ? W[row * NDQ + q] : (T)0;
            }
            for (int q = threadIdx.x; q < NA; q += 256) s_y[sl][q] = q < np ? R.dwq_y[(int64_t)r * NDQ + q] : 0;
            if (threadIdx.x == 0) s_n[sl] = np;
        } else {
            const int i = I[d];
            const int xs = R.xs[d][i], nw = R.nwin[d][i];
            const T* W = wt_tab<T>(R, d) + (int64_t)i * 2 * M * NW;
            for (int k = threadIdx.x; k < 2 * M * NA; k += 256) {
                const int q = k % NA, row = k / NA;
                s_w[sl][k] = q < NW ? W[row * NW + q] : (T)0;
            }
            for (int q = threadIdx.x; q < NA; q += 256) s_y[sl][q] = q < nw ? R.x2y[d][xs + q] : 0;
            if (threadIdx.x == 0) s_n[sl] = nw;
        }
    }
    // gather the cotangent row into the local window, ordered [jC][jB][jA]
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    for (int k = threadIdx.x; k < M3; k += 256) {
        const int jj0 = k / (M * M), jj1 = (k / M) % M, jj2 = k % M;
        const int o = pos[k];
        // the component of (jj0, jj1, jj2) along direction d
        auto along = [&](int d) { return d == 0 ? jj0 : (d == 1 ? jj1 : jj2); };
        const int l = (along(dC) * M + along(dB)) * M + along(dA);
        s_g[0][l] = (o >= 0 && MASS) ? gm[rb + o] : (T)0;
        s_g[1][l] = (o >= 0 && STIFF) ? gk[rb + o] : (T)0;
    }
    __syncthreads();
    const int nA = s_n[0], nB = s_n[1], nC = s_n[2];
    // C^T: C0[qC][jB jA] = sum_jC W_C^0 GM + W_C^1 GK; C1 = sum_jC W_C^0 GK
    for (int it = threadIdx.x; it < nC * MM; it += 256) {
        const int qC = it / MM, cc = it % MM;
        T c0 = 0, c1 = 0;
        for (int jC = 0; jC < M; ++jC) {
            const T w0 = s_w[2][jC * NA + qC];
            if (MASS) c0 += w0 * s_g[0][jC * MM + cc];
            if (STIFF) { c0 += s_w[2][(M + jC) * NA + qC] * s_g[1][jC * MM + cc]; c1 += w0 * s_g[1][jC * MM + cc]; }
        }
        s_c[0][qC * MM + cc] = c0;
        if (STIFF) s_c[1][qC * MM + cc] = c1;
    }
    __syncthreads();
    // B^T and A^T per (qC, qB): b[jA] = sum_jB W_B C; dk(qA, qB, qC) += sum_jA W_A b
    for (int it = threadIdx.x; it < nC * nB; it += 256) {
        const int qC = it / nB, qB = it % nB;
        T b0[M], b1[M];
#pragma unroll
        for (int jA = 0; jA < M; ++jA) {
            T s0 = 0, s1 = 0;
            for (int jB = 0; jB < M; ++jB) {
                const T w0 = s_w[1][jB * NA + qB];
                const T c0 = s_c[0][qC * MM + jB * M + jA];
                s0 += w0 * c0;
                if (STIFF) {
                    const T c1 = s_c[1][qC * MM + jB * M + jA];
                    s0 += s_w[1][(M + jB) * NA + qB] * c1;
                    s1 += w0 * c1;
                }
            }
            b0[jA] = s0; b1[jA] = s1;
        }
        const int yB = s_y[1][qB], yC = s_y[2][qC];
        for (int qA = 0; qA < nA; ++qA) {
            const int yA = s_y[0][qA];
            T v = 0;
#pragma unroll
            for (int jA = 0; jA < M; ++jA) {
                v += s_w[0][jA * NA + qA] * b0[jA];
                if (STIFF) v += s_w[0][(M + jA) * NA + qA] * b1[jA];
            }
            atomicAdd(&dk[slot_of(R, pick3(0, dA, dB, yA, yB, yC), pick3(1, dA, dB, yA, yB, yC),
                                  pick3(2, dA, dB, yA, yB, yC))], v);
        }
    }
}

// ----------------------------------------------------------------------------------------
// remainder elements (element Gauss) of cut rows
// ----------------------------------------------------------------------------------------
template <typename T> __device__ inline const T* rem_tab_a(const DevRules& R, int d);
template <> __device__ inline const double* rem_tab_a<double>(const DevRules& R, int d) { return R.rem_w64[d]; }
template <> __device__ inline const float* rem_tab_a<float>(const DevRules& R, int d) { return R.rem_w32[d]; }

template <int P> struct RemAdjCfg {
    static constexpr int P1 = P + 1, NP = P1 * P1 * P1, P2 = P1 * P1;
    static constexpr int SLOT = ((NP + 63) / 64) * 64;         // threads per element in flight
    static constexpr int NT = SLOT >= 256 ? SLOT : 256;
    static constexpr int NSLOT = NT / SLOT;
};

// One workgroup per cut row; NSLOT remainder elements in flight, one thread per Gauss point
// (or per intermediate entry) of each, transposed contractions in the order 1, 2, 3.  The
// row's 1D weights and cotangent block sit in LDS; slot indices are loaded one pass ahead.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(RemAdjCfg<P>::NT)
k_adj_remainder(DevRules R, const T* __restrict__ gm, const T* __restrict__ gk, T* __restrict__ dk) {
    using C = RemAdjCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, M = 2 * P + 1, M3 = M * M * M, NT = C::NT, SLOT = C::SLOT;
    constexpr int NSLOT = C::NSLOT;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_g[2][M3];
    __shared__ T s_wt[3][P1][2 * P2];                 // [d][I_d - e_d][a][k][g]
    __shared__ T s_c[NSLOT][2][NP];
    __shared__ T s_b[NSLOT][2][NP];
    __shared__ int2 s_list[NP];
    const int64_t cr = blockIdx.x;
    const int ra = R.cut_rows[cr];
    int I[3];
    unlex3a(R.act2lex[ra], R.nfun, I);
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    const int t = threadIdx.x;
    const int l0 = R.rem_ptr[cr], nrem = R.rem_ptr[cr + 1] - l0;
    if (nrem == 0) return;
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        s_g[0][k] = (o >= 0 && MASS) ? gm[rb + o] : (T)0;
        s_g[1][k] = (o >= 0 && STIFF) ? gk[rb + o] : (T)0;
    }
    for (int q = t; q < 3 * P1 * 2 * P2; q += NT) {
        const int d = q / (P1 * 2 * P2), kI = (q / (2 * P2)) % P1, rest = q % (2 * P2);
        const int e = I[d] - kI;
        s_wt[d][kI][rest] = (e >= 0 && e < R.nel[d]) ? rem_tab_a<T>(R, d)[((int64_t)e * P1 + kI) * 2 * P2 + rest] : (T)0;
    }
    for (int k = t; k < nrem; k += NT) s_list[k] = R.rem_list[l0 + k];
    __syncthreads();
    const int sl = t / SLOT, u = t % SLOT;
    const bool act_u = u < NP;
    const int d1 = u / P2, d2 = (u / P1) % P1, d3 = u % P1;       // u = (d1, d2, d3)
    int bs_c = (act_u && sl < nrem) ? R.blk_slot[(int64_t)s_list[sl].y * NP + u] : 0;
    for (int r0 = 0; r0 < nrem; r0 += NSLOT) {
        const int r = r0 + sl;
        const bool active = r < nrem;
        const int bs = bs_c;
        bs_c = (act_u && r + NSLOT < nrem) ? R.blk_slot[(int64_t)s_list[r + NSLOT].y * NP + u] : 0;
        const int pk = active ? s_list[r].x : 0;
        const int kI0 = pk & 15, kI1 = (pk >> 4) & 15, kI2 = (pk >> 8) & 15;
        const T* W1 = s_wt[0][kI0];
        const T* W2 = s_wt[1][kI1];
        const T* W3 = s_wt[2][kI2];
        if (active && act_u) {      // 1^T: C[v][g1][k2][k3] = sum_k1 W1[k1][g1] G[k1][k2][k3], u = (g1, k2, k3)
            T c0 = 0, c1 = 0;
            const int j23 = (d2 - kI1 + P) * M + (d3 - kI2 + P);
#pragma unroll
            for (int k1 = 0; k1 < P1; ++k1) {
                const int jj = (k1 - kI0 + P) * M * M + j23;
                const T w0 = W1[k1 * P1 + d1];
                if (MASS) c0 += w0 * s_g[0][jj];
                if (STIFF) { c0 += W1[P2 + k1 * P1 + d1] * s_g[1][jj]; c1 += w0 * s_g[1][jj]; }
            }
            s_c[sl][0][u] = c0;
            if (STIFF) s_c[sl][1][u] = c1;
        }
        __syncthreads();
        if (active && act_u) {      // 2^T: B[v][g1][g2][k3], u = (g1, g2, k3)
            T b0 = 0, b1 = 0;
#pragma unroll
            for (int k2 = 0; k2 < P1; ++k2) {
                const T c0 = s_c[sl][0][(d1 * P1 + k2) * P1 + d3];
                const T w0 = W2[k2 * P1 + d2];
                b0 += w0 * c0;
                if (STIFF) {
                    const T c1 = s_c[sl][1][(d1 * P1 + k2) * P1 + d3];
                    b0 += W2[P2 + k2 * P1 + d2] * c1;
                    b1 += w0 * c1;
                }
            }
            s_b[sl][0][u] = b0;
            if (STIFF) s_b[sl][1][u] = b1;
        }
        __syncthreads();
        if (active && act_u) {      // 3^T: dk(g1, g2, g3), u = (g1, g2, g3)
            T v = 0;
#pragma unroll
            for (int k3 = 0; k3 < P1; ++k3) {
                v += W3[k3 * P1 + d3] * s_b[sl][0][(d1 * P1 + d2) * P1 + k3];
                if (STIFF) v += W3[P2 + k3 * P1 + d3] * s_b[sl][1][(d1 * P1 + d2) * P1 + k3];
            }
            atomicAdd(&dk[bs], v);
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------
// octree cut elements: dk_g = w_g sum_ab (GM_ab phi_a phi_b + GK_ab grad phi_a . grad phi_b)
// ----------------------------------------------------------------------------------------
template <int P> struct OctAdjCfg {
    static constexpr int P1 = P + 1, NP = P1 * P1 * P1, P2 = P1 * P1;
    static constexpr int NT = ((NP + 63) / 64) * 64;
    static constexpr int AG = P <= 4 ? P1 : (P == 5 ? 3 : 4);
    static constexpr int NAG = (P1 + AG - 1) / AG;
};

template <typename T> __device__ inline const T* oct_wt_a(const DevRules& R);
template <> __device__ inline const double* oct_wt_a<double>(const DevRules& R) { return R.oct_w; }
template <> __device__ inline const float* oct_wt_a<float>(const DevRules& R) { return R.oct_w32; }
template <typename T> __device__ inline const T* oct_tab_a(const DevRules& R, int d);
template <> __device__ inline const double* oct_tab_a<double>(const DevRules& R, int d) { return R.oct_pp64[d]; }
template <> __device__ inline const float* oct_tab_a<float>(const DevRules& R, int d) { return R.oct_pp32[d]; }

// One workgroup per cut element (it owns the element's octree slots, so dkappa is updated
// without atomics).  For each a3 (and group of a1) the cotangent block G[a1 b1][a2 b2 b3] is
// contracted with direction 1 once per x-group, with direction 2 once per column, and with
// direction 3 per leaf, in the same leaf order as the forward kernel.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(OctAdjCfg<P>::NT)
k_adj_octree(DevRules R, const int32_t* __restrict__ act2cut, const T* __restrict__ gm, const T* __restrict__ gk,
             T* __restrict__ dk) {
    using C = OctAdjCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, AG = C::AG, M = 2 * P + 1, NT = C::NT;
    constexpr int NPP = 2 * P2 * P1, KP = (NPP + NT - 1) / NT, MAXC = 512;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ int s_cell[MAXC], s_key[MAXC];
    __shared__ T s_pz[2][NPP], s_py[NPP], s_px[NPP];
    __shared__ T s_q[2][P1 * NP];                    // [v][g1][a2 b2 b3]
    __shared__ T s_r[2][P2 * P1];                    // [v][g1 g2][b3]
    const int ce = blockIdx.x;
    const int64_t eid = R.cut_elems[ce];
    int e[3];
    unlex3a(eid, R.nel, e);
    const int t = threadIdx.x;
    const bool own = t < NP;
    const int a2 = t / P2, b2 = (t / P1) % P1, b3 = t % P1;     // c2 = (a2, b2, b3) = t
    const int g12R = t / P1;                                     // R item (g1 g2, b3) = t
    const int64_t oct0 = R.n_grid + R.n_block;
    const int cb = R.cell_begin[ce], cend = R.cell_begin[ce + 1];
    const int ni = (2 << R.levels) - 1;
    const T* tx = oct_tab_a<T>(R, 0) + (int64_t)e[0] * ni * NPP;
    const T* ty = oct_tab_a<T>(R, 1) + (int64_t)e[1] * ni * NPP;
    const T* tz = oct_tab_a<T>(R, 2) + (int64_t)e[2] * ni * NPP;
    auto ivl = [](int key, int d) { return (1 << (key & 7)) - 1 + ((key >> (3 + 6 * d)) & 63); };
    const int xmask = (1 << 9) - 1, cmask = (1 << 15) - 1;
    for (int c0 = cb; c0 < cend; c0 += MAXC) {
        const int nc = cend - c0 < MAXC ? cend - c0 : MAXC;
        __syncthreads();
        for (int j = t; j < nc; j += NT) {
            const int cell = R.cell_perm[c0 + j];
            s_cell[j] = cell;
            s_key[j] = R.cell_key[cell];
        }
        __syncthreads();
        for (int a3 = 0; a3 < P1; ++a3) {
            for (int ag0 = 0; ag0 < P1; ag0 += AG) {
                T gmv[AG][P1], gkv[AG][P1];
#pragma unroll
                for (int i = 0; i < AG; ++i) {
                    const int a1 = ag0 + i;
#pragma unroll
                    for (int b1 = 0; b1 < P1; ++b1) { gmv[i][b1] = 0; gkv[i][b1] = 0; }
                    if (!own || a1 >= P1) continue;
                    const int64_t alex = ((int64_t)(e[0] + a1) * R.nfun[1] + (e[1] + a2)) * R.nfun[2] + (e[2] + a3);
                    const int ra = R.lex2act[alex];
                    const int cr = act2cut[ra];
                    const int32_t* pos = R.pos_map + (int64_t)cr * M * M * M;
                    const int64_t rb = R.row_ptr[ra];
#pragma unroll
                    for (int b1 = 0; b1 < P1; ++b1) {
                        const int o = pos[((b1 - a1 + P) * M + (b2 - a2 + P)) * M + (b3 - a3 + P)];
                        if (o < 0) continue;
                        if (MASS) gmv[i][b1] = gm[rb + o];
                        if (STIFF) gkv[i][b1] = gk[rb + o];
                    }
                }
                T w_n = 0, pz_n[KP], py_n[KP], px_n[KP];
                {
                    const int cell = s_cell[0], key = s_key[0];
                    if (own) w_n = oct_wt_a<T>(R)[(int64_t)cell * NP + t];
#pragma unroll
                    for (int i = 0; i < KP; ++i) {
                        const int q = t + i * NT;
                        pz_n[i] = q < NPP ? tz[(int64_t)ivl(key, 2) * NPP + q] : (T)0;
                        py_n[i] = q < NPP ? ty[(int64_t)ivl(key, 1) * NPP + q] : (T)0;
                        px_n[i] = q < NPP ? tx[(int64_t)ivl(key, 0) * NPP + q] : (T)0;
                    }
                }
                int kprev = -1, buf = 0;
                for (int j = 0; j < nc; ++j) {
                    const int cell = s_cell[j], key = s_key[j];
                    const bool new_x = kprev < 0 || (key & xmask) != (kprev & xmask);
                    const bool new_col = kprev < 0 || (key & cmask) != (kprev & cmask);
                    kprev = key;
                    const T w = w_n;
#pragma unroll
                    for (int i = 0; i < KP; ++i) {
                        const int q = t + i * NT;
                        if (q < NPP) {
                            s_pz[buf][q] = pz_n[i];
                            if (new_col) s_py[q] = py_n[i];
                            if (new_x) s_px[q] = px_n[i];
                        }
                    }
                    if (j + 1 < nc) {
                        const int cn = s_cell[j + 1], kn = s_key[j + 1];
                        if (own) w_n = oct_wt_a<T>(R)[(int64_t)cn * NP + t];
                        const bool nc_next = (kn & cmask) != (key & cmask), nx_next = (kn & xmask) != (key & xmask);
#pragma unroll
                        for (int i = 0; i < KP; ++i) {
                            const int q = t + i * NT;
                            if (q < NPP) {
                                pz_n[i] = tz[(int64_t)ivl(kn, 2) * NPP + q];
                                if (nc_next) py_n[i] = ty[(int64_t)ivl(kn, 1) * NPP + q];
                                if (nx_next) px_n[i] = tx[(int64_t)ivl(kn, 0) * NPP + q];
                            }
                        }
                    }
                    __syncthreads();
                    if (new_x) {
                        // Q0[g1][c2] = sum_{a1,b1} px[0] GM + px[1] GK; Q1 = sum px[0] GK
                        if (own) {
#pragma unroll
                            for (int g1 = 0; g1 < P1; ++g1) {
                                T q0 = 0, q1 = 0;
#pragma unroll
                                for (int i = 0; i < AG; ++i) {
                                    const int a1 = ag0 + i;
                                    if (a1 >= P1) break;
#pragma unroll
                                    for (int b1 = 0; b1 < P1; ++b1) {
                                        const T w0 = s_px[(a1 * P1 + b1) * P1 + g1];
                                        if (MASS) q0 += w0 * gmv[i][b1];
                                        if (STIFF) { q0 += s_px[P2 * P1 + (a1 * P1 + b1) * P1 + g1] * gkv[i][b1]; q1 += w0 * gkv[i][b1]; }
                                    }
                                }
                                s_q[0][g1 * NP + t] = q0;
                                if (STIFF) s_q[1][g1 * NP + t] = q1;
                            }
                        }
                        __syncthreads();
                    }
                    if (new_col) {
                        // R0[g1 g2][b3] = sum_{a2 b2} py[0][a2 b2][g2] Q0[g1][a2 b2 b3] + py[1] Q1; R1 = sum py[0] Q1
                        if (t < P2 * P1) {
                            const int g1 = g12R / P1, g2 = g12R % P1;
                            T r0 = 0, r1 = 0;
#pragma unroll
                            for (int ab2 = 0; ab2 < P2; ++ab2) {
                                const T q0 = s_q[0][g1 * NP + ab2 * P1 + b3];
                                const T w0 = s_py[ab2 * P1 + g2];
                                r0 += w0 * q0;
                                if (STIFF) {
                                    const T q1 = s_q[1][g1 * NP + ab2 * P1 + b3];
                                    r0 += s_py[P2 * P1 + ab2 * P1 + g2] * q1;
                                    r1 += w0 * q1;
                                }
                            }
                            s_r[0][t] = r0;
                            if (STIFF) s_r[1][t] = r1;
                        }
                        __syncthreads();
                    }
                    // dk_g += w_g sum_b3 pz[.][a3 b3][g3] R[.][g1 g2][b3]
                    if (own && w != (T)0) {
                        const int g12 = t / P1, g3 = t % P1;
                        T v = 0;
#pragma unroll
                        for (int bb3 = 0; bb3 < P1; ++bb3) {
                            v += s_pz[buf][(a3 * P1 + bb3) * P1 + g3] * s_r[0][g12 * P1 + bb3];
                            if (STIFF) v += s_pz[buf][P2 * P1 + (a3 * P1 + bb3) * P1 + g3] * s_r[1][g12 * P1 + bb3];
                        }
                        dk[oct0 + (int64_t)cell * NP + t] += w * v;
                    }
                    buf ^= 1;
                }
                __syncthreads();
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------------------
// ----------------------------------------------------------------------------------------
// cut elements in moment form (p <= 4, octree depth <= 3): for a point g of a leaf of cut
// element e,  dL/dkappa_g = w_g sum_k Gmom[k] B_k1(x_g) B_k2(y_g) B_k3(z_g)  with
//   Gmom = sum_ab GM_ab QX0 QY0 QZ0 + GK_ab (QX1 QY0 QZ0 + QX0 QY1 QZ0 + QX0 QY0 QZ1)
// (the transposed contraction of the forward moment form).
// ----------------------------------------------------------------------------------------
// k_adj_local: one workgroup per (cut element, a3): gathers the cotangents of the rows
// a = (a1, a2, a3) from the CSR values and contracts them with Q^T, direction 1 on matrix
// cores (U0 = QX0^T GM + QX1^T GK, Us = QX0^T GK), then directions 2 and 3 on the vector ALU;
// writes this a3's share of Gmom to part[(ce P1 + a3) NK^3 + k].
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_adj_local(DevRules R, const int32_t* __restrict__ act2cut, const T* __restrict__ gm, const T* __restrict__ gk,
            T* __restrict__ part) {
    using C = MomCfg<P>;
    using MF = MfmaOp<T>;
    using v4 = typename MF::v4;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int M = 2 * P + 1, M3 = M * M * M, NTC = C::NTC, NTW = C::NTW, QN = 2 * P2 * NK;
    constexpr int NBLK = P2 * NP, NU = NK * NP, NV = NK2 * P1;
    constexpr int KA = (2 * P2 + 3) / 4, KB = (P2 + 3) / 4;        // k steps of U0 and Us
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_q[3][QN];
    __shared__ T s_g[2][NBLK];                      // cotangent blocks [(a1 b1)][(a2 b2) b3]
    __shared__ T s_u[2][NU];                        // U0, Us [k1][(a2 b2) b3]
    static_assert(2 * NV <= 2 * NBLK, "VA/VB reuse the cotangent block");
    T (*s_v)[NV] = reinterpret_cast<T (*)[NV]>(&s_g[0][0]);   // VA, VB [k1 k2][b3] after direction 1
    __shared__ int64_t s_rb[P2];
    __shared__ int32_t s_cr[P2];
    const int ce = blockIdx.x / P1, a3 = blockIdx.x % P1;
    int e[3];
    unlex3a(R.cut_elems[ce], R.nel, e);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    if (t < P2) {
        const int a1 = t / P1, a2 = t % P1;
        const int64_t alex = ((int64_t)(e[0] + a1) * R.nfun[1] + (e[1] + a2)) * R.nfun[2] + (e[2] + a3);
        const int ra = R.lex2act[alex];
        s_rb[t] = R.row_ptr[ra];
        s_cr[t] = act2cut[ra];
    }
    for (int i = t; i < 3 * QN; i += NT) {
        const int d = i / QN;
        s_q[d][i % QN] = bern_q<T>(R, d)[(int64_t)e[d] * QN + i % QN];
    }
    __syncthreads();
    for (int i = t; i < NBLK; i += NT) {
        const int r = i / NP, b = i % NP, a1 = r / P1, a2 = r % P1;
        const int b1 = b / P2, b2 = (b / P1) % P1, b3 = b % P1;
        const int jj = ((b1 - a1 + P) * M + (b2 - a2 + P)) * M + (b3 - a3 + P);
        const int o = R.pos_map[(int64_t)s_cr[r] * M3 + jj];
        const int dst = (a1 * P1 + b1) * NP + (a2 * P1 + b2) * P1 + b3;
        s_g[0][dst] = (MASS && o >= 0) ? gm[s_rb[r] + o] : (T)0;
        s_g[1][dst] = (STIFF && o >= 0) ? gk[s_rb[r] + o] : (T)0;
    }
    __syncthreads();
    const T* qx = s_q[0];
    const T* qy = s_q[1];
    const T* qz = s_q[2];
    // direction 1 on matrix cores: rows k1 (< NK <= 16), columns n = (a2 b2 b3), K = (a1 b1)
#pragma unroll
    for (int ti = 0; ti < NTW; ++ti) {
        const int nt = wv + ti * C::NWAVE;
        if (nt >= NTC) break;
        const int n = nt * 16 + lm;
        const bool nv = n < NP;
        v4 u0 = {0, 0, 0, 0}, us = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < KA; ++k) {              // U0 = [QX0^T | QX1^T] [GM ; GK]
            const int kk = 4 * k + lk;
            T av = 0, bv = 0;
            if (kk < P2) {
                if (MASS) { av = lm < NK ? qx[kk * NK + lm] : (T)0; bv = nv ? s_g[0][kk * NP + n] : (T)0; }
            } else if (kk < 2 * P2) {
                if (STIFF) {
                    av = lm < NK ? qx[P2 * NK + (kk - P2) * NK + lm] : (T)0;
                    bv = nv ? s_g[1][(kk - P2) * NP + n] : (T)0;
                }
            }
            u0 = MF::mma(av, bv, u0);
        }
        if (STIFF) {
#pragma unroll
            for (int k = 0; k < KB; ++k) {          // Us = QX0^T GK
                const int kk = 4 * k + lk;
                const T av = (kk < P2 && lm < NK) ? qx[kk * NK + lm] : (T)0;
                const T bv = (kk < P2 && nv) ? s_g[1][kk * NP + n] : (T)0;
                us = MF::mma(av, bv, us);
            }
        }
        if (nv) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int k1 = MF::row(lane, r);
                if (k1 < NK) {
                    s_u[0][k1 * NP + n] = u0[r];
                    if (STIFF) s_u[1][k1 * NP + n] = us[r];
                }
            }
        }
    }
    __syncthreads();
    // direction 2: VA = QY0^T U0 + QY1^T Us, VB = QY0^T Us
    for (int i = t; i < NV; i += NT) {
        const int k1 = i / (NK * P1), k2 = (i / P1) % NK, b3 = i % P1;
        T va = 0, vb = 0;
#pragma unroll 5
        for (int ab2 = 0; ab2 < P2; ++ab2) {
            const T y0 = qy[ab2 * NK + k2];
            va += y0 * s_u[0][k1 * NP + ab2 * P1 + b3];
            if (STIFF) {
                const T u = s_u[1][k1 * NP + ab2 * P1 + b3];
                va += qy[P2 * NK + ab2 * NK + k2] * u;
                vb += y0 * u;
            }
        }
        s_v[0][i] = va;
        if (STIFF) s_v[1][i] = vb;
    }
    __syncthreads();
    // direction 3: Gmom share = QZ0^T VA + QZ1^T VB for this a3
    for (int i = t; i < NK3; i += NT) {
        const int k12 = i / NK, k3 = i % NK;
        T g = 0;
#pragma unroll
        for (int b3 = 0; b3 < P1; ++b3) {
            g += qz[(a3 * P1 + b3) * NK + k3] * s_v[0][k12 * P1 + b3];
            if (STIFF) g += qz[P2 * NK + (a3 * P1 + b3) * NK + k3] * s_v[1][k12 * P1 + b3];
        }
        part[((int64_t)ce * P1 + a3) * NK3 + i] = g;
    }
}

// k_adj_local_a2 (degrees 5 and 6): as k_adj_local, with the rows a = (a1, a2, a3) of the
// workgroup's a3 taken one a2 at a time, so that LDS holds the cotangent block of one a2
// ([(a1 b1)][(b2 b3)]) instead of all of them; the direction-2 sums VA, VB are accumulated
// over a2 in registers.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_adj_local_a2(DevRules R, const int32_t* __restrict__ act2cut, const T* __restrict__ gm, const T* __restrict__ gk,
               T* __restrict__ part) {
    using C = MomCfg<P>;
    using MF = MfmaOp<T>;
    using v4 = typename MF::v4;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int M = 2 * P + 1, M3 = M * M * M, QN = 2 * P2 * NK;
    constexpr int NB2 = P2 * P2, NU = NK * P2, NV = NK2 * P1, RV = (NV + NT - 1) / NT;
    constexpr int NTC = (P2 + 15) / 16, NTW = (NTC + C::NWAVE - 1) / C::NWAVE;
    constexpr int KA = (2 * P2 + 3) / 4, KB = (P2 + 3) / 4;        // k steps of U0 and Us
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    static_assert(NK <= 16, "rows k1 of one MFMA tile");
    __shared__ T s_q[3][QN];
    __shared__ T s_g[2][NB2];                       // cotangents of one a2: [(a1 b1)][(b2 b3)]
    __shared__ T s_u[2][NU];                        // U0, Us [k1][(b2 b3)]
    __shared__ T s_v[2][NV];                        // VA, VB [k1 k2][b3]
    __shared__ int64_t s_rb[P2];
    __shared__ int32_t s_cr[P2];
    const int ce = blockIdx.x / P1, a3 = blockIdx.x % P1;
    int e[3];
    unlex3a(R.cut_elems[ce], R.nel, e);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    if (t < P2) {
        const int a1 = t / P1, a2 = t % P1;
        const int64_t alex = ((int64_t)(e[0] + a1) * R.nfun[1] + (e[1] + a2)) * R.nfun[2] + (e[2] + a3);
        const int ra = R.lex2act[alex];
        s_rb[t] = R.row_ptr[ra];
        s_cr[t] = act2cut[ra];
    }
    for (int i = t; i < 3 * QN; i += NT) {
        const int d = i / QN;
        s_q[d][i % QN] = bern_q<T>(R, d)[(int64_t)e[d] * QN + i % QN];
    }
    const T* qx = s_q[0];
    const T* qy = s_q[1];
    const T* qz = s_q[2];
    T va_acc[RV], vb_acc[RV];
#pragma unroll
    for (int r = 0; r < RV; ++r) { va_acc[r] = 0; vb_acc[r] = 0; }
    __syncthreads();
    for (int a2 = 0; a2 < P1; ++a2) {
        for (int i = t; i < P1 * NP; i += NT) {
            const int a1 = i / NP, b = i % NP, r = a1 * P1 + a2;
            const int b1 = b / P2, b2 = (b / P1) % P1, b3 = b % P1;
            const int jj = ((b1 - a1 + P) * M + (b2 - a2 + P)) * M + (b3 - a3 + P);
            const int o = R.pos_map[(int64_t)s_cr[r] * M3 + jj];
            const int dst = (a1 * P1 + b1) * P2 + b2 * P1 + b3;
            s_g[0][dst] = (MASS && o >= 0) ? gm[s_rb[r] + o] : (T)0;
            s_g[1][dst] = (STIFF && o >= 0) ? gk[s_rb[r] + o] : (T)0;
        }
        __syncthreads();
        // direction 1 on matrix cores: rows k1, columns n = (b2 b3), K = (a1 b1)
#pragma unroll
        for (int ti = 0; ti < NTW; ++ti) {
            const int nt = wv + ti * C::NWAVE;
            if (nt >= NTC) break;
            const int n = nt * 16 + lm;
            const bool nv = n < P2;
            v4 u0 = {0, 0, 0, 0}, us = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < KA; ++k) {          // U0 = [QX0^T | QX1^T] [GM ; GK]
                const int kk = 4 * k + lk;
                T av = 0, bv = 0;
                if (kk < P2) {
                    if (MASS) { av = lm < NK ? qx[kk * NK + lm] : (T)0; bv = nv ? s_g[0][kk * P2 + n] : (T)0; }
                } else if (kk < 2 * P2) {
                    if (STIFF) {
                        av = lm < NK ? qx[P2 * NK + (kk - P2) * NK + lm] : (T)0;
                        bv = nv ? s_g[1][(kk - P2) * P2 + n] : (T)0;
                    }
                }
                u0 = MF::mma(av, bv, u0);
            }
            if (STIFF) {
#pragma unroll
                for (int k = 0; k < KB; ++k) {      // Us = QX0^T GK
                    const int kk = 4 * k + lk;
                    const T av = (kk < P2 && lm < NK) ? qx[kk * NK + lm] : (T)0;
                    const T bv = (kk < P2 && nv) ? s_g[1][kk * P2 + n] : (T)0;
                    us = MF::mma(av, bv, us);
                }
            }
            if (nv) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int k1 = MF::row(lane, r);
                    if (k1 < NK) {
                        s_u[0][k1 * P2 + n] = u0[r];
                        if (STIFF) s_u[1][k1 * P2 + n] = us[r];
                    }
                }
            }
        }
        __syncthreads();
        // direction 2 for this a2: VA += QY0^T U0 + QY1^T Us, VB += QY0^T Us (sums over b2)
#pragma unroll
        for (int r = 0; r < RV; ++r) {
            const int i = t + r * NT;
            if (i >= NV) break;
            const int k1 = i / (NK * P1), k2 = (i / P1) % NK, b3 = i % P1;
#pragma unroll
            for (int b2 = 0; b2 < P1; ++b2) {
                const int ab2 = a2 * P1 + b2;
                const T y0 = qy[ab2 * NK + k2];
                va_acc[r] += y0 * s_u[0][k1 * P2 + b2 * P1 + b3];
                if (STIFF) {
                    const T u = s_u[1][k1 * P2 + b2 * P1 + b3];
                    va_acc[r] += qy[P2 * NK + ab2 * NK + k2] * u;
                    vb_acc[r] += y0 * u;
                }
            }
        }
        // the next a2 rewrites s_g, then s_u after the barrier that follows its gather
    }
#pragma unroll
    for (int r = 0; r < RV; ++r) {
        const int i = t + r * NT;
        if (i < NV) {
            s_v[0][i] = va_acc[r];
            s_v[1][i] = vb_acc[r];
        }
    }
    __syncthreads();
    // direction 3: Gmom share = QZ0^T VA + QZ1^T VB for this a3
    for (int i = t; i < NK3; i += NT) {
        const int k12 = i / NK, k3 = i % NK;
        T g = 0;
#pragma unroll
        for (int b3 = 0; b3 < P1; ++b3) {
            g += qz[(a3 * P1 + b3) * NK + k3] * s_v[0][k12 * P1 + b3];
            if (STIFF) g += qz[P2 * NK + (a3 * P1 + b3) * NK + k3] * s_v[1][k12 * P1 + b3];
        }
        part[((int64_t)ce * P1 + a3) * NK3 + i] = g;
    }
}

// k_adj_leaves: one workgroup per cut element sums the a3 shares of Gmom and evaluates
// dL/dkappa at every point of its leaves: direction 1 once per x-group, direction 2 once per
// column, direction 3 per leaf.  Every octree slot belongs to one element: plain stores.
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_adj_leaves(DevRules R, const T* __restrict__ part, T* __restrict__ dk) {
    using C = MomCfg<P>;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int NB = C::NB, KW = C::KW, MAXC = C::MAXC, NZ = C::NZ, NY = C::NY;
    __shared__ int s_cell[MAXC], s_key[MAXC];
    __shared__ T s_bi[C::NIMAX * NK * P1];
    __shared__ T s_gmom[NK3];
    __shared__ T s_gy[NY];                          // [g1][k2 k3]
    __shared__ T s_gz[NZ];                          // [g1 g2][k3]
    __shared__ T s_w[2][NB * NP];                   // octree weights of a batch of leaves
    const int ce = blockIdx.x;
    const int t = threadIdx.x;
    const int ni = (2 << R.levels) - 1;
    for (int i = t; i < ni * NK * P1; i += NT) s_bi[i] = bern_i<T>(R)[i];
    for (int i = t; i < NK3; i += NT) {
        T g = 0;
#pragma unroll
        for (int a3 = 0; a3 < P1; ++a3) g += part[((int64_t)ce * P1 + a3) * NK3 + i];
        s_gmom[i] = g;
    }
    const int64_t oct0 = R.n_grid + R.n_block;
    const T* __restrict__ ow = oct_wt_a<T>(R);
    const int cb = R.cell_begin[ce], cend = R.cell_begin[ce + 1];
    auto ivl = [](int key, int d) { return (1 << (key & 7)) - 1 + ((key >> (3 + 6 * d)) & 63); };
    const int xmask = (1 << 9) - 1, cmask = (1 << 15) - 1;
    int kprev = -1;
    T pw[KW];
    for (int c0 = cb; c0 < cend; c0 += MAXC) {
        const int nc = cend - c0 < MAXC ? cend - c0 : MAXC;
        __syncthreads();
        for (int j = t; j < nc; j += NT) {
            const int cell = R.cell_perm[c0 + j];
            s_cell[j] = cell;
            s_key[j] = R.cell_key[cell];
        }
        __syncthreads();
        auto issue = [&](int jb, int nb) {
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const int idx = t + i * NT;
                if (idx < nb * NP) pw[i] = ow[(int64_t)s_cell[jb + idx / NP] * NP + idx % NP];
            }
        };
        const int nbat = (nc + NB - 1) / NB;
        issue(0, nc < NB ? nc : NB);
        for (int b = 0; b < nbat; ++b) {
            const int jb = b * NB, nb = nc - jb < NB ? nc - jb : NB, buf = b & 1;
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const int idx = t + i * NT;
                if (idx < nb * NP) s_w[buf][idx] = pw[i];
            }
            __syncthreads();
            if (b + 1 < nbat) issue(jb + NB, nc - jb - NB < NB ? nc - jb - NB : NB);
            for (int jl = 0; jl < nb; ++jl) {
                const int j = jb + jl;
                const int key = s_key[j];
                const bool new_x = kprev < 0 || (key & xmask) != (kprev & xmask);
                const bool new_col = kprev < 0 || (key & cmask) != (kprev & cmask);
                kprev = key;
                if (new_col) {
                    __syncthreads();                // earlier leaves are done with s_gz (and s_gy)
                    if (new_x) {                    // Gy[g1][k2 k3] = sum_k1 B_k1(x_g1) Gmom[k1][k2 k3]
                        const T* bx = s_bi + ivl(key, 0) * NK * P1;
                        for (int i = t; i < NY; i += NT) {
                            const int g1 = i / NK2, k23 = i % NK2;
                            T s = 0;
#pragma unroll
                            for (int k1 = 0; k1 < NK; ++k1) s += bx[k1 * P1 + g1] * s_gmom[k1 * NK2 + k23];
                            s_gy[i] = s;
                        }
                        __syncthreads();
                    }
                    // Gz[g1 g2][k3] = sum_k2 B_k2(y_g2) Gy[g1][k2][k3]
                    const T* by = s_bi + ivl(key, 1) * NK * P1;
                    for (int i = t; i < NZ; i += NT) {
                        const int g1 = i / (P1 * NK), g2 = (i / NK) % P1, k3 = i % NK;
                        T s = 0;
#pragma unroll
                        for (int k2 = 0; k2 < NK; ++k2) s += by[k2 * P1 + g2] * s_gy[g1 * NK2 + k2 * NK + k3];
                        s_gz[i] = s;
                    }
                    __syncthreads();
                }
                // this leaf: dk(g) = w_g sum_k3 B_k3(z_g3) Gz[g1 g2][k3]
                for (int g = t; g < NP; g += NT) {         // NP > NT from p = 6 on
                    const T* bz = s_bi + ivl(key, 2) * NK * P1;
                    const int g12 = g / P1, g3 = g % P1;
                    T s = 0;
#pragma unroll
                    for (int k3 = 0; k3 < NK; ++k3) s += bz[k3 * P1 + g3] * s_gz[g12 * NK + k3];
                    dk[oct0 + (int64_t)s_cell[j] * NP + g] = s_w[buf][jl * NP + g] * s;
                }
            }
        }
    }
}

template <typename T> __device__ inline const T* fit_v_a(const DevRules& R);
template <> __device__ inline const double* fit_v_a<double>(const DevRules& R) { return R.fit_V64; }
template <> __device__ inline const float* fit_v_a<float>(const DevRules& R) { return R.fit_V32; }

// Fitted cut rule: dkappa at the NK^3 points of a cut element, w_g sum_k Gmom[k] B_k1(tau_g1)
// B_k2(tau_g2) B_k3(tau_g3), Gmom the element's moment cotangent (sum of its a3 shares);
// contracted direction by direction, one workgroup per cut element (it owns the points).
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_adj_fit(DevRules R, const T* __restrict__ part, T* __restrict__ dk) {
    using C = MomCfg<P>;
    constexpr int P1 = C::P1, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    __shared__ T s_a[NK3], s_b[NK3];
    __shared__ T s_v[NK * NK];
    const int64_t ce = blockIdx.x;
    const int t = threadIdx.x;
    for (int i = t; i < NK * NK; i += NT) s_v[i] = fit_v_a<T>(R)[i];
    for (int i = t; i < NK3; i += NT) {
        T g = 0;
#pragma unroll
        for (int a3 = 0; a3 < P1; ++a3) g += part[(ce * P1 + a3) * NK3 + i];
        s_a[i] = g;                                 // [k1][k2 k3]
    }
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {             // [g1][k2 k3]
        const int g1 = i / NK2, k23 = i % NK2;
        T v = 0;
#pragma unroll
        for (int k1 = 0; k1 < NK; ++k1) v += s_v[k1 * NK + g1] * s_a[k1 * NK2 + k23];
        s_b[i] = v;
    }
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {             // [g1 g2][k3]
        const int g1 = i / NK2, g2 = (i / NK) % NK, k3 = i % NK;
        T v = 0;
#pragma unroll
        for (int k2 = 0; k2 < NK; ++k2) v += s_v[k2 * NK + g2] * s_b[(g1 * NK + k2) * NK + k3];
        s_a[i] = v;
    }
    __syncthreads();
    const int64_t s0 = R.n_grid + R.n_block + ce * NK3;
    for (int i = t; i < NK3; i += NT) {             // [g1 g2][g3]
        const int g12 = i / NK, g3 = i % NK;
        T v = 0;
#pragma unroll
        for (int k3 = 0; k3 < NK; ++k3) v += s_v[k3 * NK + g3] * s_a[g12 * NK + k3];
        dk[s0 + i] = oct_wt_a<T>(R)[ce * NK3 + i] * v;
    }
}

// The octree part writes only the octree slots (one owner each) and the other parts add into
// the grid and block slots with atomics, so with a second stream the octree part runs beside
// the rest: forked after the zero fill, joined before the call returns.
template <typename T, int P, int WHICH>
static int launch_adj_octree(const wq_rules* H, const T* gm, const T* gk, T* dk, T* part, hipStream_t s) {
    const DevRules& R = H->R;
    using C = MomCfg<P>;
    if constexpr (P <= 4)
        hipLaunchKernelGGL((k_adj_local<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1)), dim3(256), 0, s, R, H->act2cut,
                           gm, gk, part);
    else
        hipLaunchKernelGGL((k_adj_local_a2<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1)), dim3(256), 0, s, R,
                           H->act2cut, gm, gk, part);
    if (R.fit)
        hipLaunchKernelGGL((k_adj_fit<T, P>), dim3((unsigned)R.n_cut_elems), dim3(256), 0, s, R, (const T*)part, dk);
    else
        hipLaunchKernelGGL((k_adj_leaves<T, P>), dim3((unsigned)R.n_cut_elems), dim3(256), 0, s, R, (const T*)part, dk);
    return WQ_OK;
}

template <typename T, int P, int WHICH>
static int launch_adj_p(const wq_rules* H, const T* gm, const T* gk, T* dk, hipStream_t s) {
    const DevRules& R = H->R;
    if (H->side && R.n_cut_elems > 0 && R.levels <= 3) {
        using C = MomCfg<P>;
        T* part = nullptr;
        hipError_t err = H->scratch_alloc((void**)&part, sizeof(T) * (size_t)R.n_cut_elems * C::P1 * C::NK3, s);
        if (err != hipSuccess)
            return wq_set_error(WQ_ENOMEM, "wq_assemble_adjoint: scratch allocation failed: %s", hipGetErrorString(err));
        std::lock_guard<std::mutex> lock(*H->side_mu);
        const bool forked = hipEventRecord(H->ev_fork, s) == hipSuccess && hipStreamWaitEvent(H->side, H->ev_fork, 0) == hipSuccess;
        if (!forked) (void)hipGetLastError();
        launch_adj_octree<T, P, WHICH>(H, gm, gk, dk, part, forked ? H->side : s);
        if (R.n_lblocks > 0) {
            if constexpr (P <= 4) {
                using A = AdjCfg<T, P, WHICH, 16>;
                hipLaunchKernelGGL((k_adj_interior<T, P, WHICH, 16>), dim3((unsigned)R.n_lblocks), dim3(A::NT), 0, s, R, gm, gk,
                                   dk);
            } else {
                using A = AdjCfg<T, P, WHICH, 8>;
                hipLaunchKernelGGL((k_adj_interior<T, P, WHICH, 8>), dim3((unsigned)R.n_lblocks), dim3(A::NT), 0, s, R, gm, gk,
                                   dk);
            }
        }
        if (R.n_cut > 0) {
            if (R.n_box > 0)
                hipLaunchKernelGGL((k_adj_cut<T, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, gm, gk, dk);
            hipLaunchKernelGGL((k_adj_remainder<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemAdjCfg<P>::NT), 0, s, R, gm,
                               gk, dk);
        }
        if (forked && (hipEventRecord(H->ev_join, H->side) != hipSuccess || hipStreamWaitEvent(s, H->ev_join, 0) != hipSuccess)) {
            (void)hipGetLastError();
            (void)hipStreamSynchronize(H->side);
        }
        err = hipFreeAsync(part, s);
        if (err != hipSuccess)
            return wq_set_error(WQ_EHIP, "wq_assemble_adjoint: scratch release failed: %s", hipGetErrorString(err));
        return WQ_OK;
    }
    if (R.n_lblocks > 0) {
        if constexpr (P <= 4) {
            using C = AdjCfg<T, P, WHICH, 16>;
            hipLaunchKernelGGL((k_adj_interior<T, P, WHICH, 16>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0, s, R, gm, gk, dk);
        } else {
            using C = AdjCfg<T, P, WHICH, 8>;
            hipLaunchKernelGGL((k_adj_interior<T, P, WHICH, 8>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0, s, R, gm, gk, dk);
        }
    }
    if (R.n_cut > 0) {
        if (R.n_box > 0)
            hipLaunchKernelGGL((k_adj_cut<T, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, gm, gk, dk);
        hipLaunchKernelGGL((k_adj_remainder<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemAdjCfg<P>::NT), 0, s, R, gm, gk,
                           dk);
    }
    if (R.n_cut_elems > 0) {
        {
            if (R.levels <= 3) {
                using C = MomCfg<P>;
                T* part = nullptr;
                hipError_t err = H->scratch_alloc((void**)&part, sizeof(T) * (size_t)R.n_cut_elems * C::P1 * C::NK3, s);
                if (err != hipSuccess)
                    return wq_set_error(WQ_ENOMEM, "wq_assemble_adjoint: scratch allocation failed: %s", hipGetErrorString(err));
                if constexpr (P <= 4)
                    hipLaunchKernelGGL((k_adj_local<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1)), dim3(256), 0, s,
                                       R, H->act2cut, gm, gk, part);
                else
                    hipLaunchKernelGGL((k_adj_local_a2<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1)), dim3(256), 0,
                                       s, R, H->act2cut, gm, gk, part);
                if (R.fit)
        hipLaunchKernelGGL((k_adj_fit<T, P>), dim3((unsigned)R.n_cut_elems), dim3(256), 0, s, R, (const T*)part, dk);
    else
        hipLaunchKernelGGL((k_adj_leaves<T, P>), dim3((unsigned)R.n_cut_elems), dim3(256), 0, s, R, (const T*)part, dk);
                err = hipFreeAsync(part, s);
                if (err != hipSuccess)
                    return wq_set_error(WQ_EHIP, "wq_assemble_adjoint: scratch release failed: %s", hipGetErrorString(err));
                return WQ_OK;
            }
        }
        using C = OctAdjCfg<P>;
        hipLaunchKernelGGL((k_adj_octree<T, P, WHICH>), dim3((unsigned)R.n_cut_elems), dim3(C::NT), 0, s, R,
                           H->act2cut, gm, gk, dk);
    }
    return WQ_OK;
}

template <typename T, int P>
static int launch_adj_w(const wq_rules* H, uint32_t which, const T* gm, const T* gk, T* dk, hipStream_t s) {
    if (which == 1) return launch_adj_p<T, P, 1>(H, gm, gk, dk, s);
    if (which == 2) return launch_adj_p<T, P, 2>(H, gm, gk, dk, s);
    return launch_adj_p<T, P, 3>(H, gm, gk, dk, s);
}

template <typename T>
int launch_adjoint(const wq_rules* H, uint32_t which, const T* gm, const T* gk, T* dk, hipStream_t s) {
    const int64_t n = H->R.n_kappa;
    if (n > 0) hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dk, n, (T)0);
    if (H->nnz == 0) return WQ_OK;
    switch (H->R.p) {
        case 1: return launch_adj_w<T, 1>(H, which, gm, gk, dk, s);
        case 2: return launch_adj_w<T, 2>(H, which, gm, gk, dk, s);
        case 3: return launch_adj_w<T, 3>(H, which, gm, gk, dk, s);
        case 4: return launch_adj_w<T, 4>(H, which, gm, gk, dk, s);
        case 5: return launch_adj_w<T, 5>(H, which, gm, gk, dk, s);
        case 6: return launch_adj_w<T, 6>(H, which, gm, gk, dk, s);
    }
    return WQ_OK;
}

#ifndef WQ_ONLY_F32
template int launch_adjoint<double>(const wq_rules*, uint32_t, const double*, const double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template int launch_adjoint<float>(const wq_rules*, uint32_t, const float*, const float*, float*, hipStream_t);
#endif
