// cut_assemble: the part of Eq. (1) that is integrated element by element.
//
// (i) Remainder elements: for every cut row, the interior elements of its support that lie
//     outside its DWQ box are integrated with the (p+1)^3 element Gauss rule, test weights
//     omega_g B_I(x_g) (gradient for stiffness).  One workgroup per cut row; each wave
//     takes elements in turn, contracts the three directions over the element's tensor
//     Gauss grid and adds into a row accumulator in LDS, which is then added into the row
//     (a row is owned by one workgroup, so no global atomics).
// (ii) Cut elements: octree leaves with (p+1)^3 Gauss points each (weight 0 outside the
//     domain at cut leaves).  One workgroup per (cut element, a2, group of a1), with (a1,
//     a2, a3) the local index of the test function on the element; per leaf the local
//     matrix is contracted direction 3, then 2, then 1 and accumulated in registers over
//     all leaves; the local rows are added into the CSR values with atomics at the end.
#include "rows.h"

__device__ inline void unlex3i(int64_t k, const int* n, int* I) {
    I[2] = (int)(k % n[2]);
    I[1] = (int)((k / n[2]) % n[1]);
    I[0] = (int)(k / ((int64_t)n[1] * n[2]));
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------------------------------------
// (i) remainder element Gauss, one workgroup per cut row
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_cut_remainder(DevRules R, const int32_t* __restrict__ box, const T* __restrict__ kappa, T* __restrict__ vm,
                T* __restrict__ vk) {
    constexpr int P1 = P + 1, NP = P1 * P1 * P1, M = 2 * P + 1, M3 = M * M * M, NWAVE = 4;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_accm[MASS ? M3 : 1], s_acck[STIFF ? M3 : 1];
    __shared__ T s_kap[NWAVE][NP];
    __shared__ T s_w[NWAVE][3][2][P1 * P1];          // [dir][a][k][g]
    __shared__ T s_t1[NWAVE][2][NP];
    __shared__ T s_t2[NWAVE][2][NP];
    const int64_t cr = blockIdx.x;
    const int ra = R.cut_rows[cr];
    int I[3];
    unlex3i(R.act2lex[ra], R.nfun, I);
    for (int k = threadIdx.x; k < M3; k += 256) {
        if (MASS) s_accm[k] = 0;
        if (STIFF) s_acck[k] = 0;
    }
    int lo[3], hi[3], blo[3], bhi[3];
    const bool has_box = R.split[cr].x >= 0;
    for (int d = 0; d < 3; ++d) {
        lo[d] = I[d] - P < 0 ? 0 : I[d] - P;
        hi[d] = I[d] < R.nel[d] - 1 ? I[d] : R.nel[d] - 1;
        blo[d] = box[cr * 6 + 2 * d];
        bhi[d] = box[cr * 6 + 2 * d + 1];
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int n2 = hi[1] - lo[1] + 1, n3 = hi[2] - lo[2] + 1;
    const int ne = (hi[0] - lo[0] + 1) * n2 * n3;
    for (int k = wave; k < ne; k += NWAVE) {
        const int e[3] = {lo[0] + k / (n2 * n3), lo[1] + (k / n3) % n2, lo[2] + k % n3};
        const int64_t eid = ((int64_t)e[0] * R.nel[1] + e[1]) * R.nel[2] + e[2];
        if (R.ecls[eid] != CLS_IN) continue;
        if (has_box && e[0] >= blo[0] && e[0] <= bhi[0] && e[1] >= blo[1] && e[1] <= bhi[1] && e[2] >= blo[2] &&
            e[2] <= bhi[2])
            continue;
        // W_d[a][k][g] = omega_g (h/2) B_{I_d}^(a)(y_g) B_{e_d+k}^(a)(y_g)
        for (int t = lane; t < 3 * 2 * P1 * P1; t += 64) {
            const int d = t / (2 * P1 * P1), a = (t / (P1 * P1)) % 2, kk = (t / P1) % P1, g = t % P1;
            const int64_t y = (int64_t)e[d] * P1 + g;
            const double* tab = a ? R.dBval[d] : R.Bval[d];
            const double om = R.gw[g] * R.h[d] * 0.5;
            s_w[wave][d][a][kk * P1 + g] = (T)(om * tab[y * P1 + (I[d] - e[d])] * tab[y * P1 + kk]);
        }
        for (int t = lane; t < NP; t += 64) {
            const int g1 = t / (P1 * P1), g2 = (t / P1) % P1, g3 = t % P1;
            s_kap[wave][t] = kappa[slot_of(R, e[0] * P1 + g1, e[1] * P1 + g2, e[2] * P1 + g3)];
        }
        wave_sync();
        for (int t = lane; t < NP; t += 64) {          // T1[v][g1][g2][k3]
            const int g12 = t / P1, k3 = t % P1;
            T a0 = 0, a1 = 0;
            for (int g3 = 0; g3 < P1; ++g3) {
                const T kv = s_kap[wave][g12 * P1 + g3];
                a0 += s_w[wave][2][0][k3 * P1 + g3] * kv;
                if (STIFF) a1 += s_w[wave][2][1][k3 * P1 + g3] * kv;
            }
            s_t1[wave][0][t] = a0;
            if (STIFF) s_t1[wave][1][t] = a1;
        }
        wave_sync();
        for (int t = lane; t < NP; t += 64) {          // T2[v][g1][k2][k3]
            const int g1 = t / (P1 * P1), k2 = (t / P1) % P1, k3 = t % P1;
            T m0 = 0, ms = 0;
            for (int g2 = 0; g2 < P1; ++g2) {
                const T t0 = s_t1[wave][0][(g1 * P1 + g2) * P1 + k3];
                const T w0 = s_w[wave][1][0][k2 * P1 + g2];
                m0 += w0 * t0;
                if (STIFF) ms += s_w[wave][1][1][k2 * P1 + g2] * t0 + w0 * s_t1[wave][1][(g1 * P1 + g2) * P1 + k3];
            }
            s_t2[wave][0][t] = m0;
            if (STIFF) s_t2[wave][1][t] = ms;
        }
        wave_sync();
        for (int t = lane; t < NP; t += 64) {          // out[k1][k2][k3] into the row window
            const int k1 = t / (P1 * P1), k23 = t % (P1 * P1);
            const int k2 = k23 / P1, k3 = k23 % P1;
            T am = 0, ak = 0;
            for (int g1 = 0; g1 < P1; ++g1) {
                const T t0 = s_t2[wave][0][g1 * P1 * P1 + k23];
                const T w0 = s_w[wave][0][0][k1 * P1 + g1];
                am += w0 * t0;
                if (STIFF) ak += s_w[wave][0][1][k1 * P1 + g1] * t0 + w0 * s_t2[wave][1][g1 * P1 * P1 + k23];
            }
            const int jj = ((e[0] + k1 - I[0] + P) * M + (e[1] + k2 - I[1] + P)) * M + (e[2] + k3 - I[2] + P);
            if (MASS) atomicAdd(&s_accm[jj], am);
            if (STIFF) atomicAdd(&s_acck[jj], ak);
        }
        wave_sync();
    }
    __syncthreads();
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    for (int k = threadIdx.x; k < M3; k += 256) {
        const int o = pos[k];
        if (o < 0) continue;
        if (MASS) vm[rb + o] += s_accm[k];
        if (STIFF) vk[rb + o] += s_acck[k];
    }
}

// ----------------------------------------------------------------------------------------
// (ii) octree cut elements
// ----------------------------------------------------------------------------------------
template <int P> struct OctCfg {
    static constexpr int P1 = P + 1, NP = P1 * P1 * P1, P2 = P1 * P1;
    static constexpr int NT = ((NP + 63) / 64) * 64;
    static constexpr int AG = P <= 4 ? P1 : (P == 5 ? 3 : 4);       // a1 per workgroup
    static constexpr int NAG = (P1 + AG - 1) / AG;
    static constexpr int KA = (P2 * P2 + NT - 1) / NT;               // stage-A items per thread
    static constexpr int KB = (P1 * P1 * P2 + NT - 1) / NT;          // stage-B items per thread
};

template <typename T> __device__ inline const T* oct_tab(const DevRules& R, int d);
template <> __device__ inline const double* oct_tab<double>(const DevRules& R, int d) { return R.oct_pp64[d]; }
template <> __device__ inline const float* oct_tab<float>(const DevRules& R, int d) { return R.oct_pp32[d]; }

// Leaves are visited in the per-element sorted order: leaves with the same x-interval are
// contiguous (one x-group), and inside an x-group leaves with the same y-interval are
// contiguous (one column).  Stage A (direction 3) runs per leaf and accumulates over the
// column, stage B (direction 2) runs once per column and accumulates over the x-group,
// stage C (direction 1) runs once per x-group: each stage is applied to the sum of the
// partial results that share its 1D basis products.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(OctCfg<P>::NT)
k_cut_octree(DevRules R, const int32_t* __restrict__ act2cut, const T* __restrict__ kappa, T* __restrict__ vm,
             T* __restrict__ vk) {
    using C = OctCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, AG = C::AG, M = 2 * P + 1, NT = C::NT;
    constexpr int KA = C::KA, KB = C::KB;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_wk[NP];
    __shared__ T s_pp[3][2 * P2 * P1];                  // x-group, column, leaf products
    __shared__ T s_p1[2][P2 * P2];                      // column result [v][g1 g2][a3 b3]
    __shared__ T s_p2[2][P1 * P1 * P2];                 // x-group result [v][g1][b2][a3 b3]
    const int ce = blockIdx.x / (P1 * C::NAG);
    const int a2 = (blockIdx.x / C::NAG) % P1;
    const int ag0 = (blockIdx.x % C::NAG) * AG;
    const int64_t eid = R.cut_elems[ce];
    int e[3];
    unlex3i(eid, R.nel, e);
    const int t = threadIdx.x;
    const bool own = t < NP;
    const int b2 = t / P2, a3 = (t / P1) % P1, b3 = t % P1;   // stage-C column c2 = (b2, a3, b3)
    T accA[2][KA], accB[2][KB], accm[AG][P1], acck[AG][P1];
#pragma unroll
    for (int i = 0; i < AG; ++i)
#pragma unroll
        for (int j = 0; j < P1; ++j) { accm[i][j] = 0; acck[i][j] = 0; }
    const int64_t oct0 = R.n_grid + R.n_block;
    const int cb = R.cell_begin[ce], cend = R.cell_begin[ce + 1];
    // software pipeline: the next leaf's weight * kappa (one point per thread), key and its
    // direction-3 basis products are loaded while the current leaf is contracted
    constexpr int NPP = 2 * P2 * P1, KP = (NPP + NT - 1) / NT;
    const int ni = (2 << R.levels) - 1;
    const T* tab[3] = {oct_tab<T>(R, 0) + (int64_t)e[0] * ni * NPP, oct_tab<T>(R, 1) + (int64_t)e[1] * ni * NPP,
                       oct_tab<T>(R, 2) + (int64_t)e[2] * ni * NPP};
    auto ivl = [](int key, int d) { const int dep = key & 7; return (1 << dep) - 1 + ((key >> (3 + 6 * d)) & 63); };
    int cell_n = cb < cend ? R.cell_perm[cb] : 0;
    int key_n = cb < cend ? R.cell_key[cell_n] : 0;
    T wk_n = (own && cb < cend) ? (T)R.oct_w[(int64_t)cell_n * NP + t] * kappa[oct0 + (int64_t)cell_n * NP + t] : (T)0;
    T pz_n[KP];
#pragma unroll
    for (int i = 0; i < KP; ++i) {
        const int j = t + i * NT;
        pz_n[i] = (cb < cend && j < NPP) ? tab[2][(int64_t)ivl(key_n, 2) * NPP + j] : (T)0;
    }
    int kprev = -1;
    for (int k = cb; k < cend; ++k) {
        const int cell = cell_n, key = key_n;
        const T wk = wk_n;
        T pz[KP];
#pragma unroll
        for (int i = 0; i < KP; ++i) pz[i] = pz_n[i];
        if (k + 1 < cend) {
            cell_n = R.cell_perm[k + 1];
            key_n = R.cell_key[cell_n];
            if (own) wk_n = (T)R.oct_w[(int64_t)cell_n * NP + t] * kappa[oct0 + (int64_t)cell_n * NP + t];
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const int j = t + i * NT;
                if (j < NPP) pz_n[i] = tab[2][(int64_t)ivl(key_n, 2) * NPP + j];
            }
        }
        const int knext = k + 1 < cend ? key_n : -1;
        const int xmask = (1 << 9) - 1, cmask = (1 << 15) - 1;
        const bool new_x = kprev < 0 || (key & xmask) != (kprev & xmask);
        const bool new_col = kprev < 0 || (key & cmask) != (kprev & cmask);
        const bool end_col = knext < 0 || (key & cmask) != (knext & cmask);
        const bool end_x = knext < 0 || (key & xmask) != (knext & xmask);
        kprev = key;
        if (new_col) {
#pragma unroll
            for (int i = 0; i < KA; ++i) { accA[0][i] = 0; accA[1][i] = 0; }
        }
        if (new_x) {
#pragma unroll
            for (int i = 0; i < KB; ++i) { accB[0][i] = 0; accB[1][i] = 0; }
        }
        if (own) s_wk[t] = wk;
#pragma unroll
        for (int i = 0; i < KP; ++i) {
            const int j = t + i * NT;
            if (j < NPP) {
                s_pp[2][j] = pz[i];
                if (new_col) s_pp[1][j] = tab[1][(int64_t)ivl(key, 1) * NPP + j];
                if (new_x) s_pp[0][j] = tab[0][(int64_t)ivl(key, 0) * NPP + j];
            }
        }
        __syncthreads();
        // stage A: accA[v][g1 g2][a3 b3] += sum_g3 pp3[v][a3 b3][g3] wk[g1 g2 g3]
#pragma unroll
        for (int i = 0; i < KA; ++i) {
            const int it = t + i * NT;
            if (it < P2 * P2) {
                const int g12 = it / P2, ab3 = it % P2;
                T s0 = 0, s1 = 0;
#pragma unroll
                for (int g3 = 0; g3 < P1; ++g3) {
                    const T w = s_wk[g12 * P1 + g3];
                    s0 += s_pp[2][ab3 * P1 + g3] * w;
                    if (STIFF) s1 += s_pp[2][P2 * P1 + ab3 * P1 + g3] * w;
                }
                accA[0][i] += s0;
                accA[1][i] += s1;
            }
        }
        if (end_col) {
#pragma unroll
            for (int i = 0; i < KA; ++i) {
                const int it = t + i * NT;
                if (it < P2 * P2) {
                    s_p1[0][it] = accA[0][i];
                    if (STIFF) s_p1[1][it] = accA[1][i];
                }
            }
            __syncthreads();
            // stage B: accB[g1][b2][a3 b3] += sum_g2 pp2[0][a2 b2][g2] P1_0 (+ stiffness terms)
#pragma unroll
            for (int i = 0; i < KB; ++i) {
                const int it = t + i * NT;
                if (it < P1 * P1 * P2) {
                    const int g1 = it / (P1 * P2), bb2 = (it / P2) % P1, ab3 = it % P2;
                    T s0 = 0, ss = 0;
#pragma unroll
                    for (int g2 = 0; g2 < P1; ++g2) {
                        const T v0 = s_p1[0][(g1 * P1 + g2) * P2 + ab3];
                        const T w0 = s_pp[1][(a2 * P1 + bb2) * P1 + g2];
                        s0 += w0 * v0;
                        if (STIFF) ss += s_pp[1][P2 * P1 + (a2 * P1 + bb2) * P1 + g2] * v0 + w0 * s_p1[1][(g1 * P1 + g2) * P2 + ab3];
                    }
                    accB[0][i] += s0;
                    accB[1][i] += ss;
                }
            }
            if (end_x) {
#pragma unroll
                for (int i = 0; i < KB; ++i) {
                    const int it = t + i * NT;
                    if (it < P1 * P1 * P2) {
                        s_p2[0][it] = accB[0][i];
                        if (STIFF) s_p2[1][it] = accB[1][i];
                    }
                }
                __syncthreads();
                // stage C: acc[a1][b1] += sum_g1 pp1[.][a1 b1][g1] P2[.][g1][c2]
                if (own) {
                    T v0[P1], vs[P1];
#pragma unroll
                    for (int g1 = 0; g1 < P1; ++g1) {
                        v0[g1] = s_p2[0][g1 * P1 * P2 + t];
                        vs[g1] = STIFF ? s_p2[1][g1 * P1 * P2 + t] : (T)0;
                    }
#pragma unroll
                    for (int i = 0; i < AG; ++i) {
                        const int a1 = ag0 + i;
                        if (a1 >= P1) break;
#pragma unroll
                        for (int b1 = 0; b1 < P1; ++b1) {
                            T sm = 0, sk = 0;
#pragma unroll
                            for (int g1 = 0; g1 < P1; ++g1) {
                                const T w0 = s_pp[0][(a1 * P1 + b1) * P1 + g1];
                                sm += w0 * v0[g1];
                                if (STIFF) sk += s_pp[0][P2 * P1 + (a1 * P1 + b1) * P1 + g1] * v0[g1] + w0 * vs[g1];
                            }
                            accm[i][b1] += sm;
                            acck[i][b1] += sk;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    if (!own) return;
    // scatter: row a = e + (a1, a2, a3), column b = e + (b1, b2, b3)
#pragma unroll
    for (int i = 0; i < AG; ++i) {
        const int a1 = ag0 + i;
        if (a1 >= P1) break;
        const int64_t alex = ((int64_t)(e[0] + a1) * R.nfun[1] + (e[1] + a2)) * R.nfun[2] + (e[2] + a3);
        const int ra = R.lex2act[alex];
        const int cr = act2cut[ra];
        const int32_t* pos = R.pos_map + (int64_t)cr * M * M * M;
        const int64_t rb = R.row_ptr[ra];
#pragma unroll
        for (int b1 = 0; b1 < P1; ++b1) {
            const int jj = ((b1 - a1 + P) * M + (b2 - a2 + P)) * M + (b3 - a3 + P);
            const int o = pos[jj];
            if (o < 0) continue;
            if (MASS) atomicAdd(&vm[rb + o], accm[i][b1]);
            if (STIFF) atomicAdd(&vk[rb + o], acck[i][b1]);
        }
    }
}

// ----------------------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH>
static void launch_cut_p(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if (R.n_cut > 0)
        hipLaunchKernelGGL((k_cut_remainder<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(256), 0, s, R, H->box, kappa, vm, vk);
    if (R.n_cut_elems > 0) {
        using C = OctCfg<P>;
        hipLaunchKernelGGL((k_cut_octree<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1 * C::NAG)), dim3(C::NT), 0, s, R,
                           H->act2cut, kappa, vm, vk);
    }
}

template <typename T, int P>
static void launch_cut_w(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s) {
    if (which == 1) launch_cut_p<T, P, 1>(H, kappa, vm, vk, s);
    else if (which == 2) launch_cut_p<T, P, 2>(H, kappa, vm, vk, s);
    else launch_cut_p<T, P, 3>(H, kappa, vm, vk, s);
}

template <typename T>
void launch_cut(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s) {
    switch (H->R.p) {
        case 1: launch_cut_w<T, 1>(H, which, kappa, vm, vk, s); break;
        case 2: launch_cut_w<T, 2>(H, which, kappa, vm, vk, s); break;
        case 3: launch_cut_w<T, 3>(H, which, kappa, vm, vk, s); break;
        case 4: launch_cut_w<T, 4>(H, which, kappa, vm, vk, s); break;
        case 5: launch_cut_w<T, 5>(H, which, kappa, vm, vk, s); break;
        case 6: launch_cut_w<T, 6>(H, which, kappa, vm, vk, s); break;
    }
}

#ifndef WQ_ONLY_F32
template void launch_cut<double>(const wq_rules*, uint32_t, const double*, double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template void launch_cut<float>(const wq_rules*, uint32_t, const float*, float*, float*, hipStream_t);
#endif
