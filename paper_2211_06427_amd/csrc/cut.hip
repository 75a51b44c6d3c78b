// cut_assemble: the part of Eq. (1) that is integrated element by element.
//
// (i) Remainder elements: for every cut row, the interior elements of its support that lie
//     outside its DWQ box are integrated with the (p+1)^3 element Gauss rule, test weights
//     omega_g B_I(x_g) (gradient for stiffness).  One workgroup per cut row; each wave
//     takes elements in turn, contracts the three directions over the element's tensor
//     Gauss grid and adds into a row accumulator in LDS, which is then added into the row
//     (a row is owned by one workgroup, so no global atomics).
// (ii) Cut elements: octree leaves with (p+1)^3 Gauss points each (weight 0 outside the
//     domain at cut leaves).  For octrees of depth <= 3 (the default) in moment form:
//     k_cut_moments forms each cut element's Bernstein moments of w kappa over its leaves,
//     k_cut_local (k_cut_local_a2 at p = 5, 6) contracts them with the Bernstein tables of
//     the basis products into the element's local rows, and k_cut_gather adds every cut
//     row's local rows in a fixed order (one workgroup per row, no atomics).  Deeper
//     octrees take k_cut_octree: one workgroup per (cut element, a3, group of a1), the
//     local matrix contracted leaf by leaf and added into the CSR values with atomics.
//     Under the fitted cut rule (WQ_OPT_MOMENT_FIT) the moments come from the element's
//     (2p+1)^3 fitted points instead (k_cut_moments_fit); the rest is unchanged.
// (iii) The coefficient-tensor stiffness reuses (ii): moments of each of the six tensor
//     components, local stiffness rows per element (k_tensor_local), the same gather.
#include <algorithm>
#include <mutex>

#include "rows.h"
#include "moments.h"

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
template <int P> struct RemCfg {
    static constexpr int P1 = P + 1, NP = P1 * P1 * P1, P2 = P1 * P1;
    static constexpr int SLOT = ((NP + 63) / 64) * 64;         // threads per element in flight
    static constexpr int NT = SLOT >= 256 ? SLOT : 256;
    static constexpr int NSLOT = NT / SLOT;                    // elements in flight per workgroup
};

template <typename T> __device__ inline const T* rem_tab(const DevRules& R, int d);
template <> __device__ inline const double* rem_tab<double>(const DevRules& R, int d) { return R.rem_w64[d]; }
template <> __device__ inline const float* rem_tab<float>(const DevRules& R, int d) { return R.rem_w32[d]; }

// One workgroup per cut row, NSLOT remainder elements in flight, one thread per Gauss point
// (stage 1) or per partial / output entry (stages 2, 3).  The row's 1D weights sit in LDS;
// kappa of the next element is loaded while the current one is contracted.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(RemCfg<P>::NT)
k_cut_remainder(DevRules R, const T* __restrict__ kappa, T* __restrict__ vm, T* __restrict__ vk) {
    using C = RemCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, M = 2 * P + 1, M3 = M * M * M, NT = C::NT, SLOT = C::SLOT;
    constexpr int NSLOT = C::NSLOT;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    // per-slot accumulators: inside one pass every output of a slot has one writer, so
    // they are updated without atomics and summed over the slots at the end
    __shared__ T s_accm[NSLOT][MASS ? M3 : 1], s_acck[NSLOT][STIFF ? M3 : 1];
    __shared__ T s_wt[3][P1][2 * P2];                 // [d][I_d - e_d][a][k][g]
    __shared__ T s_kap[NSLOT][NP];
    __shared__ T s_t1[NSLOT][2][NP];
    __shared__ T s_t2[NSLOT][2][NP];
    __shared__ int2 s_list[NP];
    const int64_t cr = blockIdx.x;
    const int ra = R.cut_rows[cr];
    int I[3];
    unlex3i(R.act2lex[ra], R.nfun, I);
    const int t = threadIdx.x;
    const int l0 = R.rem_ptr[cr], nrem = R.rem_ptr[cr + 1] - l0;
    if (nrem == 0) return;
    for (int k = t; k < NSLOT * M3; k += NT) {
        if (MASS) s_accm[k / M3][k % M3] = 0;
        if (STIFF) s_acck[k / M3][k % M3] = 0;
    }
    for (int q = t; q < 3 * P1 * 2 * P2; q += NT) {
        const int d = q / (P1 * 2 * P2), kI = (q / (2 * P2)) % P1, rest = q % (2 * P2);
        const int e = I[d] - kI;
        s_wt[d][kI][rest] = (e >= 0 && e < R.nel[d]) ? rem_tab<T>(R, d)[((int64_t)e * P1 + kI) * 2 * P2 + rest] : (T)0;
    }
    for (int k = t; k < nrem; k += NT) s_list[k] = R.rem_list[l0 + k];
    __syncthreads();
    const int sl = t / SLOT, u = t % SLOT;
    const bool act_u = u < NP;
    const int d1 = u / P2, d2 = (u / P1) % P1, d3 = u % P1;       // u = (d1, d2, d3)
    // pipeline: kappa one pass ahead, its slot index two passes ahead
    T kap_c = 0;
    int bs_n = 0;
    if (act_u && sl < nrem) kap_c = kappa[R.blk_slot[(int64_t)s_list[sl].y * NP + u]];
    if (act_u && sl + NSLOT < nrem) bs_n = R.blk_slot[(int64_t)s_list[sl + NSLOT].y * NP + u];
    for (int r0 = 0; r0 < nrem; r0 += NSLOT) {
        const int r = r0 + sl;
        const bool active = r < nrem;
        if (active && act_u) s_kap[sl][u] = kap_c;
        kap_c = (act_u && r + NSLOT < nrem) ? kappa[bs_n] : (T)0;
        bs_n = (act_u && r + 2 * NSLOT < nrem) ? R.blk_slot[(int64_t)s_list[r + 2 * NSLOT].y * NP + u] : 0;
        const int pk = active ? s_list[r].x : 0;
        const int kI0 = pk & 15, kI1 = (pk >> 4) & 15, kI2 = (pk >> 8) & 15;
        const T* W1 = s_wt[0][kI0];
        const T* W2 = s_wt[1][kI1];
        const T* W3 = s_wt[2][kI2];
        __syncthreads();
        if (active && act_u) {                      // stage 1: T1[v][g1 g2][k3], u = (g1, g2, k3)
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int g3 = 0; g3 < P1; ++g3) {
                const T kv = s_kap[sl][(d1 * P1 + d2) * P1 + g3];
                a0 += W3[d3 * P1 + g3] * kv;
                if (STIFF) a1 += W3[P2 + d3 * P1 + g3] * kv;
            }
            s_t1[sl][0][u] = a0;
            if (STIFF) s_t1[sl][1][u] = a1;
        }
        __syncthreads();
        if (active && act_u) {                      // stage 2: T2[v][g1][k2][k3], u = (g1, k2, k3)
            T m0 = 0, ms = 0;
#pragma unroll
            for (int g2 = 0; g2 < P1; ++g2) {
                const T t0 = s_t1[sl][0][(d1 * P1 + g2) * P1 + d3];
                const T w0 = W2[d2 * P1 + g2];
                m0 += w0 * t0;
                if (STIFF) ms = fmat(w0, s_t1[sl][1][(d1 * P1 + g2) * P1 + d3], fmat(W2[P2 + d2 * P1 + g2], t0, ms));
            }
            s_t2[sl][0][u] = m0;
            if (STIFF) s_t2[sl][1][u] = ms;
        }
        __syncthreads();
        if (active && act_u) {                      // stage 3: out[k1][k2][k3], u = (k1, k2, k3)
            T am = 0, ak = 0;
#pragma unroll
            for (int g1 = 0; g1 < P1; ++g1) {
                const T t0 = s_t2[sl][0][g1 * P2 + d2 * P1 + d3];
                const T w0 = W1[d1 * P1 + g1];
                am += w0 * t0;
                if (STIFF) ak = fmat(w0, s_t2[sl][1][g1 * P2 + d2 * P1 + d3], fmat(W1[P2 + d1 * P1 + g1], t0, ak));
            }
            // trial J = e + (d1, d2, d3) = I + (d - kI): local index d - kI + P
            const int jj = ((d1 - kI0 + P) * M + (d2 - kI1 + P)) * M + (d3 - kI2 + P);
            if (MASS) s_accm[sl][jj] += am;
            if (STIFF) s_acck[sl][jj] += ak;
        }
        __syncthreads();
    }
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        if (o < 0) continue;
        T am = 0, ak = 0;
#pragma unroll
        for (int i = 0; i < NSLOT; ++i) {
            if (MASS) am += s_accm[i][k];
            if (STIFF) ak += s_acck[i][k];
        }
        if (MASS) vm[rb + o] += am;
        if (STIFF) vk[rb + o] += ak;
    }
}

// Eight consecutive values from LDS (16-byte aligned) in two or four vector loads.
__device__ inline void lds8(const float* p, float (&r)[8]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 a = *reinterpret_cast<const f4*>(p), b = *reinterpret_cast<const f4*>(p + 4);
    r[0] = a.x; r[1] = a.y; r[2] = a.z; r[3] = a.w; r[4] = b.x; r[5] = b.y; r[6] = b.z; r[7] = b.w;
}
__device__ inline void lds8(const double* p, double (&r)[8]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const d2 a = *reinterpret_cast<const d2*>(p + 2 * i);
        r[2 * i] = a.x;
        r[2 * i + 1] = a.y;
    }
}

// k_cut_remainder with every contracted operand a run of P1 consecutive values in LDS, padded
// to 8 and read with vector loads: the row's 1D weights [d][I_d - e_d][a][k][g], kappa
// [g1 g2][g3], the stage-1 result [g1 k3][g2] and the stage-2 result [k2 k3][g1].  Fewer LDS
// instructions, more registers and LDS per workgroup: faster for FP32 at p = 5, 6 (64^3 p = 6:
// 15.5 ms instead of 18.4), slower at p <= 4 and in FP64, where k_cut_remainder runs.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(RemCfg<P>::NT)
k_cut_remainder_v8(DevRules R, const T* __restrict__ kappa, T* __restrict__ vm, T* __restrict__ vk) {
    using C = RemCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, M = 2 * P + 1, M3 = M * M * M, NT = C::NT, SLOT = C::SLOT;
    constexpr int NSLOT = C::NSLOT, G8 = 8;
    static_assert(P1 <= G8, "runs of at most 8");
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    // per-slot accumulators: inside one pass every output of a slot has one writer, so
    // they are updated without atomics and summed over the slots at the end
    __shared__ T s_accm[NSLOT][MASS ? M3 : 1], s_acck[NSLOT][STIFF ? M3 : 1];
    __shared__ __align__(16) T s_wt[3][P1][2][P1][G8];     // [d][I_d - e_d][a][k][g]
    __shared__ __align__(16) T s_kap[NSLOT][P2][G8];        // [g1 g2][g3]
    __shared__ __align__(16) T s_t1[NSLOT][2][P2][G8];      // [v][g1 k3][g2]
    __shared__ __align__(16) T s_t2[NSLOT][2][P2][G8];      // [v][k2 k3][g1]
    __shared__ int2 s_list[NP];
    const int64_t cr = blockIdx.x;
    const int ra = R.cut_rows[cr];
    int I[3];
    unlex3i(R.act2lex[ra], R.nfun, I);
    const int t = threadIdx.x;
    const int l0 = R.rem_ptr[cr], nrem = R.rem_ptr[cr + 1] - l0;
    if (nrem == 0) return;
    for (int k = t; k < NSLOT * M3; k += NT) {
        if (MASS) s_accm[k / M3][k % M3] = 0;
        if (STIFF) s_acck[k / M3][k % M3] = 0;
    }
    for (int q = t; q < 3 * P1 * 2 * P2; q += NT) {
        const int d = q / (P1 * 2 * P2), kI = (q / (2 * P2)) % P1, rest = q % (2 * P2);
        const int a = rest / P2, k = (rest / P1) % P1, g = rest % P1;
        const int e = I[d] - kI;
        s_wt[d][kI][a][k][g] = (e >= 0 && e < R.nel[d]) ? rem_tab<T>(R, d)[((int64_t)e * P1 + kI) * 2 * P2 + rest] : (T)0;
    }
    for (int k = t; k < nrem; k += NT) s_list[k] = R.rem_list[l0 + k];
    __syncthreads();
    const int sl = t / SLOT, u = t % SLOT;
    const bool act_u = u < NP;
    const int d1 = u / P2, d2 = (u / P1) % P1, d3 = u % P1;       // u = (d1, d2, d3)
    // pipeline: kappa one pass ahead, its slot index two passes ahead
    T kap_c = 0;
    int bs_n = 0;
    if (act_u && sl < nrem) kap_c = kappa[R.blk_slot[(int64_t)s_list[sl].y * NP + u]];
    if (act_u && sl + NSLOT < nrem) bs_n = R.blk_slot[(int64_t)s_list[sl + NSLOT].y * NP + u];
    for (int r0 = 0; r0 < nrem; r0 += NSLOT) {
        const int r = r0 + sl;
        const bool active = r < nrem;
        if (active && act_u) s_kap[sl][d1 * P1 + d2][d3] = kap_c;
        kap_c = (act_u && r + NSLOT < nrem) ? kappa[bs_n] : (T)0;
        bs_n = (act_u && r + 2 * NSLOT < nrem) ? R.blk_slot[(int64_t)s_list[r + 2 * NSLOT].y * NP + u] : 0;
        const int pk = active ? s_list[r].x : 0;
        const int kI0 = pk & 15, kI1 = (pk >> 4) & 15, kI2 = (pk >> 8) & 15;
        __syncthreads();
        if (active && act_u) {                      // stage 1: T1[v][g1 k3][g2], u = (g1, g2, k3)
            T kv[G8], w0[G8], w1[G8];
            lds8(s_kap[sl][d1 * P1 + d2], kv);
            lds8(s_wt[2][kI2][0][d3], w0);
            T a0 = 0, a1 = 0;
            if (STIFF) lds8(s_wt[2][kI2][1][d3], w1);
#pragma unroll
            for (int g3 = 0; g3 < P1; ++g3) {
                a0 += w0[g3] * kv[g3];
                if (STIFF) a1 += w1[g3] * kv[g3];
            }
            s_t1[sl][0][d1 * P1 + d3][d2] = a0;
            if (STIFF) s_t1[sl][1][d1 * P1 + d3][d2] = a1;
        }
        __syncthreads();
        if (active && act_u) {                      // stage 2: T2[v][k2 k3][g1], u = (g1, k2, k3)
            T t0[G8], t1[G8], w0[G8], w1[G8];
            lds8(s_t1[sl][0][d1 * P1 + d3], t0);
            lds8(s_wt[1][kI1][0][d2], w0);
            if (STIFF) {
                lds8(s_t1[sl][1][d1 * P1 + d3], t1);
                lds8(s_wt[1][kI1][1][d2], w1);
            }
            T m0 = 0, ms = 0;
#pragma unroll
            for (int g2 = 0; g2 < P1; ++g2) {
                m0 += w0[g2] * t0[g2];
                if (STIFF) ms = fmat(w0[g2], t1[g2], fmat(w1[g2], t0[g2], ms));
            }
            s_t2[sl][0][d2 * P1 + d3][d1] = m0;
            if (STIFF) s_t2[sl][1][d2 * P1 + d3][d1] = ms;
        }
        __syncthreads();
        if (active && act_u) {                      // stage 3: out[k1][k2][k3], u = (k1, k2, k3)
            T t0[G8], t1[G8], w0[G8], w1[G8];
            lds8(s_t2[sl][0][d2 * P1 + d3], t0);
            lds8(s_wt[0][kI0][0][d1], w0);
            if (STIFF) {
                lds8(s_t2[sl][1][d2 * P1 + d3], t1);
                lds8(s_wt[0][kI0][1][d1], w1);
            }
            T am = 0, ak = 0;
#pragma unroll
            for (int g1 = 0; g1 < P1; ++g1) {
                am += w0[g1] * t0[g1];
                if (STIFF) ak = fmat(w0[g1], t1[g1], fmat(w1[g1], t0[g1], ak));
            }
            // trial J = e + (d1, d2, d3) = I + (d - kI): local index d - kI + P
            const int jj = ((d1 - kI0 + P) * M + (d2 - kI1 + P)) * M + (d3 - kI2 + P);
            if (MASS) s_accm[sl][jj] += am;
            if (STIFF) s_acck[sl][jj] += ak;
        }
        __syncthreads();
    }
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        if (o < 0) continue;
        T am = 0, ak = 0;
#pragma unroll
        for (int i = 0; i < NSLOT; ++i) {
            if (MASS) am += s_accm[i][k];
            if (STIFF) ak += s_acck[i][k];
        }
        if (MASS) vm[rb + o] += am;
        if (STIFF) vk[rb + o] += ak;
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
};

template <typename T> __device__ inline const T* oct_wt(const DevRules& R);
template <> __device__ inline const double* oct_wt<double>(const DevRules& R) { return R.oct_w; }
template <> __device__ inline const float* oct_wt<float>(const DevRules& R) { return R.oct_w32; }
template <typename T> __device__ inline const T* oct_tab(const DevRules& R, int d);
template <> __device__ inline const double* oct_tab<double>(const DevRules& R, int d) { return R.oct_pp64[d]; }
template <> __device__ inline const float* oct_tab<float>(const DevRules& R, int d) { return R.oct_pp32[d]; }

// One workgroup per (cut element, a3, group of a1), (a1, a2, a3) the local index of the test
// function on the element.  With a3 fixed, the direction-3 stage per leaf is
// P1[g1 g2][b3] = sum_g3 pz[a3 b3][g3] wk[g1 g2 g3].  Leaves are visited in the per-element
// sorted order: leaves with the same x-interval are contiguous (x-group), and inside an
// x-group leaves with the same y-interval are contiguous (column).  The direction-3 stage
// accumulates over a column, the direction-2 stage runs once per column and accumulates
// over the x-group, the direction-1 stage runs once per x-group.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(OctCfg<P>::NT)
k_cut_octree(DevRules R, const int32_t* __restrict__ act2cut, const T* __restrict__ kappa, T* __restrict__ vm,
             T* __restrict__ vk) {
    using C = OctCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, AG = C::AG, M = 2 * P + 1, NT = C::NT;
    constexpr int NPP = 2 * P2 * P1, KP = (NPP + NT - 1) / NT, MAXC = 512;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ int s_cell[MAXC], s_key[MAXC];          // this chunk of the sorted leaves
    __shared__ T s_wk[2][NP];                           // weight * kappa, double buffered
    __shared__ T s_pz[2][NPP];                          // direction-3 products, double buffered
    __shared__ T s_py[NPP], s_px[NPP];                  // column / x-group products
    __shared__ T s_p1[2][P2 * P1];                      // column result [v][g1 g2][b3]
    __shared__ T s_p2[2][P1 * NP];                      // x-group result [v][g1][a2 b2 b3]
    // the P1 * NAG workgroups of one cut element read the same leaves: keep them on one XCD
    const int bid = xcd_logical(blockIdx.x, gridDim.x);
    const int ce = bid / (P1 * C::NAG);
    const int a3 = (bid / C::NAG) % P1;
    const int ag0 = (bid % C::NAG) * AG;
    const T* __restrict__ ow = oct_wt<T>(R);
    const int64_t eid = R.cut_elems[ce];
    int e[3];
    unlex3i(eid, R.nel, e);
    const int t = threadIdx.x;
    const bool own = t < NP;
    // stage C column c2 = t = (a2, b2, b3); stage A item (g1 g2, b3) = t; stage B item (g1, a2, b3)
    const int a2 = t / P2, b2 = (t / P1) % P1, b3 = t % P1;
    const int g12A = t / P1;
    const int g1B = t / P2, a2B = (t / P1) % P1;
    T accA0 = 0, accA1 = 0, accB[2][P1], accm[AG][P1], acck[AG][P1];
#pragma unroll
    for (int i = 0; i < AG; ++i)
#pragma unroll
        for (int j = 0; j < P1; ++j) { accm[i][j] = 0; acck[i][j] = 0; }
    const int64_t oct0 = R.n_grid + R.n_block;
    const int cb = R.cell_begin[ce], cend = R.cell_begin[ce + 1];
    const int ni = (2 << R.levels) - 1;
    const T* tx = oct_tab<T>(R, 0) + (int64_t)e[0] * ni * NPP;
    const T* ty = oct_tab<T>(R, 1) + (int64_t)e[1] * ni * NPP;
    const T* tz = oct_tab<T>(R, 2) + (int64_t)e[2] * ni * NPP;
    auto ivl = [](int key, int d) { return (1 << (key & 7)) - 1 + ((key >> (3 + 6 * d)) & 63); };
    const int xmask = (1 << 9) - 1, cmask = (1 << 15) - 1;
    int kprev = -1, buf = 0;
    for (int c0 = cb; c0 < cend; c0 += MAXC) {
        const int nc = cend - c0 < MAXC ? cend - c0 : MAXC;
        __syncthreads();
        for (int j = t; j < nc; j += NT) {
            const int cell = R.cell_perm[c0 + j];
            s_cell[j] = cell;
            s_key[j] = R.cell_key[cell];
        }
        const int key_after = c0 + nc < cend ? R.cell_key[R.cell_perm[c0 + nc]] : -1;
        __syncthreads();
        // software pipeline: the next leaf's data is loaded while the current one is contracted
        T wk_n = 0, pz_n[KP], py_n[KP], px_n[KP];
        {
            const int cell = s_cell[0], key = s_key[0];
            if (own) wk_n = ow[(int64_t)cell * NP + t] * kappa[oct0 + (int64_t)cell * NP + t];
#pragma unroll
            for (int i = 0; i < KP; ++i) {
                const int q = t + i * NT;
                pz_n[i] = q < NPP ? tz[(int64_t)ivl(key, 2) * NPP + q] : (T)0;
                py_n[i] = q < NPP ? ty[(int64_t)ivl(key, 1) * NPP + q] : (T)0;
                px_n[i] = q < NPP ? tx[(int64_t)ivl(key, 0) * NPP + q] : (T)0;
            }
        }
        for (int j = 0; j < nc; ++j) {
            const int key = s_key[j];
            const int knext = j + 1 < nc ? s_key[j + 1] : key_after;
            const bool new_x = kprev < 0 || (key & xmask) != (kprev & xmask);
            const bool new_col = kprev < 0 || (key & cmask) != (kprev & cmask);
            const bool end_col = knext < 0 || (key & cmask) != (knext & cmask);
            const bool end_x = knext < 0 || (key & xmask) != (knext & xmask);
            kprev = key;
            if (new_col) { accA0 = 0; accA1 = 0; }
            if (new_x) {
#pragma unroll
                for (int b = 0; b < P1; ++b) { accB[0][b] = 0; accB[1][b] = 0; }
            }
            if (own) s_wk[buf][t] = wk_n;
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
                const int cell = s_cell[j + 1];
                if (own) wk_n = ow[(int64_t)cell * NP + t] * kappa[oct0 + (int64_t)cell * NP + t];
                const bool nc_next = (knext & cmask) != (key & cmask), nx_next = (knext & xmask) != (key & xmask);
#pragma unroll
                for (int i = 0; i < KP; ++i) {
                    const int q = t + i * NT;
                    if (q < NPP) {
                        pz_n[i] = tz[(int64_t)ivl(knext, 2) * NPP + q];
                        if (nc_next) py_n[i] = ty[(int64_t)ivl(knext, 1) * NPP + q];
                        if (nx_next) px_n[i] = tx[(int64_t)ivl(knext, 0) * NPP + q];
                    }
                }
            }
            __syncthreads();
            // stage A: P1[v][g1 g2][b3] += sum_g3 pz[v][a3 b3][g3] wk[g1 g2 g3]
            if (t < P2 * P1) {
#pragma unroll
                for (int g3 = 0; g3 < P1; ++g3) {
                    const T w = s_wk[buf][g12A * P1 + g3];
                    accA0 += s_pz[buf][(a3 * P1 + b3) * P1 + g3] * w;
                    if (STIFF) accA1 += s_pz[buf][P2 * P1 + (a3 * P1 + b3) * P1 + g3] * w;
                }
            }
            buf ^= 1;
            if (end_col) {
                if (t < P2 * P1) {
                    s_p1[0][t] = accA0;
                    if (STIFF) s_p1[1][t] = accA1;
                }
                __syncthreads();
                // stage B: P2[g1][a2 b2][b3] += sum_g2 py[0][a2 b2][g2] P1_0[g1 g2][b3] (+ stiffness)
                if (own) {
                    T u0[P1], u1[P1];
#pragma unroll
                    for (int g2 = 0; g2 < P1; ++g2) {
                        u0[g2] = s_p1[0][(g1B * P1 + g2) * P1 + b3];
                        u1[g2] = STIFF ? s_p1[1][(g1B * P1 + g2) * P1 + b3] : (T)0;
                    }
#pragma unroll
                    for (int bb2 = 0; bb2 < P1; ++bb2) {
                        T s0 = 0, ss = 0;
#pragma unroll
                        for (int g2 = 0; g2 < P1; ++g2) {
                            const T w0 = s_py[(a2B * P1 + bb2) * P1 + g2];
                            s0 += w0 * u0[g2];
                            if (STIFF) ss = fmat(w0, u1[g2], fmat(s_py[P2 * P1 + (a2B * P1 + bb2) * P1 + g2], u0[g2], ss));
                        }
                        accB[0][bb2] += s0;
                        accB[1][bb2] += ss;
                    }
                }
                if (end_x) {
                    if (own) {
#pragma unroll
                        for (int bb2 = 0; bb2 < P1; ++bb2) {
                            const int c = (a2B * P1 + bb2) * P1 + b3;
                            s_p2[0][g1B * NP + c] = accB[0][bb2];
                            if (STIFF) s_p2[1][g1B * NP + c] = accB[1][bb2];
                        }
                    }
                    __syncthreads();
                    // stage C: acc[a1][b1] += sum_g1 px[.][a1 b1][g1] P2[.][g1][c2]
                    if (own) {
                        T v0[P1], vs[P1];
#pragma unroll
                        for (int g1 = 0; g1 < P1; ++g1) {
                            v0[g1] = s_p2[0][g1 * NP + t];
                            vs[g1] = STIFF ? s_p2[1][g1 * NP + t] : (T)0;
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
                                    const T w0 = s_px[(a1 * P1 + b1) * P1 + g1];
                                    sm += w0 * v0[g1];
                                    if (STIFF) sk = fmat(w0, vs[g1], fmat(s_px[P2 * P1 + (a1 * P1 + b1) * P1 + g1], v0[g1], sk));
                                }
                                accm[i][b1] += sm;
                                acck[i][b1] += sk;
                            }
                        }
                    }
                }
                __syncthreads();       // s_py / s_px / s_p1 / s_p2 are rewritten by the next column
            }
        }
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
// (ii') octree cut elements for p <= 4: the column (direction 2) and x-group (direction 1)
// contractions on matrix cores
// ----------------------------------------------------------------------------------------
// Cut elements in moment form.  On an element every product phi_a phi_b (and phi_a' phi_b')
// of one direction is a degree-2p polynomial with Bernstein coefficients Q_v[ab][k], so with
// the moments
//   Mom[k1 k2 k3] = sum over the element's octree points of w kappa B_k1(x) B_k2(y) B_k3(z)
// (B the degree-2p Bernstein polynomials of the element) the local matrices are
//   M[a][b] = sum_k QX0[a1 b1][k1] QY0[a2 b2][k2] QZ0[a3 b3][k3] Mom[k],
//   K[a][b] = the same with Q1 in one direction, summed over the three directions.
// Exact up to rounding: the Bernstein expansion is an identity.
//
// k_cut_moments: one workgroup per cut element forms Mom leaf by leaf (direction 3 per
// leaf, direction 2 per column, direction 1 per x-group) and writes it to a scratch buffer.
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_cut_moments(DevRules R, const T* __restrict__ kappa, T* __restrict__ mom, int ce0) {
    using C = MomCfg<P>;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int NB = C::NB, KW = C::KW, MAXC = C::MAXC;
    constexpr int NZ = C::NZ, NY = C::NY, RZ = C::RZ, RY = C::RY, RX = C::RX;
    __shared__ int s_cell[MAXC], s_key[MAXC];
    __shared__ T s_bi[C::NIMAX * NK * P1];
    __shared__ T s_wk[2 * NB * NP];                 // weight * kappa of a batch of leaves
    __shared__ T s_mz[2 * NZ];                      // column sums, double buffered
    __shared__ T s_my[NY];                          // x-group sums

    const int ce = ce0 + blockIdx.x;                // mom holds the elements from ce0 on
    const int t = threadIdx.x;
    const int ni = (2 << R.levels) - 1;
    for (int i = t; i < ni * NK * P1; i += NT) s_bi[i] = bern_i<T>(R)[i];
    const int64_t oct0 = R.n_grid + R.n_block;
    const T* __restrict__ ow = oct_wt<T>(R);
    const int cb = R.cell_begin[ce], cend = R.cell_begin[ce + 1];
    auto ivl = [](int key, int d) { return (1 << (key & 7)) - 1 + ((key >> (3 + 6 * d)) & 63); };
    const int xmask = (1 << 9) - 1, cmask = (1 << 15) - 1;

    // ---------------- phase 1: moments ----------------
    T accZ[RZ], accY[RY], accX[RX];
#pragma unroll
    for (int r = 0; r < RZ; ++r) accZ[r] = 0;
#pragma unroll
    for (int r = 0; r < RY; ++r) accY[r] = 0;
#pragma unroll
    for (int r = 0; r < RX; ++r) accX[r] = 0;
    T pw[KW], pk[KW];
    int kprev = -1, zbuf = 0;
    for (int c0 = cb; c0 < cend; c0 += MAXC) {
        const int nc = cend - c0 < MAXC ? cend - c0 : MAXC;
        __syncthreads();
        for (int j = t; j < nc; j += NT) {
            const int cell = R.cell_perm[c0 + j];
            s_cell[j] = cell;
            s_key[j] = R.cell_key[cell];
        }
        const int key_after = c0 + nc < cend ? R.cell_key[R.cell_perm[c0 + nc]] : -1;
        __syncthreads();
        auto issue = [&](int jb, int nb) {
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const int idx = t + i * NT;
                if (idx < nb * NP) {
                    const int64_t o = (int64_t)s_cell[jb + idx / NP] * NP + idx % NP;
                    pw[i] = ow[o];
                    pk[i] = kappa[oct0 + o];
                }
            }
        };
        const int nbat = (nc + NB - 1) / NB;
        issue(0, nc < NB ? nc : NB);
        for (int b = 0; b < nbat; ++b) {
            const int jb = b * NB, nb = nc - jb < NB ? nc - jb : NB;
            T* wkb = s_wk + (b & 1) * NB * NP;
#pragma unroll
            for (int i = 0; i < KW; ++i) {
                const int idx = t + i * NT;
                if (idx < nb * NP) wkb[idx] = pw[i] * pk[i];
            }
            __syncthreads();
            if (b + 1 < nbat) issue(jb + NB, nc - jb - NB < NB ? nc - jb - NB : NB);
            for (int jl = 0; jl < nb; ++jl) {
                const int j = jb + jl;
                const int key = s_key[j];
                const int knext = j + 1 < nc ? s_key[j + 1] : key_after;
                const bool end_col = knext < 0 || (key & cmask) != (knext & cmask);
                const bool end_x = knext < 0 || (key & xmask) != (knext & xmask);
                kprev = key;
                {   // direction 3: Mz[g1 g2][k3] += sum_g3 B_k3(z_g3) wk[g1 g2 g3]
                    const T* bz = s_bi + ivl(key, 2) * NK * P1;
                    const T* wk = wkb + jl * NP;
#pragma unroll
                    for (int r = 0; r < RZ; ++r) {
                        const int i = t + r * NT;
                        if (i < NZ) {
                            const int g12 = i / NK, k3 = i % NK;
                            T s = 0;
#pragma unroll
                            for (int g3 = 0; g3 < P1; ++g3) s += bz[k3 * P1 + g3] * wk[g12 * P1 + g3];
                            accZ[r] += s;
                        }
                    }
                }
                if (!end_col) continue;
                T* mz = s_mz + zbuf * NZ;
#pragma unroll
                for (int r = 0; r < RZ; ++r) {
                    const int i = t + r * NT;
                    if (i < NZ) mz[i] = accZ[r];
                    accZ[r] = 0;
                }
                __syncthreads();
                {   // direction 2: My[g1][k2 k3] += sum_g2 B_k2(y_g2) Mz[g1 g2][k3]
                    const T* by = s_bi + ivl(key, 1) * NK * P1;
#pragma unroll
                    for (int r = 0; r < RY; ++r) {
                        const int i = t + r * NT;
                        if (i < NY) {
                            const int g1 = i / NK2, k2 = (i / NK) % NK, k3 = i % NK;
                            T s = 0;
#pragma unroll
                            for (int g2 = 0; g2 < P1; ++g2) s += by[k2 * P1 + g2] * mz[(g1 * P1 + g2) * NK + k3];
                            accY[r] += s;
                        }
                    }
                }
                zbuf ^= 1;
                if (!end_x) continue;
#pragma unroll
                for (int r = 0; r < RY; ++r) {
                    const int i = t + r * NT;
                    if (i < NY) s_my[i] = accY[r];
                    accY[r] = 0;
                }
                __syncthreads();
                {   // direction 1: Mom[k1][k2 k3] += sum_g1 B_k1(x_g1) My[g1][k2 k3]
                    const T* bx = s_bi + ivl(key, 0) * NK * P1;
#pragma unroll
                    for (int r = 0; r < RX; ++r) {
                        const int i = t + r * NT;
                        if (i < NK3) {
                            const int k1 = i / NK2, k23 = i % NK2;
                            T s = 0;
#pragma unroll
                            for (int g1 = 0; g1 < P1; ++g1) s += bx[k1 * P1 + g1] * s_my[g1 * NK2 + k23];
                            accX[r] += s;
                        }
                    }
                }
            }
        }
    }
    (void)kprev;
#pragma unroll
    for (int r = 0; r < RX; ++r) {
        const int i = t + r * NT;
        if (i < NK3) mom[(int64_t)blockIdx.x * NK3 + i] = accX[r];
    }
}


// Moments of one cut element on its fitted rule: Mom[k1 k2 k3] = sum_g w_g kappa_g
// B_k1(tau_g1) B_k2(tau_g2) B_k3(tau_g3) over the NK^3 tensor points, contracted direction by
// direction (3, then 2, then 1).  One workgroup per cut element from ce0 on.  The fitted
// weights have both signs, so these sums cancel; they run in FP64 for both dtypes (FP64
// weights and Bernstein values, kappa read in T) and the moments are rounded to T once.
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_cut_moments_fit(DevRules R, const T* __restrict__ kappa, T* __restrict__ mom, int ce0) {
    using C = MomCfg<P>;
    constexpr int NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    __shared__ double s_a[NK3], s_b[NK3];
    __shared__ double s_v[NK * NK];
    const int64_t ce = (int64_t)ce0 + blockIdx.x;
    const int t = threadIdx.x;
    const int64_t s0 = R.n_grid + R.n_block + ce * NK3;
    for (int i = t; i < NK * NK; i += NT) s_v[i] = R.fit_V64[i];
    for (int i = t; i < NK3; i += NT) s_a[i] = R.oct_w[ce * NK3 + i] * (double)kappa[s0 + i];
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {             // [g1 g2][k3]
        const int g12 = i / NK, k3 = i % NK;
        double v = 0;
#pragma unroll
        for (int g3 = 0; g3 < NK; ++g3) v += s_v[k3 * NK + g3] * s_a[g12 * NK + g3];
        s_b[i] = v;
    }
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {             // [g1][k2 k3]
        const int g1 = i / NK2, k2 = (i / NK) % NK, k3 = i % NK;
        double v = 0;
#pragma unroll
        for (int g2 = 0; g2 < NK; ++g2) v += s_v[k2 * NK + g2] * s_b[(g1 * NK + g2) * NK + k3];
        s_a[i] = v;
    }
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {             // [k1][k2 k3]
        const int k1 = i / NK2, k23 = i % NK2;
        double v = 0;
#pragma unroll
        for (int g1 = 0; g1 < NK; ++g1) v += s_v[k1 * NK + g1] * s_a[g1 * NK2 + k23];
        mom[(int64_t)blockIdx.x * NK3 + i] = (T)v;
    }
}

// moments of cut elements [c0, c0 + n) by the octree or the fitted rule
template <typename T, int P>
static void launch_moments(const wq_rules* H, const T* kappa, T* mom, int64_t c0, int64_t n, hipStream_t s) {
    if (H->R.fit)
        hipLaunchKernelGGL((k_cut_moments_fit<T, P>), dim3((unsigned)n), dim3(256), 0, s, H->R, kappa, mom, (int)c0);
    else
        hipLaunchKernelGGL((k_cut_moments<T, P>), dim3((unsigned)n), dim3(256), 0, s, H->R, kappa, mom, (int)c0);
}


// k_cut_local: one workgroup per (cut element, a3) contracts Mom with the Q tables
// (directions 3 and 2 on the vector ALU, direction 1 on matrix cores) and stores the local
// rows a = (a1, a2, a3) of both matrices, loc[((ce P1 + a3) 2 + v) P1^2 + (a1 P1 + a2)][b],
// through LDS so that every row is one contiguous run.
// SCATTER = false: store the local rows (cut-element path).  SCATTER = true: add them into
// the CSR values with atomics, element by element (the conventional assembly).
template <typename T, int P, int WHICH, bool SCATTER = false>
__global__ void __launch_bounds__(256)
k_cut_local(DevRules R, const int32_t* __restrict__ elems, const T* __restrict__ mom, T* __restrict__ loc,
            const int32_t* __restrict__ act2cut, T* __restrict__ vm, T* __restrict__ vk, int ce0) {
    using C = MomCfg<P>;
    using MF = MfmaOp<T>;
    using v4 = typename MF::v4;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int M = 2 * P + 1, M3 = M * M * M, NS1 = C::NS1, NS2 = C::NS2;
    constexpr int MT = C::MT, NTC = C::NTC, NTW = C::NTW, KS1 = C::KS1, KS2 = C::KS2, QN = 2 * P2 * NK;
    constexpr int NBLK = P2 * NP;                   // one matrix's block: rows (a1 a2) x columns b
    constexpr int NSU = (2 * NS1 + 2 * NS2) > NBLK ? (2 * NS1 + 2 * NS2) : NBLK;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_q[3][QN];
    __shared__ T s_mom[NK3];
    __shared__ T s_u[NSU];
    T* s_s1 = s_u;                                  // [2][NS1]
    T* s_s2 = s_u + 2 * NS1;                        // [2][NS2]
    T* s_blk = s_u;                                 // [(a1 a2)][b] after the contractions

    __shared__ int64_t s_rb[SCATTER ? P2 : 1];
    __shared__ int32_t s_cr[SCATTER ? P2 : 1];
    const int ce = blockIdx.x / P1, a3 = blockIdx.x % P1;    // ce counts from element ce0 of elems
    const int64_t eid = elems[ce0 + ce];
    int e[3];
    unlex3i(eid, R.nel, e);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    for (int i = t; i < 3 * QN; i += NT) {
        const int d = i / QN;
        s_q[d][i % QN] = bern_q<T>(R, d)[(int64_t)e[d] * QN + i % QN];
    }
    for (int i = t; i < NK3; i += NT) s_mom[i] = mom[(int64_t)ce * NK3 + i];
    if (SCATTER && t < P2) {                        // rows a = e + (a1, a2, a3)
        const int a1 = t / P1, a2 = t % P1;
        const int64_t alex = ((int64_t)(e[0] + a1) * R.nfun[1] + (e[1] + a2)) * R.nfun[2] + (e[2] + a3);
        const int ra = R.lex2act[alex];
        s_rb[t] = R.row_ptr[ra];
        s_cr[t] = act2cut[ra];
    }
    __syncthreads();
    const T* qx = s_q[0];
    const T* qy = s_q[1];
    const T* qz = s_q[2];
    // S1_v[k1 k2][b3] = sum_k3 QZ_v[a3 b3][k3] Mom[k1 k2 k3]
    for (int i = t; i < NS1; i += NT) {
        const int k12 = i / P1, b3 = i % P1;
        const T* z0 = qz + (a3 * P1 + b3) * NK;
        const T* z1 = qz + P2 * NK + (a3 * P1 + b3) * NK;
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int k3 = 0; k3 < NK; ++k3) {
            const T mo = s_mom[k12 * NK + k3];
            s0 += z0[k3] * mo;
            if (STIFF) s1 += z1[k3] * mo;
        }
        s_s1[i] = s0;
        if (STIFF) s_s1[NS1 + i] = s1;
    }
    __syncthreads();
    // S2_0[k1][(a2 b2) b3] = sum_k2 QY0 S1_0,  S2_s = sum_k2 (QY1 S1_0 + QY0 S1_1)
    for (int i = t; i < NS2; i += NT) {
        const int k1 = i / NP, c = i % NP, ab2 = c / P1, b3 = c % P1;
        const T* y0 = qy + ab2 * NK;
        const T* y1 = qy + P2 * NK + ab2 * NK;
        T m0 = 0, ms = 0;
#pragma unroll
        for (int k2 = 0; k2 < NK; ++k2) {
            const T u0 = s_s1[(k1 * NK + k2) * P1 + b3];
            m0 += y0[k2] * u0;
            if (STIFF) ms = fmat(y0[k2], s_s1[NS1 + (k1 * NK + k2) * P1 + b3], fmat(y1[k2], u0, ms));
        }
        s_s2[i] = m0;
        if (STIFF) s_s2[NS2 + i] = ms;
    }
    __syncthreads();
    // direction 1 on matrix cores: rows m = (a1 b1), columns n = (a2 b2 b3), K = k1
    v4 accM[NTW][MT], accK[NTW][MT];
#pragma unroll
    for (int ti = 0; ti < NTW; ++ti)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) { accM[ti][mt] = v4{0, 0, 0, 0}; accK[ti][mt] = v4{0, 0, 0, 0}; }
#pragma unroll
    for (int ti = 0; ti < NTW; ++ti) {
        const int nt = wv + ti * C::NWAVE;
        if (nt >= NTC) break;
        const int n = nt * 16 + lm;
        const bool nv = n < NP;
        if (MASS) {
#pragma unroll
            for (int k = 0; k < KS1; ++k) {
                const int k1 = 4 * k + lk;
                const T bv = (nv && k1 < NK) ? s_s2[k1 * NP + n] : (T)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int m = mt * 16 + lm;
                    const T av = (m < P2 && k1 < NK) ? qx[m * NK + k1] : (T)0;
                    accM[ti][mt] = MF::mma(av, bv, accM[ti][mt]);
                }
            }
        }
        if (STIFF) {                                // K = [QX1 | QX0] [S2_0 ; S2_s]
#pragma unroll
            for (int k = 0; k < KS2; ++k) {
                const int kk = 4 * k + lk;
                T bv = 0;
                if (nv && kk < NK) bv = s_s2[kk * NP + n];
                else if (nv && kk < 2 * NK) bv = s_s2[NS2 + (kk - NK) * NP + n];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int m = mt * 16 + lm;
                    T av = 0;
                    if (m < P2 && kk < NK) av = qx[P2 * NK + m * NK + kk];
                    else if (m < P2 && kk < 2 * NK) av = qx[m * NK + (kk - NK)];
                    accK[ti][mt] = MF::mma(av, bv, accK[ti][mt]);
                }
            }
        }
    }
    // stage each matrix's block as [(a1 a2)][(b1 b2 b3)] and store (or add) it
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        if ((v == 0 && !MASS) || (v == 1 && !STIFF)) continue;
        T* out = SCATTER ? (v == 0 ? vm : vk) : loc + ((int64_t)(ce * P1 + a3) * 2 + v) * NBLK;
        __syncthreads();                            // s_u is free (contractions / previous scatter done)
#pragma unroll
        for (int ti = 0; ti < NTW; ++ti) {
            const int nt = wv + ti * C::NWAVE;
            if (nt >= NTC) break;
            const int n = nt * 16 + lm;
            if (n >= NP) continue;
            const int a2 = n / P2, b2 = (n / P1) % P1, b3 = n % P1;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = mt * 16 + MF::row(lane, r);
                    if (m >= P2) continue;
                    const int a1 = m / P1, b1 = m % P1;
                    s_blk[(a1 * P1 + a2) * NP + (b1 * P1 + b2) * P1 + b3] = v == 0 ? accM[ti][mt][r] : accK[ti][mt][r];
                }
        }
        __syncthreads();
        if (!SCATTER) {
            for (int i = t; i < NBLK; i += NT) out[i] = s_blk[i];
        } else {
            for (int i = t; i < NBLK; i += NT) {
                const int r = i / NP, b = i % NP, a1 = r / P1, a2 = r % P1;
                const int b1 = b / P2, b2 = (b / P1) % P1, b3 = b % P1;
                const int jj1 = b1 - a1 + P, jj2 = b2 - a2 + P, jj3 = b3 - a3 + P;
                int o;
                if (s_cr[r] >= 0) {
                    o = R.pos_map[(int64_t)s_cr[r] * M3 + (jj1 * M + jj2) * M + jj3];
                } else {                            // interior row: its full window is stored
                    const int I1 = e[0] + a1, I2 = e[1] + a2, I3 = e[2] + a3;
                    const int lo1 = I1 - P < 0 ? P - I1 : 0;
                    const int lo2 = I2 - P < 0 ? P - I2 : 0, hi2 = I2 + P > R.nfun[1] - 1 ? R.nfun[1] - 1 - I2 + P : 2 * P;
                    const int lo3 = I3 - P < 0 ? P - I3 : 0, hi3 = I3 + P > R.nfun[2] - 1 ? R.nfun[2] - 1 - I3 + P : 2 * P;
                    o = ((jj1 - lo1) * (hi2 - lo2 + 1) + (jj2 - lo2)) * (hi3 - lo3 + 1) + (jj3 - lo3);
                }
                if (o >= 0) atomicAdd(&out[s_rb[r] + o], s_blk[i]);
            }
        }
    }
}

// k_cut_local_a2 (degrees 5 and 6): as k_cut_local with one workgroup per (cut element,
// a3, a2), so that the LDS block of one workgroup is P1 local rows (a1) instead of P1^2:
// direction 3 is contracted for every a2 (recomputed per workgroup), direction 2 for this
// a2 only, direction 1 on matrix cores with rows (a1 b1) and columns (b2 b3).
// SCATTER = true: add the rows into the CSR values with atomics (the conventional assembly).
template <typename T, int P, int WHICH, bool SCATTER = false>
__global__ void __launch_bounds__(256)
k_cut_local_a2(DevRules R, const int32_t* __restrict__ elems, const T* __restrict__ mom, T* __restrict__ loc, int ce0,
               const int32_t* __restrict__ act2cut = nullptr, T* __restrict__ vm = nullptr, T* __restrict__ vk = nullptr) {
    using C = MomCfg<P>;
    using MF = MfmaOp<T>;
    using v4 = typename MF::v4;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    constexpr int NS1 = C::NS1, NS2 = NK * P2, QN = 2 * P2 * NK;
    constexpr int MT = (P2 + 15) / 16, NTC = (P2 + 15) / 16, NTW = (NTC + C::NWAVE - 1) / C::NWAVE;
    constexpr int KS1 = C::KS1, KS2 = C::KS2;
    constexpr int NROW = P1 * NP;                   // this workgroup's rows a1 x columns b
    constexpr int NBLK = P2 * NP;                   // one (element, a3, matrix) block of loc
    constexpr int NSU = (2 * NS1 + 2 * NS2) > NROW ? (2 * NS1 + 2 * NS2) : NROW;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_q[3][QN];
    __shared__ T s_mom[NK3];
    __shared__ T s_u[NSU];
    T* s_s1 = s_u;                                  // [2][NS1]
    T* s_s2 = s_u + 2 * NS1;                        // [2][NS2]
    T* s_blk = s_u;                                 // [a1][b] after the contractions

    const int ce = blockIdx.x / P2, a3 = (blockIdx.x / P1) % P1, a2 = blockIdx.x % P1;   // from element ce0
    const int64_t eid = elems[ce0 + ce];
    int e[3];
    unlex3i(eid, R.nel, e);
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    for (int i = t; i < 3 * QN; i += NT) {
        const int d = i / QN;
        s_q[d][i % QN] = bern_q<T>(R, d)[(int64_t)e[d] * QN + i % QN];
    }
    for (int i = t; i < NK3; i += NT) s_mom[i] = mom[(int64_t)ce * NK3 + i];
    __syncthreads();
    const T* qx = s_q[0];
    const T* qy = s_q[1];
    const T* qz = s_q[2];
    // S1_v[k1 k2][b3] = sum_k3 QZ_v[a3 b3][k3] Mom[k1 k2 k3]
    for (int i = t; i < NS1; i += NT) {
        const int k12 = i / P1, b3 = i % P1;
        const T* z0 = qz + (a3 * P1 + b3) * NK;
        const T* z1 = qz + P2 * NK + (a3 * P1 + b3) * NK;
        T s0 = 0, s1 = 0;
#pragma unroll
        for (int k3 = 0; k3 < NK; ++k3) {
            const T mo = s_mom[k12 * NK + k3];
            s0 += z0[k3] * mo;
            if (STIFF) s1 += z1[k3] * mo;
        }
        s_s1[i] = s0;
        if (STIFF) s_s1[NS1 + i] = s1;
    }
    __syncthreads();
    // S2_0[k1][b2 b3] = sum_k2 QY0[a2 b2][k2] S1_0,  S2_s = sum_k2 (QY1 S1_0 + QY0 S1_1)
    for (int i = t; i < NS2; i += NT) {
        const int k1 = i / P2, c = i % P2, b2 = c / P1, b3 = c % P1;
        const T* y0 = qy + (a2 * P1 + b2) * NK;
        const T* y1 = qy + P2 * NK + (a2 * P1 + b2) * NK;
        T m0 = 0, ms = 0;
#pragma unroll
        for (int k2 = 0; k2 < NK; ++k2) {
            const T u0 = s_s1[(k1 * NK + k2) * P1 + b3];
            m0 += y0[k2] * u0;
            if (STIFF) ms = fmat(y0[k2], s_s1[NS1 + (k1 * NK + k2) * P1 + b3], fmat(y1[k2], u0, ms));
        }
        s_s2[i] = m0;
        if (STIFF) s_s2[NS2 + i] = ms;
    }
    __syncthreads();
    // direction 1 on matrix cores: rows m = (a1 b1), columns n = (b2 b3), K = k1
    v4 accM[NTW][MT], accK[NTW][MT];
#pragma unroll
    for (int ti = 0; ti < NTW; ++ti)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) { accM[ti][mt] = v4{0, 0, 0, 0}; accK[ti][mt] = v4{0, 0, 0, 0}; }
#pragma unroll
    for (int ti = 0; ti < NTW; ++ti) {
        const int nt = wv + ti * C::NWAVE;
        if (nt >= NTC) break;
        const int n = nt * 16 + lm;
        const bool nv = n < P2;
        if (MASS) {
#pragma unroll
            for (int k = 0; k < KS1; ++k) {
                const int k1 = 4 * k + lk;
                const T bv = (nv && k1 < NK) ? s_s2[k1 * P2 + n] : (T)0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int m = mt * 16 + lm;
                    const T av = (m < P2 && k1 < NK) ? qx[m * NK + k1] : (T)0;
                    accM[ti][mt] = MF::mma(av, bv, accM[ti][mt]);
                }
            }
        }
        if (STIFF) {                                // K = [QX1 | QX0] [S2_0 ; S2_s]
#pragma unroll
            for (int k = 0; k < KS2; ++k) {
                const int kk = 4 * k + lk;
                T bv = 0;
                if (nv && kk < NK) bv = s_s2[kk * P2 + n];
                else if (nv && kk < 2 * NK) bv = s_s2[NS2 + (kk - NK) * P2 + n];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int m = mt * 16 + lm;
                    T av = 0;
                    if (m < P2 && kk < NK) av = qx[P2 * NK + m * NK + kk];
                    else if (m < P2 && kk < 2 * NK) av = qx[m * NK + (kk - NK)];
                    accK[ti][mt] = MF::mma(av, bv, accK[ti][mt]);
                }
            }
        }
    }
    // stage each matrix's rows as [a1][(b1 b2 b3)] and store them at rows (a1 P1 + a2)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
        if ((v == 0 && !MASS) || (v == 1 && !STIFF)) continue;
        T* out = SCATTER ? nullptr : loc + ((int64_t)(ce * P1 + a3) * 2 + v) * NBLK;
        __syncthreads();                            // s_u is free (contractions / previous matrix done)
#pragma unroll
        for (int ti = 0; ti < NTW; ++ti) {
            const int nt = wv + ti * C::NWAVE;
            if (nt >= NTC) break;
            const int n = nt * 16 + lm;
            if (n >= P2) continue;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = mt * 16 + MF::row(lane, r);
                    if (m >= P2) continue;
                    const int a1 = m / P1, b1 = m % P1;
                    s_blk[a1 * NP + b1 * P2 + n] = v == 0 ? accM[ti][mt][r] : accK[ti][mt][r];
                }
        }
        __syncthreads();
        if (!SCATTER) {
            for (int i = t; i < NROW; i += NT) {
                const int a1 = i / NP, b = i % NP;
                out[(int64_t)(a1 * P1 + a2) * NP + b] = s_blk[i];
            }
        } else {
            T* dst = v == 0 ? vm : vk;
            for (int i = t; i < NROW; i += NT) {
                const int a1 = i / NP, b = i % NP;
                const int b1 = b / P2, b2 = (b / P1) % P1, b3 = b % P1;
                const int I1 = e[0] + a1, I2 = e[1] + a2, I3 = e[2] + a3;
                const int ra = R.lex2act[((int64_t)I1 * R.nfun[1] + I2) * R.nfun[2] + I3];
                const int cr = act2cut[ra];
                const int jj1 = b1 - a1 + P, jj2 = b2 - a2 + P, jj3 = b3 - a3 + P;
                int o;
                if (cr >= 0) {
                    o = R.pos_map[(int64_t)cr * (2 * P + 1) * (2 * P + 1) * (2 * P + 1) +
                                  (jj1 * (2 * P + 1) + jj2) * (2 * P + 1) + jj3];
                } else {                            // interior row: its full window is stored
                    const int lo1 = I1 - P < 0 ? P - I1 : 0;
                    const int lo2 = I2 - P < 0 ? P - I2 : 0, hi2 = I2 + P > R.nfun[1] - 1 ? R.nfun[1] - 1 - I2 + P : 2 * P;
                    const int lo3 = I3 - P < 0 ? P - I3 : 0, hi3 = I3 + P > R.nfun[2] - 1 ? R.nfun[2] - 1 - I3 + P : 2 * P;
                    o = ((jj1 - lo1) * (hi2 - lo2 + 1) + (jj2 - lo2)) * (hi3 - lo3 + 1) + (jj3 - lo3);
                }
                if (o >= 0) atomicAdd(&dst[R.row_ptr[ra] + o], s_blk[i]);
            }
        }
    }
}

// k_cut_gather: one workgroup per cut row adds the local rows of its cut elements (a fixed
// order, no atomics): NSLOT elements in flight, one lane per column b of the element,
// per-slot LDS accumulators over the row's (2p+1)^3 window, then one pass over the row.
// Only the cut elements ce0 <= ce < ce1 are added (loc holds their local rows from ce0 on);
// the workgroups cover the cut rows from cr0 on.
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(RemCfg<P>::NT)
k_cut_gather(DevRules R, const T* __restrict__ loc, T* __restrict__ vm, T* __restrict__ vk, int ce0, int ce1,
             int64_t cr0) {
    using C = RemCfg<P>;
    constexpr int P1 = C::P1, NP = C::NP, P2 = C::P2, M = 2 * P + 1, M3 = M * M * M, NT = C::NT, SLOT = C::SLOT;
    constexpr int NSLOT = C::NSLOT, NBLK = P2 * NP;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_accm[NSLOT][MASS ? M3 : 1], s_acck[NSLOT][STIFF ? M3 : 1];
    __shared__ int2 s_list[NP];
    __shared__ int s_n;
    const int64_t cr = cr0 + blockIdx.x;
    const int t = threadIdx.x;
    const int l0 = R.rcut_ptr[cr], nall = R.rcut_ptr[cr + 1] - l0;
    if (nall == 0) return;
    // this row's cut elements inside [ce0, ce1), in list order (one wave compacts them)
    if (t < 64) {
        int base = 0;
        for (int k0 = 0; k0 < nall; k0 += 64) {
            const int k = k0 + t;
            int2 en = make_int2(0, 0);
            bool in = false;
            if (k < nall) {
                en = R.rcut_list[l0 + k];
                in = en.x >= ce0 && en.x < ce1;
            }
            const uint64_t mask = __ballot(in);
            if (in) {
                en.x -= ce0;
                s_list[base + __popcll(mask & ((1ull << t) - 1))] = en;
            }
            base += __popcll(mask);
        }
        if (t == 0) s_n = base;
    }
    for (int k = t; k < NSLOT * M3; k += NT) {
        if (MASS) s_accm[k / M3][k % M3] = 0;
        if (STIFF) s_acck[k / M3][k % M3] = 0;
    }
    __syncthreads();
    const int n = s_n;
    if (n == 0) return;
    const int sl = t / SLOT, u = t % SLOT;
    const bool act_u = u < NP;
    const int b1 = u / P2, b2 = (u / P1) % P1, b3 = u % P1;
    auto src = [&](int r, int v) -> const T* {
        const int2 en = s_list[r];
        const int k0 = en.y & 15, k1 = (en.y >> 4) & 15, k2 = (en.y >> 8) & 15;
        return loc + ((int64_t)(en.x * P1 + k2) * 2 + v) * NBLK + (k0 * P1 + k1) * NP;
    };
    T cm = 0, ck = 0;                               // values of the element in flight
    if (act_u && sl < n) {
        if (MASS) cm = src(sl, 0)[u];
        if (STIFF) ck = src(sl, 1)[u];
    }
    for (int r0 = 0; r0 < n; r0 += NSLOT) {
        const int r = r0 + sl;
        const bool active = r < n;
        T nm = 0, nk = 0;                           // next pass, loaded before this one is added
        if (act_u && r + NSLOT < n) {
            if (MASS) nm = src(r + NSLOT, 0)[u];
            if (STIFF) nk = src(r + NSLOT, 1)[u];
        }
        if (active && act_u) {
            const int pk = s_list[r].y;
            const int a1 = pk & 15, a2 = (pk >> 4) & 15, a3 = (pk >> 8) & 15;
            const int jj = ((b1 - a1 + P) * M + (b2 - a2 + P)) * M + (b3 - a3 + P);
            if (MASS) s_accm[sl][jj] += cm;
            if (STIFF) s_acck[sl][jj] += ck;
        }
        cm = nm; ck = nk;
        __syncthreads();
    }
    const int ra = R.cut_rows[cr];
    const int32_t* pos = R.pos_map + cr * (int64_t)M3;
    const int64_t rb = R.row_ptr[ra];
    for (int k = t; k < M3; k += NT) {
        const int o = pos[k];
        if (o < 0) continue;
        T am = 0, ak = 0;
#pragma unroll
        for (int i = 0; i < NSLOT; ++i) {
            if (MASS) am += s_accm[i][k];
            if (STIFF) ak += s_acck[i][k];
        }
        if (MASS) vm[rb + o] += am;
        if (STIFF) vk[rb + o] += ak;
    }
}

// ----------------------------------------------------------------------------------------
// Conventional element-by-element Gauss assembly (the reference scheme of Section 3.1:
// Gauss rules on every interior element, the octree on cut elements), for comparison.
// Every element's local matrices are formed from its moments (Gauss points for interior
// elements, octree points for cut elements) and added into the values with atomics.
// ----------------------------------------------------------------------------------------
// Moments of one interior element from its (p+1)^3 Gauss points (kappa_gauss in the
// element's lexicographic Gauss order); the Bernstein values at the Gauss points of the
// whole element are the depth-0 row of the interval table.
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_gauss_moments(DevRules R, const T* __restrict__ kg, const double* __restrict__ gw, T* __restrict__ mom) {
    using C = MomCfg<P>;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK2 = C::NK2, NK3 = C::NK3, NT = C::NT;
    __shared__ T s_wk[NP], s_mz[P2 * NK], s_my[P1 * NK2], s_b[NK * P1];
    const int64_t el = blockIdx.x;
    const int t = threadIdx.x;
    const double vol = R.h[0] * R.h[1] * R.h[2] / 8.0;
    for (int i = t; i < NP; i += NT) {
        const int g1 = i / P2, g2 = (i / P1) % P1, g3 = i % P1;
        s_wk[i] = (T)(gw[g1] * gw[g2] * gw[g3] * vol) * kg[el * NP + i];
    }
    if (t < NK * P1) s_b[t] = bern_i<T>(R)[t];
    __syncthreads();
    for (int i = t; i < P2 * NK; i += NT) {          // [g1 g2][k3]
        const int g12 = i / NK, k3 = i % NK;
        T s = 0;
#pragma unroll
        for (int g3 = 0; g3 < P1; ++g3) s += s_b[k3 * P1 + g3] * s_wk[g12 * P1 + g3];
        s_mz[i] = s;
    }
    __syncthreads();
    for (int i = t; i < P1 * NK2; i += NT) {         // [g1][k2 k3]
        const int g1 = i / NK2, k2 = (i / NK) % NK, k3 = i % NK;
        T s = 0;
#pragma unroll
        for (int g2 = 0; g2 < P1; ++g2) s += s_b[k2 * P1 + g2] * s_mz[(g1 * P1 + g2) * NK + k3];
        s_my[i] = s;
    }
    __syncthreads();
    for (int i = t; i < NK3; i += NT) {              // [k1][k2 k3]
        const int k1 = i / NK2, k23 = i % NK2;
        T s = 0;
#pragma unroll
        for (int g1 = 0; g1 < P1; ++g1) s += s_b[k1 * P1 + g1] * s_my[g1 * NK2 + k23];
        mom[el * NK3 + i] = s;
    }
}

template <typename T>
__global__ void k_zero(T* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (T)0;
}

template <typename T, int P, int WHICH>
static int launch_gauss_p(const wq_rules* H, const T* kg, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    using C = MomCfg<P>;
    const int64_t ni = H->n_int_elems, nc = R.n_cut_elems, ne = ni + nc;
    const unsigned zb = (unsigned)((H->nnz + 255) / 256);
    if ((WHICH & 1)) hipLaunchKernelGGL(k_zero<T>, dim3(zb), dim3(256), 0, s, vm, H->nnz);
    if ((WHICH & 2)) hipLaunchKernelGGL(k_zero<T>, dim3(zb), dim3(256), 0, s, vk, H->nnz);
    if (ne == 0) return WQ_OK;
    T* mom = nullptr;
    hipError_t err = H->scratch_alloc((void**)&mom, sizeof(T) * (size_t)ne * C::NK3, s);
    if (err != hipSuccess) return wq_set_error(WQ_ENOMEM, "gauss_assemble: scratch allocation failed: %s", hipGetErrorString(err));
    auto scatter = [&](const int32_t* elems, int64_t n, const T* m) {
        if constexpr (P <= 4)
            hipLaunchKernelGGL((k_cut_local<T, P, WHICH, true>), dim3((unsigned)(n * (P + 1))), dim3(256), 0, s, R, elems,
                               m, (T*)nullptr, H->act2cut, vm, vk, 0);
        else
            hipLaunchKernelGGL((k_cut_local_a2<T, P, WHICH, true>), dim3((unsigned)(n * (P + 1) * (P + 1))), dim3(256), 0,
                               s, R, elems, m, (T*)nullptr, 0, H->act2cut, vm, vk);
    };
    if (ni > 0) {
        hipLaunchKernelGGL((k_gauss_moments<T, P>), dim3((unsigned)ni), dim3(256), 0, s, R, kg, (const double*)H->gw, mom);
        scatter(H->int_elems, ni, (const T*)mom);
    }
    if (nc > 0) {
        T* mc = mom + (size_t)ni * C::NK3;
        launch_moments<T, P>(H, kappa, mc, 0, nc, s);
        scatter(R.cut_elems, nc, (const T*)mc);
    }
    err = hipFreeAsync(mom, s);
    if (err != hipSuccess) return wq_set_error(WQ_EHIP, "gauss_assemble: scratch release failed: %s", hipGetErrorString(err));
    return WQ_OK;
}

template <typename T>
int launch_gauss(const wq_rules* H, uint32_t which, const T* kg, const T* kappa, T* vm, T* vk, hipStream_t s) {
    if (H->R.levels > 3) return wq_set_error(WQ_EUNSUPPORTED, "gauss_assemble: octree depth above 3 is not supported");
    switch (H->R.p) {
#define WQ_GAUSS_CASE(PP)                                                                                          \
    case PP:                                                                                                       \
        if (which == 1) return launch_gauss_p<T, PP, 1>(H, kg, kappa, vm, vk, s);                                  \
        if (which == 2) return launch_gauss_p<T, PP, 2>(H, kg, kappa, vm, vk, s);                                  \
        return launch_gauss_p<T, PP, 3>(H, kg, kappa, vm, vk, s);
        WQ_GAUSS_CASE(1)
        WQ_GAUSS_CASE(2)
        WQ_GAUSS_CASE(3)
        WQ_GAUSS_CASE(4)
        WQ_GAUSS_CASE(5)
        WQ_GAUSS_CASE(6)
#undef WQ_GAUSS_CASE
    }
    return WQ_OK;
}

#ifndef WQ_ONLY_F32
// coordinates of the Gauss points of every interior element (lexicographic elements, then
// lexicographic Gauss points), the order kappa_gauss is read in
__global__ void k_gauss_coords(DevRules R, const int32_t* elems, int64_t n, const double* gxi, double* xyz) {
    const int p1 = R.p + 1, np = p1 * p1 * p1;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n * np) return;
    const int64_t el = id / np;
    const int q = (int)(id % np), g[3] = {q / (p1 * p1), (q / p1) % p1, q % p1};
    int e[3];
    unlex3i(elems[el], R.nel, e);
    for (int d = 0; d < 3; ++d) xyz[id * 3 + d] = R.lo[d] + (e[d] + (1.0 + gxi[g[d]]) / 2.0) * R.h[d];
}

int launch_gauss_coords(const wq_rules* H, double* xyz, hipStream_t s) {
    const int64_t n = H->n_int_elems * (int64_t)(H->R.p + 1) * (H->R.p + 1) * (H->R.p + 1);
    if (n > 0)
        hipLaunchKernelGGL(k_gauss_coords, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, H->R, H->int_elems,
                           H->n_int_elems, (const double*)H->gxi, xyz);
    return WQ_OK;
}
template int launch_gauss<double>(const wq_rules*, uint32_t, const double*, const double*, double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template int launch_gauss<float>(const wq_rules*, uint32_t, const float*, const float*, float*, float*, hipStream_t);
#endif

// ----------------------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------------------
// Cut elements in moment form, in batches of at most nb elements whose moments and local
// rows fit in buf; the gather of a batch covers the cut rows whose support can reach it
// (cut elements and cut rows are in lexicographic order, so a batch's first direction-1
// element index bounds them).
template <typename T, int P, int WHICH>
static void launch_moment_form(const wq_rules* H, const T* kappa, T* vm, T* vk, T* buf, int64_t nb, hipStream_t s) {
    const DevRules& R = H->R;
    using C = MomCfg<P>;
    const int64_t nce = R.n_cut_elems;
    for (int64_t c0 = 0; c0 < nce; c0 += nb) {
        const int64_t c1 = c0 + nb < nce ? c0 + nb : nce, n = c1 - c0;
        T* mom = buf;
        T* loc = buf + n * C::NK3;
        launch_moments<T, P>(H, kappa, mom, c0, n, s);
        if constexpr (P <= 4)
            hipLaunchKernelGGL((k_cut_local<T, P, WHICH>), dim3((unsigned)(n * (P + 1))), dim3(256), 0, s, R, R.cut_elems,
                               (const T*)mom, loc, nullptr, nullptr, nullptr, (int)c0);
        else
            hipLaunchKernelGGL((k_cut_local_a2<T, P, WHICH>), dim3((unsigned)(n * (P + 1) * (P + 1))), dim3(256), 0, s, R,
                               R.cut_elems, (const T*)mom, loc, (int)c0);
        int64_t r0 = 0, r1 = R.n_cut;
        if (c0 > 0 || c1 < nce) {
            const int e1lo = H->h_cut_elem_e1[c0], e1hi = H->h_cut_elem_e1[c1 - 1];
            const auto& ri = H->h_cut_row_i1;
            r0 = std::lower_bound(ri.begin(), ri.end(), e1lo) - ri.begin();
            r1 = std::upper_bound(ri.begin(), ri.end(), e1hi + P) - ri.begin();
        }
        if (r1 > r0)
            hipLaunchKernelGGL((k_cut_gather<T, P, WHICH>), dim3((unsigned)(r1 - r0)), dim3(RemCfg<P>::NT), 0, s, R,
                               (const T*)loc, vm, vk, (int)c0, (int)c1, r0);
    }
}

// scratch values per cut element of the moment form: moments and local rows
template <int P>
static constexpr int64_t moment_form_per_elem() {
    using C = MomCfg<P>;
    return (int64_t)C::NK3 + (int64_t)C::P1 * 2 * C::P2 * C::NP;
}

// buf == nullptr: scratch from the handle's stream-ordered pool; else the caller's buffer of
// cap bytes, filled batch by batch (allocation-free variant)
template <typename T, int P, int WHICH>
static void launch_remainder(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if constexpr (sizeof(T) == 4 && P >= 5)
        hipLaunchKernelGGL((k_cut_remainder_v8<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemCfg<P>::NT), 0, s, R, kappa,
                           vm, vk);
    else
        hipLaunchKernelGGL((k_cut_remainder<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemCfg<P>::NT), 0, s, R, kappa, vm,
                           vk);
}

template <typename T, int P, int WHICH>
static int launch_cut_p(const wq_rules* H, uint32_t parts, const T* kappa, T* vm, T* vk, hipStream_t s, void* buf,
                        size_t cap) {
    const DevRules& R = H->R;
    // both parts in one call, default scratch, moment form: the remainder overlaps the octree
    // moments and local rows (launched below); otherwise the parts run one after the other
    const bool overlap = (parts & WQ_CUT_REMAINDER) && (parts & WQ_CUT_OCTREE) && R.n_cut > 0 && R.n_cut_elems > 0 &&
                         R.levels <= 3 && !buf && H->side;
    if ((parts & WQ_CUT_REMAINDER) && R.n_cut > 0 && !overlap) launch_remainder<T, P, WHICH>(H, kappa, vm, vk, s);
    if ((parts & WQ_CUT_OCTREE) && R.n_cut_elems > 0) {
        if (R.levels <= 3) {
            const int64_t per = moment_form_per_elem<P>();
            if (buf) {
                const int64_t nb = (int64_t)(cap / sizeof(T)) / per;
                if (nb < 1)
                    return wq_set_error(WQ_EINVAL, "cut_assemble_noalloc: one cut element needs %lld bytes of scratch, "
                                                   "more than the fixed %zu", (long long)(per * sizeof(T)), cap);
                launch_moment_form<T, P, WHICH>(H, kappa, vm, vk, (T*)buf, nb, s);
                return WQ_OK;
            }
            T* mom = nullptr;
            hipError_t err = H->scratch_alloc((void**)&mom, sizeof(T) * (size_t)(per * R.n_cut_elems), s);
            if (err != hipSuccess)
                return wq_set_error(WQ_ENOMEM, "cut_assemble: scratch allocation failed: %s", hipGetErrorString(err));
            if (overlap) {
                // moments and local rows on the side stream while the remainder runs on s (they
                // touch no values); the gather waits for both
                using C = MomCfg<P>;
                const int64_t n = R.n_cut_elems;
                T* loc = mom + n * C::NK3;
                std::lock_guard<std::mutex> lock(*H->side_mu);
                if (hipEventRecord(H->ev_fork, s) == hipSuccess && hipStreamWaitEvent(H->side, H->ev_fork, 0) == hipSuccess) {
                    launch_moments<T, P>(H, kappa, mom, 0, n, H->side);
                    if constexpr (P <= 4)
                        hipLaunchKernelGGL((k_cut_local<T, P, WHICH>), dim3((unsigned)(n * (P + 1))), dim3(256), 0, H->side, R,
                                           R.cut_elems, (const T*)mom, loc, nullptr, nullptr, nullptr, 0);
                    else
                        hipLaunchKernelGGL((k_cut_local_a2<T, P, WHICH>), dim3((unsigned)(n * (P + 1) * (P + 1))), dim3(256), 0,
                                           H->side, R, R.cut_elems, (const T*)mom, loc, 0);
                    launch_remainder<T, P, WHICH>(H, kappa, vm, vk, s);
                    if (hipEventRecord(H->ev_join, H->side) != hipSuccess || hipStreamWaitEvent(s, H->ev_join, 0) != hipSuccess) {
                        (void)hipGetLastError();
                        (void)hipStreamSynchronize(H->side);
                    }
                    hipLaunchKernelGGL((k_cut_gather<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemCfg<P>::NT), 0, s, R,
                                       (const T*)loc, vm, vk, 0, (int)n, (int64_t)0);
                } else {
                    (void)hipGetLastError();
                    launch_remainder<T, P, WHICH>(H, kappa, vm, vk, s);
                    launch_moment_form<T, P, WHICH>(H, kappa, vm, vk, mom, R.n_cut_elems, s);
                }
            } else {
                launch_moment_form<T, P, WHICH>(H, kappa, vm, vk, mom, R.n_cut_elems, s);
            }
            err = hipFreeAsync(mom, s);
            if (err != hipSuccess)
                return wq_set_error(WQ_EHIP, "cut_assemble: scratch release failed: %s", hipGetErrorString(err));
            return WQ_OK;
        }
        using C = OctCfg<P>;
        hipLaunchKernelGGL((k_cut_octree<T, P, WHICH>), dim3((unsigned)(R.n_cut_elems * C::P1 * C::NAG)), dim3(C::NT), 0, s, R,
                           H->act2cut, kappa, vm, vk);
    }
    return WQ_OK;
}

template <typename T, int P>
static int launch_cut_w(const wq_rules* H, uint32_t which, uint32_t parts, const T* kappa, T* vm, T* vk, hipStream_t s,
                        void* buf, size_t cap) {
    if (which == 1) return launch_cut_p<T, P, 1>(H, parts, kappa, vm, vk, s, buf, cap);
    if (which == 2) return launch_cut_p<T, P, 2>(H, parts, kappa, vm, vk, s, buf, cap);
    return launch_cut_p<T, P, 3>(H, parts, kappa, vm, vk, s, buf, cap);
}

// ----------------------------------------------------------------------------------------
// Cut elements of the coefficient-tensor stiffness (wq_assemble_tensor): the moments of each
// of the six components C_c of the tensor (w C_c in place of w kappa, octree or fitted points),
// then per element the local stiffness rows
//   K[a][b] = sum_{d,e} sum_k Q1^f(x=0)[a1 b1][k1] Q2^f(x=1)[a2 b2][k2] Q3^f(x=2)[a3 b3][k3] Mom_{C_de}[k],
// with the family f of direction x in term (d, e): phi_a phi_b (x not d, e), phi_a' phi_b'
// (x = d = e), phi_a' phi_b (x = d only), phi_a phi_b' (x = e only), all as degree-2p
// Bernstein coefficients; the row gather of the scalar path then adds them into the cut rows.
// ----------------------------------------------------------------------------------------
template <typename T> __device__ inline const T* bern_qx(const DevRules& R, int d);
template <> __device__ inline const double* bern_qx<double>(const DevRules& R, int d) { return R.bern_qx64[d]; }
template <> __device__ inline const float* bern_qx<float>(const DevRules& R, int d) { return R.bern_qx32[d]; }

// one workgroup per (cut element, a3); mom: [component][cut element][k]; loc: the gather's
// layout, stiffness half (v = 1)
template <typename T, int P>
__global__ void __launch_bounds__(256)
k_tensor_local(DevRules R, const T* __restrict__ mom, int64_t n, T* __restrict__ loc) {
    using C = MomCfg<P>;
    constexpr int P1 = C::P1, P2 = C::P2, NP = C::NP, NK = C::NK, NK3 = C::NK3, NT = 256;
    constexpr int NBLK = P2 * NP, NI = P2 * P2 * P1, KR = (NI + NT - 1) / NT;
    __shared__ T s_m[NK3];
    __shared__ T s_q[3][4][P2][NK];                  // [direction][family][a b][k]
    __shared__ T s_t1[NK * NK * P1];                 // [k1 k2][b3]
    __shared__ T s_t2[NK * P1 * P2];                 // [k1][a2 b2 b3]
    const int64_t ce = blockIdx.x / P1;
    const int a3 = blockIdx.x % P1;
    const int t = threadIdx.x;
    const int64_t eid = R.cut_elems[ce];
    const int el[3] = {(int)(eid / ((int64_t)R.nel[1] * R.nel[2])), (int)((eid / R.nel[2]) % R.nel[1]), (int)(eid % R.nel[2])};
    for (int i = t; i < 3 * 4 * P2 * NK; i += NT) {
        const int d = i / (4 * P2 * NK), f = (i / (P2 * NK)) % 4, ab = (i / NK) % P2, k = i % NK;
        const int a = ab / P1, b = ab % P1;
        T v;
        if (f < 2) v = bern_q<T>(R, d)[(((int64_t)el[d] * 2 + f) * P2 + ab) * NK + k];
        else if (f == 2) v = bern_qx<T>(R, d)[(((int64_t)el[d] * P1 + a) * P1 + b) * NK + k];
        else v = bern_qx<T>(R, d)[(((int64_t)el[d] * P1 + b) * P1 + a) * NK + k];
        s_q[d][f][ab][k] = v;
    }
    T acc[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) acc[r] = 0;
    for (int c = 0; c < 6; ++c) {
        __syncthreads();
        for (int k = t; k < NK3; k += NT) s_m[k] = mom[((int64_t)c * n + ce) * NK3 + k];
        const int nterm = c < 3 ? 1 : 2;
        for (int tm = 0; tm < nterm; ++tm) {
            int d, e;
            if (c < 3) { d = c; e = c; }
            else {
                const int lo = c == 5 ? 1 : 0, hi = c == 3 ? 1 : 2;
                d = tm == 0 ? lo : hi; e = tm == 0 ? hi : lo;
            }
            const int f1 = d == 0 ? (e == 0 ? 1 : 2) : (e == 0 ? 3 : 0);
            const int f2 = d == 1 ? (e == 1 ? 1 : 2) : (e == 1 ? 3 : 0);
            const int f3 = d == 2 ? (e == 2 ? 1 : 2) : (e == 2 ? 3 : 0);
            __syncthreads();
            for (int i = t; i < NK * NK * P1; i += NT) {     // [k1 k2][b3] = sum_k3 Q3[a3 b3][k3] Mom[k1 k2 k3]
                const int k12 = i / P1, b3 = i % P1;
                const T* q = s_q[2][f3][a3 * P1 + b3];
                T v = 0;
#pragma unroll
                for (int k3 = 0; k3 < NK; ++k3) v = fmat(q[k3], s_m[k12 * NK + k3], v);
                s_t1[i] = v;
            }
            __syncthreads();
            for (int i = t; i < NK * P1 * P2; i += NT) {     // [k1][a2 b2 b3] = sum_k2 Q2[a2 b2][k2] T1[k1 k2][b3]
                const int k1 = i / (P1 * P2), ab2 = (i / P1) % P2, b3 = i % P1;
                const T* q = s_q[1][f2][ab2];
                T v = 0;
#pragma unroll
                for (int k2 = 0; k2 < NK; ++k2) v = fmat(q[k2], s_t1[(k1 * NK + k2) * P1 + b3], v);
                s_t2[i] = v;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < KR; ++r) {                   // [a1 b1][a2 b2 b3] += sum_k1 Q1[a1 b1][k1] T2[k1][..]
                const int i = t + r * NT;
                if (i < NI) {
                    const int ab1 = i / (P2 * P1), rest = i % (P2 * P1);
                    const T* q = s_q[0][f1][ab1];
                    T v = acc[r];
#pragma unroll
                    for (int k1 = 0; k1 < NK; ++k1) v = fmat(q[k1], s_t2[k1 * P2 * P1 + rest], v);
                    acc[r] = v;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int i = t + r * NT;
        if (i < NI) {
            const int a1 = i / (P1 * P2 * P1), b1 = (i / (P2 * P1)) % P1, a2 = (i / P2) % P1, b2 = (i / P1) % P1, b3 = i % P1;
            loc[((ce * P1 + a3) * 2 + 1) * NBLK + (a1 * P1 + a2) * NP + (b1 * P1 + b2) * P1 + b3] = acc[r];
        }
    }
}

template <typename T, int P>
static int launch_tensor_cut_p(const wq_rules* H, const T* Cc, int64_t ldc, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    const int64_t n = R.n_cut_elems;
    using C = MomCfg<P>;
    const int64_t nloc = n * C::P1 * 2 * C::P2 * C::NP;
    T* mom = nullptr;
    hipError_t err = H->scratch_alloc((void**)&mom, sizeof(T) * (size_t)(6 * n * C::NK3 + nloc), s);
    if (err != hipSuccess)
        return wq_set_error(WQ_ENOMEM, "wq_assemble_tensor: scratch allocation failed: %s", hipGetErrorString(err));
    T* loc = mom + 6 * n * C::NK3;
    for (int c = 0; c < 6; ++c) launch_moments<T, P>(H, Cc + c * ldc, mom + c * n * C::NK3, 0, n, s);
    hipLaunchKernelGGL((k_tensor_local<T, P>), dim3((unsigned)(n * C::P1)), dim3(256), 0, s, R, (const T*)mom, n, loc);
    hipLaunchKernelGGL((k_cut_gather<T, P, 2>), dim3((unsigned)R.n_cut), dim3(RemCfg<P>::NT), 0, s, R, (const T*)loc,
                       (T*)nullptr, vk, 0, (int)n, (int64_t)0);
    err = hipFreeAsync(mom, s);
    if (err != hipSuccess) return wq_set_error(WQ_EHIP, "wq_assemble_tensor: scratch release failed: %s", hipGetErrorString(err));
    return WQ_OK;
}

// returns WQ_EUNSUPPORTED when the moment form does not apply (octree depth > 3): the caller
// then integrates the cut elements row by row
template <typename T>
int launch_tensor_cut(const wq_rules* H, const T* Cc, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if (R.levels > 3 || R.p > 4) return WQ_EUNSUPPORTED;
    if (R.n_cut_elems == 0 || R.n_cut == 0) return WQ_OK;
    const int64_t ldc = R.n_kappa;
    switch (R.p) {
        case 1: return launch_tensor_cut_p<T, 1>(H, Cc, ldc, vk, s);
        case 2: return launch_tensor_cut_p<T, 2>(H, Cc, ldc, vk, s);
        case 3: return launch_tensor_cut_p<T, 3>(H, Cc, ldc, vk, s);
        default: return launch_tensor_cut_p<T, 4>(H, Cc, ldc, vk, s);
    }
}

#ifndef WQ_ONLY_F32
template int launch_tensor_cut<double>(const wq_rules*, const double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template int launch_tensor_cut<float>(const wq_rules*, const float*, float*, hipStream_t);
#endif

// Fused assembly (wq_assemble): cut_prep enqueues the octree part's element work (moments and
// local rows into stream-ordered scratch allocated on s_alloc) on s_oct and the remainder on
// s_rem; after the caller has joined both streams into s, cut_finish adds the local rows into
// the cut rows (the gather) on s and releases the scratch.  Moment form only (octree depth <= 3).
template <typename T, int P, int WHICH>
static int launch_cut_prep_p(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s_rem, hipStream_t s_oct,
                             T* mom) {
    const DevRules& R = H->R;
    using C = MomCfg<P>;
    const int64_t n = R.n_cut_elems;
    T* loc = mom + n * C::NK3;
    launch_moments<T, P>(H, kappa, mom, 0, n, s_oct);
    if constexpr (P <= 4)
        hipLaunchKernelGGL((k_cut_local<T, P, WHICH>), dim3((unsigned)(n * (P + 1))), dim3(256), 0, s_oct, R, R.cut_elems,
                           (const T*)mom, loc, nullptr, nullptr, nullptr, 0);
    else
        hipLaunchKernelGGL((k_cut_local_a2<T, P, WHICH>), dim3((unsigned)(n * (P + 1) * (P + 1))), dim3(256), 0, s_oct, R,
                           R.cut_elems, (const T*)mom, loc, 0);
    launch_remainder<T, P, WHICH>(H, kappa, vm, vk, s_rem);
    return WQ_OK;
}

template <typename T, int P, int WHICH>
static void launch_cut_finish_p(const wq_rules* H, const T* mom, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    using C = MomCfg<P>;
    const int64_t n = R.n_cut_elems;
    hipLaunchKernelGGL((k_cut_gather<T, P, WHICH>), dim3((unsigned)R.n_cut), dim3(RemCfg<P>::NT), 0, s, R,
                       mom + n * C::NK3, vm, vk, 0, (int)n, (int64_t)0);
}

template <typename T, int P>
static int launch_cut_prep_w(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_rem,
                             hipStream_t s_oct, T* mom) {
    if (which == 1) return launch_cut_prep_p<T, P, 1>(H, kappa, vm, vk, s_rem, s_oct, mom);
    if (which == 2) return launch_cut_prep_p<T, P, 2>(H, kappa, vm, vk, s_rem, s_oct, mom);
    return launch_cut_prep_p<T, P, 3>(H, kappa, vm, vk, s_rem, s_oct, mom);
}

template <typename T, int P>
static void launch_cut_finish_w(const wq_rules* H, uint32_t which, const T* mom, T* vm, T* vk, hipStream_t s) {
    if (which == 1) launch_cut_finish_p<T, P, 1>(H, mom, vm, vk, s);
    else if (which == 2) launch_cut_finish_p<T, P, 2>(H, mom, vm, vk, s);
    else launch_cut_finish_p<T, P, 3>(H, mom, vm, vk, s);
}

// bytes of scratch of the fused assembly, 0 when it does not apply (no cut elements or rows,
// octree deeper than three levels)
template <typename T>
size_t cut_fused_scratch_bytes(const wq_rules* H) {
    const DevRules& R = H->R;
    if (R.levels > 3 || R.n_cut_elems == 0 || R.n_cut == 0) return 0;
    int64_t per = 0;
    switch (R.p) {
        case 1: per = moment_form_per_elem<1>(); break;
        case 2: per = moment_form_per_elem<2>(); break;
        case 3: per = moment_form_per_elem<3>(); break;
        case 4: per = moment_form_per_elem<4>(); break;
        case 5: per = moment_form_per_elem<5>(); break;
        default: per = moment_form_per_elem<6>(); break;
    }
    return sizeof(T) * (size_t)(per * R.n_cut_elems);
}

template <typename T>
int launch_cut_prep(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_rem, hipStream_t s_oct,
                    void* scratch) {
    T* mom = (T*)scratch;
    switch (H->R.p) {
        case 1: return launch_cut_prep_w<T, 1>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
        case 2: return launch_cut_prep_w<T, 2>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
        case 3: return launch_cut_prep_w<T, 3>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
        case 4: return launch_cut_prep_w<T, 4>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
        case 5: return launch_cut_prep_w<T, 5>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
        default: return launch_cut_prep_w<T, 6>(H, which, kappa, vm, vk, s_rem, s_oct, mom);
    }
}

template <typename T>
void launch_cut_finish(const wq_rules* H, uint32_t which, const void* scratch, T* vm, T* vk, hipStream_t s) {
    const T* mom = (const T*)scratch;
    switch (H->R.p) {
        case 1: launch_cut_finish_w<T, 1>(H, which, mom, vm, vk, s); break;
        case 2: launch_cut_finish_w<T, 2>(H, which, mom, vm, vk, s); break;
        case 3: launch_cut_finish_w<T, 3>(H, which, mom, vm, vk, s); break;
        case 4: launch_cut_finish_w<T, 4>(H, which, mom, vm, vk, s); break;
        case 5: launch_cut_finish_w<T, 5>(H, which, mom, vm, vk, s); break;
        default: launch_cut_finish_w<T, 6>(H, which, mom, vm, vk, s); break;
    }
}

#ifndef WQ_ONLY_F32
template size_t cut_fused_scratch_bytes<double>(const wq_rules*);
template int launch_cut_prep<double>(const wq_rules*, uint32_t, const double*, double*, double*, hipStream_t, hipStream_t,
                                     void*);
template void launch_cut_finish<double>(const wq_rules*, uint32_t, const void*, double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template size_t cut_fused_scratch_bytes<float>(const wq_rules*);
template int launch_cut_prep<float>(const wq_rules*, uint32_t, const float*, float*, float*, hipStream_t, hipStream_t,
                                    void*);
template void launch_cut_finish<float>(const wq_rules*, uint32_t, const void*, float*, float*, hipStream_t);
#endif

template <typename T>
int launch_cut(const wq_rules* H, uint32_t which, uint32_t parts, const T* kappa, T* vm, T* vk, hipStream_t s, void* buf,
               size_t cap) {
    switch (H->R.p) {
        case 1: return launch_cut_w<T, 1>(H, which, parts, kappa, vm, vk, s, buf, cap);
        case 2: return launch_cut_w<T, 2>(H, which, parts, kappa, vm, vk, s, buf, cap);
        case 3: return launch_cut_w<T, 3>(H, which, parts, kappa, vm, vk, s, buf, cap);
        case 4: return launch_cut_w<T, 4>(H, which, parts, kappa, vm, vk, s, buf, cap);
        case 5: return launch_cut_w<T, 5>(H, which, parts, kappa, vm, vk, s, buf, cap);
        case 6: return launch_cut_w<T, 6>(H, which, parts, kappa, vm, vk, s, buf, cap);
    }
    return WQ_OK;
}

#ifndef WQ_ONLY_F32
template int launch_cut<double>(const wq_rules*, uint32_t, uint32_t, const double*, double*, double*, hipStream_t, void*,
                                size_t);
#endif
#ifndef WQ_ONLY_F64
template int launch_cut<float>(const wq_rules*, uint32_t, uint32_t, const float*, float*, float*, hipStream_t, void*,
                               size_t);
#endif

#ifndef WQ_ONLY_F32
// octree moments of every cut element in the basis of table (interval layout of bern_i: the
// rule build fits the cut rule from Legendre moments)
int launch_octree_moments_f64(const wq_rules* H, const double* table, const double* kappa, double* mom, hipStream_t s) {
    const int64_t n = H->R.n_cut_elems;
    if (n == 0) return WQ_OK;
    DevRules R = H->R;
    R.bern_i64 = table;
    switch (R.p) {
        case 1: hipLaunchKernelGGL((k_cut_moments<double, 1>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
        case 2: hipLaunchKernelGGL((k_cut_moments<double, 2>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
        case 3: hipLaunchKernelGGL((k_cut_moments<double, 3>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
        case 4: hipLaunchKernelGGL((k_cut_moments<double, 4>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
        case 5: hipLaunchKernelGGL((k_cut_moments<double, 5>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
        default: hipLaunchKernelGGL((k_cut_moments<double, 6>), dim3((unsigned)n), dim3(256), 0, s, R, kappa, mom, 0); break;
    }
    return WQ_OK;
}
#endif
