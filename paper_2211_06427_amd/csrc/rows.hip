// Row assembly by sum factorization over weighted-quadrature rules (Section 1: sum
// factorization, weighted quadrature and the row loop; Section 2.2 for DWQ rows).
//
// Interior rows: one workgroup per line block of consecutive interior rows along direction 1
// (fixed i2, i3).  Stages 1-2 contract directions 3 and 2 once for the whole block into an
// LDS slab T2[q1][j2 j3]; stage 3 contracts direction 1 per row, one lane per (j2, j3)
// column, and stores each row's (2p+1)^3 values with coalesced writes.  FP32 at p <= 4 uses
// k_rows_block (blocks of at most 8 rows, every contraction over the compile-time band of its
// window class, four workgroups per CU); FP64, p > 4 and the BF16x3 experiment use
// k_rows_interior.
//
// Cut rows: rows with a DWQ box use the one-sided rule in the split direction and the
// standard rules in the others (kappa gathered through the slot map): k_rows_box at p <= 4
// (the whole box in LDS), k_rows_cut otherwise; rows without a box are zeroed by k_rows_zero
// (their support is handled by cut_assemble).  The cut rows run on a second stream beside
// the interior rows.
#include <type_traits>

#include "rows.h"

template <typename T> __device__ inline const T* wt_table(const DevRules& R, int d);
template <> __device__ inline const double* wt_table<double>(const DevRules& R, int d) { return R.Wt64[d]; }
template <> __device__ inline const float* wt_table<float>(const DevRules& R, int d) { return R.Wt32[d]; }
template <typename T> __device__ inline const T* dwq_table(const DevRules& R);
template <> __device__ inline const double* dwq_table<double>(const DevRules& R) { return R.dwq_Wt64; }
template <> __device__ inline const float* dwq_table<float>(const DevRules& R) { return R.dwq_Wt32; }

__device__ inline int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ----------------------------------------------------------------------------------------
// interior rows
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH, int RB>
struct RowCfg {
    static constexpr int M = 2 * P + 1, NW = 4 * P, MM = M * M;
    static constexpr int GT = ((MM + 63) / 64) * 64;       // threads per stage-3 row group
    static constexpr int NG = GT >= 256 ? 1 : 256 / GT;    // row groups
    static constexpr int NT = NG * GT;                     // threads per block: whole groups only
    static constexpr int NQ1 = 2 * RB + 4 * P;             // q1 slab bound
    static constexpr int NWP = NW + 1;                     // padded stride of staged rows
    static constexpr bool STIFF = (WHICH & 2) != 0;
    static constexpr bool MASS = (WHICH & 1) != 0;
};

// ---- BF16x3 experiment: stage 3 on matrix cores with split operands ----
// x = hi + lo with hi = bf16(x) and lo = bf16(x - hi) (round to nearest even, finite x);
// a product is taken as hi*hi + hi*lo + lo*hi (the lo*lo term is dropped), accumulated in
// FP32 by v_mfma_f32_16x16x16_bf16.  Operand layout of that instruction: A (16 x 16, M x K)
// element (m, k) in lane m + 16 (k / 4), slot k % 4; B (K x N) element (k, n) in lane
// n + 16 (k / 4), slot k % 4; D as for the FP32 16x16x4 form (column lane % 16, row
// 4 (lane / 16) + r).
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rn(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ inline float bf16_up(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }
__device__ inline void split4(const float v[4], bf16x4_t& hi, bf16x4_t& lo) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const short h = bf16_rn(v[i]);
        hi[i] = h;
        lo[i] = bf16_rn(v[i] - bf16_up(h));
    }
}
__device__ inline f32x4_t mma3(const bf16x4_t& ah, const bf16x4_t& al, const bf16x4_t& bh, const bf16x4_t& bl,
                               f32x4_t c) {
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
}

// One wave per row of the block (rows wave, wave + nwaves, ...): out[jj1][c] = sum_q
// W1[jj1][q] T2[off + q][c] with rows m = jj1 (M <= 16), K = q in chunks of 16, columns
// c = (j2 j3) in tiles of 16.  Stiffness: W1^11 T2_00 + W1^00 T2_s.
template <int P, int WHICH>
__device__ void stage3_bf16x3(const DevRules& R, const float* s_t00, const float* s_ts, int i1s, int I2, int I3,
                              int nrows, int qbase, float* __restrict__ vm, float* __restrict__ vk) {
    constexpr int M = 2 * P + 1, NW = 4 * P, MM = M * M, KC = (NW + 15) / 16, NTILE = (MM + 15) / 16;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    static_assert(M <= 16 && NW % 4 == 0, "one M tile, float4 weight loads");
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    const int lm = lane & 15, lk = lane >> 4;
    const int p = P;
    const int lo2 = I2 - p < 0 ? p - I2 : 0, hi2 = I2 + p > R.nfun[1] - 1 ? R.nfun[1] - 1 - I2 + p : 2 * p;
    const int lo3 = I3 - p < 0 ? p - I3 : 0, hi3 = I3 + p > R.nfun[2] - 1 ? R.nfun[2] - 1 - I3 + p : 2 * p;
    const int m2 = hi2 - lo2 + 1, m3 = hi3 - lo3 + 1;
    const int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
    const float* W1 = R.Wt32[0];
    for (int r = wv; r < nrows; r += nwv) {
        const int i1 = i1s + r;
        const int ra = __builtin_amdgcn_readfirstlane(R.lex2act[(int64_t)i1 * nl + (int64_t)I2 * R.nfun[2] + I3]);
        const int64_t base = R.row_ptr[ra];
        const int off = R.xs[0][i1] - qbase;
        const int nw1 = R.nwin[0][i1];
        const int lo1 = i1 - p < 0 ? p - i1 : 0, hi1 = i1 + p > R.nfun[0] - 1 ? R.nfun[0] - 1 - i1 + p : 2 * p;
        // A operands: W1^00 and W1^11 rows m = jj1, K slots q = 16 kc + 4 lk + i
        bf16x4_t a0h[KC], a0l[KC], a1h[KC], a1l[KC];
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const int q = 16 * kc + 4 * lk;
            float w0[4] = {0, 0, 0, 0}, w1[4] = {0, 0, 0, 0};
            if (lm < M && q < NW) {
                const float4 v0 = *(const float4*)(W1 + ((int64_t)i1 * 2 * M + lm) * NW + q);
                const float4 v1 = *(const float4*)(W1 + ((int64_t)i1 * 2 * M + M + lm) * NW + q);
                w0[0] = v0.x; w0[1] = v0.y; w0[2] = v0.z; w0[3] = v0.w;
                w1[0] = v1.x; w1[1] = v1.y; w1[2] = v1.z; w1[3] = v1.w;
            }
            split4(w0, a0h[kc], a0l[kc]);
            split4(w1, a1h[kc], a1l[kc]);
        }
        for (int tile = 0; tile < NTILE; ++tile) {
            const int c = tile * 16 + lm;
            f32x4_t accM = {0, 0, 0, 0}, accK = {0, 0, 0, 0};
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float t0[4], ts[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int q = 16 * kc + 4 * lk + i;
                    const bool ok = c < MM && q < nw1;
                    t0[i] = ok ? s_t00[(off + q) * MM + c] : 0.0f;
                    ts[i] = (ok && STIFF) ? s_ts[(off + q) * MM + c] : 0.0f;
                }
                bf16x4_t b0h, b0l;
                split4(t0, b0h, b0l);
                if (MASS) accM = mma3(a0h[kc], a0l[kc], b0h, b0l, accM);
                if (STIFF) {
                    bf16x4_t bsh, bsl;
                    split4(ts, bsh, bsl);
                    accK = mma3(a1h[kc], a1l[kc], b0h, b0l, accK);
                    accK = mma3(a0h[kc], a0l[kc], bsh, bsl, accK);
                }
            }
            const int jj2 = c / M, jj3 = c % M;
            if (c < MM && jj2 >= lo2 && jj2 <= hi2 && jj3 >= lo3 && jj3 <= hi3) {
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    const int jj1 = 4 * lk + rr;
                    if (jj1 < lo1 || jj1 > hi1) continue;
                    const int64_t o = base + ((int64_t)(jj1 - lo1) * m2 + (jj2 - lo2)) * m3 + (jj3 - lo3);
                    if (MASS) vm[o] = accM[rr];
                    if (STIFF) vk[o] = accK[rr];
                }
            }
        }
    }
}

// One workgroup per line block (or half of one: SPLIT = 2 processes RB rows of a block of
// up to 2 RB).  Stages 1-2 contract directions 3 and 2 once for the block into the LDS slab
// T2[q1][j2 j3] (mass) and Ts (stiffness, directions 2 and 3); stage 3 runs row by row with
// the row's direction-1 weights staged in LDS one row ahead.
template <typename T, int P, int WHICH, int RB, int SPLIT, bool BF3 = false>
__global__ void __launch_bounds__((RowCfg<T, P, WHICH, RB>::NT))
k_rows_interior(DevRules R, const T* __restrict__ kappa, T* __restrict__ vm, T* __restrict__ vk) {
    using C = RowCfg<T, P, WHICH, RB>;
    constexpr int M = C::M, NW = C::NW, MM = C::MM, NWP = C::NWP, NT = C::NT, NG = C::NG;
    constexpr int W1N = 2 * M * NW;             // direction-1 weights of one row
    __shared__ T s_t00[C::NQ1 * MM];
    __shared__ T s_ts[C::STIFF ? C::NQ1 * MM : 1];
    __shared__ T s_w2[2 * M * NWP], s_w3[2 * M * NWP];
    __shared__ T s_w1[NG][2][W1N];              // per row group, double buffered

    const int4 blk = R.lblocks[blockIdx.x / SPLIT];
    const int half = blockIdx.x % SPLIT;
    const int i1s = blk.x + half * RB, i2 = blk.y, i3 = blk.z;
    const int nrows = blk.w - half * RB < RB ? blk.w - half * RB : RB;
    if (nrows <= 0) return;
    const int t = threadIdx.x;
    const T* W1 = wt_table<T>(R, 0);
    const T* W2 = wt_table<T>(R, 1) + (int64_t)i2 * 2 * M * NW;
    const T* W3 = wt_table<T>(R, 2) + (int64_t)i3 * 2 * M * NW;
    // Stage-3 weights of every row this lane's group will handle, loaded into registers now:
    // their loads are older than every row store, so moving them to LDS row by row never
    // waits for stores to complete.
    constexpr int RPG = (RB + NG - 1) / NG;     // rows per group
    constexpr int WPL = (W1N + C::GT - 1) / C::GT;   // weights per lane per row
    const int grp = __builtin_amdgcn_readfirstlane(t / C::GT);
    const int c = t % C::GT;
    static_assert(RPG >= 2, "the queue holds the current and the next row");
    T wq[RPG][WPL];
    // and the rows' active indices and windows (their CSR offsets are fetched after stages
    // 1-2, once these have arrived)
    int rq_act[RPG], rq_xs[RPG], rq_nw[RPG];
    int64_t rq_base[RPG];
    if constexpr (!BF3) {
        const int64_t nl0 = (int64_t)R.nfun[1] * R.nfun[2];
#pragma unroll
        for (int j = 0; j < RPG; ++j) {
            const int r = grp + j * NG;
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                const int k = c + i * C::GT;
                wq[j][i] = (r < nrows && k < W1N) ? W1[(int64_t)(i1s + r) * W1N + k] : (T)0;
            }
            const int i1 = i1s + (r < nrows ? r : 0);
            rq_act[j] = __builtin_amdgcn_readfirstlane(R.lex2act[(int64_t)i1 * nl0 + (int64_t)i2 * R.nfun[2] + i3]);
            rq_xs[j] = __builtin_amdgcn_readfirstlane(R.xs[0][i1]);
            rq_nw[j] = __builtin_amdgcn_readfirstlane(R.nwin[0][i1]);
        }
    }
    for (int k = t; k < 2 * M * NW; k += NT) {
        s_w2[(k / NW) * NWP + k % NW] = W2[k];
        s_w3[(k / NW) * NWP + k % NW] = W3[k];
    }
    const int qbase = R.xs[0][i1s];
    const int i1e = i1s + nrows - 1;
    const int nq1 = R.xs[0][i1e] + R.nwin[0][i1e] - qbase;
    const int xs2 = R.xs[1][i2], nw2 = R.nwin[1][i2];
    const int xs3 = R.xs[2][i3], nw3 = R.nwin[2][i3];
    const int nx2 = R.nx[1], nx3 = R.nx[2];

    // ---- stages 1-2: one item per (q1, j3).  For each q2 the direction-3 sums T1_v(q1,q2,j3)
    // are formed from one row of kappa (all its loads issued together) and folded at once
    // into the direction-2 sums over all j2, so only the 2M stage-2 accumulators stay live.
    __syncthreads();
    for (int it = t; it < nq1 * M; it += NT) {
        const int q1 = it / M, j3 = it % M;
        const T* kap = kappa + ((int64_t)(qbase + q1) * nx2 + xs2) * nx3 + xs3;
        T m0[M], ms[M];
#pragma unroll
        for (int j2 = 0; j2 < M; ++j2) { m0[j2] = 0; ms[j2] = 0; }
        for (int q2 = 0; q2 < nw2; ++q2) {
            const T* kq = kap + (int64_t)q2 * nx3;
            T kv[NW];
#pragma unroll
            for (int q3 = 0; q3 < NW; ++q3) kv[q3] = q3 < nw3 ? kq[q3] : (T)0;
            T a0 = 0, a1 = 0;
#pragma unroll
            for (int q3 = 0; q3 < NW; ++q3) {
                a0 += s_w3[j3 * NWP + q3] * kv[q3];
                if (C::STIFF) a1 += s_w3[(M + j3) * NWP + q3] * kv[q3];
            }
#pragma unroll
            for (int j2 = 0; j2 < M; ++j2) {
                const T w0 = s_w2[j2 * NWP + q2];
                m0[j2] += w0 * a0;
                if (C::STIFF) ms[j2] = fmat(w0, a1, fmat(s_w2[(M + j2) * NWP + q2], a0, ms[j2]));
            }
        }
#pragma unroll
        for (int j2 = 0; j2 < M; ++j2) {
            s_t00[q1 * MM + j2 * M + j3] = m0[j2];
            if (C::STIFF) s_ts[q1 * MM + j2 * M + j3] = ms[j2];
        }
    }

    if constexpr (BF3) {
        __syncthreads();                        // slab ready
        stage3_bf16x3<P, WHICH>(R, s_t00, s_ts, i1s, i2, i3, nrows, qbase, vm, vk);
        return;
    }

    // ---- stage 3: row groups of GT lanes, one lane per (j2, j3) ----
    const int jj2 = c / M, jj3 = c % M;
    const int p = P;
    const int I2 = i2, I3 = i3;
    const int lo2 = I2 - p < 0 ? p - I2 : 0, hi2 = I2 + p > R.nfun[1] - 1 ? R.nfun[1] - 1 - I2 + p : 2 * p;
    const int lo3 = I3 - p < 0 ? p - I3 : 0, hi3 = I3 + p > R.nfun[2] - 1 ? R.nfun[2] - 1 - I3 + p : 2 * p;
    const int m2 = hi2 - lo2 + 1, m3 = hi3 - lo3 + 1;
    const bool live = c < MM && jj2 >= lo2 && jj2 <= hi2 && jj3 >= lo3 && jj3 <= hi3;
    const int64_t nl = (int64_t)R.nfun[1] * R.nfun[2];
    // first row of each group: its weights; every row's CSR offset
#pragma unroll
    for (int i = 0; i < WPL; ++i) {
        const int k = c + i * C::GT;
        if (grp < nrows && k < W1N) s_w1[grp][0][k] = wq[0][i];
    }
#pragma unroll
    for (int j = 0; j < RPG; ++j) rq_base[j] = R.row_ptr[rq_act[j]];
    __syncthreads();                            // slab and first weights ready
    int wb = 0;
    for (int r0 = 0; r0 < nrows; r0 += NG) {
        const int r = r0 + grp;
        const bool active = r < nrows;
        const bool has_next = r + NG < nrows;
        if (active) {
            const int i1 = __builtin_amdgcn_readfirstlane(i1s + r);
            const int64_t base = rq_base[0];
            const int off = rq_xs[0] - qbase;
            const int nw1 = rq_nw[0];
            const int lo1 = i1 - p < 0 ? p - i1 : 0, hi1 = i1 + p > R.nfun[0] - 1 ? R.nfun[0] - 1 - i1 + p : 2 * p;
            T t00[NW], ts[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                t00[q] = 0; ts[q] = 0;
                if (live && q < nw1) {
                    t00[q] = s_t00[(off + q) * MM + c];
                    if (C::STIFF) ts[q] = s_ts[(off + q) * MM + c];
                }
            }
            const T* w10 = s_w1[grp][wb];
            const T* w11 = w10 + M * NW;
            // A row whose window has two points in each of its p+1 elements (no boundary
            // element) has W1[jj1][q] != 0 only for q in [2 max(0, jj1-p), 2 (min(p, jj1)+1)):
            // that range is a compile-time constant.  Other rows loop over the padded window.
            const bool regular = nw1 == 2 * P + 2 && lo1 == 0 && hi1 == 2 * P;
            if (regular) {
#pragma unroll
                for (int jj1 = 0; jj1 < M; ++jj1) {
                    const int qa = 2 * (jj1 - P > 0 ? jj1 - P : 0);
                    const int qb = 2 * ((jj1 < P ? jj1 : P) + 1);
                    T am = 0, ak = 0;
#pragma unroll
                    for (int q = 0; q < 2 * P + 2; ++q) {
                        if (q >= qa && q < qb) {
                            const T a = w10[jj1 * NW + q];
                            if (C::MASS) am += a * t00[q];
                            if (C::STIFF) ak = fmat(a, ts[q], fmat(w11[jj1 * NW + q], t00[q], ak));
                        }
                    }
                    if (live) {
                        const int64_t o = base + ((int64_t)jj1 * m2 + (jj2 - lo2)) * m3 + (jj3 - lo3);
                        if (C::MASS) vm[o] = am;
                        if (C::STIFF) vk[o] = ak;
                    }
                }
            } else {
#pragma unroll 1
                for (int jj1 = lo1; jj1 <= hi1; ++jj1) {
                    T am = 0, ak = 0;
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        const T a = w10[jj1 * NW + q];
                        if (C::MASS) am += a * t00[q];
                        if (C::STIFF) ak = fmat(a, ts[q], fmat(w11[jj1 * NW + q], t00[q], ak));
                    }
                    if (live) {
                        const int64_t o = base + ((int64_t)(jj1 - lo1) * m2 + (jj2 - lo2)) * m3 + (jj3 - lo3);
                        if (C::MASS) vm[o] = am;
                        if (C::STIFF) vk[o] = ak;
                    }
                }
            }
        }
        if (has_next) {
#pragma unroll
            for (int i = 0; i < WPL; ++i) {
                const int k = c + i * C::GT;
                if (k < W1N) s_w1[grp][wb ^ 1][k] = wq[1][i];
            }
        }
        // advance the register queues (static indices: the rows stay in registers)
#pragma unroll
        for (int j = 0; j + 1 < RPG; ++j) {
#pragma unroll
            for (int i = 0; i < WPL; ++i) wq[j][i] = wq[j + 1][i];
            rq_base[j] = rq_base[j + 1];
            rq_xs[j] = rq_xs[j + 1];
            rq_nw[j] = rq_nw[j + 1];
        }
        wb ^= 1;
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------
// interior rows, FP32, p <= 4: one workgroup per block of up to RB rows along direction 1
// ----------------------------------------------------------------------------------------
// A window of function i along a direction is regular when supp B_i holds p+1 elements that
// each keep two points and every trial function of the row window exists (i in
// [p+1, nel-2]): point q then lies in window element q/2 and W[jj][q] can be nonzero only for
// jj in [q/2, q/2+p], so every contraction over such a window runs over a compile-time band.
// Other windows (near the boundary) run over their points with the zero-padded tables.
// Every direction must have at least p+2 elements (windows of at most 3p+1 points).
template <int P, int RB>
struct BlkCfg {
    static constexpr int M = 2 * P + 1, MM = M * M, NT = 256;
    static constexpr int NWT = 4 * P;                  // row stride of the weight tables
    static constexpr int NWB = 3 * P + 1;              // largest window
    static constexpr int NQB = 2 * RB + 4 * P - 2;     // direction-1 points of a block
    // the slab plane stride is padded so that threads with consecutive (plane, j) indices hit
    // consecutive banks (a plane starts M banks after the previous one, 32 banks); the
    // stage-1 planes are not, to keep the workgroup's LDS within a quarter of the CU's
    static constexpr int pad_to(int n) { return n + (((M - n) % 32) + 32) % 32; }
    static constexpr int P1S = 2 * NWB * M;            // stage-1 plane stride
    static constexpr int PSL = pad_to(2 * MM);         // slab plane stride
    static constexpr int BUFN = NQB * (P1S > PSL ? P1S : PSL);
    static constexpr int W1S = 2 * M * NWT + 4;        // row stride of the staged direction-1 weights
    static constexpr int IPL1 = (NQB * NWB + NT - 1) / NT;   // stage-1 items per thread
};

// Window classes of the 1D rule of function i along a direction with at least p+2 elements:
//   0        regular, i in [p+1, nel-2]: elements i-p..i, two points each (2p+2 points);
//   1+k      low end, i = k in [0, p]: elements 0..k, element 0 with all p+1 points;
//   p+1+m    high end, i = nel+p-m, m in [1, p+1]: the last m elements, the last one with all
//            p+1 points.
// For each class the window element of every point and the trial range are known at compile
// time, hence the band of trial functions jj that are nonzero at a point (B_j vanishes off
// its p+1 elements).
template <int P, int CLS>
struct Win {
    static constexpr bool LOW = CLS >= 1 && CLS <= P + 1, HIGH = CLS >= P + 2;
    static constexpr int K = LOW ? CLS - 1 : 0, MEL = HIGH ? CLS - P - 1 : 0;
    static constexpr int NW = LOW ? P + 1 + 2 * K : (HIGH ? 2 * (MEL - 1) + P + 1 : 2 * P + 2);
    static constexpr int JLO = LOW ? P - K : 0, JHI = HIGH ? MEL - 1 + P : 2 * P;
    static constexpr int el(int q) {
        return LOW ? (q < P + 1 ? 0 : 1 + (q - P - 1) / 2) : (HIGH ? (q < 2 * (MEL - 1) ? q / 2 : MEL - 1) : q / 2);
    }
    static constexpr int jlo(int q) { return (LOW ? el(q) + P - K : el(q)) > JLO ? (LOW ? el(q) + P - K : el(q)) : JLO; }
    static constexpr int jhi(int q) { return (LOW ? el(q) + 2 * P - K : el(q) + P) < JHI ? (LOW ? el(q) + 2 * P - K : el(q) + P) : JHI; }
};

__device__ inline int window_class(int i, int p, int nel) {
    if (i <= p) return 1 + i;
    if (i >= nel - 1) return p + 1 + (nel + p - i);
    return 0;
}

// calls f(std::integral_constant<int, CLS>) for the runtime class cls
template <int P, int C = 0, typename F>
__device__ inline void with_window(int cls, F&& f) {
    if constexpr (C < 2 * P + 3) {
        if (cls == C) f(std::integral_constant<int, C>{});
        else with_window<P, C + 1>(cls, f);
    }
}

// Stages, for the block's rows i1s..i1s+nrows-1 at fixed (i2, i3) and the union of their
// direction-1 windows (planes q1 of the kappa grid):
//   1. T1_v[q1][q2][j3] = sum_q3 W3_v[j3][q3] kappa[q1][q2][q3], v = 00 / 11 rules
//      (one thread per (q1, q2); its kappa row is loaded before the first barrier);
//   2. T2[q1][j2 j3] = sum_q2 W2_00[j2][q2] T1_00, Ts = sum_q2 W2_11 T1_00 + W2_00 T1_11
//      (one thread per (q1, j3));
//   3. row r, column c = (j2, j3): M[j1][c] = sum_q W1_00[j1][q] T2[off_r + q][c],
//      K = sum_q W1_11 T2 + W1_00 Ts (one thread per (row, column); all of a block's rows
//      share the slab), stored at the row's CSR offsets (contiguous per j1).
// Every contraction runs over the compile-time band of its window class; stiffness sums are
// accumulated one product per fused multiply-add.
template <int P, int WHICH, int RB>
__global__ void __launch_bounds__(256, 4)
k_rows_block(DevRules R, const float* __restrict__ kappa, float* __restrict__ vm, float* __restrict__ vk) {
    using C = BlkCfg<P, RB>;
    constexpr int M = C::M, MM = C::MM, NT = C::NT, NWT = C::NWT, NWB = C::NWB, NQB = C::NQB;
    constexpr int P1S = C::P1S, PSL = C::PSL, W1S = C::W1S, IPL1 = C::IPL1;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ float s_buf[C::BUFN];
    __shared__ float s_w1[RB * W1S];
    __shared__ float s_w2[2 * M * NWT], s_w3[2 * M * NWT];
    __shared__ int64_t s_base[RB];
    __shared__ int s_off[RB], s_cls[RB];

    const int4 blk = R.fblocks[xcd_logical(blockIdx.x, gridDim.x)];
    const int i1s = blk.x, i2 = blk.y, i3 = blk.z, nrows = blk.w;
    const int t = threadIdx.x;
    const int n2 = R.nfun[1], n3 = R.nfun[2];
    const int qbase = R.xs[0][i1s];
    const int i1e = i1s + nrows - 1;
    const int nq1 = R.xs[0][i1e] + R.nwin[0][i1e] - qbase;
    const int xs2 = R.xs[1][i2], nw2 = R.nwin[1][i2];
    const int xs3 = R.xs[2][i3], nw3 = R.nwin[2][i3];
    const int cls2 = window_class(i2, P, R.nel[1]);
    const int cls3 = window_class(i3, P, R.nel[2]);
    const int nx2 = R.nx[1], nx3 = R.nx[2];
    // kappa row of this thread's first stage-1 item, issued together with the table loads
    // below (a block with more than NT items loads the rest in stage 1)
    auto kappa_row = [&](int it, float* kv) {
        const int q1 = it / nw2, q2 = it - q1 * nw2;
        const bool on = it < nq1 * nw2;
        const float* kr = kappa + ((int64_t)(qbase + (on ? q1 : 0)) * nx2 + xs2 + (on ? q2 : 0)) * nx3 + xs3;
#pragma unroll
        for (int q = 0; q < NWB; ++q) kv[q] = (on && q < nw3) ? kr[q] : 0.f;
    };
    float kv[NWB];
    kappa_row(t, kv);
    {
        const float* W1 = R.Wt32[0] + (int64_t)i1s * 2 * M * NWT;
        for (int k = t; k < nrows * 2 * M * NWT; k += NT) {
            const int r = k / (2 * M * NWT);
            s_w1[r * W1S + (k - r * 2 * M * NWT)] = W1[k];
        }
        const float* W2 = R.Wt32[1] + (int64_t)i2 * 2 * M * NWT;
        const float* W3 = R.Wt32[2] + (int64_t)i3 * 2 * M * NWT;
        for (int k = t; k < 2 * M * NWT; k += NT) {
            s_w2[k] = W2[k];
            s_w3[k] = W3[k];
        }
    }
    if (t < nrows) {
        const int i1 = i1s + t;
        const int ra = R.lex2act[((int64_t)i1 * n2 + i2) * n3 + i3];
        s_base[t] = R.row_ptr[ra];
        s_off[t] = R.xs[0][i1] - qbase;
        s_cls[t] = window_class(i1, P, R.nel[0]);
    }
    __syncthreads();

    // ---- stage 1: items (q1, q2).  Layouts in s_buf, plane by plane: stage-1 sums
    // [q1][v][q2][j3] (stride P1S), slab [q1][v][j2 j3] (stride PSL) ----
    with_window<P>(cls3, [&](auto cc) {
        using Wn = Win<P, decltype(cc)::value>;
#pragma unroll 1
        for (int k = 0; k < IPL1; ++k) {
            const int it = t + k * NT;
            if (it >= nq1 * nw2) break;
            if (k > 0) kappa_row(it, kv);
            // keep the weight loads inside the loop: hoisted, the uniform weights of a
            // class take over a hundred registers for at most two items
            asm volatile("" ::: "memory");
            const int q1 = it / nw2, q2 = it - q1 * nw2;
            float a0[M], a1[M];
#pragma unroll
            for (int j = 0; j < M; ++j) { a0[j] = 0.f; a1[j] = 0.f; }
#pragma unroll
            for (int q = 0; q < Wn::NW; ++q)
#pragma unroll
                for (int j = Wn::jlo(q); j <= Wn::jhi(q); ++j) {
                    a0[j] = __builtin_fmaf(s_w3[j * NWT + q], kv[q], a0[j]);
                    if (STIFF) a1[j] = __builtin_fmaf(s_w3[(M + j) * NWT + q], kv[q], a1[j]);
                }
            float* o0 = s_buf + q1 * P1S + q2 * M;
#pragma unroll
            for (int j = Wn::JLO; j <= Wn::JHI; ++j) {
                o0[j] = a0[j];
                if (STIFF) o0[NWB * M + j] = a1[j];
            }
        }
    });
    __syncthreads();

    // ---- stage 2: items (q1, j3), in rounds of NT items ordered by q1.  A round keeps its
    // results in registers until all its threads have read their stage-1 sums, then writes
    // them over the slab planes of its q1; when a block needs several rounds, slab plane q1
    // ends below stage-1 plane q1 + 1 (PSL < P1S), so a round never overwrites sums that a
    // later round reads.  Entries of trial indices outside the windows' ranges are never
    // written and never read ----
    static_assert(NQB * M <= NT || (PSL < P1S && (NT / M) * (P1S - PSL) >= PSL),
                  "a round's slab planes end below the stage-1 planes of later rounds");
    for (int base = 0; base < nq1 * M; base += NT) {
        asm volatile("" ::: "memory");             // weight loads stay inside the round
        const int it = base + t;
        const int q1 = it / M, j3 = it - q1 * M;
        float r0[M], rs[M];
#pragma unroll
        for (int j = 0; j < M; ++j) { r0[j] = 0.f; rs[j] = 0.f; }
        const bool on = it < nq1 * M;
        int jlo2 = 0, jhi2 = -1;
        with_window<P>(cls2, [&](auto cc) {
            using Wn = Win<P, decltype(cc)::value>;
            jlo2 = Wn::JLO; jhi2 = Wn::JHI;
            if (on) {
                const float* t0 = s_buf + q1 * P1S + j3;
                const float* t1 = t0 + NWB * M;
#pragma unroll
                for (int q = 0; q < Wn::NW; ++q) {
                    const float x0 = t0[q * M];
                    const float x1 = STIFF ? t1[q * M] : 0.f;
#pragma unroll
                    for (int j = Wn::jlo(q); j <= Wn::jhi(q); ++j) {
                        const float w0 = s_w2[j * NWT + q];
                        r0[j] = __builtin_fmaf(w0, x0, r0[j]);
                        if (STIFF) {
                            rs[j] = __builtin_fmaf(s_w2[(M + j) * NWT + q], x0, rs[j]);
                            rs[j] = __builtin_fmaf(w0, x1, rs[j]);
                        }
                    }
                }
            }
        });
        __syncthreads();
        if (on) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j >= jlo2 && j <= jhi2) {
                    s_buf[q1 * PSL + j * M + j3] = r0[j];
                    if (STIFF) s_buf[q1 * PSL + MM + j * M + j3] = rs[j];
                }
            }
        }
        __syncthreads();
    }

    // ---- stage 3: items (row, column) ----
    const int lo2 = i2 - P < 0 ? P - i2 : 0, hi2 = i2 + P > n2 - 1 ? n2 - 1 - i2 + P : 2 * P;
    const int lo3 = i3 - P < 0 ? P - i3 : 0, hi3 = i3 + P > n3 - 1 ? n3 - 1 - i3 + P : 2 * P;
    const int m2 = hi2 - lo2 + 1, m3 = hi3 - lo3 + 1;
    for (int it = t; it < nrows * MM; it += NT) {
        const int r = it / MM, c = it - r * MM;
        const int jj2 = c / M, jj3 = c - jj2 * M;
        const bool live = jj2 >= lo2 && jj2 <= hi2 && jj3 >= lo3 && jj3 <= hi3;
        const int64_t ob = s_base[r] + (int64_t)(jj2 - lo2) * m3 + (jj3 - lo3);
        const int step = m2 * m3;
        const float* w10 = s_w1 + r * W1S;
        const float* w11 = w10 + M * NWT;
        const float* x0 = s_buf + s_off[r] * PSL + c;
        const float* xs = x0 + MM;
        with_window<P>(s_cls[r], [&](auto cc) {
            using Wn = Win<P, decltype(cc)::value>;
            float t0[Wn::NW], ts[Wn::NW];
#pragma unroll
            for (int q = 0; q < Wn::NW; ++q) {
                t0[q] = live ? x0[q * PSL] : 0.f;
                ts[q] = (STIFF && live) ? xs[q * PSL] : 0.f;
            }
#pragma unroll
            for (int jj1 = Wn::JLO; jj1 <= Wn::JHI; ++jj1) {
                float am = 0.f, ak = 0.f;
#pragma unroll
                for (int q = 0; q < Wn::NW; ++q) {
                    if (jj1 >= Wn::jlo(q) && jj1 <= Wn::jhi(q)) {
                        const float a = w10[jj1 * NWT + q];
                        if (MASS) am = __builtin_fmaf(a, t0[q], am);
                        if (STIFF) {
                            ak = __builtin_fmaf(w11[jj1 * NWT + q], t0[q], ak);
                            ak = __builtin_fmaf(a, ts[q], ak);
                        }
                    }
                }
                if (live) {
                    const int64_t o = ob + (int64_t)(jj1 - Wn::JLO) * step;
                    if (MASS) vm[o] = am;
                    if (STIFF) vk[o] = ak;
                }
            }
        });
    }
}

// ----------------------------------------------------------------------------------------
// cut rows (general kernel): contraction order A (split direction first), B, C
// ----------------------------------------------------------------------------------------
template <typename T, int P, int WHICH>
struct CutCfg {
    static constexpr int M = 2 * P + 1, NW = 4 * P, NDQ = P * (P + 1), MM = M * M;
    static constexpr int NA = NDQ > NW ? NDQ : NW;         // the split direction may hold a DWQ rule
    static constexpr int NT = 256;
    static constexpr int QCH = sizeof(T) == 8 && P > 4 ? 4 : 2;   // direction-C points per chunk (small: occupancy)
    static constexpr bool STIFF = (WHICH & 2) != 0;
    static constexpr bool MASS = (WHICH & 1) != 0;
};

// Cut rows without a DWQ box: one wave per row writes zeros over the row (their values come
// from cut_assemble alone), 16-byte stores over the aligned middle of the row.
template <typename T, int WHICH>
__global__ void __launch_bounds__(256)
k_rows_zero(DevRules R, T* __restrict__ vm, T* __restrict__ vk) {
    const int64_t cr = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (cr >= R.n_cut || R.split[cr].x >= 0) return;
    const int lane = threadIdx.x & 63;
    const int ra = R.cut_rows[cr];
    const int64_t rb = R.row_ptr[ra], re = R.row_ptr[ra + 1];
    constexpr int V = 16 / sizeof(T);           // values per 16-byte store
    if (((uintptr_t)vm | (uintptr_t)vk) % 16 != 0) {   // arrays not 16-byte aligned: plain stores
        for (int64_t k = rb + lane; k < re; k += 64) {
            if (WHICH & 1) vm[k] = 0;
            if (WHICH & 2) vk[k] = 0;
        }
        return;
    }
    // head up to the first 16-byte boundary, then whole vectors, then the tail
    int64_t a = (rb + V - 1) / V * V;
    if (a > re) a = re;
    const int64_t b = a + (re - a) / V * V;
    if (rb + lane < a) {
        if (WHICH & 1) vm[rb + lane] = 0;
        if (WHICH & 2) vk[rb + lane] = 0;
    }
    if (b + lane < re) {
        if (WHICH & 1) vm[b + lane] = 0;
        if (WHICH & 2) vk[b + lane] = 0;
    }
    const int4 z = make_int4(0, 0, 0, 0);
    for (int64_t k = a / V + lane; k < b / V; k += 64) {
        if (WHICH & 1) reinterpret_cast<int4*>(vm)[k] = z;
        if (WHICH & 2) reinterpret_cast<int4*>(vk)[k] = z;
    }
}

// One workgroup per cut row with a DWQ box (the box-row list).  The contraction runs split
// direction first (A, with the one-sided rule), then B, then C; kappa of a chunk of C points
// is gathered into LDS with independent loads (through the slot map; the next chunk's loads
// are issued before the current chunk is contracted), then stage A (items (qC, qB, jA)),
// stage B (items (qC, jB, jA)) and, after all chunks, stage C (items (jC, jB, jA)) write
// the row through its position map (read at the start).
template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_rows_cut(DevRules R, const T* __restrict__ kappa, T* __restrict__ vm, T* __restrict__ vk) {
    using C = CutCfg<T, P, WHICH>;
    constexpr int M = C::M, NW = C::NW, NDQ = C::NDQ, MM = C::MM, NA = C::NA, QCH = C::QCH, NT = C::NT;
    __shared__ T s_w[3][2 * M * NA];
    __shared__ int s_y[3][NA];
    __shared__ int s_n[3];
    __shared__ T s_k[QCH * NW * NA];                // kappa [qC in chunk][qB][qA]
    __shared__ T s_t1[2 * QCH * NW * M];            // [v][qC in chunk][qB][jA]
    __shared__ T s_t2[2 * NW * MM];                 // [v][qC][jB jA]

    const int64_t cr = R.box_rows[blockIdx.x];
    const int ra = R.cut_rows[cr];
    const int4 sp = R.split[cr];
    const int64_t rb = R.row_ptr[ra];
    if (sp.x < 0) return;
    const int t = threadIdx.x;
    const int lex = R.act2lex[ra];
    int I[3];
    I[2] = lex % R.nfun[2]; I[1] = (lex / R.nfun[2]) % R.nfun[1]; I[0] = lex / (R.nfun[1] * R.nfun[2]);
    // contraction order: A = split direction, then the other two ascending
    const int dA = sp.x, dB = dA == 0 ? 1 : 0, dC = dA == 2 ? 1 : 2;
    const int dirs[3] = {dA, dB, dC};
    // position map entries of this thread's stage-C items, loaded now
    constexpr int NPOS = (M * MM + NT - 1) / NT;
    const int32_t* pos = R.pos_map + cr * (int64_t)M * M * M;
    int pq[NPOS];
#pragma unroll
    for (int i = 0; i < NPOS; ++i) {
        const int it = t + i * NT;
        pq[i] = -1;
        if (it < M * MM) {
            const int jA = it % M, jB = (it / M) % M, jC = it / MM;
            pq[i] = pos[(pick3(0, dA, dB, jA, jB, jC) * M + pick3(1, dA, dB, jA, jB, jC)) * M + pick3(2, dA, dB, jA, jB, jC)];
        }
    }
    // rules into LDS: s_w[slot][a][jj][q] with q stride NA
    for (int sl = 0; sl < 3; ++sl) {
        const int d = dirs[sl];
        if (sl == 0) {
            const int r = sp.w;
            const int np = R.dwq_np[r];
            const T* W = dwq_table<T>(R) + (int64_t)r * 2 * M * NDQ;
            for (int k = t; k < 2 * M * NA; k += NT) {
                const int q = k % NA, row = k / NA;
                s_w[sl][k] = q < NDQ ? W[row * NDQ + q] : (T)0;
            }
            for (int q = t; q < NA; q += NT) s_y[sl][q] = q < np ? R.dwq_y[(int64_t)r * NDQ + q] : 0;
            if (t == 0) s_n[sl] = np;
        } else {
            const int i = I[d];
            const int xs = R.xs[d][i], nw = R.nwin[d][i];
            const T* W = wt_table<T>(R, d) + (int64_t)i * 2 * M * NW;
            for (int k = t; k < 2 * M * NA; k += NT) {
                const int q = k % NA, row = k / NA;
                s_w[sl][k] = q < NW ? W[row * NW + q] : (T)0;
            }
            for (int q = t; q < NA; q += NT) s_y[sl][q] = q < nw ? R.x2y[d][xs + q] : 0;
            if (t == 0) s_n[sl] = nw;
        }
    }
    __syncthreads();
    const int nA = s_n[0], nB = s_n[1], nCc = s_n[2];
    // kappa of a chunk: KQ values per thread, all loads independent
    constexpr int KQ = (QCH * NW * NA + NT - 1) / NT;
    T kq[KQ];
    auto gather = [&](int qc0) {
        const int nch = nCc - qc0 < QCH ? nCc - qc0 : QCH;
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            const int k = t + i * NT;
            if (k < nch * nB * nA) {
                const int qCl = k / (nB * nA), qB = (k / nA) % nB, qA = k % nA;
                const int yA = s_y[0][qA], yB = s_y[1][qB], yC = s_y[2][qc0 + qCl];
                kq[i] = kappa[slot_of(R, pick3(0, dA, dB, yA, yB, yC), pick3(1, dA, dB, yA, yB, yC),
                                      pick3(2, dA, dB, yA, yB, yC))];
            }
        }
    };
    gather(0);
    for (int qc0 = 0; qc0 < nCc; qc0 += QCH) {
        const int nch = nCc - qc0 < QCH ? nCc - qc0 : QCH;
#pragma unroll
        for (int i = 0; i < KQ; ++i) {
            const int k = t + i * NT;
            if (k < nch * nB * nA) {
                const int qCl = k / (nB * nA), qB = (k / nA) % nB, qA = k % nA;
                s_k[(qCl * NW + qB) * NA + qA] = kq[i];
            }
        }
        __syncthreads();
        if (qc0 + QCH < nCc) gather(qc0 + QCH);     // in flight during this chunk's stages
        // stage A: T1[v][qC][qB][jA] = sum_qA W_A^v[jA][qA] kappa(qA, qB, qC)
        for (int it = t; it < nch * nB * M; it += NT) {
            const int qCl = it / (nB * M), qB = (it / M) % nB, jA = it % M;
            const T* kr = s_k + (qCl * NW + qB) * NA;
            T a0 = 0, a1 = 0;
            for (int qA = 0; qA < nA; ++qA) {
                const T kv = kr[qA];
                a0 += s_w[0][jA * NA + qA] * kv;
                if (C::STIFF) a1 += s_w[0][(M + jA) * NA + qA] * kv;
            }
            s_t1[((0 * QCH + qCl) * NW + qB) * M + jA] = a0;
            if (C::STIFF) s_t1[((1 * QCH + qCl) * NW + qB) * M + jA] = a1;
        }
        __syncthreads();
        // stage B: T2_00[qC][jB jA] = sum_qB W_B^0 T1_0; T2_s = sum W_B^1 T1_0 + W_B^0 T1_1
        for (int it = t; it < nch * MM; it += NT) {
            const int qCl = it / MM, jB = (it / M) % M, jA = it % M;
            const int qC = qc0 + qCl;
            T m0 = 0, ms = 0;
            for (int qB = 0; qB < nB; ++qB) {
                const T t0 = s_t1[((0 * QCH + qCl) * NW + qB) * M + jA];
                const T w0 = s_w[1][jB * NA + qB];
                m0 += w0 * t0;
                if (C::STIFF) ms = fmat(w0, s_t1[((1 * QCH + qCl) * NW + qB) * M + jA], fmat(s_w[1][(M + jB) * NA + qB], t0, ms));
            }
            s_t2[(0 * NW + qC) * MM + jB * M + jA] = m0;
            if (C::STIFF) s_t2[(1 * NW + qC) * MM + jB * M + jA] = ms;
        }
        __syncthreads();                            // s_k / s_t1 are rewritten by the next chunk
    }
    // stage C: items (jC, jB, jA); out[jC][jB][jA]
#pragma unroll
    for (int i = 0; i < NPOS; ++i) {
        const int it = t + i * NT;
        if (it >= M * MM) break;
        const int jC = it / MM, cc = it % MM, jB = cc / M, jA = cc % M;
        T am = 0, ak = 0;
        for (int qC = 0; qC < nCc; ++qC) {
            const T t0 = s_t2[(0 * NW + qC) * MM + cc];
            const T a = s_w[2][jC * NA + qC];
            if (C::MASS) am += a * t0;
            if (C::STIFF) ak = fmat(a, s_t2[(1 * NW + qC) * MM + cc], fmat(s_w[2][(M + jC) * NA + qC], t0, ak));
        }
        const int k = pq[i];
        if (k >= 0) {
            if (C::MASS) vm[rb + k] = am;
            if (C::STIFF) vk[rb + k] = ak;
        }
    }
}

// ----------------------------------------------------------------------------------------
// cut rows with a DWQ box, p <= 4: the whole box at once
// ----------------------------------------------------------------------------------------
// One workgroup per box row.  The row's points are the one-sided DWQ rule's points in the
// split direction A and the standard windows in B and C (directions ascending).  kappa of
// every point of the box is gathered into LDS first (one batch of independent loads; the
// slot of a point follows from per-direction tables: a grid point when its A point is a WQ
// point, else the Gauss block of its element), then three contractions:
//   A: T1_v[qC][qB][jA] = sum_qA W_A^v[jA][qA] kappa[qC][qB][qA];
//   B: T2_00[qC][jB jA] = sum_qB W_B^00 T1_00, T2_s = sum_qB W_B^11 T1_00 + W_B^00 T1_11;
//   C: M[jC jB jA] = sum_qC W_C^00 T2_00, K = sum_qC W_C^11 T2_00 + W_C^00 T2_s,
// each thread holding one output index j of the contracted direction and a few values of
// the others, so a weight read from LDS serves several products.  Values go to the row
// through its position map.  Needs windows of at most 3p+1 points (p+2 elements per direction).
template <typename T, int P>
struct BoxCfg {
    static constexpr int M = 2 * P + 1, MM = M * M, NT = 256;
    static constexpr int NDQ = P * (P + 1), NWT = 4 * P, NWB = 3 * P + 1;
    static constexpr int NQM = NDQ > NWB ? NDQ : NWB;       // points of the longest of the three rules
    static constexpr int KS = NDQ + 1;                      // odd stride of a kappa row
    static constexpr int NK = NWB * NWB * KS;                // kappa of the box [qC qB][qA]
    static constexpr int NT2 = 2 * NWB * MM;                 // stage-B sums (reuse the kappa space)
    static constexpr int NKB = NK > NT2 ? NK : NT2;
    static constexpr int NT1 = 2 * NWB * NWB * M;            // stage-A sums [v][qC qB][jA]
    static constexpr int NG = (NDQ * NWB * NWB + NT - 1) / NT;   // kappa gathers per thread
    static constexpr int GA = 4, GB = 4, GC = 3;             // outputs per thread and weight read
};

template <typename T, int P, int WHICH>
__global__ void __launch_bounds__(256)
k_rows_box(DevRules R, const T* __restrict__ kappa, T* __restrict__ vm, T* __restrict__ vk) {
    using C = BoxCfg<T, P>;
    constexpr int M = C::M, MM = C::MM, NT = C::NT, NDQ = C::NDQ, NWT = C::NWT, NWB = C::NWB, KS = C::KS;
    constexpr int P1 = P + 1, P13 = P1 * P1 * P1;
    constexpr bool MASS = (WHICH & 1) != 0, STIFF = (WHICH & 2) != 0;
    __shared__ T s_kb[C::NKB];                   // kappa, then the stage-B sums
    __shared__ T s_t1[C::NT1];
    __shared__ T s_wa[2 * M * NDQ], s_wb[2 * M * NWT], s_wc[2 * M * NWT];
    __shared__ int s_g[3][C::NQM], s_e[3][C::NQM], s_l[3][C::NQM];   // per direction and point: slot parts
    __shared__ int s_n[3];
    __shared__ int s_qa[2][M];                   // nonzero point range [s_qa[0][j], s_qa[1][j]) of W_A[.][j][.]

    const int64_t cr = R.box_rows[blockIdx.x];
    const int ra = R.cut_rows[cr];
    const int4 sp = R.split[cr];
    const int64_t rb = R.row_ptr[ra];
    const int t = threadIdx.x;
    const int lex = R.act2lex[ra];
    int I[3];
    I[2] = lex % R.nfun[2]; I[1] = (lex / R.nfun[2]) % R.nfun[1]; I[0] = lex / (R.nfun[1] * R.nfun[2]);
    const int dA = sp.x, dB = dA == 0 ? 1 : 0, dC = dA == 2 ? 1 : 2;
    // strides of the grid and of the element / point indices of a Gauss block along
    // direction d (selects, not indexed arrays, so nothing goes to scratch)
    auto gstr = [&](int d) { return d == 0 ? R.nx[1] * R.nx[2] : (d == 1 ? R.nx[2] : 1); };
    auto estr = [&](int d) { return d == 0 ? R.nel[1] * R.nel[2] : (d == 1 ? R.nel[2] : 1); };
    auto lstr = [&](int d) { return d == 0 ? P1 * P1 : (d == 1 ? P1 : 1); };
    // rules and per-point slot parts
    {
        const int r = sp.w;
        const int np = R.dwq_np[r];
        const T* W = dwq_table<T>(R) + (int64_t)r * 2 * M * NDQ;
        for (int k = t; k < 2 * M * NDQ; k += NT) s_wa[k] = W[k];
        const int IB = dB == 0 ? I[0] : I[1], IC = dC == 1 ? I[1] : I[2];
        const T* WB = wt_table<T>(R, dB) + (int64_t)IB * 2 * M * NWT;
        const T* WC = wt_table<T>(R, dC) + (int64_t)IC * 2 * M * NWT;
        for (int k = t; k < 2 * M * NWT; k += NT) {
            s_wb[k] = WB[k];
            s_wc[k] = WC[k];
        }
        if (t < NDQ) {
            if (t < np) {
                const int y = R.dwq_y[(int64_t)r * NDQ + t];
                const int x = R.y2x[dA][y];
                s_g[0][t] = x >= 0 ? x * gstr(dA) : -1;
                s_e[0][t] = (y / P1) * estr(dA);
                s_l[0][t] = (y % P1) * lstr(dA);
            }
        }
#pragma unroll
        for (int s = 1; s < 3; ++s) {
            const int d = s == 1 ? dB : dC;
            const int Id = d == 0 ? I[0] : (d == 1 ? I[1] : I[2]);
            const int xs = R.xs[d][Id], nw = R.nwin[d][Id];
            if (t < nw) {
                const int x = xs + t;
                const int y = R.x2y[d][x];
                s_g[s][t] = x * gstr(d);
                s_e[s][t] = (y / P1) * estr(d);
                s_l[s][t] = (y % P1) * lstr(d);
            }
            if (t == 0) s_n[s] = nw;
        }
        if (t == 0) s_n[0] = np;
    }
    // position map entries of this thread's outputs in stage C
    const int32_t* pos = R.pos_map + cr * (int64_t)M * MM;
    __syncthreads();
    const int nA = s_n[0], nB = s_n[1], nC = s_n[2];
    // W_A[v][jA][qA] vanishes unless point qA lies in the support of trial function jA: the
    // nonzero points of each jA form one range (the points are ordered)
    if (t < M) {
        int lo = nA, hi = 0;
        for (int q = 0; q < nA; ++q)
            if (s_wa[t * NDQ + q] != (T)0 || s_wa[(M + t) * NDQ + q] != (T)0) {
                lo = q < lo ? q : lo;
                hi = q + 1;
            }
        s_qa[0][t] = lo < hi ? lo : 0;
        s_qa[1][t] = lo < hi ? hi : 0;
    }
    // regular standard windows (2p+2 points, two per element): W[j][q] != 0 only for
    // q in [2 max(0, j-p), 2 (min(j, p) + 1))
    const int IBr = dB == 0 ? I[0] : I[1], ICr = dC == 1 ? I[1] : I[2];
    const bool regB = IBr >= P + 1 && IBr <= R.nel[dB] - 2;
    const bool regC = ICr >= P + 1 && ICr <= R.nel[dC] - 2;
    const int npts = nA * nB * nC;
    // ---- kappa of the box: [qC qB][qA] ----
    {
        T kv[C::NG];
#pragma unroll
        for (int i = 0; i < C::NG; ++i) {
            const int k = t + i * NT;
            kv[i] = (T)0;
            if (k < npts) {
                const int qA = k % nA, pr = k / nA, qB = pr % nB, qC = pr / nB;
                const int ga = s_g[0][qA];
                int64_t slot;
                if (ga >= 0) {
                    slot = (int64_t)ga + s_g[1][qB] + s_g[2][qC];
                } else {
                    const int b = R.elem_block[s_e[0][qA] + s_e[1][qB] + s_e[2][qC]];
                    slot = R.n_grid + (int64_t)b * P13 + s_l[0][qA] + s_l[1][qB] + s_l[2][qC];
                }
                kv[i] = kappa[slot];
            }
        }
#pragma unroll
        for (int i = 0; i < C::NG; ++i) {
            const int k = t + i * NT;
            if (k < npts) {
                const int qA = k % nA, pr = k / nA;
                s_kb[pr * KS + qA] = kv[i];
            }
        }
    }
    __syncthreads();
    // ---- stage A: thread (jA, group), pairs pr = group + k * ngroups ----
    {
        constexpr int G = C::GA;
        const int npair = nB * nC, ngrp = (npair + G - 1) / G;
        for (int it = t; it < M * ngrp; it += NT) {
            const int jA = it / ngrp, grp = it - jA * ngrp;
            T a0[G], a1[G];
            int prk[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                a0[k] = 0; a1[k] = 0;
                const int pr = grp + k * ngrp;
                prk[k] = pr < npair ? pr : npair - 1;
            }
            const T* w0p = s_wa + jA * NDQ;
            const T* w1p = s_wa + (M + jA) * NDQ;
            const int qlo = s_qa[0][jA], qhi = s_qa[1][jA];
#pragma unroll 2
            for (int qA = qlo; qA < qhi; ++qA) {
                const T w0 = w0p[qA];
                const T w1 = STIFF ? w1p[qA] : (T)0;
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const T kk = s_kb[prk[k] * KS + qA];
                    a0[k] += w0 * kk;
                    if (STIFF) a1[k] += w1 * kk;
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int pr = grp + k * ngrp;
                if (pr < npair) {
                    s_t1[pr * M + jA] = a0[k];
                    if (STIFF) s_t1[NWB * NWB * M + pr * M + jA] = a1[k];
                }
            }
        }
    }
    __syncthreads();
    // ---- stage B: thread (jB, group), pairs (qC, jA) ----
    {
        constexpr int G = C::GB;
        const int npair = nC * M, ngrp = (npair + G - 1) / G;
        for (int it = t; it < M * ngrp; it += NT) {
            const int jB = it / ngrp, grp = it - jB * ngrp;
            T m0[G], ms[G];
            int base[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                m0[k] = 0; ms[k] = 0;
                int pr = grp + k * ngrp;
                pr = pr < npair ? pr : npair - 1;
                const int qC = pr / M, jA = pr - qC * M;
                base[k] = qC * nB * M + jA;
            }
            const T* w0p = s_wb + jB * NWT;
            const T* w1p = s_wb + (M + jB) * NWT;
            const int qlo = regB ? 2 * (jB - P > 0 ? jB - P : 0) : 0;
            const int qhi = regB ? 2 * ((jB < P ? jB : P) + 1) : nB;
#pragma unroll 2
            for (int qB = qlo; qB < qhi; ++qB) {
                const T w0 = w0p[qB];
                const T w1 = STIFF ? w1p[qB] : (T)0;
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const T t0 = s_t1[base[k] + qB * M];
                    m0[k] += w0 * t0;
                    if (STIFF) ms[k] = fmat(w0, s_t1[NWB * NWB * M + base[k] + qB * M], fmat(w1, t0, ms[k]));
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int pr = grp + k * ngrp;
                if (pr < npair) {
                    const int qC = pr / M, jA = pr - qC * M;
                    s_kb[qC * MM + jB * M + jA] = m0[k];
                    if (STIFF) s_kb[NWB * MM + qC * MM + jB * M + jA] = ms[k];
                }
            }
        }
    }
    __syncthreads();
    // ---- stage C: thread (jC, group), pairs c = (jB, jA); stores through the position map ----
    {
        constexpr int G = C::GC;
        constexpr int ngrp = (MM + G - 1) / G;
        for (int it = t; it < M * ngrp; it += NT) {
            const int jC = it / ngrp, grp = it - jC * ngrp;
            T am[G], ak[G];
            int ck[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                am[k] = 0; ak[k] = 0;
                const int c = grp + k * ngrp;
                ck[k] = c < MM ? c : MM - 1;
            }
            const T* w0p = s_wc + jC * NWT;
            const T* w1p = s_wc + (M + jC) * NWT;
            const int qlo = regC ? 2 * (jC - P > 0 ? jC - P : 0) : 0;
            const int qhi = regC ? 2 * ((jC < P ? jC : P) + 1) : nC;
#pragma unroll 2
            for (int qC = qlo; qC < qhi; ++qC) {
                const T w0 = w0p[qC];
                const T w1 = STIFF ? w1p[qC] : (T)0;
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    const T t0 = s_kb[qC * MM + ck[k]];
                    if (MASS) am[k] += w0 * t0;
                    if (STIFF) ak[k] = fmat(w0, s_kb[NWB * MM + qC * MM + ck[k]], fmat(w1, t0, ak[k]));
                }
            }
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int c = grp + k * ngrp;
                if (c < MM) {
                    const int jB = c / M, jA = c - jB * M;
                    const int o = pos[(pick3(0, dA, dB, jA, jB, jC) * M + pick3(1, dA, dB, jA, jB, jC)) * M +
                                      pick3(2, dA, dB, jA, jB, jC)];
                    if (o >= 0) {
                        if (MASS) vm[rb + o] = am[k];
                        if (STIFF) vk[rb + o] = ak[k];
                    }
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------------------
// windows of at most 3p+1 points: p + 2 elements in every direction
static bool windows_fit(const DevRules& R) {
    return R.nel[0] >= R.p + 2 && R.nel[1] >= R.p + 2 && R.nel[2] >= R.p + 2;
}
static bool block_kernel_fits(const DevRules& R) { return R.p <= 4 && R.n_fblocks > 0 && windows_fit(R); }

template <typename T, int P, int WHICH>
static void launch_interior_rows(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if constexpr (sizeof(T) == 4 && P <= 4) {
        if (block_kernel_fits(R)) {
            hipLaunchKernelGGL((k_rows_block<P, WHICH, 8>), dim3((unsigned)R.n_fblocks), dim3(256), 0, s, R,
                               (const float*)kappa, (float*)vm, (float*)vk);
            return;
        }
    }
    if (R.n_lblocks > 0) {
        // line blocks hold up to 16 rows for p <= 4 and 8 above; FP64 at p <= 4 takes half a
        // block per workgroup to bound its LDS slab
        if constexpr (P <= 4 && sizeof(T) == 4) {
            using C = RowCfg<T, P, WHICH, 16>;
            hipLaunchKernelGGL((k_rows_interior<T, P, WHICH, 16, 1>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0, s, R, kappa,
                               vm, vk);
        } else if constexpr (P <= 4) {
            using C = RowCfg<T, P, WHICH, 8>;
            hipLaunchKernelGGL((k_rows_interior<T, P, WHICH, 8, 2>), dim3((unsigned)(2 * R.n_lblocks)), dim3(C::NT), 0, s, R,
                               kappa, vm, vk);
        } else {
            using C = RowCfg<T, P, WHICH, 8>;
            hipLaunchKernelGGL((k_rows_interior<T, P, WHICH, 8, 1>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0, s, R, kappa,
                               vm, vk);
        }
    }
}

template <typename T, int P, int WHICH>
static void launch_cut_rows(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if (R.n_box > 0) {
        bool done = false;
        if constexpr (P <= 4) {
            if (windows_fit(R)) {
                hipLaunchKernelGGL((k_rows_box<T, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, kappa, vm, vk);
                done = true;
            }
        }
        if (!done)
            hipLaunchKernelGGL((k_rows_cut<T, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, kappa, vm, vk);
    }
    if (R.n_cut > R.n_box)
        hipLaunchKernelGGL((k_rows_zero<T, WHICH>), dim3((unsigned)((R.n_cut + 3) / 4)), dim3(256), 0, s, R, vm, vk);
}

// The cut rows run on the handle's side stream beside the interior rows on the caller's
// stream (they write disjoint rows): forked after the caller's earlier work, joined back
// before anything the caller enqueues later.
template <typename T, int P, int WHICH>
static void launch_rows_p(const wq_rules* H, const T* kappa, T* vm, T* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if (!(H->side && R.n_cut > 0)) {
        launch_cut_rows<T, P, WHICH>(H, kappa, vm, vk, s);
        launch_interior_rows<T, P, WHICH>(H, kappa, vm, vk, s);
        return;
    }
    std::lock_guard<std::mutex> lock(*H->side_mu);
    if (hipEventRecord(H->ev_fork, s) != hipSuccess || hipStreamWaitEvent(H->side, H->ev_fork, 0) != hipSuccess) {
        (void)hipGetLastError();
        launch_cut_rows<T, P, WHICH>(H, kappa, vm, vk, s);
        launch_interior_rows<T, P, WHICH>(H, kappa, vm, vk, s);
        return;
    }
    launch_cut_rows<T, P, WHICH>(H, kappa, vm, vk, H->side);
    launch_interior_rows<T, P, WHICH>(H, kappa, vm, vk, s);
    if (hipEventRecord(H->ev_join, H->side) != hipSuccess || hipStreamWaitEvent(s, H->ev_join, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(H->side);    // the join failed: finish the side stream's work here
    }
}

#ifndef WQ_ONLY_F64
// BF16x3 experiment: interior rows with the split-operand stage 3, cut rows as in FP32
template <int P, int WHICH>
static void launch_rows_bf3_p(const wq_rules* H, const float* kappa, float* vm, float* vk, hipStream_t s) {
    const DevRules& R = H->R;
    if (R.n_lblocks > 0) {
        if constexpr (P <= 4) {
            using C = RowCfg<float, P, WHICH, 16>;
            hipLaunchKernelGGL((k_rows_interior<float, P, WHICH, 16, 1, true>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0,
                               s, R, kappa, vm, vk);
        } else {
            using C = RowCfg<float, P, WHICH, 8>;
            hipLaunchKernelGGL((k_rows_interior<float, P, WHICH, 8, 1, true>), dim3((unsigned)R.n_lblocks), dim3(C::NT), 0,
                               s, R, kappa, vm, vk);
        }
    }
    if (R.n_box > 0) {
        bool done = false;
        if constexpr (P <= 4) {
            if (windows_fit(R)) {
                hipLaunchKernelGGL((k_rows_box<float, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, kappa, vm,
                                   vk);
                done = true;
            }
        }
        if (!done)
            hipLaunchKernelGGL((k_rows_cut<float, P, WHICH>), dim3((unsigned)R.n_box), dim3(256), 0, s, R, kappa, vm,
                               vk);
    }
    if (R.n_cut > R.n_box)
        hipLaunchKernelGGL((k_rows_zero<float, WHICH>), dim3((unsigned)((R.n_cut + 3) / 4)), dim3(256), 0, s, R, vm, vk);
}

template <int P>
static void launch_rows_bf3_w(const wq_rules* H, uint32_t which, const float* kappa, float* vm, float* vk,
                              hipStream_t s) {
    if (which == 1) launch_rows_bf3_p<P, 1>(H, kappa, vm, vk, s);
    else if (which == 2) launch_rows_bf3_p<P, 2>(H, kappa, vm, vk, s);
    else launch_rows_bf3_p<P, 3>(H, kappa, vm, vk, s);
}

void launch_rows_bf16x3(const wq_rules* H, uint32_t which, const float* kappa, float* vm, float* vk, hipStream_t s) {
    switch (H->R.p) {
        case 1: launch_rows_bf3_w<1>(H, which, kappa, vm, vk, s); break;
        case 2: launch_rows_bf3_w<2>(H, which, kappa, vm, vk, s); break;
        case 3: launch_rows_bf3_w<3>(H, which, kappa, vm, vk, s); break;
        case 4: launch_rows_bf3_w<4>(H, which, kappa, vm, vk, s); break;
        case 5: launch_rows_bf3_w<5>(H, which, kappa, vm, vk, s); break;
        case 6: launch_rows_bf3_w<6>(H, which, kappa, vm, vk, s); break;
    }
}
#endif

template <typename T, int P>
static void launch_rows_w(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s) {
    if (which == 1) launch_rows_p<T, P, 1>(H, kappa, vm, vk, s);
    else if (which == 2) launch_rows_p<T, P, 2>(H, kappa, vm, vk, s);
    else launch_rows_p<T, P, 3>(H, kappa, vm, vk, s);
}

template <typename T>
void launch_rows(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s) {
    switch (H->R.p) {
        case 1: launch_rows_w<T, 1>(H, which, kappa, vm, vk, s); break;
        case 2: launch_rows_w<T, 2>(H, which, kappa, vm, vk, s); break;
        case 3: launch_rows_w<T, 3>(H, which, kappa, vm, vk, s); break;
        case 4: launch_rows_w<T, 4>(H, which, kappa, vm, vk, s); break;
        case 5: launch_rows_w<T, 5>(H, which, kappa, vm, vk, s); break;
        case 6: launch_rows_w<T, 6>(H, which, kappa, vm, vk, s); break;
    }
}

// interior rows on s_int and cut rows on s_cut, with no fork or join (the fused assembly orders
// the streams itself)
template <typename T, int P>
static void launch_rows_split_p(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_int,
                                hipStream_t s_cut) {
    if (which == 1) {
        launch_cut_rows<T, P, 1>(H, kappa, vm, vk, s_cut);
        launch_interior_rows<T, P, 1>(H, kappa, vm, vk, s_int);
    } else if (which == 2) {
        launch_cut_rows<T, P, 2>(H, kappa, vm, vk, s_cut);
        launch_interior_rows<T, P, 2>(H, kappa, vm, vk, s_int);
    } else {
        launch_cut_rows<T, P, 3>(H, kappa, vm, vk, s_cut);
        launch_interior_rows<T, P, 3>(H, kappa, vm, vk, s_int);
    }
}

template <typename T>
void launch_rows_split(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_int,
                       hipStream_t s_cut) {
    switch (H->R.p) {
        case 1: launch_rows_split_p<T, 1>(H, which, kappa, vm, vk, s_int, s_cut); break;
        case 2: launch_rows_split_p<T, 2>(H, which, kappa, vm, vk, s_int, s_cut); break;
        case 3: launch_rows_split_p<T, 3>(H, which, kappa, vm, vk, s_int, s_cut); break;
        case 4: launch_rows_split_p<T, 4>(H, which, kappa, vm, vk, s_int, s_cut); break;
        case 5: launch_rows_split_p<T, 5>(H, which, kappa, vm, vk, s_int, s_cut); break;
        case 6: launch_rows_split_p<T, 6>(H, which, kappa, vm, vk, s_int, s_cut); break;
    }
}

#ifndef WQ_ONLY_F32
template void launch_rows_split<double>(const wq_rules*, uint32_t, const double*, double*, double*, hipStream_t,
                                        hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template void launch_rows_split<float>(const wq_rules*, uint32_t, const float*, float*, float*, hipStream_t, hipStream_t);
#endif

#ifndef WQ_ONLY_F32
template void launch_rows<double>(const wq_rules*, uint32_t, const double*, double*, double*, hipStream_t);
#endif
#ifndef WQ_ONLY_F64
template void launch_rows<float>(const wq_rules*, uint32_t, const float*, float*, float*, hipStream_t);
#endif
