// Shared pieces of the cut-element kernels in moment form (forward and adjoint).
#pragma once
#include "rows.h"

// 16x16x4 MFMA: A (16x4) element (m, k) in lane m + 16 k, B (4x16) element (k, n) in lane
// n + 16 k; D (16x16) column n = lane % 16, row given by MfmaOp<T>::row(lane, r) for the
// accumulator register r (FP32: 4 (lane / 16) + r, FP64: lane / 16 + 4 r).
template <typename T> struct MfmaOp;
template <> struct MfmaOp<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};
template <> struct MfmaOp<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ inline v4 mma(double a, double b, v4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};

template <int P> struct MomCfg {
    static constexpr int P1 = P + 1, P2 = P1 * P1, NP = P2 * P1;
    static constexpr int NK = 2 * P + 1, NK2 = NK * NK, NK3 = NK2 * NK;
    static constexpr int NT = 256, NWAVE = 4;
    static constexpr int NB = 8;                              // leaves per load batch
    static constexpr int KW = (NB * NP + NT - 1) / NT;        // weight / kappa loads per thread per batch
    static constexpr int NIMAX = 15, MAXC = 512;              // octree depth <= 3
    static constexpr int NZ = P2 * NK, NY = P1 * NK2;         // column sums [g1 g2][k3], x-group sums [g1][k2 k3]
    static constexpr int RZ = (NZ + NT - 1) / NT, RY = (NY + NT - 1) / NT, RX = (NK3 + NT - 1) / NT;
    static constexpr int NS1 = NK2 * P1, NS2 = NK * NP;       // [k1 k2][b3], [k1][(a2 b2) b3]
    static constexpr int MT = (P2 + 15) / 16, NTC = (NP + 15) / 16, NTW = (NTC + NWAVE - 1) / NWAVE;
    static constexpr int KS1 = (NK + 3) / 4, KS2 = (2 * NK + 3) / 4;
};

template <typename T> __device__ inline const T* bern_q(const DevRules& R, int d);
template <> __device__ inline const double* bern_q<double>(const DevRules& R, int d) { return R.bern_q64[d]; }
template <> __device__ inline const float* bern_q<float>(const DevRules& R, int d) { return R.bern_q32[d]; }
template <typename T> __device__ inline const T* bern_i(const DevRules& R);
template <> __device__ inline const double* bern_i<double>(const DevRules& R) { return R.bern_i64; }
template <> __device__ inline const float* bern_i<float>(const DevRules& R) { return R.bern_i32; }

