// MFMA operand/accumulator helpers and the extended index map shared by the
// S-build and its adjoint.
#pragma once

#include "common.h"

namespace prony {

template <typename T>
struct Pair;
template <>
struct Pair<float> {
    using type = float2;
};
template <>
struct Pair<double> {
    using type = double2;
};
template <typename T>
using pair_t = typename Pair<T>::type;

// 16x16x4 MFMA in T with FP32/FP64 accumulation. Operand layout (both types):
// lane l holds A[l%16][l/16] and B[l/16][l%16]. Accumulator element r of lane l
// holds row row(l/16, r), column l%16 of the 16x16 result (measured on gfx950).
template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
    typedef float acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t fma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
    static __device__ __forceinline__ int group_of_row(int i) { return i >> 2; }
    static __device__ __forceinline__ int elem_of_row(int i) { return i & 3; }
};
template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t fma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
    static __device__ __forceinline__ int group_of_row(int i) { return i & 3; }
    static __device__ __forceinline__ int elem_of_row(int i) { return i >> 2; }
};

// Value of the neighbouring lane (lane ^ 1) through a DPP quad permutation
// [1, 0, 3, 2]; every lane of the wave must be active.
constexpr int kDppSwapPairs = 0xB1;
__device__ __forceinline__ float swap_lane_pair(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), kDppSwapPairs, 0xF, 0xF, false));
}
__device__ __forceinline__ double swap_lane_pair(double x) {
    const long long v = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(v & 0xffffffffll), kDppSwapPairs, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(v >> 32), kDppSwapPairs, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Grid offset G(k') = sum_l k'_l (2n+2)^(d-l) of the row-extended index k',
// row-major over {0..n+1}^d (digits in base n+2).
__host__ __device__ inline int rowext_offset(int r, int d, int n) {
    const int E = n + 2, Q = 2 * n + 2;
    int g = 0, scale = 1;
    for (int l = d - 1; l >= 0; --l) {
        const int q = r / E;
        g += (r - q * E) * scale;
        r = q;
        scale *= Q;
    }
    return g;
}

// Grid offset of the extended index h' (row-major over {-1..n}^d).
__host__ __device__ inline int ext_offset(int hx, int d, int n) {
    const int E = n + 2, Q = 2 * n + 2;
    int g = 0, scale = 1;
    for (int l = d - 1; l >= 0; --l) {
        const int q = hx / E;
        g += (hx - q * E - 1) * scale;
        hx = q;
        scale *= Q;
    }
    return g;
}

}  // namespace prony
