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
};
template <>
struct Mfma<double> {
    typedef double acc_t __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc_t fma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};

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
