// Matrix-core (MFMA) primitives shared by the translation kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace imq {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 matrix-core step: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// item v of lane l holds D[row(l/16, v)][l%16], where the FP32 form keeps four
// consecutive rows per lane group and the FP64 form interleaves them.
template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = f32x4;
    static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int q, int v) { return 4 * v + q; }
};

// Four consecutive values of one lane of a packed table (one 16- or 32-byte load).
template <typename T> struct alignas(4 * sizeof(T)) Quad { T v[4]; };

}  // namespace imq
