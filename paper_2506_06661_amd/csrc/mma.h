// Matrix-core steps used by the kernels: one 16x16x4 product per element type.
// Operands: lane l supplies A[l%16][l/16] and B[l/16][l%16]; result element r
// of lane l is row row(l, r), column l%16.  The FP64 and FP32 instructions
// place result rows differently (measured with a one-hot probe on gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace dfjk {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mma;
template <>
struct Mma<double> {
    typedef v4d acc_t;
    __device__ static acc_t zero() { return v4d{0.0, 0.0, 0.0, 0.0}; }
    __device__ static acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mma<float> {
    typedef v4f acc_t;
    __device__ static acc_t zero() { return v4f{0.f, 0.f, 0.f, 0.f}; }
    __device__ static acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

}  // namespace dfjk
