// Sustained matrix-core rate, measured with register-only kernels (no memory
// traffic): every wavefront repeats independent steps on several
// accumulators (8 for FP64 16x16x4, 16 for FP32 16x16x4, 4 for BF16
// 32x32x16: enough independent chains for each shape to reach its measured
// best on MI355X), eight wavefronts per SIMD.  Used to state how far the
// exchange kernels sit from what the matrix cores sustain, beside the
// published peaks.  Likewise the sustained HBM read rate of a plain
// streaming kernel, the measured ceiling of the J passes.
#include "internal.h"
#include "mma.h"

namespace dfjk {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kAcc = 8, kAcc32 = 16, kAccBf = 4;

__global__ __launch_bounds__(256) void probe_f64(double* out, int iters) {
    v4d acc[kAcc];
    for (int t = 0; t < kAcc; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    const double a = threadIdx.x * 1e-3, b = 1.0 + threadIdx.x * 1e-4;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int t = 0; t < kAcc; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
    double s = 0.0;
    for (int t = 0; t < kAcc; ++t) s += acc[t][0] + acc[t][3];
    if (s == -1.0) out[0] = s;  // keeps the work; never true for these inputs
}

__global__ __launch_bounds__(256) void probe_f32(double* out, int iters) {
    v4f acc[kAcc32];
    for (int t = 0; t < kAcc32; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const float a = threadIdx.x * 1e-3f, b = 1.0f;
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int t = 0; t < kAcc32; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
    float s = 0.f;
    for (int t = 0; t < kAcc32; ++t) s += acc[t][0];
    if (s == -1.f) out[0] = s;
}

__global__ __launch_bounds__(256) void probe_bf16(double* out, int iters) {
    v16f acc[kAccBf];
    for (int t = 0; t < kAccBf; ++t)
        for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
    v8bf a, b;
    for (int j = 0; j < 8; ++j) {
        a[j] = (__bf16)(threadIdx.x * 1e-3f);
        b[j] = (__bf16)1.0f;
    }
    for (int it = 0; it < iters; ++it)
#pragma unroll
        for (int t = 0; t < kAccBf; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[t], 0, 0, 0);
    float s = 0.f;
    for (int t = 0; t < kAccBf; ++t) s += acc[t][0];
    if (s == -1.f) out[0] = s;
}

// Streaming read of n 16-byte vectors: workgroup b reads the contiguous
// range [b*per, (b+1)*per) with eight independent non-temporal loads in
// flight per thread (32 KB per workgroup per step), folded with XOR so that
// no load can be dropped.
__global__ __launch_bounds__(256) void probe_read(const u32x4* __restrict__ x, int64_t n, int64_t per,
                                                  uint32_t* out) {
    constexpr int U = 8;
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = beg + per < n ? beg + per : n;
    u32x4 s = u32x4{0u, 0u, 0u, 0u};
    int64_t i = beg + threadIdx.x;
    for (; i + (U - 1) * 256 < end; i += U * 256) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(x + i + u * 256);
#pragma unroll
        for (int u = 0; u < U; ++u) s ^= v[u];
    }
    for (; i < end; i += 256) s ^= __builtin_nontemporal_load(x + i);
    const uint32_t v = s[0] ^ s[1] ^ s[2] ^ s[3];
    if (v == 0x9e3779b9u) out[0] = v;  // practically never true: keeps the loads
}

}  // namespace
}  // namespace dfjk

using namespace dfjk;

extern "C" int dfjk_probe_hbm_read(const void* buf_dev, size_t bytes, double* gbs) {
    clear_error();
    if (!buf_dev || !gbs || bytes < 16 || (reinterpret_cast<uintptr_t>(buf_dev) & 15u)) {
        set_error("dfjk_probe_hbm_read: need a 16-byte aligned device buffer of at least 16 bytes");
        return DFJK_E_INVALID;
    }
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_probe_hbm_read: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    DFJK_HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    DFJK_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    uint32_t* out = nullptr;
    DFJK_HIP_TRY(hipMalloc(&out, 64));
    hipEvent_t e0, e1;
    DFJK_HIP_TRY(hipEventCreate(&e0));
    DFJK_HIP_TRY(hipEventCreate(&e1));
    const int64_t n = (int64_t)(bytes / 16);
    float best = 1e30f;
    // several grid sizes (workgroups per CU); the best rate is the ceiling
    for (int wpc : {2, 4, 8, 16}) {
        const int64_t blocks = (int64_t)cus * wpc;
        const int64_t per = (n + blocks - 1) / blocks;
        for (int rep = 0; rep < 3; ++rep) {  // the first launch warms the clocks
            float ms = 0.f;
            (void)hipEventRecord(e0, nullptr);
            probe_read<<<(unsigned)blocks, 256>>>(static_cast<const u32x4*>(buf_dev), n, per, out);
            (void)hipEventRecord(e1, nullptr);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0 && ms < best) best = ms;
        }
    }
    const hipError_t le = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (le != hipSuccess) {
        set_error("dfjk_probe_hbm_read: launch failed: %s", hipGetErrorString(le));
        return DFJK_E_HIP;
    }
    *gbs = (double)n * 16.0 / (best * 1e6);
    return DFJK_OK;
}

extern "C" int dfjk_probe_mfma(int dtype, double* tflops) {
    clear_error();
    if (!tflops || (dtype != DFJK_F64 && dtype != DFJK_F32 && dtype != DFJK_BF16)) {
        set_error("dfjk_probe_mfma: dtype must be DFJK_F64, DFJK_F32 or DFJK_BF16");
        return DFJK_E_INVALID;
    }
    int ndev = 0, dev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_probe_mfma: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    DFJK_HIP_TRY(hipGetDevice(&dev));
    int cus = 0;
    DFJK_HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    double* out = nullptr;
    DFJK_HIP_TRY(hipMalloc(&out, 64));
    hipEvent_t e0, e1;
    DFJK_HIP_TRY(hipEventCreate(&e0));
    DFJK_HIP_TRY(hipEventCreate(&e1));
    const int blocks = cus * 8, iters = 2000;  // 8 workgroups of 4 waves per CU
    // flop per step times steps per iteration
    const double per = dtype == DFJK_BF16 ? 32768.0 * kAccBf : 2048.0 * (dtype == DFJK_F32 ? kAcc32 : kAcc);
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {  // the first launch warms the clocks
        (void)hipEventRecord(e0, nullptr);
        if (dtype == DFJK_F64) probe_f64<<<blocks, 256>>>(out, iters);
        else if (dtype == DFJK_F32) probe_f32<<<blocks, 256>>>(out, iters);
        else probe_bf16<<<blocks, 256>>>(out, iters);
        (void)hipEventRecord(e1, nullptr);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
    }
    const hipError_t le = hipGetLastError();
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (le != hipSuccess) {
        set_error("dfjk_probe_mfma: launch failed: %s", hipGetErrorString(le));
        return DFJK_E_HIP;
    }
    *tflops = per * iters * (double)blocks * 4.0 / (ms * 1e9);
    return DFJK_OK;
}
