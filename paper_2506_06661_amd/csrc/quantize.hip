// One-step round-to-nearest-even conversion of FP64 values to FP32, BF16 or
// FP16, used to store B at reduced precision.
//
// FP32: the hardware double -> float conversion rounds to nearest even.
// BF16 / FP16: the double is first narrowed to float with round-to-odd, then
// rounded to nearest even in the 16-bit format.  Round-to-odd into a format
// with at least two more significand bits than the target makes the second
// rounding equal to a single correct rounding (Boldo and Melquiond, "Emulation
// of FMA and correctly rounded sums: proved algorithms using rounding to odd",
// IEEE Trans. Computers 57(4), 2008); float carries 24 bits against 8 (bf16)
// and 11 (fp16), and covers both formats' subnormal ranges.
#include "internal.h"
#include "numerics.h"

namespace dfjk {

namespace {

__global__ void quantize_kernel(const double* __restrict__ src, void* __restrict__ dst, int dtype,
                                int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const double x = src[i];
        if (dtype == DFJK_F32) {
            static_cast<float*>(dst)[i] = (float)x;
        } else if (dtype == DFJK_BF16) {
            static_cast<uint16_t*>(dst)[i] = float_to_bf16_rne(to_float_round_odd(x));
        } else {
            const _Float16 hv = (_Float16)to_float_round_odd(x);
            static_cast<_Float16*>(dst)[i] = hv;
        }
    }
}

}  // namespace

int quantize(const double* src, void* dst, int dtype, int64_t n, hipStream_t s) {
    if (n == 0) return DFJK_OK;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    quantize_kernel<<<dim3((unsigned)blocks), 256, 0, s>>>(src, dst, dtype, n);
    DFJK_LAUNCH_CHECK("quantize_kernel");
    return DFJK_OK;
}

}  // namespace dfjk
