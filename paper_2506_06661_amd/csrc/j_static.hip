// Coulomb build without device allocation: dfjk_build_J's kernels run on a
// workspace carved out of a fixed array in device memory that the library
// holds for the life of the process (one copy per GPU), for callers that
// cannot call hipMalloc (HIP graph capture, tight serving loops, hosts that
// forbid allocation).
//
// The array's host-side name only stands in for it; the device address of
// each GPU's copy comes from hipGetSymbolAddress with that GPU current, once
// per device, and only that address is handed to kernels.
#include <mutex>

#include "internal.h"

namespace dfjk {

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;  // 128 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

inline size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

// Device address of the current GPU's scratch array (looked up once per GPU).
int scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
        (void)hipGetLastError();
        set_error("dfjk_build_J_static: no current HIP device");
        return DFJK_E_NO_DEVICE;
    }
    if (dev >= kMaxDevices) {
        set_error("dfjk_build_J_static: device %d beyond the %d supported", dev, kMaxDevices);
        return DFJK_E_INVALID;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("dfjk_build_J_static: hipGetSymbolAddress of the scratch array failed: %s",
                      hipGetErrorString(e));
            return DFJK_E_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return DFJK_OK;
}

}  // namespace

}  // namespace dfjk

using namespace dfjk;

extern "C" {

size_t dfjk_static_scratch_bytes(void) { return kScratchBytes; }

int dfjk_build_J_static(const void* B_dev, int dtype, int64_t nao, int64_t naux, int64_t ldB, void* stream,
                        const dfjk_options* opts, const double* D_dev, double* J_dev, double* rho_dev) {
    clear_error();
    if (!B_dev || !D_dev || !J_dev) {
        set_error("dfjk_build_J_static: null B, D or J");
        return DFJK_E_INVALID;
    }
    if (dtype < DFJK_F64 || dtype > DFJK_F16) {
        set_error("dfjk_build_J_static: unknown dtype %d", dtype);
        return DFJK_E_INVALID;
    }
    if (nao < 1 || nao > 65535 || naux < 1 || naux > (int64_t(1) << 31)) {
        set_error("dfjk_build_J_static: nao=%lld naux=%lld out of range", (long long)nao, (long long)naux);
        return DFJK_E_INVALID;
    }
    const int64_t npair = nao * (nao + 1) / 2;
    if (ldB < npair) {
        set_error("dfjk_build_J_static: ldB=%lld < nao(nao+1)/2=%lld", (long long)ldB, (long long)npair);
        return DFJK_E_INVALID;
    }
    // A handle on the stack: same fields and kernels as dfjk_init + dfjk_build_J,
    // its workspace pointing into the scratch array (nothing here allocates).
    dfjk_ctx h;
    h.stream = (hipStream_t)stream;
    h.B = B_dev;
    h.dtype = dtype;
    h.nao = nao;
    h.naux = naux;
    h.ldB = ldB;
    h.npair = npair;
    if (opts)
        h.opts = *opts;
    else
        dfjk_default_options(&h.opts);
    if (h.opts.compensated_j < 0 || h.opts.compensated_j > 2) {
        set_error("dfjk_build_J_static: compensated_j must be 0, 1 or 2");
        return DFJK_E_INVALID;
    }
    JWork w;
    j_plan(&h, &w);
    // the handle reserves pass-2 partials for every column width; this build
    // uses the default width only
    w.jpart = sizeof(double) * (size_t)npair * (size_t)j_splits_used(&h);
    const size_t o_rho_part = align256(w.dt);
    const size_t o_rho = o_rho_part + align256(w.rho_part);
    const size_t o_jpart = o_rho + align256(w.rho);
    const size_t need = o_jpart + align256(w.jpart);
    if (need > kScratchBytes) {
        set_error("dfjk_build_J_static: nao=%lld, naux=%lld need %zu bytes of scratch, more than the "
                  "%zu the library holds; use dfjk_init + dfjk_build_J",
                  (long long)nao, (long long)naux, need, kScratchBytes);
        return DFJK_E_INVALID;
    }
    void* base = nullptr;
    if (int rc = scratch_address(&base)) return rc;
    unsigned char* s = static_cast<unsigned char*>(base);
    h.dt.ptr = s;
    h.dt.bytes = w.dt;
    h.rho_part.ptr = s + o_rho_part;
    h.rho_part.bytes = w.rho_part;
    h.rho.ptr = s + o_rho;
    h.rho.bytes = w.rho;
    h.jpart.ptr = s + o_jpart;
    h.jpart.bytes = w.jpart;
    // every workspace element a build reads is first written by that build
    // (packed density, per-chunk and per-split partial sums), so the scratch
    // left by an earlier call needs no clearing
    const int rc = j_build(&h, D_dev, J_dev, rho_dev, nullptr);
    // the stack handle only borrowed the scratch: forget it before h goes
    h.dt.ptr = h.rho_part.ptr = h.rho.ptr = h.jpart.ptr = nullptr;
    return rc;
}

}  // extern "C"
