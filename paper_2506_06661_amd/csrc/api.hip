// C-ABI entry points of libdfjk: argument checks, handle lifetime, dispatch.
#include <cstdarg>
#include <cstring>
#include <new>

#include "internal.h"

namespace dfjk {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int DevBuf::ensure(size_t want) {
    if (want <= bytes && ptr) return DFJK_OK;
    if (fixed) {
        set_error("the call needs %zu bytes of a workspace buffer reserved at init with %zu "
                  "(raise max_ncol / max_ndm in dfjk_options)", want, bytes);
        return DFJK_E_INVALID;
    }
    release();
    if (want == 0) want = 256;
    if (hipMalloc(&ptr, want) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
        bytes = 0;
        set_error("device allocation of %zu bytes failed", want);
        return DFJK_E_OOM;
    }
    bytes = want;
    return DFJK_OK;
}

void DevBuf::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

// Reserve every workspace buffer for the sizes the options allow, make the
// 16-bit copy of B if the handle uses one, then fix the buffers so that no
// later call allocates.
static int reserve_all(dfjk_ctx* h) {
    int rc;
    if ((rc = j_reserve(h, h->opts.max_ndm))) return rc;
    if ((rc = k_reserve(h, h->opts.max_ncol))) return rc;
    if ((h->dtype == DFJK_BF16 || h->dtype == DFJK_F16) && h->opts.k16) {
        if ((rc = k16_reserve(h, h->opts.max_ncol))) return rc;
        if ((rc = k16_make_dense(h))) return rc;
    }
    if (h->nao <= 4096 && (rc = scf_reserve(h))) return rc;
    DevBuf* all[] = {&h->dt, &h->rho_part, &h->rho, &h->jpart, &h->dpart, &h->mdt, &h->mpart, &h->mrho,
                     &h->mjpart, &h->X, &h->kpart, &h->ones, &h->Cw, &h->eig, &h->Bdense};
    for (DevBuf* b : all) b->fixed = true;
    return DFJK_OK;
}

// With workspace reserved at init, a call whose K needs more factor columns
// than reserved is refused before anything is enqueued.
static int check_reserved(const dfjk_ctx* h, int64_t ncol, const char* what) {
    if (h->opts.max_ncol > 0 && ncol > h->opts.max_ncol) {
        set_error("%s: needs workspace for %lld factor columns, the handle reserved %d (max_ncol)", what,
                  (long long)ncol, h->opts.max_ncol);
        return DFJK_E_INVALID;
    }
    return DFJK_OK;
}

static int check_handle(const dfjk_ctx* h) {
    if (!h) {
        set_error("null handle");
        return DFJK_E_INVALID;
    }
    return DFJK_OK;
}

}  // namespace dfjk

using namespace dfjk;

extern "C" {

void dfjk_default_options(dfjk_options* o) {
    if (!o) return;
    o->diis_space = 8;
    o->conv_tol = 1e-9;
    o->conv_tol_grad = 3e-5;
    o->max_cycle = 100;
    o->compensated_j = 2;
    o->k16 = 0;
    o->max_ncol = 0;
    o->max_ndm = 8;
}

const char* dfjk_last_error(void) { return g_err; }

int dfjk_init(dfjk_handle* out, const void* B_dev, int dtype, int64_t nao, int64_t naux, int64_t ldB,
              void* stream, const dfjk_options* opts) {
    clear_error();
    if (!out) {
        set_error("dfjk_init: null handle pointer");
        return DFJK_E_INVALID;
    }
    *out = nullptr;
    if (!B_dev) {
        set_error("dfjk_init: null B");
        return DFJK_E_INVALID;
    }
    if (dtype < DFJK_F64 || dtype > DFJK_F16) {
        set_error("dfjk_init: unknown dtype %d", dtype);
        return DFJK_E_INVALID;
    }
    if (nao < 1 || nao > 65535 || naux < 1 || naux > (int64_t(1) << 31)) {
        set_error("dfjk_init: nao=%lld naux=%lld out of range", (long long)nao, (long long)naux);
        return DFJK_E_INVALID;
    }
    const int64_t npair = nao * (nao + 1) / 2;
    if (ldB < npair) {
        set_error("dfjk_init: ldB=%lld < nao(nao+1)/2=%lld", (long long)ldB, (long long)npair);
        return DFJK_E_INVALID;
    }
    dfjk_options o;
    if (opts)
        o = *opts;
    else
        dfjk_default_options(&o);
    if (o.diis_space < 1 || o.diis_space > 15 || o.max_cycle < 1 || o.compensated_j < 0 || o.compensated_j > 2 ||
        o.k16 < 0 || o.k16 > 1 || o.max_ncol < 0 || o.max_ncol > nao || o.max_ndm < 1) {
        set_error("dfjk_init: options out of range (diis_space 1..15, compensated_j 0..2, k16 0..1, "
                  "max_ncol 0..nao, max_ndm >= 1)");
        return DFJK_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_init: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    dfjk_ctx* h = new (std::nothrow) dfjk_ctx();
    if (!h) {
        set_error("dfjk_init: host allocation failed");
        return DFJK_E_OOM;
    }
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        set_error("dfjk_init: hipGetDevice failed");
        return DFJK_E_HIP;
    }
    h->stream = (hipStream_t)stream;
    h->B = B_dev;
    h->dtype = dtype;
    h->nao = nao;
    h->naux = naux;
    h->ldB = ldB;
    h->npair = npair;
    h->opts = o;
    int rc = j_setup(h);
    if (rc == DFJK_OK && h->opts.max_ncol > 0) rc = reserve_all(h);
    if (rc != DFJK_OK) {
        dfjk_destroy(h);
        return rc;
    }
    *out = h;
    return DFJK_OK;
}

int dfjk_update_B(dfjk_handle h) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!h->dense_ready) return DFJK_OK;  // nothing derived from B's contents yet
    return k16_make_dense(h);
}

int dfjk_build_J(dfjk_handle h, const double* D_dev, double* J_dev, double* rho_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!D_dev || !J_dev) {
        set_error("dfjk_build_J: null D or J");
        return DFJK_E_INVALID;
    }
    return j_build(h, D_dev, J_dev, rho_dev, nullptr);
}

int dfjk_form_B(int64_t naux, int64_t ncol, double* M_dev, double* Q_dev, int64_t ldQ, void* stream) {
    clear_error();
    if (naux < 1 || ncol < 1 || ldQ < ncol || !M_dev || !Q_dev) {
        set_error("dfjk_form_B: need naux >= 1, ncol >= 1, ldQ >= ncol and non-null M, Q");
        return DFJK_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_form_B: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    return form_B(naux, ncol, M_dev, Q_dev, ldQ, (hipStream_t)stream);
}

int dfjk_build_J_multi(dfjk_handle h, int64_t ndm, const double* D_dev, double* J_dev, double* rho_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (ndm < 1 || !D_dev || !J_dev) {
        set_error("dfjk_build_J_multi: ndm must be >= 1 and D, J non-null");
        return DFJK_E_INVALID;
    }
    return j_build_multi(h, ndm, D_dev, J_dev, rho_dev);
}

int dfjk_build_J_diag(dfjk_handle h, const double* D_dev, double* J_dev, double* rho_dev, double* diag_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!D_dev || !J_dev || !diag_dev) {
        set_error("dfjk_build_J_diag: null D, J or diag");
        return DFJK_E_INVALID;
    }
    return j_build(h, D_dev, J_dev, rho_dev, diag_dev);
}

int dfjk_build_K_factored(dfjk_handle h, const double* C_dev, int64_t ncol, const double* sign_dev,
                          double scale, double* K_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!C_dev || !K_dev) {
        set_error("dfjk_build_K_factored: null C or K");
        return DFJK_E_INVALID;
    }
    if (ncol < 1 || ncol > h->nao) {
        set_error("dfjk_build_K_factored: ncol=%lld outside [1, nao=%lld]", (long long)ncol,
                  (long long)h->nao);
        return DFJK_E_INVALID;
    }
    if (int rc = check_reserved(h, ncol, "dfjk_build_K_factored")) return rc;
    return k_build_factored(h, C_dev, ncol, sign_dev, scale, K_dev);
}

int dfjk_build_K_pair(dfjk_handle h, const double* L_dev, const double* R_dev, int64_t ncol, int sym,
                      double scale, double* K_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!L_dev || !R_dev || !K_dev) {
        set_error("dfjk_build_K_pair: null L, R or K");
        return DFJK_E_INVALID;
    }
    if (ncol < 1 || ncol > h->nao) {
        set_error("dfjk_build_K_pair: ncol=%lld outside [1, nao=%lld]", (long long)ncol, (long long)h->nao);
        return DFJK_E_INVALID;
    }
    if (sym != 0 && sym != 1) {
        set_error("dfjk_build_K_pair: sym=%d is neither 0 nor 1", sym);
        return DFJK_E_INVALID;
    }
    if (int rc = check_reserved(h, 2 * ncol, "dfjk_build_K_pair")) return rc;
    return k_build_pair(h, L_dev, R_dev, ncol, sym, scale, K_dev);
}

int dfjk_build_K(dfjk_handle h, const double* Cocc_dev, int64_t nocc, const double* D_dev,
                 double* K_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!K_dev) {
        set_error("dfjk_build_K: null K");
        return DFJK_E_INVALID;
    }
    if (Cocc_dev) {
        if (nocc < 1 || nocc > h->nao) {
            set_error("dfjk_build_K: nocc=%lld outside [1, nao=%lld]", (long long)nocc,
                      (long long)h->nao);
            return DFJK_E_INVALID;
        }
        if (int rc = check_reserved(h, nocc, "dfjk_build_K")) return rc;
        return k_build_factored(h, Cocc_dev, nocc, nullptr, 2.0, K_dev);
    }
    if (!D_dev) {
        set_error("dfjk_build_K: both Cocc and D are null");
        return DFJK_E_INVALID;
    }
    if (int rc = check_reserved(h, h->nao, "dfjk_build_K (from D)")) return rc;
    return k_build_from_D(h, D_dev, K_dev);
}

int dfjk_scf_step(dfjk_handle h, const double* H_dev, double* D_dev, double* Cocc_dev, int64_t nocc,
                  int flags, dfjk_scf_info* info) {
    static_assert(sizeof(dfjk_scf_info) == 6 * sizeof(double) + 2 * sizeof(int), "record layout");
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!H_dev || !D_dev || !Cocc_dev) {
        set_error("dfjk_scf_step: null H, D or Cocc");
        return DFJK_E_INVALID;
    }
    if (nocc < 1 || nocc > h->nao) {
        set_error("dfjk_scf_step: nocc=%lld outside [1, nao=%lld]", (long long)nocc, (long long)h->nao);
        return DFJK_E_INVALID;
    }
    if (flags & ~DFJK_SCF_C_VALID) {
        set_error("dfjk_scf_step: unknown flags 0x%x", flags);
        return DFJK_E_INVALID;
    }
    if (int rc = check_reserved(h, (flags & DFJK_SCF_C_VALID) ? nocc : h->nao, "dfjk_scf_step")) return rc;
    return scf_step(h, H_dev, D_dev, Cocc_dev, nocc, flags, info);
}

int dfjk_aufbau(dfjk_handle h, const double* F_dev, int64_t nocc, double* Cocc_dev, double* D_dev) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!F_dev || !Cocc_dev || nocc < 1 || nocc > h->nao) {
        set_error("dfjk_aufbau: null F or Cocc, or nocc outside [1, nao]");
        return DFJK_E_INVALID;
    }
    return aufbau(h, F_dev, nocc, Cocc_dev, D_dev);
}

int dfjk_scf_reset(dfjk_handle h) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    return scf_reset(h);
}

int dfjk_tile_count(int kernel) {
    clear_error();
    if (kernel == DFJK_TILE_GEMM1) return k_tile_count();
    if (kernel == DFJK_TILE_J_OUT) return j_out_count();
    if (kernel == DFJK_TILE_K16) return k16_tile_count();
    if (kernel == DFJK_TILE_K16_SYRK) return k16_syrk_tile_count();
    set_error("dfjk_tile_count: unknown kernel %d", kernel);
    return DFJK_E_INVALID;
}

int dfjk_tile_info(int kernel, int index, int* p0, int* p1) {
    clear_error();
    if ((kernel != DFJK_TILE_GEMM1 && kernel != DFJK_TILE_J_OUT && kernel != DFJK_TILE_K16 &&
         kernel != DFJK_TILE_K16_SYRK) ||
        !p0 || !p1) {
        set_error("dfjk_tile_info: unknown kernel or null output");
        return DFJK_E_INVALID;
    }
    if (kernel == DFJK_TILE_K16) {
        if (k16_tile_info(index, p0, p1) != DFJK_OK) {
            set_error("dfjk_tile_info: index %d out of range", index);
            return DFJK_E_INVALID;
        }
        return DFJK_OK;
    }
    if (kernel == DFJK_TILE_K16_SYRK) {
        if (index < 0 || index >= k16_syrk_tile_count()) {
            set_error("dfjk_tile_info: index %d out of range", index);
            return DFJK_E_INVALID;
        }
        *p0 = *p1 = k16_syrk_tile_size(index);
        return DFJK_OK;
    }
    if (kernel == DFJK_TILE_J_OUT) {
        static const int widths[] = {2, 4, 8, 16};
        if (index < 0 || index >= j_out_count()) {
            set_error("dfjk_tile_info: index %d out of range", index);
            return DFJK_E_INVALID;
        }
        *p0 = 512 * widths[index];
        *p1 = 0;
        return DFJK_OK;
    }
    if (k_tile_info(index, p0, p1) != DFJK_OK) {
        set_error("dfjk_tile_info: index %d out of range", index);
        return DFJK_E_INVALID;
    }
    return DFJK_OK;
}

int dfjk_set_tile(dfjk_handle h, int kernel, int index) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    const int count = kernel == DFJK_TILE_GEMM1 ? k_tile_count()
                      : kernel == DFJK_TILE_J_OUT ? j_out_count()
                      : kernel == DFJK_TILE_K16 ? k16_tile_count()
                      : kernel == DFJK_TILE_K16_SYRK ? k16_syrk_tile_count() : 0;
    if (count == 0 || index < -1 || index >= count) {
        set_error("dfjk_set_tile: kernel %d / index %d invalid", kernel, index);
        return DFJK_E_INVALID;
    }
    if (kernel == DFJK_TILE_GEMM1 && index >= 0 && !k_tile_has_dtype(index, h->dtype)) {
        set_error("dfjk_set_tile: GEMM1 tile %d has no form for B dtype %d", index, h->dtype);
        return DFJK_E_DTYPE;
    }
    if (kernel == DFJK_TILE_GEMM1)
        h->g1_tile = index;
    else if (kernel == DFJK_TILE_J_OUT)
        h->jout_tile = index;
    else if (kernel == DFJK_TILE_K16)
        h->k16_tile = index;
    else
        h->k16_syrk_tile = index;
    return DFJK_OK;
}

int dfjk_workspace_bytes(dfjk_handle h, size_t* bytes) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!bytes) {
        set_error("dfjk_workspace_bytes: null output");
        return DFJK_E_INVALID;
    }
    *bytes = h->dt.bytes + h->rho_part.bytes + h->rho.bytes + h->jpart.bytes + h->dpart.bytes + h->mdt.bytes + h->mpart.bytes +
             h->mrho.bytes + h->mjpart.bytes + h->X.bytes +
             h->kpart.bytes + h->ones.bytes + h->Cw.bytes + h->eig.bytes + h->Bdense.bytes;
    return DFJK_OK;
}

static void prof_free(dfjk_ctx* h) {
    for (int p = 0; p < PH_COUNT; ++p) {
        if (h->prof.ev[p]) {
            for (int i = 0; i < 2 * h->prof.cap; ++i) (void)hipEventDestroy(h->prof.ev[p][i]);
            delete[] h->prof.ev[p];
            h->prof.ev[p] = nullptr;
        }
        h->prof.n[p] = 0;
    }
    h->prof.cap = 0;
    h->prof.on = false;
}

int dfjk_profile(dfjk_handle h, int capacity) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (capacity < 0 || capacity > 4096) {
        set_error("dfjk_profile: capacity %d outside [0, 4096]", capacity);
        return DFJK_E_INVALID;
    }
    DFJK_HIP_TRY(hipStreamSynchronize(h->stream));
    prof_free(h);
    if (capacity == 0) return DFJK_OK;
    h->prof.cap = capacity;  // phases before a failing one hold all 2*cap events
    for (int p = 0; p < PH_COUNT; ++p) {
        h->prof.ev[p] = new (std::nothrow) hipEvent_t[2 * capacity];
        if (!h->prof.ev[p]) {
            prof_free(h);
            set_error("dfjk_profile: host allocation failed");
            return DFJK_E_OOM;
        }
        for (int i = 0; i < 2 * capacity; ++i) {
            if (hipEventCreate(&h->prof.ev[p][i]) != hipSuccess) {
                for (int j = 0; j < i; ++j) (void)hipEventDestroy(h->prof.ev[p][j]);
                delete[] h->prof.ev[p];
                h->prof.ev[p] = nullptr;
                prof_free(h);
                set_error("dfjk_profile: hipEventCreate failed");
                return DFJK_E_HIP;
            }
        }
    }
    h->prof.on = true;
    return DFJK_OK;
}

int dfjk_profile_read(dfjk_handle h, double* total_ms, int* counts, int nphase) {
    clear_error();
    if (int rc = check_handle(h)) return rc;
    if (!total_ms || !counts || nphase < 1) {
        set_error("dfjk_profile_read: null output or nphase < 1");
        return DFJK_E_INVALID;
    }
    DFJK_HIP_TRY(hipStreamSynchronize(h->stream));
    for (int p = 0; p < nphase; ++p) {
        total_ms[p] = 0.0;
        counts[p] = 0;
        if (p >= PH_COUNT || !h->prof.on) continue;
        for (int i = 0; i < h->prof.n[p]; ++i) {
            float ms = 0.f;
            DFJK_HIP_TRY(hipEventElapsedTime(&ms, h->prof.ev[p][2 * i], h->prof.ev[p][2 * i + 1]));
            total_ms[p] += ms;
        }
        counts[p] = h->prof.n[p];
        h->prof.n[p] = 0;
    }
    return DFJK_OK;
}

void dfjk_destroy(dfjk_handle h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    prof_free(h);
    h->dt.release();
    h->rho_part.release();
    h->rho.release();
    h->jpart.release();
    h->dpart.release();
    h->mdt.release();
    h->mpart.release();
    h->mrho.release();
    h->mjpart.release();
    h->X.release();
    h->kpart.release();
    h->ones.release();
    h->Cw.release();
    h->eig.release();
    h->Bdense.release();
    delete h;
}

int dfjk_quantize(const double* src_dev, void* dst_dev, int dtype, int64_t n, void* stream) {
    clear_error();
    if (!src_dev || !dst_dev || n < 0) {
        set_error("dfjk_quantize: null pointer or negative n");
        return DFJK_E_INVALID;
    }
    if (dtype < DFJK_F32 || dtype > DFJK_F16) {
        set_error("dfjk_quantize: dtype %d is not a reduced format", dtype);
        return DFJK_E_INVALID;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_quantize: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    return quantize(src_dev, dst_dev, dtype, n, (hipStream_t)stream);
}

}  // extern "C"
