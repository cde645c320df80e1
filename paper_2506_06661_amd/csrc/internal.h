// Internal declarations shared by the libdfjk translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/dfjk.h"

namespace dfjk {

// Thread-local error text behind dfjk_last_error().
void set_error(const char* fmt, ...);
void clear_error();

#define DFJK_HIP_TRY(expr)                                                                     \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) {                                                                \
            ::dfjk::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                              __LINE__);                                                       \
            return DFJK_E_HIP;                                                                 \
        }                                                                                      \
    } while (0)

#define DFJK_LAUNCH_CHECK(what)                                                                   \
    do {                                                                                          \
        hipError_t e_ = hipGetLastError();                                                        \
        if (e_ != hipSuccess) {                                                                   \
            ::dfjk::set_error("launch of %s failed: %s", what, hipGetErrorString(e_));            \
            return DFJK_E_HIP;                                                                    \
        }                                                                                         \
    } while (0)

// Grow-only device buffer owned by a handle.  Once `fixed` (workspace
// reserved at init), ensure() never allocates: a larger request fails with
// DFJK_E_INVALID.
struct DevBuf {
    void* ptr = nullptr;
    size_t bytes = 0;
    bool fixed = false;
    int ensure(size_t want);  // returns DFJK_OK / DFJK_E_OOM / DFJK_E_INVALID
    void release();
};

// Per-phase event timing (dfjk_profile): a ring of event pairs per phase,
// recorded on the handle's stream around each kernel when enabled.
enum ProfPhase { PH_J = 0, PH_J_RHO, PH_J_OUT, PH_K, PH_K_GEMM1, PH_K_SYRK, PH_K_FINISH, PH_COUNT };

struct Prof {
    bool on = false;
    int cap = 0;
    hipEvent_t* ev[PH_COUNT] = {};  // 2*cap events per phase
    int n[PH_COUNT] = {};           // pairs recorded since the last read
    void begin(int ph, hipStream_t s) {
        if (on && n[ph] < cap) (void)hipEventRecord(ev[ph][2 * n[ph]], s);
    }
    void end(int ph, hipStream_t s) {
        if (on && n[ph] < cap) (void)hipEventRecord(ev[ph][2 * n[ph] + 1], s), ++n[ph];
    }
};

}  // namespace dfjk

struct dfjk_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    const void* B = nullptr;
    int dtype = DFJK_F64;
    int64_t nao = 0, naux = 0, ldB = 0, npair = 0;
    dfjk_options opts{};

    // J workspace
    dfjk::DevBuf dt;        // packed density, npair doubles (plus FP32 hi/lo for reduced B)
    dfjk::DevBuf rho_part;  // naux x j_chunks partial sums
    dfjk::DevBuf rho;       // naux
    dfjk::DevBuf jpart;     // j_splits x npair partial sums
    dfjk::DevBuf dpart;     // j_splits x npair partial sums of B^2 (DF diagonal, on request)
    dfjk::DevBuf mdt, mpart, mrho, mjpart;  // several-density J workspace (on request)
    int j_chunks = 1, j_splits = 1;

    // K workspace
    dfjk::DevBuf X;         // (naux * ncol) x ldx, element type per path
    dfjk::DevBuf kpart;     // split partial tiles
    dfjk::DevBuf ones;      // default +1 signs
    dfjk::DevBuf Cw;        // staged (converted) C
    dfjk::DevBuf eig;       // eigen-work for the D path
    dfjk::DevBuf Bdense;    // dense 16-bit copy of B for the 16-bit exchange (opts.k16)
    bool dense_ready = false;

    int g1_tile = -1;       // GEMM1 tile index (-1: heuristic)
    int jout_tile = -1;     // J pass-2 column width index (-1: default)
    int k16_tile = -1;      // 16-bit GEMM1 column tile index (-1: default)
    int k16_syrk_tile = -1; // 16-bit SYRK output tile index (-1: default)

    // SCF state (scf.hip): iterations done, DIIS vectors stored
    int scf_iter = 0, scf_count = 0;
    bool scf_ready = false;
    bool scf_v_warm = false;  // eigensolver buffer V holds the last SCF eigenbasis

    dfjk::Prof prof;
};

namespace dfjk {

// J launchers (j_kernels.hip)
struct JWork {  // bytes of each J workspace buffer for a handle's sizes
    size_t dt, rho_part, rho, jpart;
};
void j_plan(dfjk_ctx* h, JWork* w);  // also sets h->j_chunks, h->j_splits
int64_t j_splits_used(const dfjk_ctx* h);  // pass-2 row slices j_build uses (after j_plan)
int j_setup(dfjk_ctx* h);
int j_build(dfjk_ctx* h, const double* D, double* J, double* rho_out, double* diag);
int j_build_multi(dfjk_ctx* h, int64_t ndm, const double* D, double* J, double* rho_out);
int form_B(int64_t naux, int64_t ncol, double* M, double* Q, int64_t ldQ, hipStream_t st);
int j_out_count();

// Workspace reservation at init (options max_ncol > 0): each build path
// sizes its buffers with the same function it uses when it runs.
int j_reserve(dfjk_ctx* h, int64_t max_ndm);
int k_reserve(dfjk_ctx* h, int64_t max_ncol);
int k16_reserve(dfjk_ctx* h, int64_t max_ncol);
int k16_make_dense(dfjk_ctx* h);
int scf_reserve(dfjk_ctx* h);

// K launchers (k_kernels.hip)
int k_build_factored(dfjk_ctx* h, const double* C, int64_t ncol, const double* sign, double scale,
                     double* K);
int k_build_pair(dfjk_ctx* h, const double* L, const double* R, int64_t ncol, int sym, double scale,
                 double* K);
int k_build_from_D(dfjk_ctx* h, const double* D, double* K);
int k_build_16(dfjk_ctx* h, const double* C, int64_t ncol, double scale, double* K);
int scf_step(dfjk_ctx* h, const double* H, double* D, double* C, int64_t nocc, int flags,
             dfjk_scf_info* info);
int scf_reset(dfjk_ctx* h);
int scf_tail(dfjk_ctx* h, const double* H, double* D, double* C, int64_t nocc, const double* J,
             const double* K, const void** rec);
int scf_read_info(dfjk_ctx* h, const void* rec, dfjk_scf_info* info);
int aufbau(dfjk_ctx* h, const double* F, int64_t nocc, double* C, double* D);
int k_tile_count();
bool k_tile_has_dtype(int t, int dtype);  // GEMM1 tile t has a form for B of this dtype
int k_tile_info(int t, int* ni, int* wm);
int k16_tile_count();
int k16_tile_info(int t, int* cols, int* rows);
int k16_syrk_tile_count();
int k16_syrk_tile_size(int t);

// Batched builds (batch.hip drives; j_kernels.hip / k_kernels.hip launch).
// One descriptor per molecule; all pointers are device pointers.
struct MolDesc {
    const void* B;
    int64_t ldB, nao, naux, npair, nocc;
    const double* D;
    const double* C;
    double* J;
    double* K;
    double* dt;        // npair
    double* rho_part;  // naux x j_chunks
    double* rho;       // naux
    double* jpart;     // j_splits x npair
    float* Cf;         // nao x nocc, rows ldcf apart
    float* X;          // naux*nocc x nao, rows ldx apart
    int64_t ldcf, ldx; // nocc and nao rounded up to whole 16-byte vectors
    float* kpart;      // nsplit x ntl x 128 x 128
    int64_t j_chunks, j_splits, chunk, prows;
    int64_t nsplit, kchunk, ntl;
    int64_t g1_nib, g1_nmb;
    int vec;
    // 16-bit exchange (BF16 / FP16 B on the 16-bit matrix cores)
    void* Ct16;        // ncp16 x rs16, C^T rounded to the storage format
    void* X16;         // naux x nao x ncp16
    float* kpart16;    // nsplit16 x ntl x 128 x 128
    int64_t ncp16, ldd16, rs16, pchunk16, nsplit16;
};

// A phase launch over a subset of molecules: ids (device, n entries, in
// dispatch order) and prefix (device, n+1 entries) of per-molecule block counts.
struct PhaseList {
    const int* ids;
    const int64_t* prefix;
    int n;
    int64_t nblk;
};

enum BatchPhaseKind {
    BP_PACK = 0, BP_RHO, BP_RHO_FIN, BP_OUT, BP_JFIN, BP_CF32, BP_SYRK, BP_KFIN,
    BP_CT16, BP_G16, BP_SYRK16, BP_KFIN16, BP_NKIND
};
int j_batch_phase(hipStream_t st, int kind, int dtype, const MolDesc* mols, const PhaseList& pl);
int k_batch_phase(hipStream_t st, int kind, int dtype, const MolDesc* mols, const PhaseList& pl);
int k_batch_gemm1(hipStream_t st, int dtype, int tile, const MolDesc* mols, const PhaseList& pl);
int pick_tile(int64_t ncol);
// 16-bit exchange over a batch (k16.hip): per-molecule geometry (sets the
// *16 fields except the pointers; bytes of Ct16, X16, kpart16), the GEMM1
// bucket of a molecule, the blocks of a phase, and the launch of a phase
// (BP_CT16, BP_G16 with its bucket, BP_SYRK16, BP_KFIN16).
void k16_batch_geometry(MolDesc& d, size_t* ct_bytes, size_t* x_bytes, size_t* kpart_bytes);
int k16_batch_bucket(const MolDesc& d);
int64_t k16_batch_blocks(int kind, int bucket, const MolDesc& d);
int k16_batch_phase(hipStream_t st, int kind, int bucket, int dtype, const MolDesc* mols, const PhaseList& pl);
int tile_nb(int tile, int64_t nao, int64_t ncol, int64_t* nib, int64_t* nmb);

// quantisation (quantize.hip)
int quantize(const double* src, void* dst, int dtype, int64_t n, hipStream_t s);

inline size_t dtype_size(int dt) { return dt == DFJK_F64 ? 8 : dt == DFJK_F32 ? 4 : 2; }

}  // namespace dfjk
