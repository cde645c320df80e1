/*
 * dfjk.h -- C-ABI of libdfjk, the density-fitted Coulomb/exchange (J/K)
 * build for AMD Instinct MI355X (gfx950).
 *
 * What it computes (paper Sec. IV.C.2, Eq. eq:df:eri and the metric
 * factorisation after it): electron-repulsion integrals approximated as
 *     (mu nu|ka la) = sum_P B[P, mu nu] B[P, ka la],   B = L^-1 (Q|mu nu),
 * and, for a density matrix D, the Coulomb and exchange matrices that the
 * paper's get_jk(mol, dm) returns (Sec. II and Sec. III):
 *     J[mu,nu] = sum_P rho_P B_P[mu,nu],   rho_P = sum_{ka,la} B_P[ka,la] D[ka,la]
 *     K[mu,nu] = sum_P (B_P D B_P)[mu,nu]
 * With occupied orbitals C (nao x nocc) and D = 2 C C^T this is
 *     K = 2 sum_P X_P X_P^T,   X_P = B_P C.
 *
 * Layouts (all row-major, all device pointers unless stated):
 *   B   naux rows of length ldB >= npair = nao(nao+1)/2; row P holds the
 *       packed lower triangle of the symmetric B_P, element (mu, nu) at
 *       p = max(mu,nu)*(max(mu,nu)+1)/2 + min(mu,nu) (numpy.tril_indices
 *       order, the aosym='s2' layout of the paper's three-index arrays).
 *       Columns p >= npair are never read.  Element type per dfjk_dtype.
 *   D, J, K, H, F   nao x nao FP64.
 *   C   nao x nocc FP64 (row mu, column i).
 *
 * Ownership: the caller owns every array.  dfjk_init borrows B for the life
 * of the handle and never writes it.  The handle owns its workspace, which
 * it allocates in dfjk_init and, when a call needs more (a larger nocc),
 * in that call.
 *
 * Streams: every call enqueues its work on the stream given to dfjk_init
 * and returns without waiting, except where stated.
 *
 * Errors: 0 on success, a negative DFJK_E_* code on failure (nothing is
 * enqueued when argument checks fail), a positive DFJK_W_* code for a
 * warning.  No call aborts the process; dfjk_last_error() returns a
 * message for the calling thread's most recent failure.
 */
#ifndef DFJK_H
#define DFJK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfjk_ctx* dfjk_handle;

/* Element type of B. */
typedef enum {
    DFJK_F64 = 0,
    DFJK_F32 = 1,
    DFJK_BF16 = 2,
    DFJK_F16 = 3
} dfjk_dtype;

enum {
    DFJK_OK = 0,
    DFJK_E_INVALID = -1,   /* bad argument: null pointer, size out of range */
    DFJK_E_NO_DEVICE = -2, /* no usable GPU */
    DFJK_E_HIP = -3,       /* a HIP runtime call or kernel launch failed */
    DFJK_E_OOM = -4,       /* device allocation failed */
    DFJK_E_DTYPE = -5,     /* operation not provided for this B dtype */
    DFJK_E_NONFINITE = -6, /* non-finite value met where it must not be */
    DFJK_W_NOT_CONVERGED = 1
};

/* Options; pass NULL to dfjk_init for the defaults shown. */
typedef struct {
    int diis_space;       /* Pulay DIIS history length (8) */
    double conv_tol;      /* |E_k - E_{k-1}| threshold (1e-9) */
    double conv_tol_grad; /* ||FD - DF||_F threshold (3e-5) */
    int max_cycle;        /* SCF iteration cap (100) */
    int compensated_j;    /* reduced-precision B: 1 = two-term FP32 sums in J (1) */
} dfjk_options;

/* Fills *o with the defaults. */
void dfjk_default_options(dfjk_options* o);

/*
 * Create a handle over B.
 *   h       out: the new handle (host pointer to a handle variable).
 *   B_dev   device pointer to B (see layout above), dtype `dtype`.
 *   nao     number of basis functions, 1 <= nao <= 65535.
 *   naux    number of auxiliary functions, >= 1.
 *   ldB     row stride of B in elements, >= nao(nao+1)/2.
 *   stream  hipStream_t to enqueue on (NULL = the default stream).
 *   opts    options or NULL.
 * Errors: DFJK_E_INVALID, DFJK_E_NO_DEVICE, DFJK_E_OOM, DFJK_E_HIP.
 */
int dfjk_init(dfjk_handle* h, const void* B_dev, int dtype, int64_t nao, int64_t naux,
              int64_t ldB, void* stream, const dfjk_options* opts);

/*
 * J = sum_P rho_P B_P with rho_P = sum_{ka,la} B_P[ka,la] D[ka,la]
 * (paper Eq. eq:df:eri contracted with D).  D may be any real nao x nao
 * matrix; J is written in full (both triangles).  rho_dev, if non-NULL,
 * receives the naux values rho_P (FP64).  Deterministic: the same inputs
 * give bitwise the same J.
 */
int dfjk_build_J(dfjk_handle h, const double* D_dev, double* J_dev, double* rho_dev);

/*
 * Exchange matrix, written in full (both triangles):
 *   Cocc_dev != NULL: K = 2 sum_P (B_P C)(B_P C)^T with C = Cocc_dev
 *                     (nao x nocc, 1 <= nocc <= nao), i.e. K for D = 2 C C^T.
 *   Cocc_dev == NULL: K = sum_P B_P D B_P for the symmetric D_dev, through
 *                     the signed eigen-factors of D (paper Sec. IV.A.1: a
 *                     guess density need not be idempotent).
 * Deterministic.
 */
int dfjk_build_K(dfjk_handle h, const double* Cocc_dev, int64_t nocc, const double* D_dev,
                 double* K_dev);

/*
 * Exchange with per-column signs: K = s * sum_P sum_i sign_i X_P[:,i] X_P[:,i]^T,
 * X_P = B_P C, sign_dev[i] in {+1, -1} (FP64, nocc entries, NULL = all +1).
 * Used by the D path (signed eigen-factors) and available to callers that
 * factor their own density.
 */
int dfjk_build_K_factored(dfjk_handle h, const double* C_dev, int64_t ncol,
                          const double* sign_dev, double scale, double* K_dev);

/*
 * Per-kernel timing.  dfjk_profile(h, cap) (cap > 0) makes later calls record
 * HIP events on the handle's stream around each phase, for up to cap calls
 * per phase; cap = 0 turns it off.  dfjk_profile_read waits for the stream
 * and returns, per phase, the summed milliseconds and the number of timed
 * launches since the last read.  Phases, in order: 0 J build, 1 J pass 1
 * (rho), 2 J pass 2 (J), 3 K build, 4 K GEMM1 (X = B C), 5 K GEMM2 (SYRK
 * splits), 6 K split reduction.
 */
int dfjk_profile(dfjk_handle h, int capacity);
int dfjk_profile_read(dfjk_handle h, double* total_ms, int* counts, int nphase);

/*
 * Tile shapes (for autotuning).  DFJK_TILE_GEMM1 selects the X = B_P C
 * kernel's workgroup tile.  dfjk_tile_count returns the number of compiled
 * tiles; dfjk_tile_info gives tile `index` as (p0, p1) = (row tiles of 16
 * occupied orbitals, column tiles of 16 basis functions per wavefront);
 * dfjk_set_tile makes the handle use tile `index` (-1 = built-in heuristic).
 * Every tile computes the same X up to summation order.
 */
enum { DFJK_TILE_GEMM1 = 0 };
int dfjk_tile_count(int kernel);
int dfjk_tile_info(int kernel, int index, int* p0, int* p1);
int dfjk_set_tile(dfjk_handle h, int kernel, int index);

/* Device workspace currently held by the handle, in bytes. */
int dfjk_workspace_bytes(dfjk_handle h, size_t* bytes);

/* Release the handle and its workspace (waits for its stream). NULL is a no-op. */
void dfjk_destroy(dfjk_handle h);

/* Message of the calling thread's most recent failure ("" if none). */
const char* dfjk_last_error(void);

/*
 * Round n FP64 values to `dtype` with one round-to-nearest-even step
 * (never through an intermediate format), writing the packed elements to
 * dst_dev (4 bytes each for DFJK_F32, 2 for DFJK_BF16/DFJK_F16, gradual
 * underflow, overflow to infinity).  Used to store B at reduced precision.
 */
int dfjk_quantize(const double* src_dev, void* dst_dev, int dtype, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DFJK_H */
