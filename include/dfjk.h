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
 * of the handle and never writes it (with the k16 option the handle also keeps
 * a dense 16-bit copy of it).  The handle owns its workspace, which
 * it allocates in dfjk_init and, when a call needs more (a larger nocc),
 * in that call -- unless dfjk_options.max_ncol > 0, which reserves all of it
 * in dfjk_init.
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

/*
 * Options; pass NULL to dfjk_init for the defaults shown.  There is no
 * determinism switch: every build sums its split partials in a fixed order,
 * so J and K are bitwise reproducible for a given tile choice.  Tile choices
 * are made per handle with dfjk_set_tile and, for batches, by
 * dfjk_batch_autotune, whose cache_path argument is the tuning cache.
 */
typedef struct {
    int diis_space;       /* Pulay DIIS history length (8) */
    double conv_tol;      /* |E_k - E_{k-1}| threshold (1e-9) */
    double conv_tol_grad; /* ||FD - DF||_F threshold (3e-5) */
    int max_cycle;        /* SCF iteration cap (100) */
    int compensated_j;    /* reduced-precision B, J accumulation: 2 = FP64 (default),
                             1 = compensated FP32 (Dot2), 0 = plain FP32 */
    int k16;              /* BF16/FP16 B, exchange from C: 1 = 16-bit matrix cores
                             (with the default GEMM1 tile the handle keeps a
                             dense 16-bit copy of B, naux * ceil64(nao) *
                             (ceil64(nao) + 64) elements, made in dfjk_init
                             when max_ncol > 0, else on the first K call; K
                             then uses B's contents as they were when the copy
                             was made: call dfjk_update_B after changing them;
                             the packed-triangle GEMM1 tiles, DFJK_TILE_K16
                             8..12, read B itself and use no copy; C and X
                             rounded to the 16-bit format); 0 = B dequantised
                             on load, FP32 matrix cores (default) */
    int max_ncol;         /* 0 (default): workspace grows on demand, so a call
                             may allocate.  1..nao: dfjk_init reserves every
                             workspace buffer for K with up to max_ncol columns
                             of C (two-factor K: up to max_ncol / 2; K from a
                             density, and SCF steps without valid Cocc, need
                             max_ncol = nao), J of up to max_ndm densities at
                             a time, the DF diagonal and the SCF state; later
                             calls never allocate (they can be captured in a
                             HIP graph), and one that would need more returns
                             DFJK_E_INVALID before enqueuing anything */
    int max_ndm;          /* densities per dfjk_build_J_multi pass reserved
                             with max_ncol > 0 (8; at most 8 are used) */
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
 * dfjk_build_J without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, hosts that
 * forbid hipMalloc.  Takes dfjk_init's arguments (B_dev, dtype, nao, naux,
 * ldB, stream, opts; only opts->compensated_j is used, NULL = defaults) and
 * dfjk_build_J's (D_dev, J_dev, rho_dev), and computes bitwise what a handle
 * made with them would.  Its workspace is a fixed array of
 * dfjk_static_scratch_bytes() bytes (128 MiB) in device memory that the
 * library holds on each GPU it runs on until the process ends; sizes whose
 * workspace does not fit are rejected with DFJK_E_INVALID before anything is
 * enqueued.  The workspace is the packed density (3 npair doubles), naux x
 * (a few) partial sums of rho and the pass-2 partials (npair doubles per row
 * slice: about 4096 * 2048 / npair slices for FP64 B, more for reduced B):
 * nao = 1024 with naux = 4096 and FP64 B needs 80 MB and fits; the same size
 * with FP32 or 16-bit B, or nao = 2048, does not.  Every call on one GPU shares that
 * array, so calls that overlap on one GPU (two streams, two threads) race and
 * give wrong results: serialise them.  Each call writes every workspace
 * element it reads, so no clearing is needed between calls.  The device is
 * the current one; its scratch address is looked up on the first call there.
 * Asynchronous on `stream`.  Errors: as dfjk_init and dfjk_build_J.
 */
int dfjk_build_J_static(const void* B_dev, int dtype, int64_t nao, int64_t naux, int64_t ldB, void* stream,
                        const dfjk_options* opts, const double* D_dev, double* J_dev, double* rho_dev);
size_t dfjk_static_scratch_bytes(void);

/*
 * The 3-index factor of Eq. eq:df:eri (Sec. IV.C.2): with the auxiliary
 * metric M = L L^T (Cholesky, lower L) and the 3-index integrals Q = (P|mu
 * nu), B = L^-1 Q.  No handle needed.
 *   naux    auxiliary functions; ncol columns of Q (npair for a packed B).
 *   M_dev   device, naux x naux row-major FP64, symmetric positive definite;
 *           overwritten by L (strict upper triangle set to zero).
 *   Q_dev   device, naux x ldQ row-major FP64; columns < ncol overwritten by
 *           B (the result is directly a B for dfjk_init, dtype DFJK_F64).
 *   stream  hipStream_t or NULL; the call waits for the stream at the end.
 * Blocked by 64: Cholesky with FP64 matrix-core trailing updates, then
 * forward substitution with matrix-core updates; deterministic.
 * Errors: DFJK_E_INVALID, DFJK_E_NO_DEVICE, DFJK_E_OOM, DFJK_E_HIP,
 * DFJK_E_NONFINITE (M not positive definite; M and Q then hold partial
 * results).
 */
int dfjk_form_B(int64_t naux, int64_t ncol, double* M_dev, double* Q_dev, int64_t ldQ, void* stream);

/*
 * J for ndm densities (the paper's get_jk takes any number of density
 * matrices, Sec. II): D_dev and J_dev hold ndm row-major nao x nao FP64
 * matrices back to back, rho_dev (or NULL) ndm x naux.  With FP64 B both
 * passes read B once for up to 8 densities at a time (each B element is
 * multiplied with all of them), so ndm densities cost about ceil(ndm/8)
 * single-density passes of HBM traffic; with reduced-precision B the
 * densities are streamed one after another.  Each J equals dfjk_build_J's up
 * to summation order (FP64).  The handle allocates its workspace on the first
 * call.  Errors: DFJK_E_INVALID (ndm < 1, null D or J), as dfjk_build_J.
 */
int dfjk_build_J_multi(dfjk_handle h, int64_t ndm, const double* D_dev, double* J_dev, double* rho_dev);

/*
 * dfjk_build_J plus the DF diagonal from the same pass over B:
 *   diag_dev[p(mu,nu)] = sum_P B[P, p(mu,nu)]^2,  p = max(mu,nu)(max+1)/2 + min,
 * the density-fitted (mu nu|mu nu), whose difference from the exact diagonal
 * integrals is the fitting error measure of Sec. IV.C.2.  diag_dev: device,
 * npair = nao(nao+1)/2 FP64 values, caller-owned.  Products and sums in FP64
 * of the stored B values (exact squares for FP32/BF16/FP16 B); deterministic.
 * J and rho are bitwise those of dfjk_build_J.  The handle allocates
 * j-splits x npair FP64 of workspace on the first call.
 * Errors: as dfjk_build_J; DFJK_E_INVALID if diag_dev is NULL.
 */
int dfjk_build_J_diag(dfjk_handle h, const double* D_dev, double* J_dev, double* rho_dev, double* diag_dev);

/*
 * Exchange matrix, written in full (both triangles):
 *   Cocc_dev != NULL: K = 2 sum_P (B_P C)(B_P C)^T with C = Cocc_dev
 *                     (nao x nocc, 1 <= nocc <= nao), i.e. K for D = 2 C C^T.
 *   Cocc_dev == NULL: K = sum_P B_P D B_P for the symmetric D_dev (paper
 *                     Sec. IV.A.1: a guess density need not be idempotent),
 *                     through the signed eigen-factors of D for nao < 256
 *                     or a reserved workspace (max_ncol > 0), else as the
 *                     two-factor form of dfjk_build_K_pair with L = D,
 *                     R = I, sym = 1, scale 1/2 (workspace: X for
 *                     2 * naux * nao rows).
 * Deterministic.
 */
int dfjk_build_K(dfjk_handle h, const double* Cocc_dev, int64_t nocc, const double* D_dev,
                 double* K_dev);

/* One SCF iteration's record (host struct). */
typedef struct {
    double e_tot;    /* E_k = tr(D H) + tr(D J)/2 - tr(D K)/4 of the input density */
    double e_1e;     /* tr(D H) */
    double e_j;      /* tr(D J)/2 = (1/2) sum_P rho_P^2 */
    double e_k;      /* -tr(D K)/4 */
    double err_norm; /* ||F D - D F||_F */
    double d_e;      /* E_k - E_{k-1} (E_1 on the first iteration) */
    int iter;        /* k, counted from 1 since the last dfjk_scf_reset */
    int converged;   /* k > 1, |d_e| < conv_tol and err_norm < conv_tol_grad */
} dfjk_scf_info;

/* dfjk_scf_step flag: on entry Cocc_dev holds orbitals with D = 2 C C^T. */
enum { DFJK_SCF_C_VALID = 1 };

/*
 * One restricted closed-shell SCF iteration in an orthonormal AO basis
 * (paper Sec. IV.A: a mean-field run starts from a guess density, which need
 * not be idempotent; Sec. IV.B: Pulay DIIS is the default accelerator):
 *   J, K of D (K through Cocc when flags has DFJK_SCF_C_VALID, else through
 *   the eigen-factors of D); F = H + J - K/2; E = tr(D(H+F))/2;
 *   e = FD - DF; DIIS over the last diis_space (F, e) pairs (the oldest
 *   dropped for good while the Gram matrix of the error vectors has a
 *   condition number above 1e12); aufbau on the
 *   extrapolated F; D <- 2 C C^T, Cocc <- C (nao x nocc).
 *   H_dev    nao x nao FP64 core Hamiltonian (symmetric).
 *   D_dev    in: the density of this iteration; out: the next density.
 *   Cocc_dev out: the next occupied orbitals (in: see flags).
 *   info     host pointer or NULL.  When given, the call waits for the stream,
 *            fills it, and returns DFJK_W_NOT_CONVERGED until converged.
 * nao <= 4096.  Iteration count and DIIS history live in the handle; call
 * dfjk_scf_reset before starting another system.
 */
int dfjk_scf_step(dfjk_handle h, const double* H_dev, double* D_dev, double* Cocc_dev, int64_t nocc,
                  int flags, dfjk_scf_info* info);

/*
 * Aufbau occupation of a symmetric nao x nao matrix F (e.g. the core
 * Hamiltonian for the core guess): Cocc <- eigenvectors of the nocc lowest
 * eigenvalues (nao x nocc), and, if D_dev is not NULL, D <- 2 C C^T.  Uses
 * the handle's eigensolver workspace and stream (nao <= 4096).
 */
int dfjk_aufbau(dfjk_handle h, const double* F_dev, int64_t nocc, double* Cocc_dev, double* D_dev);

/* Forget the SCF iteration count and the DIIS history. */
int dfjk_scf_reset(dfjk_handle h);

/*
 * Exchange with per-column signs: K = s * sum_P sum_i sign_i X_P[:,i] X_P[:,i]^T,
 * X_P = B_P C, sign_dev[i] in {+1, -1} (FP64, nocc entries, NULL = all +1).
 * Used by the D path (signed eigen-factors) and available to callers that
 * factor their own density.
 */
int dfjk_build_K_factored(dfjk_handle h, const double* C_dev, int64_t ncol,
                          const double* sign_dev, double scale, double* K_dev);

/*
 * Exchange for a density given by two factors, D = L R^T (Sec. IV.C.2, Eq.
 * eq:df:eri, with K_{mu nu} = sum_{ka la} (mu ka|nu la) D_{ka la}; D need not
 * be symmetric).  Such densities are what the second-order SCF's orbital
 * Hessian contracts (Sec. IV.B, SOSCF): for an occupied-virtual rotation x
 * the trial density is C_vir x C_occ^T plus its transpose, i.e. L = C_vir x,
 * R = C_occ, sym = 1, at the cost of two K(C_occ) builds instead of a full-
 * rank factorisation of D.
 *   L_dev, R_dev  nao x ncol FP64 device matrices, row-major (1 <= ncol <= nao).
 *   sym = 0       K = scale * sum_P (B_P L)(B_P R)^T         (not symmetric)
 *   sym = 1       K = scale * sum_P [(B_P L)(B_P R)^T + (B_P R)(B_P L)^T],
 *                 exactly symmetric (K of D + D^T).
 *   K_dev         nao x nao FP64 output, overwritten.
 * FP64 B runs on the FP64 matrix cores; FP32, BF16 and FP16 B on the FP32
 * matrix cores (the k16 option does not apply: its path takes one factor).
 * Workspace: X for 2 * naux * ncol rows.  DFJK_E_INVALID for a null pointer,
 * ncol outside [1, nao] or sym not 0/1.  Asynchronous on the handle's stream.
 */
int dfjk_build_K_pair(dfjk_handle h, const double* L_dev, const double* R_dev, int64_t ncol, int sym,
                      double scale, double* K_dev);

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
 * kernel's workgroup tile: dfjk_tile_info gives (p0, p1) = (row tiles of 16
 * occupied orbitals, column tiles of 16 basis functions per wavefront); the
 * last three run on the FP32 32 x 32 x 2 matrix-core steps and have no FP64
 * form (dfjk_set_tile returns DFJK_E_DTYPE for them on an FP64 handle).
 * DFJK_TILE_J_OUT selects the FP64 J pass-2 column width: (p0, p1) =
 * (packed columns per workgroup, 0).  DFJK_TILE_K16 selects the 16-bit
 * exchange's GEMM1 tile: (p0, p1) = (occupied orbitals, basis functions) per
 * workgroup.  DFJK_TILE_K16_SYRK selects the 16-bit exchange's GEMM2 output
 * tile: p0 = p1 = its edge (128 or 256).  dfjk_tile_count returns the number of
 * compiled tiles; dfjk_set_tile makes the handle use tile `index` (-1 =
 * default).  Every tile computes the same result up to summation order.
 */
enum { DFJK_TILE_GEMM1 = 0, DFJK_TILE_J_OUT = 1, DFJK_TILE_K16 = 2, DFJK_TILE_K16_SYRK = 3 };
int dfjk_tile_count(int kernel);
int dfjk_tile_info(int kernel, int index, int* p0, int* p1);
int dfjk_set_tile(dfjk_handle h, int kernel, int index);

/*
 * Batched builds: J and K for many molecules of uneven size in one pass
 * (each phase of the build is one launch over every molecule; molecules are
 * dispatched longest first).  Per molecule (all device pointers, held by the
 * caller for the life of the batch; contents may change between builds):
 *   B (naux x ldB packed, element type `dtype` = DFJK_F32, DFJK_BF16 or
 *   DFJK_F16), D and J, K (nao x nao FP64), Cocc (nao x nocc FP64).
 * Each build writes J(D) and K = 2 sum_P (B_P C)(B_P C)^T for every molecule;
 * J accumulates in FP64, the K products run on the FP32 matrix cores.
 *   dfjk_batch_build    enqueue the whole batch on the stream.
 *   dfjk_batch_capture  record one build into a HIP graph (no allocation,
 *                       synchronisation or memset inside a build).
 *   dfjk_batch_launch   replay the recorded graph on the stream.
 *   dfjk_batch_autotune time every compiled GEMM1 tile per bucket of
 *                       molecules (bucket = ceil(nocc/16) - 1, 0..7), keep the
 *                       fastest whose K matches the default tile's within
 *                       1e-5 relative, and store the choice in cache_path
 *                       (text lines "dtype bucket tile ms"; read instead of
 *                       timing when present, and then checked against the
 *                       default tile's K the same way).  best_ms (8 doubles)
 *                       or NULL.  Drops a recorded graph first; waits; leaves
 *                       J and K of every molecule written.
 */
typedef struct dfjk_batch_ctx* dfjk_batch;
typedef struct {
    const void* B;
    int64_t nao, naux, ldB, nocc;
    const double* D;
    const double* Cocc;
    double* J;
    double* K;
} dfjk_mol;
int dfjk_batch_init(dfjk_batch* b, const dfjk_mol* mols, int nmol, int dtype, void* stream);
int dfjk_batch_build(dfjk_batch b);
int dfjk_batch_capture(dfjk_batch b);
int dfjk_batch_launch(dfjk_batch b);
int dfjk_batch_autotune(dfjk_batch b, int reps, const char* cache_path, double* best_ms);
int dfjk_batch_get_tile(dfjk_batch b, int bucket, int* tile);
int dfjk_batch_set_tile(dfjk_batch b, int bucket, int tile);
/*
 * dfjk_batch_set_k16(b, 1): K of every molecule on the 16-bit matrix cores
 * (BF16 / FP16 B only; DFJK_E_DTYPE otherwise), Eq. eq:df:eri contracted
 * with the occupied orbitals as in the single-molecule 16-bit exchange:
 * C^T rounded once to the storage format, X_P = B_P C accumulated in FP32
 * from the packed triangle and rounded to 16 bits, K = 2 sum X X^T in FP32
 * with the split partials added in FP64.  Error against the FP64 oracle on
 * the stored B with C rounded the same way: below 2u max|K| plus the FP32
 * sums (u = 2^-8 BF16, 2^-11 FP16).  J is unchanged.  Allocates the 16-bit
 * workspace (C^T, X, split partials: about naux nao ceil32(nocc) 2 bytes per
 * molecule) on the first call; drops a recorded graph.  0 returns to the
 * FP32 exchange.
 */
int dfjk_batch_set_k16(dfjk_batch b, int on);
int dfjk_batch_workspace_bytes(dfjk_batch b, size_t* bytes);
void dfjk_batch_destroy(dfjk_batch b);

/*
 * SCF over a batch: dfjk_scf_step for every molecule at once (Sec. IV.A and
 * IV.B: each molecule's mean-field iteration, DIIS by default).
 *   H_list  host array of nmol device pointers, molecule i's core
 *           Hamiltonian (nao_i x nao_i FP64, symmetric), in dfjk_batch_init
 *           order.
 *   dfjk_batch_scf_guess  core guess for every molecule: Cocc <- the nocc
 *           lowest eigenvectors of H, D <- 2 Cocc Cocc^T, written into the
 *           molecules' Cocc and D buffers; forgets the SCF histories.
 *   dfjk_batch_scf_step   one iteration for every molecule: J(D) and
 *           K(Cocc) with the batch build (on entry D = 2 Cocc Cocc^T, as the
 *           guess and every step leave it; the molecules' J and K buffers
 *           receive them), then F = H + J - K/2, E, e = FD - DF, DIIS (with
 *           dfjk_scf_step's rule for dropping old vectors), aufbau, and the
 *           next D and Cocc written in place.  info: host array of nmol
 *           records or NULL; when given, the call waits and returns
 *           DFJK_W_NOT_CONVERGED until every molecule has converged
 *           (dfjk_scf_step's criteria and defaults), DFJK_E_NONFINITE for a
 *           non-finite energy.
 *   dfjk_batch_scf_reset  forget the SCF histories.
 * The molecules' dense steps run on up to 8 worker streams forked from and
 * joined back to the batch stream (not graph-capturable); each molecule keeps
 * its own DIIS history and eigensolver workspace (about (5 + 2 * 8) nao^2
 * doubles), allocated on first use.  nao <= 4096 per molecule.
 */
int dfjk_batch_scf_guess(dfjk_batch b, const double* const* H_list);
int dfjk_batch_scf_step(dfjk_batch b, const double* const* H_list, dfjk_scf_info* info);
int dfjk_batch_scf_reset(dfjk_batch b);

/*
 * Learned initial guess (a guess density need not be idempotent, paper
 * Sec. IV.A.1).  A perceptron d_in -> hidden -> hidden -> 1 with SiLU
 * activations, FP32, trained on the GPU:
 *   dfjk_mlp_init        allocate for batches of up to max_batch rows.
 *   dfjk_mlp_nparam      number of FP32 parameters, laid out as
 *                        W1 (hidden x d_in), b1, W2 (hidden x hidden), b2,
 *                        W3 (hidden), b3, each row-major.
 *   dfjk_mlp_set_params  upload parameters (host array) and clear Adam state.
 *   dfjk_mlp_get         download parameters (which = 0) or the gradient of
 *                        the last dfjk_mlp_loss_grad (which = 1); waits.
 *   dfjk_mlp_forward     y = f(X) for n rows (X: n x d_in FP32, device).
 *   dfjk_mlp_loss_grad   L = mean((f(X) - t)^2) and its gradient (kept in
 *                        the handle); L to loss_dev (device, may be NULL).
 *   dfjk_mlp_adam        one Adam step (Kingma & Ba) with the kept gradient.
 *   dfjk_mlp_set_compute DFJK_F32 (default) or DFJK_BF16: with BF16 the
 *                        hidden x hidden products of the forward pass, of
 *                        the input gradient and of the weight gradient round
 *                        their FP32 operands once to bfloat16 and run on the
 *                        16-bit matrix cores (FP32 sums); parameters, Adam
 *                        state and every other step stay FP32.
 * Features and guess for one system (nao <= 65535, device pointers):
 *   dfjk_guess_features  X (npair x 8 FP32, packed pair order) from H, the
 *                        core-guess density Dcore and positions R (nao x 3).
 *   dfjk_guess_assemble  D = Dcore + y, symmetric, from y (npair FP32).
 *   dfjk_guess_target    t (npair FP32, packed pair order) = D - Dcore on the
 *                        pairs: the training target for a converged D.
 *   dfjk_guess_check     out (2 FP64, device) = [tr D, number of non-finite
 *                        entries of D]: the checks that decide whether a
 *                        guess is used or the core guess takes its place.
 *   dfjk_gather_rows     Y[r] = X[idx[r]] for n rows of d FP32 values (idx:
 *                        n int64 row indices < rows of X, device), e.g. a
 *                        shuffled training order.
 * All asynchronous on `stream`.
 */
typedef struct dfjk_mlp_ctx* dfjk_mlp;
int dfjk_mlp_init(dfjk_mlp* m, int d_in, int hidden, int64_t max_batch, void* stream);
int64_t dfjk_mlp_nparam(dfjk_mlp m);
int dfjk_mlp_set_params(dfjk_mlp m, const float* host_params);
int dfjk_mlp_get(dfjk_mlp m, int which, float* host_out);
int dfjk_mlp_forward(dfjk_mlp m, const float* X_dev, int64_t n, float* y_dev);
int dfjk_mlp_loss_grad(dfjk_mlp m, const float* X_dev, const float* t_dev, int64_t n, float* loss_dev);
int dfjk_mlp_adam(dfjk_mlp m, float lr, float beta1, float beta2, float eps);
int dfjk_mlp_set_compute(dfjk_mlp m, int dtype);
void dfjk_mlp_destroy(dfjk_mlp m);
int dfjk_guess_features(const double* H_dev, const double* Dcore_dev, const double* R_dev, int64_t nao,
                        float* X_dev, void* stream);
int dfjk_guess_assemble(const float* y_dev, const double* Dcore_dev, int64_t nao, double* D_dev,
                        void* stream);
int dfjk_guess_target(const double* D_dev, const double* Dcore_dev, int64_t nao, float* t_dev, void* stream);
int dfjk_guess_check(const double* D_dev, int64_t nao, double* out_dev, void* stream);
int dfjk_gather_rows(const float* X_dev, const int64_t* idx_dev, int64_t n, int d, float* Y_dev, void* stream);

/*
 * Sustained matrix-core rate (TFLOP/s) of v_mfma_f64_16x16x4f64 (DFJK_F64),
 * v_mfma_f32_16x16x4f32 (DFJK_F32) or v_mfma_f32_32x32x16_bf16 (DFJK_BF16),
 * measured with register-only kernels on the current device (waits).
 */
int dfjk_probe_mfma(int dtype, double* tflops);

/*
 * Sustained HBM read rate (GB/s) of a plain streaming kernel over the first
 * bytes (rounded down to 16) of a caller-owned device buffer, e.g. B itself:
 * the measured ceiling of the bandwidth-bound J passes.  Contiguous ranges per
 * workgroup at 2, 4, 8 and 16 workgroups per CU, each timed twice after one
 * warm-up; the best rate is returned.  Waits.  DFJK_E_INVALID for a null or unaligned
 * buffer or fewer than 16 bytes.
 */
int dfjk_probe_hbm_read(const void* buf_dev, size_t bytes, double* gbs);

/*
 * Tell the handle that the contents of B changed (same pointer, layout and
 * dtype).  J and K read B on every call, except the k16 exchange, which
 * reads the handle's dense 16-bit copy: this remakes that copy (no
 * allocation; asynchronous on the handle's stream).  A no-op for handles
 * without a copy.
 */
int dfjk_update_B(dfjk_handle h);

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
