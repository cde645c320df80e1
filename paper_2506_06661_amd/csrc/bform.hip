// The 3-index factor of the density-fitted integrals (Sec. IV.C.2, the T of
// Eq. eq:df:eri): M = L L^T (Cholesky of the auxiliary metric, lower L) and
// T = L^-1 Q for the 3-index integrals Q = (P|mu nu), one column per packed
// pair.  Both factorisation and substitution are blocked by 64 rows:
//   Cholesky, for each diagonal block k: factor L_kk and invert it in LDS
//     (one workgroup); panel L_ik = M_ik L_kk^-T and trailing update
//     M_ij -= L_ik L_jk^T as FP64 matrix-core GEMMs.
//   Substitution, for each block row k: Q_k <- L_kk^-1 Q_k and
//     Q_i -= L_ik Q_k for the rows i > k of its 256-row panel, then one
//     rank-256 update of the rows below the panel; all matrix-core GEMMs.
// The 64 x 64 diagonal blocks are applied through their explicit inverses
// (forward substitution on the identity), which keeps every large step on
// the matrix cores; the accuracy is that of the diagonal blocks' condition.
// All sums run in a fixed order: the result is bitwise reproducible.
#include "dense.h"
#include "internal.h"

namespace dfjk {
namespace {

constexpr int NB = 64;    // block size (diagonal blocks, Cholesky panels)
constexpr int NB2 = 256;  // row panel of the substitution (a multiple of NB)
constexpr int kT = 256;

// Factor the kb x kb diagonal block at (k0, k0) of A (row-major, lda) in
// place (lower triangle <- L_kk, strict upper <- 0) and write its inverse,
// padded to 64 x 64 with the identity, to Linv.  A non-positive (or
// non-finite) pivot sets *flag.
__global__ __launch_bounds__(kT) void chol_diag(double* __restrict__ A, int64_t lda, int64_t k0, int kb,
                                                double* __restrict__ Linv, int* __restrict__ flag) {
    __shared__ double T[NB][NB + 1];
    const int tid = threadIdx.x;
    for (int e = tid; e < NB * NB; e += kT) {
        const int i = e / NB, j = e % NB;
        T[i][j] = (i < kb && j < kb) ? A[(k0 + i) * lda + k0 + j] : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int j = 0; j < kb; ++j) {
        if (tid == 0) {
            const double d = T[j][j];
            if (!(d > 0.0) || !(d < 1e300)) flag[0] = 1;
            T[j][j] = sqrt(d);  // NaN for a non-positive pivot; reported through flag
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < kb; i += kT) T[i][j] /= T[j][j];
        __syncthreads();
        const int m = kb - j - 1;  // trailing (i, l), j < l <= i < kb
        for (int e = tid; e < m * m; e += kT) {
            const int i = j + 1 + e / m, l = j + 1 + e % m;
            if (l <= i) T[i][l] = fma(-T[i][j], T[l][j], T[i][l]);
        }
        __syncthreads();
    }
    for (int e = tid; e < kb * kb; e += kT) {
        const int i = e / kb, j = e % kb;
        A[(k0 + i) * lda + k0 + j] = j <= i ? T[i][j] : 0.0;
    }
    // inverse: column c solves L x = e_c (thread c, rows in order; it reads
    // back only its own earlier entries)
    if (tid < NB) {
        const int c = tid;
        for (int j = 0; j < NB; ++j) {
            double sum = j == c ? 1.0 : 0.0;
            for (int l = c; l < j; ++l) sum = fma(-T[j][l], Linv[l * NB + c], sum);
            Linv[j * NB + c] = j < c ? 0.0 : sum / T[j][j];
        }
    }
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int form_B(int64_t naux, int64_t ncol, double* M, double* Q, int64_t ldQ, hipStream_t st) {
    // workspace: the flag, the 64 x 64 inverse of every diagonal block and a
    // 64-row staging buffer
    const int64_t wrows = naux > ncol ? naux : ncol;
    const int64_t nblk = cdiv(naux, NB);
    char* ws = nullptr;
    const size_t bytes = 256 + sizeof(double) * (size_t)(NB * NB * nblk + NB * wrows);
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        set_error("dfjk_form_B: out of device memory");
        return DFJK_E_OOM;
    }
    int* flag = reinterpret_cast<int*>(ws);
    double* Linv_all = reinterpret_cast<double*>(ws + 256);
    double* tmp = Linv_all + NB * NB * nblk;
    int rc = DFJK_OK;
    if (hipMemsetAsync(flag, 0, sizeof(int), st) != hipSuccess) rc = DFJK_E_HIP;
    // Cholesky of M, in place
    for (int64_t k0 = 0; rc == DFJK_OK && k0 < naux; k0 += NB) {
        const int kb = (int)(naux - k0 < NB ? naux - k0 : NB);
        double* Linv = Linv_all + (k0 / NB) * NB * NB;
        chol_diag<<<1, kT, 0, st>>>(M, naux, k0, kb, Linv, flag);
        const int64_t n2 = naux - k0 - kb;
        if (n2 > 0) {
            double* panel = M + (k0 + kb) * naux + k0;
            // tmp (n2 x kb) = M_ik L_kk^-T, then back into the panel
            rc = dgemm(st, false, true, n2, kb, kb, 1.0, panel, naux, Linv, NB, 0.0, tmp, kb);
            if (rc == DFJK_OK &&
                hipMemcpy2DAsync(panel, naux * sizeof(double), tmp, kb * sizeof(double), kb * sizeof(double), n2,
                                 hipMemcpyDeviceToDevice, st) != hipSuccess)
                rc = DFJK_E_HIP;
            if (rc == DFJK_OK)
                rc = dgemm(st, false, true, n2, n2, kb, -1.0, panel, naux, panel, naux, 1.0,
                           M + (k0 + kb) * naux + k0 + kb, naux);
        }
        if (rc == DFJK_OK && hipGetLastError() != hipSuccess) rc = DFJK_E_HIP;
    }
    // strict upper triangle of M outside the diagonal blocks <- 0 (M holds L)
    for (int64_t k0 = 0; rc == DFJK_OK && k0 + NB < naux; k0 += NB) {
        const int64_t w = naux - k0 - NB;
        if (hipMemset2DAsync(M + k0 * naux + k0 + NB, naux * sizeof(double), 0, w * sizeof(double), NB, st) !=
            hipSuccess)
            rc = DFJK_E_HIP;
    }
    // forward substitution T = L^-1 Q, in place, blocked twice: within a
    // panel of NB2 rows by the 64-row diagonal blocks, then one rank-NB2
    // update of all rows below (a rank-64 update per block would rewrite Q
    // naux/64 times)
    for (int64_t K0 = 0; rc == DFJK_OK && K0 < naux; K0 += NB2) {
        const int64_t K1 = K0 + NB2 < naux ? K0 + NB2 : naux;
        for (int64_t k0 = K0; rc == DFJK_OK && k0 < K1; k0 += NB) {
            const int kb = (int)(K1 - k0 < NB ? K1 - k0 : NB);
            const double* Linv = Linv_all + (k0 / NB) * NB * NB;
            double* Qk = Q + k0 * ldQ;
            rc = dgemm(st, false, false, kb, ncol, kb, 1.0, Linv, NB, Qk, ldQ, 0.0, tmp, ncol);
            if (rc == DFJK_OK &&
                hipMemcpy2DAsync(Qk, ldQ * sizeof(double), tmp, ncol * sizeof(double), ncol * sizeof(double), kb,
                                 hipMemcpyDeviceToDevice, st) != hipSuccess)
                rc = DFJK_E_HIP;
            const int64_t n2 = K1 - k0 - kb;  // rows of this panel below the block
            if (rc == DFJK_OK && n2 > 0)
                rc = dgemm(st, false, false, n2, ncol, kb, -1.0, M + (k0 + kb) * naux + k0, naux, Qk, ldQ, 1.0,
                           Q + (k0 + kb) * ldQ, ldQ);
        }
        const int64_t n3 = naux - K1;
        if (rc == DFJK_OK && n3 > 0)
            rc = dgemm(st, false, false, n3, ncol, K1 - K0, -1.0, M + K1 * naux + K0, naux, Q + K0 * ldQ, ldQ, 1.0,
                       Q + K1 * ldQ, ldQ);
        if (rc == DFJK_OK && hipGetLastError() != hipSuccess) rc = DFJK_E_HIP;
    }
    int host_flag = 0;
    if (rc == DFJK_OK &&
        (hipMemcpyAsync(&host_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
         hipStreamSynchronize(st) != hipSuccess))
        rc = DFJK_E_HIP;
    (void)hipFree(ws);
    if (rc == DFJK_E_HIP) {
        set_error("dfjk_form_B: HIP error %s", hipGetErrorString(hipGetLastError()));
        return rc;
    }
    if (rc != DFJK_OK) return rc;
    if (host_flag) {
        set_error("dfjk_form_B: the metric is not positive definite (non-positive Cholesky pivot)");
        return DFJK_E_NONFINITE;
    }
    return DFJK_OK;
}

}  // namespace dfjk
