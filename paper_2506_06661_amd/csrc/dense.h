// Dense FP64 helpers (dense.hip): matrix product, deterministic dot
// products, symmetric eigensolver.
#pragma once

#include "internal.h"

namespace dfjk {

constexpr int kMaxEighN = 4096;
constexpr int kMaxDots = 16;

// Up to kMaxDots dot products of length n, passed by value to the kernel.
struct DotList {
    const double* a[kMaxDots];
    const double* b[kMaxDots];
};

// C = alpha op(A) op(B) + beta C (row-major; op = transpose when ta / tb).
int dgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc);

int sgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha,
          const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
          int64_t ldc);

// C = op(A) op(B) (no scaling, C overwritten) with the FP32 operands rounded
// once to bfloat16 and products on the 16-bit matrix cores, FP32 sums.
int bgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
          const float* B, int64_t ldb, float* C, int64_t ldc);

// out[t] = a_t . b_t for t < nd, summed in a fixed order (bitwise reproducible).
// part needs dots_part_elems(nd) doubles.
int dots(hipStream_t st, const DotList& list, int nd, int64_t n, double* part, double* out);
size_t dots_part_elems(int nd);

// Symmetric eigendecomposition by parallel cyclic Jacobi in one workgroup.
// A (n x n) is overwritten; V (n x n) holds a basis as ROWS (set to the
// identity first when v_identity): on entry A must be expressed in that basis
// (A = V F V^T); on exit row k of V is the eigenvector of F with eigenvalue
// A[k][k].
// work: >= n + 2 doubles; iwork: >= n + 2 ints (iwork[0] = sweeps used,
// iwork[1 + r] = index of the r-th smallest eigenvalue); w: n eigenvalues in
// ascending order.
int eigh(hipStream_t st, double* A, double* V, int n, bool v_identity, double* work, int* iwork,
         double* w);

// out (n x ncol) = eigenvector columns of the ncol smallest eigenvalues; mode 1
// scales column c by sqrt|w_c| and writes sign(w_c) to sign.
int eig_gather(hipStream_t st, const double* V, int n, const int* iwork, int ncol, const double* w,
               int mode, double* out, double* sign);

}  // namespace dfjk
