// Dense FP64 helpers for the SCF step and the density path of K:
// a general matrix product on the FP64 matrix cores, deterministic
// reductions, and a one-workgroup parallel cyclic Jacobi eigensolver.
#include "dense.h"

#include "mma.h"
#include "numerics.h"

namespace dfjk {

namespace {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- GEMM
// C = alpha * op(A) op(B) + beta * C, row-major, op(X) = X or X^T.
// 64x64 tile per workgroup, 2x2 waves of 32x32 (2x2 f64 16x16x4 steps).
constexpr int GT = 64, GK = 16;

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_kernel(int64_t M, int64_t N, int64_t K, T alpha,
                                                    const T* __restrict__ A, int64_t lda,
                                                    const T* __restrict__ B, int64_t ldb, T beta,
                                                    T* __restrict__ C, int64_t ldc) {
    __shared__ T sA[GK][GT + 1];  // sA[k][m] = op(A)[m][k]
    __shared__ T sB[GK][GT + 1];  // sB[k][n] = op(B)[k][n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
    typename Mma<T>::acc_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = Mma<T>::zero();
    for (int64_t k0 = 0; k0 < K; k0 += GK) {
        for (int e = tid; e < GK * GT; e += 256) {
            // element (k, m) of op(A) and (k, n) of op(B); the mapping reads
            // memory contiguously
            int k, m;
            if (TA) { k = e / GT; m = e % GT; } else { m = e / GK; k = e % GK; }
            const int64_t gm = m0 + m, gk = k0 + k;
            T v = T(0);
            if (gm < M && gk < K) v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
            sA[k][m] = v;
            int kb, n;
            if (TB) { n = e / GK; kb = e % GK; } else { kb = e / GT; n = e % GT; }
            const int64_t gn = n0 + n, gkb = k0 + kb;
            T w = T(0);
            if (gn < N && gkb < K) w = TB ? B[gn * ldb + gkb] : B[gkb * ldb + gn];
            sB[kb][n] = w;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < GK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            T a[2], b[2];
            for (int q = 0; q < 2; ++q) {
                a[q] = sA[kr][wm * 32 + q * 16 + (lane & 15)];
                b[q] = sB[kr][wn * 32 + q * 16 + (lane & 15)];
            }
            for (int ti = 0; ti < 2; ++ti)
                for (int tj = 0; tj < 2; ++tj) acc[ti][tj] = Mma<T>::step(a[ti], b[tj], acc[ti][tj]);
        }
        __syncthreads();
    }
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj)
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * 32 + ti * 16 + Mma<T>::row(lane, r);
                const int64_t gn = n0 + wn * 32 + tj * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    const T old = beta == T(0) ? T(0) : beta * C[gm * ldc + gn];
                    C[gm * ldc + gn] = alpha * acc[ti][tj][r] + old;
                }
            }
}

// C = alpha A B + beta C for large row-major FP64 products (no transposes):
// 128 x 128 tile per workgroup, 2 x 2 waves of 64 x 64 (4 x 4 steps of
// 16 x 16 x 4 per wavefront, the accumulators in the matrix-core registers),
// K in 16-deep chunks double-buffered in LDS with the next chunk loaded into
// registers while the current one is multiplied.  Loads are pairs of
// doubles (rows start 16-byte aligned when lda, ldb are even and A, B are
// 16-byte aligned; otherwise element loads).  The k order of every sum is
// that of gemm_kernel (4-deep steps in increasing k).
constexpr int WT = 128, WK = 16;
template <bool PAIRS>
__global__ __launch_bounds__(256, 2) void gemm_nn_wide(int64_t M, int64_t N, int64_t K, double alpha,
                                                        const double* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ B, int64_t ldb, double beta,
                                                        double* __restrict__ C, int64_t ldc) {
    __shared__ double sA[2][WK][WT + 2];  // sA[k][m] = A[m0 + m][k0 + k]
    __shared__ double sB[2][WK][WT + 2];  // sB[k][n] = B[k0 + k][n0 + n]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * WT, n0 = (int64_t)blockIdx.x * WT;
    // thread's pairs: A rows m0 + tid/8 + 32 j at k pair 2 (tid%8); B rows
    // tid/64 + 4 j at n pair 2 (tid%64)
    const int am = tid >> 3, akp = 2 * (tid & 7), bk = tid >> 6, bnp = 2 * (tid & 63);
    const bool full_mn = m0 + WT <= M && n0 + WT <= N;
    double ra[4][2], rb[4][2];
    auto load = [&](int64_t k0) {
        if (PAIRS && full_mn && k0 + WK <= K) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double2 va = *reinterpret_cast<const double2*>(A + (m0 + am + 32 * j) * lda + k0 + akp);
                const double2 vb = *reinterpret_cast<const double2*>(B + (k0 + bk + 4 * j) * ldb + n0 + bnp);
                ra[j][0] = va.x;
                ra[j][1] = va.y;
                rb[j][0] = vb.x;
                rb[j][1] = vb.y;
            }
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int64_t gm = m0 + am + 32 * j, gk = k0 + akp + d;
                    ra[j][d] = (gm < M && gk < K) ? A[gm * lda + gk] : 0.0;
                    const int64_t gkb = k0 + bk + 4 * j, gn = n0 + bnp + d;
                    rb[j][d] = (gkb < K && gn < N) ? B[gkb * ldb + gn] : 0.0;
                }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sA[buf][akp][am + 32 * j] = ra[j][0];
            sA[buf][akp + 1][am + 32 * j] = ra[j][1];
            sB[buf][bk + 4 * j][bnp] = rb[j][0];
            sB[buf][bk + 4 * j][bnp + 1] = rb[j][1];
        }
    };
    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};
    const int64_t nk = cdiv(K, WK);
    load(0);
    store(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) load((kc + 1) * WK);
#pragma unroll
        for (int kk = 0; kk < WK / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = sA[buf][kr][wm * 64 + q * 16 + (lane & 15)];
                b[q] = sB[buf][kr][wn * 64 + q * 16 + (lane & 15)];
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = Mma<double>::step(a[ti], b[tj], acc[ti][tj]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * 64 + ti * 16 + Mma<double>::row(lane, r);
                const int64_t gn = n0 + wn * 64 + tj * 16 + (lane & 15);
                if (gm < M && gn < N) {
                    const double old = beta == 0.0 ? 0.0 : beta * C[gm * ldc + gn];
                    C[gm * ldc + gn] = alpha * acc[ti][tj][r] + old;
                }
            }
}

// C = op(A) op(B) with FP32 operands rounded once to bfloat16 (RNE) as they
// are staged, products on v_mfma_f32_16x16x32_bf16, FP32 accumulation and
// output.  64 x 64 tile per workgroup, 2 x 2 waves of 32 x 32 (2 x 2 steps of
// 16 x 16); K in chunks of 32, both operands held k-contiguous in LDS (row =
// m or n, 32 bfloat16 + 8 of padding: 16-byte pieces of 16 consecutive rows
// fall on distinct banks).
typedef __bf16 v8bf_d __attribute__((ext_vector_type(8)));
typedef uint32_t u4_d __attribute__((ext_vector_type(4)));
constexpr int BK = 32, BROW = BK + 8;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void bgemm_kernel(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                                     int64_t lda, const float* __restrict__ B, int64_t ldb,
                                                     float* __restrict__ C, int64_t ldc) {
    __shared__ uint16_t sA[GT][BROW];  // sA[m][k] = bf16(op(A)[m][k])
    __shared__ uint16_t sB[GT][BROW];  // sB[n][k] = bf16(op(B)[k][n])
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = v4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = 0; k0 < K; k0 += BK) {
        for (int e = tid; e < BK * GT; e += 256) {
            // element (m, k) of op(A) and (n, k) of op(B); the mapping reads
            // memory contiguously
            int k, m;
            if (TA) { k = e / GT; m = e % GT; } else { m = e / BK; k = e % BK; }
            const int64_t gm = m0 + m, gk = k0 + k;
            float v = 0.f;
            if (gm < M && gk < K) v = TA ? A[gk * lda + gm] : A[gm * lda + gk];
            sA[m][k] = float_to_bf16_rne(v);
            int kb, n;
            if (TB) { n = e / BK; kb = e % BK; } else { kb = e / GT; n = e % GT; }
            const int64_t gn = n0 + n, gkb = k0 + kb;
            float w = 0.f;
            if (gn < N && gkb < K) w = TB ? B[gn * ldb + gkb] : B[gkb * ldb + gn];
            sB[n][kb] = float_to_bf16_rne(w);
        }
        __syncthreads();
        u4_d a[2], b[2];
        for (int q = 0; q < 2; ++q) {
            a[q] = *reinterpret_cast<const u4_d*>(&sA[wm * 32 + q * 16 + (lane & 15)][8 * (lane >> 4)]);
            b[q] = *reinterpret_cast<const u4_d*>(&sB[wn * 32 + q * 16 + (lane & 15)][8 * (lane >> 4)]);
        }
        for (int ti = 0; ti < 2; ++ti)
            for (int tj = 0; tj < 2; ++tj) {
                v8bf_d av, bv;
                __builtin_memcpy(&av, &a[ti], 16);
                __builtin_memcpy(&bv, &b[tj], 16);
                acc[ti][tj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[ti][tj], 0, 0, 0);
            }
        __syncthreads();
    }
    // result row 4 (lane / 16) + r, column lane % 16 of each 16 x 16 block
    for (int ti = 0; ti < 2; ++ti)
        for (int tj = 0; tj < 2; ++tj)
            for (int r = 0; r < 4; ++r) {
                const int64_t gm = m0 + wm * 32 + ti * 16 + 4 * (lane >> 4) + r;
                const int64_t gn = n0 + wn * 32 + tj * 16 + (lane & 15);
                if (gm < M && gn < N) C[gm * ldc + gn] = acc[ti][tj][r];
            }
}

// ---------------------------------------------------------------- reductions
// part[t * nblk + b] = sum over this block's slice of a_t . b_t
constexpr int RT = 256, RBLK = 128;

__global__ __launch_bounds__(RT) void dots_partial(DotList list, int64_t n, double* __restrict__ part) {
    __shared__ double lds[RT / 64];
    const double* __restrict__ da = list.a[blockIdx.y];
    const double* __restrict__ db = list.b[blockIdx.y];
    const int64_t per = cdiv(n, RBLK);
    const int64_t beg = (int64_t)blockIdx.x * per;
    const int64_t end = beg + per < n ? beg + per : n;
    double s = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += RT) s = fma(da[i], db[i], s);
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < RT / 64; ++w) t += lds[w];
        part[blockIdx.y * RBLK + blockIdx.x] = t;
    }
}

__global__ void dots_finish(const double* __restrict__ part, int nd, double* __restrict__ out) {
    const int t = threadIdx.x;
    if (t >= nd) return;
    double s = 0.0;
    for (int b = 0; b < RBLK; ++b) s += part[t * RBLK + b];
    out[t] = s;
}

// ---------------------------------------------------------------- Jacobi
// Parallel cyclic Jacobi on a symmetric n x n matrix A (overwritten; the
// eigenvalues end on its diagonal).  Vt (n x n) holds the basis as ROWS: it
// starts as the caller's basis (rows orthonormal) and its row k ends as the
// eigenvector of diagonal entry k.  Each sweep visits every pair (p,q) once in
// the round-robin (circle) order: n-1 rounds of n/2 disjoint pairs (a dummy
// index when n is odd).  Rotations follow the symmetric Schur step of Golub &
// Van Loan (Matrix Computations, 8.5.2): with J[p][p] = J[q][q] = c,
// J[p][q] = s, J[q][p] = -s, a round applies A <- J^T A J and Vt <- J^T Vt for
// all of its pairs at once.  Because every index is in one pair, the new
// entries of rows (p, q) and columns (a, b) depend only on the old 2x2 block
// A[{p,q}][{a,b}], so one thread updates each such block in place and a round
// needs a single barrier.
constexpr int JT = 1024;
constexpr int kJacobiShN = 128;  // A in LDS up to 128 x 128 doubles (128 KB)

__device__ inline void pair_of(int r, int k, int m, int& p, int& q) {
    // circle method on m (even) players; player m-1 fixed
    if (k == 0) {
        p = r;
        q = m - 1;
    } else {
        p = (r + k) % (m - 1);
        q = (r - k + (m - 1)) % (m - 1);
    }
    if (p > q) {
        const int t = p;
        p = q;
        q = t;
    }
}

// y = J^T x on the pair (p, q): (c x_p - s x_q, s x_p + c x_q)
__device__ inline void rot(double c, double s, double xp, double xq, double& yp, double& yq) {
    yp = c * xp - s * xq;
    yq = s * xp + c * xq;
}

template <bool SH>
__global__ __launch_bounds__(JT) void jacobi_kernel(double* __restrict__ Ag, double* __restrict__ Vt,
                                                     int n, double* __restrict__ cs, int max_sweeps,
                                                     double tol, int* __restrict__ sweeps_done) {
    extern __shared__ double smem[];
    __shared__ double red[JT / 64];
    __shared__ int stop;
    double* __restrict__ A = SH ? smem : Ag;
    if (SH) {
        for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) A[e] = Ag[e];
        __syncthreads();
    }
    const int m = n + (n & 1);
    const int half = m / 2;
    double* cc = cs;
    double* ss = cs + half;
    int sweep = 0;
    for (; sweep < max_sweeps; ++sweep) {
        // convergence test: off-diagonal norm against the full norm
        double off = 0.0, all = 0.0;
        for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) {
            const double v = A[e];
            all = fma(v, v, all);
            if (e / n != e % n) off = fma(v, v, off);
        }
        off = wave_sum(off);
        all = wave_sum(all);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = off;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < JT / 64; ++w) t += red[w];
            red[0] = t;
        }
        __syncthreads();
        const double off_tot = red[0];
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = all;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < JT / 64; ++w) t += red[w];
            stop = !(off_tot > tol * tol * t) ? 1 : 0;
        }
        __syncthreads();
        if (stop) break;
        for (int r = 0; r < m - 1; ++r) {
            // rotation of each pair from the current A (dummy pairs: c = 1, s = 0)
            for (int k = threadIdx.x; k < half; k += JT) {
                int p, q;
                pair_of(r, k, m, p, q);
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[(int64_t)p * n + q];
                    if (apq != 0.0) {
                        const double app = A[(int64_t)p * n + p], aqq = A[(int64_t)q * n + q];
                        const double tau = (aqq - app) / (2.0 * apq);
                        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                cc[k] = c;
                ss[k] = s;
            }
            __syncthreads();
            // A <- J^T A J by 2x2 blocks (row pair k, column pair kk)
            for (int64_t e = threadIdx.x; e < (int64_t)half * half; e += JT) {
                const int k = (int)(e / half), kk = (int)(e % half);
                int p, q, a, b;
                pair_of(r, k, m, p, q);
                pair_of(r, kk, m, a, b);
                const double c = cc[k], s = ss[k], c2 = cc[kk], s2 = ss[kk];
                const bool qv = q < n, bv = b < n;
                // old block
                const double apa = A[(int64_t)p * n + a];
                const double apb = bv ? A[(int64_t)p * n + b] : 0.0;
                const double aqa = qv ? A[(int64_t)q * n + a] : 0.0;
                const double aqb = (qv && bv) ? A[(int64_t)q * n + b] : 0.0;
                // rows: (p, q) <- J^T
                double rpa, rqa, rpb, rqb;
                rot(c, s, apa, aqa, rpa, rqa);
                rot(c, s, apb, aqb, rpb, rqb);
                // columns: (a, b) <- J
                double npa, npb, nqa, nqb;
                rot(c2, s2, rpa, rpb, npa, npb);
                rot(c2, s2, rqa, rqb, nqa, nqb);
                if (k == kk) {  // the rotated pair's own block: off-diagonal is zero by construction
                    npb = 0.0;
                    nqa = 0.0;
                }
                A[(int64_t)p * n + a] = npa;
                if (bv) A[(int64_t)p * n + b] = npb;
                if (qv) A[(int64_t)q * n + a] = nqa;
                if (qv && bv) A[(int64_t)q * n + b] = nqb;
            }
            // Vt <- J^T Vt (row rotations; contiguous rows)
            for (int64_t e = threadIdx.x; e < (int64_t)half * n; e += JT) {
                const int k = (int)(e / n), j = (int)(e % n);
                int p, q;
                pair_of(r, k, m, p, q);
                if (q >= n) continue;
                const double c = cc[k], s = ss[k];
                double yp, yq;
                rot(c, s, Vt[(int64_t)p * n + j], Vt[(int64_t)q * n + j], yp, yq);
                Vt[(int64_t)p * n + j] = yp;
                Vt[(int64_t)q * n + j] = yq;
            }
            __syncthreads();
        }
    }
    if (SH) {
        for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += JT) Ag[e] = A[e];
    }
    if (threadIdx.x == 0) *sweeps_done = sweep;
}

// Ascending order of the diagonal of A (ties by index): rank[i] = position.
__global__ void eig_rank(const double* __restrict__ A, int n, int* __restrict__ pos_of_rank,
                         double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ai = A[(int64_t)i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
        const double aj = A[(int64_t)j * n + j];
        rank += (aj < ai || (aj == ai && j < i)) ? 1 : 0;
    }
    pos_of_rank[rank] = i;
    w[rank] = ai;
}

// out[r][c] = scale(c) * Vt[pos_of_rank[c]][r] for c < ncol (row-major n x ncol)
__global__ void gather_cols(const double* __restrict__ Vt, int n, const int* __restrict__ pos_of_rank,
                            int ncol, const double* __restrict__ w, int mode, double* __restrict__ out,
                            double* __restrict__ sign) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)n * ncol) return;
    const int r = (int)(e / ncol), c = (int)(e % ncol);
    double f = 1.0;
    if (mode == 1) f = sqrt(fabs(w[c]));  // signed square-root factor
    out[e] = f * Vt[(int64_t)pos_of_rank[c] * n + r];
    if (sign && r == 0) sign[c] = w[c] < 0.0 ? -1.0 : 1.0;
}

__global__ void set_identity(double* __restrict__ V, int n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)n * n) V[e] = (e / n == e % n) ? 1.0 : 0.0;
}

}  // namespace

template <typename T>
int gemm_t(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, T alpha, const T* A,
           int64_t lda, const T* B, int64_t ldb, T beta, T* C, int64_t ldc) {
    const dim3 grid((unsigned)cdiv(N, GT), (unsigned)cdiv(M, GT));
    if (!ta && !tb)
        gemm_kernel<T, false, false><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (ta && !tb)
        gemm_kernel<T, true, false><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (!ta && tb)
        gemm_kernel<T, false, true><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else
        gemm_kernel<T, true, true><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    DFJK_LAUNCH_CHECK("gemm_kernel");
    return DFJK_OK;
}

int dgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, double alpha,
          const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
          int64_t ldc) {
    if (!ta && !tb && M >= WT && N >= WT && K >= WK) {
        const dim3 grid((unsigned)cdiv(N, WT), (unsigned)cdiv(M, WT));
        const bool pairs = lda % 2 == 0 && ldb % 2 == 0 && (reinterpret_cast<uintptr_t>(A) & 15) == 0 &&
                           (reinterpret_cast<uintptr_t>(B) & 15) == 0;
        if (pairs)
            gemm_nn_wide<true><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
        else
            gemm_nn_wide<false><<<grid, 256, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
        DFJK_LAUNCH_CHECK("gemm_nn_wide");
        return DFJK_OK;
    }
    return gemm_t<double>(st, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

int sgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, float alpha,
          const float* A, int64_t lda, const float* B, int64_t ldb, float beta, float* C,
          int64_t ldc) {
    return gemm_t<float>(st, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

int bgemm(hipStream_t st, bool ta, bool tb, int64_t M, int64_t N, int64_t K, const float* A, int64_t lda,
          const float* B, int64_t ldb, float* C, int64_t ldc) {
    const dim3 grid((unsigned)cdiv(N, GT), (unsigned)cdiv(M, GT));
    if (!ta && !tb) bgemm_kernel<false, false><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc);
    else if (ta && !tb) bgemm_kernel<true, false><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc);
    else if (!ta && tb) bgemm_kernel<false, true><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc);
    else bgemm_kernel<true, true><<<grid, 256, 0, st>>>(M, N, K, A, lda, B, ldb, C, ldc);
    DFJK_LAUNCH_CHECK("bgemm_kernel");
    return DFJK_OK;
}

int dots(hipStream_t st, const DotList& list, int nd, int64_t n, double* part, double* out) {
    if (nd < 1 || nd > kMaxDots) {
        set_error("dots: %d products outside [1, %d]", nd, kMaxDots);
        return DFJK_E_INVALID;
    }
    dots_partial<<<dim3(RBLK, (unsigned)nd), RT, 0, st>>>(list, n, part);
    DFJK_LAUNCH_CHECK("dots_partial");
    dots_finish<<<1, 64, 0, st>>>(part, nd, out);
    DFJK_LAUNCH_CHECK("dots_finish");
    return DFJK_OK;
}

size_t dots_part_elems(int nd) { return (size_t)nd * RBLK; }

int eigh(hipStream_t st, double* A, double* V, int n, bool v_identity, double* work, int* iwork,
         double* w) {
    if (n < 1 || n > kMaxEighN) {
        set_error("eigh: n=%d outside [1, %d]", n, kMaxEighN);
        return DFJK_E_INVALID;
    }
    if (v_identity) {
        set_identity<<<dim3((unsigned)cdiv((int64_t)n * n, 256)), 256, 0, st>>>(V, n);
        DFJK_LAUNCH_CHECK("set_identity");
    }
    // stop when the off-diagonal norm is below 1e-13 of the matrix norm
    // (convergence is quadratic, so the sweep after reaching ~1e-7 lands at
    // the rounding floor; a bound at n*eps can sit below that floor and is
    // then never met)
    if (n <= kJacobiShN) {
        const size_t bytes = sizeof(double) * (size_t)n * n;
        static bool attr_set = false;
        if (!attr_set) {
            DFJK_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(&jacobi_kernel<true>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)(sizeof(double) * kJacobiShN * kJacobiShN)));
            attr_set = true;
        }
        jacobi_kernel<true><<<1, JT, bytes, st>>>(A, V, n, work, 40, 1e-13, iwork);
    } else {
        jacobi_kernel<false><<<1, JT, 0, st>>>(A, V, n, work, 40, 1e-13, iwork);
    }
    DFJK_LAUNCH_CHECK("jacobi_kernel");
    eig_rank<<<dim3((unsigned)cdiv(n, 256)), 256, 0, st>>>(A, n, iwork + 1, w);
    DFJK_LAUNCH_CHECK("eig_rank");
    return DFJK_OK;
}

int eig_gather(hipStream_t st, const double* V, int n, const int* iwork, int ncol, const double* w,
               int mode, double* out, double* sign) {
    gather_cols<<<dim3((unsigned)cdiv((int64_t)n * ncol, 256)), 256, 0, st>>>(V, n, iwork + 1, ncol, w,
                                                                               mode, out, sign);
    DFJK_LAUNCH_CHECK("gather_cols");
    return DFJK_OK;
}

}  // namespace dfjk
