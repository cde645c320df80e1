/*
 * Plain FP64 CPU oracle for the density-fitted Coulomb/exchange build.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code with the GPU path.
 *
 * What is computed (paper Sec. IV.C.2, Eq. eq:df:eri): the four-index
 * electron-repulsion tensor is approximated by
 *     (mu nu|ka la) = sum_P B[P, mu nu] B[P, ka la]
 * with B the metric-factored three-index tensor T = L^-1 (Q|mu nu).  The
 * Coulomb and exchange matrices that Sec. II's get_jk returns for a density
 * D are the standard contractions
 *     J[mu,nu] = sum_{ka,la} (mu nu|ka la) D[ka,la] = sum_P rho_P B_P[mu,nu],
 *                rho_P = sum_{ka,la} B_P[ka,la] D[ka,la]
 *     K[mu,nu] = sum_{ka,la} (mu ka|nu la) D[ka,la] = sum_P (B_P D B_P)[mu,nu]
 * and, for D = 2 C C^T with C the occupied orbitals,
 *     K = 2 sum_P X_P X_P^T,  X_P = B_P C.
 * Every function below is that definition with plain loops: B_P is read
 * through the packed index p(mu,nu) = max*(max+1)/2 + min (the aosym='s2' /
 * tril_indices order used by the paper's three-index arrays), the sums run
 * over the full index ranges, and nothing is blocked or fused.
 *
 * B is row-major [nrows][ldB]; D, J, K are nao x nao row-major; C is
 * nao x nocc row-major.  The *_acc functions add the contribution of the
 * rows they are given, so a caller can stream B in row blocks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t pidx(int64_t mu, int64_t nu) {
    int64_t a = mu > nu ? mu : nu;
    int64_t b = mu > nu ? nu : mu;
    return a * (a + 1) / 2 + b;
}

static inline double bval(const double* Brow, int64_t mu, int64_t nu) { return Brow[pidx(mu, nu)]; }

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (timing runs at one thread and at all). */
void oracle_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Unpack one packed row into a full symmetric nao x nao matrix. */
static void unpack(const double* Brow, int64_t nao, double* full) {
    for (int64_t mu = 0; mu < nao; ++mu)
        for (int64_t nu = 0; nu < nao; ++nu) full[mu * nao + nu] = bval(Brow, mu, nu);
}

/*
 * rho_P = sum_{ka,la} B_P[ka,la] D[ka,la] for each of the nrows rows: row P
 * is unpacked to the full B_P, then the double sum runs over the full index
 * range (any real D).  Returns -1 if scratch memory cannot be had.
 */
int oracle_rho(const double* B, int64_t ldB, int64_t nao, int64_t nrows, const double* D,
               double* rho) {
    const int64_t n2 = nao * nao;
    int fail = 0;
#pragma omp parallel
    {
        double* Bf = (double*)malloc((size_t)n2 * sizeof(double));
        if (!Bf) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 1)
        for (int64_t P = 0; P < nrows; ++P) {
            if (!Bf) continue;
            unpack(B + P * ldB, nao, Bf);
            double s = 0.0;
            for (int64_t ka = 0; ka < nao; ++ka)
                for (int64_t la = 0; la < nao; ++la) s += Bf[ka * nao + la] * D[ka * nao + la];
            rho[P] = s;
        }
        free(Bf);
    }
    return fail ? -1 : 0;
}

/* Sum thread-private nao x nao accumulators into out, in thread order. */
static void reduce_private(double* priv, int nt, int64_t n2, double* out) {
    for (int t = 0; t < nt; ++t)
        for (int64_t i = 0; i < n2; ++i) out[i] += priv[(int64_t)t * n2 + i];
}

/*
 * J[mu,nu] += sum_P rho_P B_P[mu,nu] over the nrows rows given: each row is
 * unpacked to the full B_P and rho_P B_P is added over the full index range.
 * Threads take fixed contiguous ranges of P (static schedule) into private
 * accumulators that are added in thread order, so the result does not depend
 * on timing.  Returns -1 if scratch memory cannot be had.
 */
int oracle_J_acc(const double* B, int64_t ldB, int64_t nao, int64_t nrows, const double* rho,
                 double* J) {
    const int nt = oracle_num_threads();
    const int64_t n2 = nao * nao;
    double* priv = (double*)calloc((size_t)nt * (size_t)n2, sizeof(double));
    if (!priv) return -1;
    int fail = 0;
#pragma omp parallel num_threads(nt)
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double* Jt = priv + (int64_t)t * n2;
        double* Bf = (double*)malloc((size_t)n2 * sizeof(double));
        if (!Bf) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(static)
        for (int64_t P = 0; P < nrows; ++P) {
            if (!Bf) continue;
            unpack(B + P * ldB, nao, Bf);
            for (int64_t mu = 0; mu < nao; ++mu)
                for (int64_t nu = 0; nu < nao; ++nu) Jt[mu * nao + nu] += rho[P] * Bf[mu * nao + nu];
        }
        free(Bf);
    }
    if (!fail) reduce_private(priv, nt, n2, J);
    free(priv);
    return fail ? -1 : 0;
}

void oracle_unpack(const double* Brow, int64_t nao, double* full) { unpack(Brow, nao, full); }

/* K[mu,nu] += 2 sum_P sum_i X_P[mu,i] X_P[nu,i],  X_P = B_P C  (D = 2 C C^T). */
int oracle_K_C_acc(const double* B, int64_t ldB, int64_t nao, int64_t nrows, const double* C,
                   int64_t nocc, double* K) {
    const int nt = oracle_num_threads();
    const int64_t n2 = nao * nao;
    double* priv = (double*)calloc((size_t)nt * (size_t)n2, sizeof(double));
    if (!priv) return -1;
    int fail = 0;
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double* Kt = priv + (int64_t)t * n2;
        double* Bf = (double*)malloc((size_t)n2 * sizeof(double));
        double* X = (double*)malloc((size_t)(nao * (nocc > 0 ? nocc : 1)) * sizeof(double));
        if (!Bf || !X) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t P = 0; P < nrows; ++P) {
                unpack(B + P * ldB, nao, Bf);
                for (int64_t mu = 0; mu < nao; ++mu)
                    for (int64_t i = 0; i < nocc; ++i) {
                        double s = 0.0;
                        for (int64_t nu = 0; nu < nao; ++nu) s += Bf[mu * nao + nu] * C[nu * nocc + i];
                        X[mu * nocc + i] = s;
                    }
                for (int64_t mu = 0; mu < nao; ++mu)
                    for (int64_t nu = 0; nu < nao; ++nu) {
                        double s = 0.0;
                        for (int64_t i = 0; i < nocc; ++i) s += X[mu * nocc + i] * X[nu * nocc + i];
                        Kt[mu * nao + nu] += 2.0 * s;
                    }
            }
        }
        free(Bf);
        free(X);
    }
    if (!fail) reduce_private(priv, nt, n2, K);
    free(priv);
    return fail ? -1 : 0;
}

/* K += sum_P B_P D B_P (any real D). */
int oracle_K_D_acc(const double* B, int64_t ldB, int64_t nao, int64_t nrows, const double* D,
                   double* K) {
    const int nt = oracle_num_threads();
    const int64_t n2 = nao * nao;
    double* priv = (double*)calloc((size_t)nt * (size_t)n2, sizeof(double));
    if (!priv) return -1;
    int fail = 0;
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        double* Kt = priv + (int64_t)t * n2;
        double* Bf = (double*)malloc((size_t)n2 * sizeof(double));
        double* Y = (double*)malloc((size_t)n2 * sizeof(double));
        if (!Bf || !Y) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t P = 0; P < nrows; ++P) {
                unpack(B + P * ldB, nao, Bf);
                /* Y = B_P D */
                for (int64_t mu = 0; mu < nao; ++mu)
                    for (int64_t la = 0; la < nao; ++la) {
                        double s = 0.0;
                        for (int64_t ka = 0; ka < nao; ++ka) s += Bf[mu * nao + ka] * D[ka * nao + la];
                        Y[mu * nao + la] = s;
                    }
                /* K += Y B_P */
                for (int64_t mu = 0; mu < nao; ++mu)
                    for (int64_t nu = 0; nu < nao; ++nu) {
                        double s = 0.0;
                        for (int64_t la = 0; la < nao; ++la) s += Y[mu * nao + la] * Bf[la * nao + nu];
                        Kt[mu * nao + nu] += s;
                    }
            }
        }
        free(Bf);
        free(Y);
    }
    if (!fail) reduce_private(priv, nt, n2, K);
    free(priv);
    return fail ? -1 : 0;
}

/*
 * Exchange entries among a set of rows, for D = 2 C C^T:
 *   Ksel[r][s] = 2 sum_P sum_i X_P[mu_r,i] X_P[mu_s,i],
 *   X_P[mu_r,i] = sum_ka B_P[mu_r,ka] C[ka,i].
 * Bsel is nsel x naux x nao with Bsel[r][P][ka] = B_P[mu_r, ka] (the packed
 * columns p(mu_r, ka) of B), so full-size checks need only those columns.
 */
int oracle_K_C_rows(const double* Bsel, int64_t nsel, int64_t nao, int64_t naux, const double* C,
                    int64_t nocc, double* Ksel) {
    double* Xs = (double*)malloc((size_t)(nsel * naux * nocc) * sizeof(double));
    if (!Xs) return -1;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
    for (int64_t r = 0; r < nsel; ++r)
        for (int64_t P = 0; P < naux; ++P)
            for (int64_t i = 0; i < nocc; ++i) {
                const double* b = Bsel + (r * naux + P) * nao;
                double x = 0.0;
                for (int64_t ka = 0; ka < nao; ++ka) x += b[ka] * C[ka * nocc + i];
                Xs[(r * naux + P) * nocc + i] = x;
            }
#pragma omp parallel for collapse(2)
    for (int64_t r = 0; r < nsel; ++r)
        for (int64_t q = 0; q < nsel; ++q) {
            double s = 0.0;
            for (int64_t P = 0; P < naux; ++P)
                for (int64_t i = 0; i < nocc; ++i)
                    s += Xs[(r * naux + P) * nocc + i] * Xs[(q * naux + P) * nocc + i];
            Ksel[r * nsel + q] = 2.0 * s;
        }
    free(Xs);
    return 0;
}
