// Exchange matrix K on the matrix cores (FP64 MFMA, v_mfma_f64_16x16x4f64).
//
// For a factor C (nao x ncol) with column signs s_i and a scale a:
//   X_P = B_P C                                  (GEMM1, per auxiliary index P)
//   K   = a * sum_P sum_i s_i X_P[:,i] X_P[:,i]^T (GEMM2, a SYRK over (P,i))
// a = 2, s = +1 gives K for D = 2 C C^T (Eq. eq:df:eri contracted twice with
// the occupied orbitals).
//
// GEMM1 computes the transposed product X_P^T = C^T B_P so that each output
// row (P,i) is contiguous in mu; X is stored as rows k = P*ncol + i of length
// ldx.  B_P is read straight from the packed triangle: a 16 x 128 (nu, mu)
// chunk that lies wholly above or below the diagonal is a set of contiguous
// runs of one packed row, and is loaded along those runs.
//
// GEMM2 accumulates only the lower block triangle of K in 128 x 128 tiles,
// with the (P,i) contraction split over workgroups; each split writes its
// own partial tile, and a last kernel adds the splits in a fixed order and
// mirrors the result, so K is bitwise reproducible.
#include "internal.h"

namespace dfjk {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int KC = 16;      // contraction chunk held in LDS
constexpr int G1_BM = 128;  // mu columns per GEMM1 workgroup
constexpr int SY_T = 128;   // SYRK output tile

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline int64_t pidx(int64_t a, int64_t b) {
    const int64_t hi = a > b ? a : b, lo = a > b ? b : a;
    return hi * (hi + 1) / 2 + lo;
}

// ---------------------------------------------------------------- GEMM1
// Global -> register staging of one (nu, mu) chunk of B_P and one (nu, i)
// chunk of C.  Each thread holds 8 elements of each.
template <int NI>
struct G1Stage {
    double b[8];
    double c[(KC * 16 * NI + kThreads - 1) / kThreads];
};

template <int NI>
__device__ inline void g1_load(G1Stage<NI>& st, const double* __restrict__ Bp, int64_t nao,
                               const double* __restrict__ C, int64_t ldc, int64_t ncol, int64_t nu0,
                               int64_t mu0, int64_t i0, int tid) {
    constexpr int BI = 16 * NI;
    // C chunk: C[nu0 + k][i0 + ii], contiguous in ii
#pragma unroll
    for (int j = 0; j < (KC * BI + kThreads - 1) / kThreads; ++j) {
        const int e = tid + j * kThreads;
        const int k = e / BI, ii = e % BI;
        const int64_t nu = nu0 + k, i = i0 + ii;
        st.c[j] = (e < KC * BI && nu < nao && i < ncol) ? C[nu * ldc + i] : 0.0;
    }
    // B chunk
    if (nu0 + KC <= mu0) {
        // every nu < mu: element (nu, mu) sits in packed row mu at column nu
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = tid % KC, m = tid / KC + 16 * j;
            const int64_t nu = nu0 + k, mu = mu0 + m;
            st.b[j] = (mu < nao) ? Bp[mu * (mu + 1) / 2 + nu] : 0.0;
        }
    } else {
        // packed row nu (or a mixed chunk on the diagonal): run along mu
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = tid / G1_BM + 2 * j, m = tid % G1_BM;
            const int64_t nu = nu0 + k, mu = mu0 + m;
            st.b[j] = (nu < nao && mu < nao) ? Bp[pidx(nu, mu)] : 0.0;
        }
    }
}

template <int NI>
__device__ inline void g1_store(const G1Stage<NI>& st, double (*sC)[16 * NI + 1],
                                double (*sB)[G1_BM + 1], bool lower, int tid) {
    constexpr int BI = 16 * NI;
#pragma unroll
    for (int j = 0; j < (KC * BI + kThreads - 1) / kThreads; ++j) {
        const int e = tid + j * kThreads;
        if (e < KC * BI) sC[e / BI][e % BI] = st.c[j];
    }
    if (lower) {
#pragma unroll
        for (int j = 0; j < 8; ++j) sB[tid % KC][tid / KC + 16 * j] = st.b[j];
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) sB[tid / G1_BM + 2 * j][tid % G1_BM] = st.b[j];
    }
}

// X[(P*ncol + i)*ldx + mu] = sum_nu C[nu][i] B_P[nu][mu]
// grid: x = i block (16*NI rows), y = mu block (128), z = P
template <int NI>
__global__ __launch_bounds__(kThreads) void k_gemm1_f64(const double* __restrict__ B, int64_t ldB,
                                                         int64_t nao, const double* __restrict__ C,
                                                         int64_t ldc, int64_t ncol,
                                                         double* __restrict__ X, int64_t ldx) {
    constexpr int BI = 16 * NI;
    __shared__ double sC[2][KC][BI + 1];
    __shared__ double sB[2][KC][G1_BM + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t i0 = (int64_t)blockIdx.x * BI;
    const int64_t mu0 = (int64_t)blockIdx.y * G1_BM;
    const int64_t P = blockIdx.z;
    const double* Bp = B + P * ldB;

    v4d acc[NI][2];
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    const int64_t nchunks = cdiv(nao, KC);
    G1Stage<NI> st;
    g1_load<NI>(st, Bp, nao, C, ldc, ncol, 0, mu0, i0, tid);
    g1_store<NI>(st, sC[0], sB[0], KC <= mu0, tid);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        const int64_t nnext = (ch + 1) * KC;
        const bool more = ch + 1 < nchunks;
        if (more) g1_load<NI>(st, Bp, nao, C, ldc, ncol, nnext, mu0, i0, tid);
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[NI], b[2];
#pragma unroll
            for (int t = 0; t < NI; ++t) a[t] = sC[buf][kr][t * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 2; ++t) b[t] = sB[buf][kr][wave * 32 + t * 16 + (lane & 15)];
#pragma unroll
            for (int ti = 0; ti < NI; ++ti)
#pragma unroll
                for (int tj = 0; tj < 2; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
        if (more) g1_store<NI>(st, sC[buf ^ 1], sB[buf ^ 1], nnext + KC <= mu0, tid);
        __syncthreads();
    }
    // v_mfma_f64_16x16x4f64 result: lane l, element r holds row 4*r + l/16,
    // column l%16 of the 16x16 tile (operands: A[l%16][l/16], B[l/16][l%16])
#pragma unroll
    for (int ti = 0; ti < NI; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + ti * 16 + 4 * r + (lane >> 4);
                const int64_t mu = mu0 + wave * 32 + tj * 16 + (lane & 15);
                if (i < ncol && mu < nao) X[(P * ncol + i) * ldx + mu] = acc[ti][tj][r];
            }
}

// ---------------------------------------------------------------- GEMM2 (SYRK)
struct SyStage {
    double a[8], b[8];
};

__device__ inline void sy_load(SyStage& st, const double* __restrict__ X, int64_t ldx, int64_t nrows,
                               int64_t nao, int64_t ncol, const double* __restrict__ sign, int64_t k0,
                               int64_t kend, int64_t mu0, int64_t nu0, int tid) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = tid / SY_T + 2 * j, m = tid % SY_T;
        const int64_t row = k0 + k;
        const bool ok = row < kend;
        const double* xr = X + row * ldx;
        st.a[j] = (ok && mu0 + m < nao) ? xr[mu0 + m] : 0.0;
        double bv = (ok && nu0 + m < nao) ? xr[nu0 + m] : 0.0;
        if (sign && ok) bv *= sign[row % ncol];
        st.b[j] = bv;
    }
}

// partial[(s*ntl + t)][m][n] = sum_{k in split s} X[k][mu0+m] * sign_k * X[k][nu0+n]
// grid: x = lower tile t (I >= J), y = split s
__global__ __launch_bounds__(kThreads) void k_syrk_f64(const double* __restrict__ X, int64_t ldx,
                                                        int64_t nrows, int64_t nao, int64_t ncol,
                                                        const double* __restrict__ sign,
                                                        int64_t kchunk, int64_t ntl,
                                                        double* __restrict__ part) {
    __shared__ double sA[2][KC][SY_T + 1];
    __shared__ double sB[2][KC][SY_T + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t t = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t mu0 = I * SY_T, nu0 = J * SY_T;
    const int64_t s = blockIdx.y;
    const int64_t kbeg = s * kchunk;
    const int64_t kend = kbeg + kchunk < nrows ? kbeg + kchunk : nrows;

    v4d acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    if (kbeg < kend) {
        const int64_t nchunks = cdiv(kend - kbeg, KC);
        SyStage st;
        sy_load(st, X, ldx, nrows, nao, ncol, sign, kbeg, kend, mu0, nu0, tid);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sA[0][tid / SY_T + 2 * j][tid % SY_T] = st.a[j];
            sB[0][tid / SY_T + 2 * j][tid % SY_T] = st.b[j];
        }
        __syncthreads();
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const int buf = ch & 1;
            const bool more = ch + 1 < nchunks;
            if (more) sy_load(st, X, ldx, nrows, nao, ncol, sign, kbeg + (ch + 1) * KC, kend, mu0, nu0, tid);
#pragma unroll
            for (int kk = 0; kk < KC / 4; ++kk) {
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
                    for (int tj = 0; tj < 4; ++tj)
                        acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
            }
            if (more) {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    sA[buf ^ 1][tid / SY_T + 2 * j][tid % SY_T] = st.a[j];
                    sB[buf ^ 1][tid / SY_T + 2 * j][tid % SY_T] = st.b[j];
                }
            }
            __syncthreads();
        }
    }
    double* out = part + (s * ntl + t) * (int64_t)(SY_T * SY_T);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * 64 + ti * 16 + 4 * r + (lane >> 4);
                const int n = wn * 64 + tj * 16 + (lane & 15);
                out[m * SY_T + n] = acc[ti][tj][r];
            }
}

// K[mu][nu] = K[nu][mu] = scale * sum_s partial[s][t][m][n] over the lower
// triangle (on diagonal tiles only m >= n is used, so K is exactly symmetric).
__global__ __launch_bounds__(kThreads) void k_syrk_finish(const double* __restrict__ part,
                                                           int64_t nsplit, int64_t ntl, int64_t nao,
                                                           double scale, double* __restrict__ K) {
    const int64_t t = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    for (int e = threadIdx.x; e < SY_T * SY_T; e += kThreads) {
        const int m = e / SY_T, n = e % SY_T;
        const int64_t mu = I * SY_T + m, nu = J * SY_T + n;
        if (mu >= nao || nu >= nao) continue;
        if (I == J && m < n) continue;
        double v = 0.0;
        for (int64_t s = 0; s < nsplit; ++s) v += part[(s * ntl + t) * (int64_t)(SY_T * SY_T) + e];
        v *= scale;
        K[mu * nao + nu] = v;
        K[nu * nao + mu] = v;
    }
}

template <int NI>
int launch_gemm1(const dfjk_ctx* h, const double* C, int64_t ncol, double* X, int64_t ldx) {
    const dim3 grid((unsigned)cdiv(ncol, 16 * NI), (unsigned)cdiv(h->nao, G1_BM), (unsigned)h->naux);
    k_gemm1_f64<NI><<<grid, kThreads, 0, h->stream>>>(static_cast<const double*>(h->B), h->ldB, h->nao,
                                                       C, ncol, ncol, X, ldx);
    DFJK_LAUNCH_CHECK("k_gemm1_f64");
    return DFJK_OK;
}

// NI in 1..8 with the least padding of ncol to a multiple of 16*NI (ties: larger NI).
int pick_ni(int64_t ncol) {
    int best = 1;
    int64_t best_pad = INT64_MAX;
    for (int ni = 1; ni <= 8; ++ni) {
        const int64_t padded = cdiv(ncol, 16 * ni) * 16 * ni;
        if (padded <= best_pad) {
            best_pad = padded;
            best = ni;
        }
    }
    return best;
}

}  // namespace

int k_build_factored(dfjk_ctx* h, const double* C, int64_t ncol, const double* sign, double scale,
                     double* K) {
    if (h->dtype != DFJK_F64) {
        set_error("K for dtype %d is not built yet", h->dtype);
        return DFJK_E_DTYPE;
    }
    const int64_t ldx = h->nao;
    const int64_t nrows = h->naux * ncol;
    int rc;
    if ((rc = h->X.ensure(sizeof(double) * (size_t)nrows * (size_t)ldx))) return rc;
    double* X = static_cast<double*>(h->X.ptr);

    h->prof.begin(PH_K, h->stream);
    h->prof.begin(PH_K_GEMM1, h->stream);
    switch (pick_ni(ncol)) {
        case 1: rc = launch_gemm1<1>(h, C, ncol, X, ldx); break;
        case 2: rc = launch_gemm1<2>(h, C, ncol, X, ldx); break;
        case 3: rc = launch_gemm1<3>(h, C, ncol, X, ldx); break;
        case 4: rc = launch_gemm1<4>(h, C, ncol, X, ldx); break;
        case 5: rc = launch_gemm1<5>(h, C, ncol, X, ldx); break;
        case 6: rc = launch_gemm1<6>(h, C, ncol, X, ldx); break;
        case 7: rc = launch_gemm1<7>(h, C, ncol, X, ldx); break;
        default: rc = launch_gemm1<8>(h, C, ncol, X, ldx); break;
    }
    h->prof.end(PH_K_GEMM1, h->stream);
    if (rc) return rc;

    const int64_t nt = cdiv(h->nao, SY_T);
    const int64_t ntl = nt * (nt + 1) / 2;
    int64_t nsplit = cdiv(2048, ntl);
    const int64_t max_split = cdiv(nrows, 256);
    if (nsplit > max_split) nsplit = max_split;
    if (nsplit < 1) nsplit = 1;
    int64_t kchunk = cdiv(cdiv(nrows, nsplit), KC) * KC;
    nsplit = cdiv(nrows, kchunk);
    if ((rc = h->kpart.ensure(sizeof(double) * (size_t)(nsplit * ntl) * SY_T * SY_T))) return rc;
    double* part = static_cast<double*>(h->kpart.ptr);
    h->prof.begin(PH_K_SYRK, h->stream);
    k_syrk_f64<<<dim3((unsigned)ntl, (unsigned)nsplit), kThreads, 0, h->stream>>>(
        X, ldx, nrows, h->nao, ncol, sign, kchunk, ntl, part);
    h->prof.end(PH_K_SYRK, h->stream);
    DFJK_LAUNCH_CHECK("k_syrk_f64");
    h->prof.begin(PH_K_FINISH, h->stream);
    k_syrk_finish<<<dim3((unsigned)ntl), kThreads, 0, h->stream>>>(part, nsplit, ntl, h->nao, scale, K);
    h->prof.end(PH_K_FINISH, h->stream);
    h->prof.end(PH_K, h->stream);
    DFJK_LAUNCH_CHECK("k_syrk_finish");
    return DFJK_OK;
}

int k_build_from_D(dfjk_ctx* h, const double* D, double* K) {
    (void)D;
    (void)K;
    set_error("K from a density matrix is not built yet (pass Cocc)");
    return DFJK_E_INVALID;
}

}  // namespace dfjk
