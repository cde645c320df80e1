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
constexpr int SY_T = 128;   // SYRK output tile

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline int64_t pidx(int64_t a, int64_t b) {
    const int64_t hi = a > b ? a : b, lo = a > b ? b : a;
    return hi * (hi + 1) / 2 + lo;
}

// ---------------------------------------------------------------- GEMM1
// Workgroup tile: BI = 16*NI rows i (all waves) x BM = 64*WM columns mu
// (each of the 4 waves owns 16*WM columns).  Per 16-deep nu chunk each thread
// stages NI elements of C and 4*WM elements of B_P in registers, then LDS.
//
// Address arithmetic is incremental: a thread's C elements and its
// below-diagonal B elements (packed row mu, column nu) advance by a constant
// per chunk; its above-diagonal B elements (packed row nu, column mu) follow
// the triangular row starts T(nu + 16) = T(nu) + 16 nu + 136.
template <int NI, int WM>
struct G1Stage {
    double b[4 * WM];
    double c[NI];
};

template <int NI, int WM>
struct G1Addr {
    int64_t c_off[NI];      // offset of C[nu0 + k][i] for the current chunk
    bool c_ok[NI];          // i < ncol
    int64_t lo_off[4 * WM]; // below-diagonal: mu(mu+1)/2 + nu0 + k
    int64_t up_row[4 * WM]; // above-diagonal: T(nu0 + k)
    bool mu_ok_lo[4 * WM], mu_ok_up;
};

template <int NI, int WM>
__device__ inline void g1_addr_init(G1Addr<NI, WM>& ad, int64_t nao, int64_t ldc, int64_t ncol,
                                    int64_t mu0, int64_t i0, int tid) {
    constexpr int BI = 16 * NI, BM = 64 * WM, ROWS = kThreads / BM;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int e = tid + j * kThreads;
        const int k = e / BI, ii = e % BI;
        ad.c_off[j] = (int64_t)k * ldc + i0 + ii;
        ad.c_ok[j] = i0 + ii < ncol;
    }
#pragma unroll
    for (int j = 0; j < 4 * WM; ++j) {
        const int64_t mu = mu0 + tid / KC + 16 * j;
        ad.lo_off[j] = mu * (mu + 1) / 2 + tid % KC;
        ad.mu_ok_lo[j] = mu < nao;
        const int64_t nu = tid / BM + ROWS * j;
        ad.up_row[j] = nu * (nu + 1) / 2;
    }
    ad.mu_ok_up = mu0 + tid % BM < nao;
}

template <int NI, int WM>
__device__ inline void g1_load(G1Stage<NI, WM>& st, const G1Addr<NI, WM>& ad,
                               const double* __restrict__ Bp, int64_t nao,
                               const double* __restrict__ C, int64_t nu0, int64_t mu0, int tid) {
    constexpr int BI = 16 * NI, BM = 64 * WM, ROWS = kThreads / BM;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int k = (tid + j * kThreads) / BI;
        st.c[j] = (ad.c_ok[j] && nu0 + k < nao) ? C[ad.c_off[j]] : 0.0;
    }
    if (nu0 + KC <= mu0) {
        // every nu < mu: packed row mu, columns nu0 .. nu0+15
#pragma unroll
        for (int j = 0; j < 4 * WM; ++j) st.b[j] = ad.mu_ok_lo[j] ? Bp[ad.lo_off[j]] : 0.0;
    } else if (nu0 >= mu0 + BM - 1) {
        // every nu >= mu: packed row nu, columns mu0 .. mu0+BM-1
        const int m = tid % BM;
#pragma unroll
        for (int j = 0; j < 4 * WM; ++j) {
            const int64_t nu = nu0 + tid / BM + ROWS * j;
            st.b[j] = (nu < nao && ad.mu_ok_up) ? Bp[ad.up_row[j] + mu0 + m] : 0.0;
        }
    } else {
        // chunk crossing the diagonal
#pragma unroll
        for (int j = 0; j < 4 * WM; ++j) {
            const int k = tid / BM + ROWS * j, m = tid % BM;
            const int64_t nu = nu0 + k, mu = mu0 + m;
            st.b[j] = (nu < nao && mu < nao) ? Bp[pidx(nu, mu)] : 0.0;
        }
    }
}

// Move the addresses from chunk nu0 to chunk nu0 + KC.
template <int NI, int WM>
__device__ inline void g1_addr_next(G1Addr<NI, WM>& ad, int64_t nu0, int64_t ldc, int tid) {
    constexpr int BM = 64 * WM, ROWS = kThreads / BM;
#pragma unroll
    for (int j = 0; j < NI; ++j) ad.c_off[j] += (int64_t)KC * ldc;
#pragma unroll
    for (int j = 0; j < 4 * WM; ++j) {
        ad.lo_off[j] += KC;
        const int64_t nu = nu0 + tid / BM + ROWS * j;
        ad.up_row[j] += (int64_t)KC * nu + (KC * (KC + 1)) / 2;
    }
}

template <int NI, int WM>
__device__ inline void g1_store(const G1Stage<NI, WM>& st, double (*sC)[16 * NI + 1],
                                double (*sB)[64 * WM + 1], bool lower, int tid) {
    constexpr int BI = 16 * NI, BM = 64 * WM, ROWS = kThreads / BM;
#pragma unroll
    for (int j = 0; j < NI; ++j) {
        const int e = tid + j * kThreads;
        sC[e / BI][e % BI] = st.c[j];
    }
    if (lower) {
#pragma unroll
        for (int j = 0; j < 4 * WM; ++j) sB[tid % KC][tid / KC + 16 * j] = st.b[j];
    } else {
#pragma unroll
        for (int j = 0; j < 4 * WM; ++j) sB[tid / BM + ROWS * j][tid % BM] = st.b[j];
    }
}

// Block order: consecutive hardware block ids go round-robin to the 8 XCDs.
// Renumber so that runs of consecutive logical ids share an XCD (and its L2):
// the i-blocks and mu-blocks of one P then read B_P through one L2.
__device__ inline int64_t xcd_logical(int64_t hw, int64_t nblk) {
    constexpr int64_t NX = 8;
    const int64_t per = nblk / NX, rem = nblk % NX;
    const int64_t x = hw % NX, q = hw / NX;
    // XCD x holds logical ids [x*per + min(x, rem), ...) ; blocks past per*NX keep their order
    if (q < per) return x * per + (x < rem ? x : rem) + q;
    return x * per + (x < rem ? x : rem) + per;  // only the first rem XCDs get one more block
}

// X[(P*ncol + i)*ldx + mu] = sum_nu C[nu][i] B_P[nu][mu]
// 1-D grid of nib * nmb * naux blocks; logical id -> (i block fastest, mu block, P)
template <int NI, int WM>
__global__ __launch_bounds__(kThreads) void k_gemm1_f64(const double* __restrict__ B, int64_t ldB,
                                                         int64_t nao, const double* __restrict__ C,
                                                         int64_t ldc, int64_t ncol,
                                                         double* __restrict__ X, int64_t ldx,
                                                         int64_t nib, int64_t nmb, int64_t nblk) {
    constexpr int BI = 16 * NI, BM = 64 * WM;
    __shared__ double sC[2][KC][BI + 1];
    __shared__ double sB[2][KC][BM + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t lid = xcd_logical(blockIdx.x, nblk);
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ib * BI, mu0 = mb * BM;
    const double* Bp = B + P * ldB;

    v4d acc[NI][WM];
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
        for (int b = 0; b < WM; ++b) acc[a][b] = v4d{0.0, 0.0, 0.0, 0.0};

    const int64_t nchunks = cdiv(nao, KC);
    G1Stage<NI, WM> st;
    G1Addr<NI, WM> ad;
    g1_addr_init<NI, WM>(ad, nao, ldc, ncol, mu0, i0, tid);
    g1_load<NI, WM>(st, ad, Bp, nao, C, 0, mu0, tid);
    g1_store<NI, WM>(st, sC[0], sB[0], KC <= mu0, tid);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        const int64_t nnext = (ch + 1) * KC;
        const bool more = ch + 1 < nchunks;
        if (more) {
            g1_addr_next<NI, WM>(ad, ch * KC, ldc, tid);
            g1_load<NI, WM>(st, ad, Bp, nao, C, nnext, mu0, tid);
        }
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            double a[NI], b[WM];
#pragma unroll
            for (int t = 0; t < NI; ++t) a[t] = sC[buf][kr][t * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < WM; ++t) b[t] = sB[buf][kr][wave * 16 * WM + t * 16 + (lane & 15)];
#pragma unroll
            for (int ti = 0; ti < NI; ++ti)
#pragma unroll
                for (int tj = 0; tj < WM; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
        if (more) g1_store<NI, WM>(st, sC[buf ^ 1], sB[buf ^ 1], nnext + KC <= mu0, tid);
        __syncthreads();
    }
    // v_mfma_f64_16x16x4f64 result: lane l, element r holds row 4*r + l/16,
    // column l%16 of the 16x16 tile (operands: A[l%16][l/16], B[l/16][l%16])
#pragma unroll
    for (int ti = 0; ti < NI; ++ti)
#pragma unroll
        for (int tj = 0; tj < WM; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + ti * 16 + 4 * r + (lane >> 4);
                const int64_t mu = mu0 + wave * 16 * WM + tj * 16 + (lane & 15);
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
                                                        int64_t kchunk, int64_t ntl, int64_t nblk,
                                                        double* __restrict__ part) {
    __shared__ double sA[2][KC][SY_T + 1];
    __shared__ double sB[2][KC][SY_T + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    // all tiles of one split run on one XCD and share its L2 copy of the X rows
    const int64_t lid = xcd_logical(blockIdx.x, nblk);
    const int64_t t = lid % ntl;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t mu0 = I * SY_T, nu0 = J * SY_T;
    const int64_t s = lid / ntl;
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

template <int NI, int WM>
int launch_gemm1(const dfjk_ctx* h, const double* C, int64_t ncol, double* X, int64_t ldx) {
    const int64_t nib = cdiv(ncol, 16 * NI), nmb = cdiv(h->nao, 64 * WM);
    const int64_t nblk = nib * nmb * h->naux;
    k_gemm1_f64<NI, WM><<<dim3((unsigned)nblk), kThreads, 0, h->stream>>>(
        static_cast<const double*>(h->B), h->ldB, h->nao, C, ncol, ncol, X, ldx, nib, nmb, nblk);
    DFJK_LAUNCH_CHECK("k_gemm1_f64");
    return DFJK_OK;
}

// Compiled GEMM1 tiles: (NI, WM) = (i tiles of 16, mu tiles of 16 per wave).
struct G1Tile {
    int ni, wm;
    int (*launch)(const dfjk_ctx*, const double*, int64_t, double*, int64_t);
};
const G1Tile kG1Tiles[] = {
    {1, 2, launch_gemm1<1, 2>}, {2, 2, launch_gemm1<2, 2>}, {3, 2, launch_gemm1<3, 2>},
    {4, 2, launch_gemm1<4, 2>}, {5, 2, launch_gemm1<5, 2>}, {6, 2, launch_gemm1<6, 2>},
    {7, 2, launch_gemm1<7, 2>}, {8, 2, launch_gemm1<8, 2>}, {13, 1, launch_gemm1<13, 1>},
    {4, 4, launch_gemm1<4, 4>}, {7, 1, launch_gemm1<7, 1>}, {5, 1, launch_gemm1<5, 1>},
};
constexpr int kNumG1Tiles = sizeof(kG1Tiles) / sizeof(kG1Tiles[0]);

// Default tile: least padded work, where each extra i block costs another
// read of the B tile (weight 1/2 of a padded column block), among the tiles
// that keep two waves per SIMD (FP64 sweep on MI355X, nao=1024, nocc=200:
// (7,1) 43.8 TFLOP/s, (5,2) 43.5, (13,1) 40.4, (1,2) 32.6).
int pick_g1_tile(int64_t ncol) {
    int best = 0;
    double best_cost = 1e300;
    for (int t = 0; t < kNumG1Tiles; ++t) {
        const int ni = kG1Tiles[t].ni, wm = kG1Tiles[t].wm;
        if (ni * wm > 7) continue;  // larger accumulator sets leave one wave per SIMD
        const double padded = (double)(cdiv(ncol, 16 * ni) * 16 * ni);
        const double cost = padded * (1.0 + 0.5 / ni);
        if (cost < best_cost) {
            best_cost = cost;
            best = t;
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
    int tile = h->g1_tile >= 0 && h->g1_tile < kNumG1Tiles ? h->g1_tile : pick_g1_tile(ncol);
    rc = kG1Tiles[tile].launch(h, C, ncol, X, ldx);
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
    k_syrk_f64<<<dim3((unsigned)(ntl * nsplit)), kThreads, 0, h->stream>>>(
        X, ldx, nrows, h->nao, ncol, sign, kchunk, ntl, ntl * nsplit, part);
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

int k_tile_count() { return kNumG1Tiles; }

int k_tile_info(int t, int* ni, int* wm) {
    if (t < 0 || t >= kNumG1Tiles) return DFJK_E_INVALID;
    *ni = kG1Tiles[t].ni;
    *wm = kG1Tiles[t].wm;
    return DFJK_OK;
}

}  // namespace dfjk
