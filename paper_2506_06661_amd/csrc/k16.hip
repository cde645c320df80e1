// Exchange on the 16-bit matrix cores (v_mfma_f32_16x16x32_bf16 / _f16) for B
// stored in BF16 or FP16.
//
// Both operands of a 16-bit matrix-core step carry 8 consecutive contraction
// indices per lane (lane l: A[l%16][8(l/16)+j], B[8(l/16)+j][l%16], j < 8;
// result row 4(l/16)+r, column l%16 in FP32).  The packed triangle is
// contiguous along the contraction index only below the diagonal, so the
// handle keeps a dense 16-bit copy of every B_P (both triangles, row length
// padded to a multiple of 64 with zeros, rows ldd + 64 elements apart), made
// once with an LDS-tiled transpose.  Then
//   GEMM1: X[P][mu][i] = sum_nu Bd_P[mu][nu] Ct[i][nu]   (Ct = C^T in 16 bits)
//   GEMM2: K[mu][nu]   = 2 sum_{P,i} X[P][mu][i] X[P][nu][i]
// with X stored in 16 bits, rows (P, mu) of ncp (nocc padded to 32) entries,
// so both products read 16-byte runs along the contraction index.  Products
// accumulate in FP32; split partials are added in FP64.
#include "internal.h"
#include "mma.h"
#include "numerics.h"

namespace dfjk {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int KS = 32;         // contraction chunk (one matrix-core step)
constexpr int64_t kMaxSum16 = 16384;  // longest FP32 running sum in the SYRK
constexpr int kFin16 = 16;            // SYRK finish: workgroups per output tile
// SYRK LDS rows: one 32-wide step, 4 pieces of 16 bytes, piece p of row r
// kept at p ^ ((r >> 1) & 3): conflict-free for the operand reads (16
// consecutive rows, one piece) and the row stores, where an 80-byte padded
// row spent half of its LDS cycles in bank conflicts (rocprofv3 on MI355X).
constexpr int LROW = KS;
__device__ inline int swz4(int row, int piece) { return (piece ^ ((row >> 1) & 3)) * 8; }

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <typename H>
struct Mma16;
template <>
struct Mma16<uint16_t> {  // bfloat16 bits
    __device__ static v4f step(u4 a, u4 b, v4f c) {
        v8bf av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c, 0, 0, 0);
    }
    __device__ static uint16_t from_float(float f) { return float_to_bf16_rne(f); }
    __device__ static uint16_t from_double(double x) { return float_to_bf16_rne(to_float_round_odd(x)); }
};
template <>
struct Mma16<_Float16> {
    __device__ static v4f step(u4 a, u4 b, v4f c) {
        v8h av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, c, 0, 0, 0);
    }
    __device__ static _Float16 from_float(float f) { return (_Float16)f; }
    __device__ static _Float16 from_double(double x) { return (_Float16)to_float_round_odd(x); }
};

// ---------------------------------------------------------------- dense copy
// Tile (I >= J) of 64 x 64 of the lower block triangle of B_P: packed rows
// nu in I, columns mu in J (mu <= nu) -> Bd[nu][mu] and Bd[mu][nu].  Elements
// outside the triangle or the matrix become zero, so the pad is zero too.
template <typename H>
__global__ __launch_bounds__(kT) void dense_copy(const H* __restrict__ B, int64_t ldB, int64_t nao,
                                                  int64_t ldd, int64_t rs, int64_t ntile, H* __restrict__ Bd) {
    __shared__ H tile[64][65];
    const int64_t P = blockIdx.y;
    const int64_t t = blockIdx.x;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t nu0 = I * 64, mu0 = J * 64;
    const H* Bp = B + P * ldB;
    H* D = Bd + P * ldd * rs;
    for (int e = threadIdx.x; e < 64 * 64; e += kT) {
        const int a = e / 64, b = e % 64;  // row nu0+a, column mu0+b
        const int64_t nu = nu0 + a, mu = mu0 + b;
        H v = H(0);
        if (nu < nao && mu <= nu) v = Bp[nu * (nu + 1) / 2 + mu];
        tile[a][b] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += kT) {
        const int a = e / 64, b = e % 64;
        const int64_t nu = nu0 + a, mu = mu0 + b;
        if (nu < ldd && mu < ldd && mu <= nu) D[nu * rs + mu] = tile[a][b];  // lower half
        // transposed: row mu0+a, column nu0+b holds B[nu0+b][mu0+a]
        const int64_t r = mu0 + a, c = nu0 + b;
        if (r < ldd && c < ldd && r < c) D[r * rs + c] = tile[b][a];
    }
    (void)ntile;
}

// Ct[i][nu] = C[nu][i] rounded once to the 16-bit format, for i < ncp,
// nu < ldd (zero outside C)
template <typename H>
__global__ void c_transpose(const double* __restrict__ C, int64_t nao, int64_t ncol, int64_t ncp,
                            int64_t ldd, int64_t rs, H* __restrict__ Ct) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ncp * ldd) return;
    const int64_t i = e / ldd, nu = e % ldd;
    const double v = (i < ncol && nu < nao) ? C[nu * ncol + i] : 0.0;
    Ct[i * rs + nu] = Mma16<H>::from_double(v);
}

// ---------------------------------------------------------------- GEMM1
// Workgroup: 128 rows mu (4 waves x 32) x 16*NI columns i, one P.  The
// contraction runs in 64-deep chunks (two matrix-core steps); the next
// chunk's 16-byte pieces are loaded into registers while the current chunk is
// multiplied from the other LDS buffer.
constexpr int KC16 = 64;
// LDS rows of one 64-deep chunk: 8 pieces of 16 bytes, piece p of row r kept
// at position p ^ (r & 7).  Measured on MI355X with rocprofv3
// (SQ_LDS_BANK_CONFLICT): the operand reads (16 consecutive rows, one piece)
// are conflict-free this way, while a padded 144-byte row spent half of its
// LDS cycles in bank conflicts.
constexpr int LROW64 = KC16;
__device__ inline int swz(int row, int piece) { return (piece ^ (row & 7)) * 8; }

template <typename H, int NI>
struct G16Stage {
    u4 a[(128 * KC16 / 8 + kT - 1) / kT];        // 1024 pieces / 256 threads = 4
    u4 b[(16 * NI * KC16 / 8 + kT - 1) / kT];    // 128*NI pieces
};

template <typename H, int NI>
__device__ inline void g16_load(G16Stage<H, NI>& st, const H* __restrict__ A, int64_t ldd, int64_t rs,
                                const H* __restrict__ Ct, int64_t ncp, int64_t mu0, int64_t i0,
                                int64_t k0, int tid) {
    constexpr int NA = 128 * KC16 / 8, NB = 16 * NI * KC16 / 8;
#pragma unroll
    for (int j = 0; j < (NA + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        const int r = e >> 3, q = e & 7;
        const int64_t mu = mu0 + r;
        st.a[j] = (e < NA && mu < ldd && k0 + 8 * q < ldd)
                      ? *reinterpret_cast<const u4*>(A + mu * rs + k0 + 8 * q)
                      : u4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int j = 0; j < (NB + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        const int r = e >> 3, q = e & 7;
        const int64_t i = i0 + r;
        st.b[j] = (e < NB && i < ncp && k0 + 8 * q < ldd)
                      ? *reinterpret_cast<const u4*>(Ct + i * rs + k0 + 8 * q)
                      : u4{0u, 0u, 0u, 0u};
    }
}

template <typename H, int NI>
__device__ inline void g16_store(const G16Stage<H, NI>& st, H (*sA)[LROW64], H (*sB)[LROW64], int tid) {
    constexpr int NA = 128 * KC16 / 8, NB = 16 * NI * KC16 / 8;
#pragma unroll
    for (int j = 0; j < (NA + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        if (e < NA) *reinterpret_cast<u4*>(&sA[e >> 3][swz(e >> 3, e & 7)]) = st.a[j];
    }
#pragma unroll
    for (int j = 0; j < (NB + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        if (e < NB) *reinterpret_cast<u4*>(&sB[e >> 3][swz(e >> 3, e & 7)]) = st.b[j];
    }
}

__device__ inline int64_t xcd_lid(int64_t hw, int64_t nblk) {
    constexpr int64_t NX = 8;
    const int64_t per = nblk / NX, rem = nblk % NX, x = hw % NX, q = hw / NX;
    return x * per + (x < rem ? x : rem) + q;
}

template <typename H, int NI>
__global__ __launch_bounds__(kT) void g1_16(const H* __restrict__ Bd, int64_t ldd, int64_t rs, int64_t nao,
                                             const H* __restrict__ Ct, int64_t ncol, int64_t ncp,
                                             H* __restrict__ X, int64_t nib, int64_t nmb, int64_t nblk) {
    constexpr int BI = 16 * NI, BM = 128;
    __shared__ H sA[2][BM][LROW64];
    __shared__ H sB[2][BI][LROW64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t lid = xcd_lid(blockIdx.x, nblk);
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ib * BI, mu0 = mb * BM;
    const H* A = Bd + P * ldd * rs;
    v4f acc[2][NI];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t nk = ldd / KC16 + (ldd % KC16 ? 1 : 0);
    G16Stage<H, NI> st;
    g16_load<H, NI>(st, A, ldd, rs, Ct, ncp, mu0, i0, 0, tid);
    g16_store<H, NI>(st, sA[0], sB[0], tid);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) g16_load<H, NI>(st, A, ldd, rs, Ct, ncp, mu0, i0, (kc + 1) * KC16, tid);
#pragma unroll
        for (int ks = 0; ks < KC16 / KS; ++ks) {
            u4 a[2];
            const int pc = ks * (KS / 8) + (lane >> 4);  // 16-byte piece of the chunk
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int r = wave * 32 + t * 16 + (lane & 15);
                a[t] = *reinterpret_cast<const u4*>(&sA[buf][r][swz(r, pc)]);
            }
#pragma unroll
            for (int n = 0; n < NI; ++n) {
                const int r = n * 16 + (lane & 15);
                const u4 b = *reinterpret_cast<const u4*>(&sB[buf][r][swz(r, pc)]);
#pragma unroll
                for (int t = 0; t < 2; ++t) acc[t][n] = Mma16<H>::step(a[t], b, acc[t][n]);
            }
        }
        if (more) g16_store<H, NI>(st, sA[buf ^ 1], sB[buf ^ 1], tid);
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int n = 0; n < NI; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t mu = mu0 + wave * 32 + t * 16 + 4 * (lane >> 4) + r;
                const int64_t i = i0 + n * 16 + (lane & 15);
                if (mu < nao && i < ncp)
                    X[(P * nao + mu) * ncp + i] = Mma16<H>::from_float(i < ncol ? acc[t][n][r] : 0.f);
            }
}

// GEMM1, direct form: no two wavefronts share rows mu, so each wavefront
// loads its A fragments (16-byte runs of dense B_P rows) straight from memory
// into the matrix-core layout; only C^T, which all four share, is staged in
// LDS.  Wavefront tile: 16*TM rows x 16*NI columns; workgroup: 4 wavefronts
// stacked along mu (64*TM rows).  The next 64-deep chunk of both operands is
// loaded into registers while the current one is multiplied.
template <int NI>
struct G16BStage {
    u4 b[(16 * NI * KC16 / 8 + kT - 1) / kT];
};

template <typename H, int NI>
__device__ inline void g16d_load_b(G16BStage<NI>& st, const H* __restrict__ Ct, int64_t ldd, int64_t rs, int64_t ncp,
                                   int64_t i0, int64_t k0, int tid) {
    constexpr int NB = 16 * NI * KC16 / 8;
#pragma unroll
    for (int j = 0; j < (NB + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        const int r = e >> 3, q = e & 7;
        const int64_t i = i0 + r;
        st.b[j] = (e < NB && i < ncp && k0 + 8 * q < ldd)
                      ? *reinterpret_cast<const u4*>(Ct + i * rs + k0 + 8 * q)
                      : u4{0u, 0u, 0u, 0u};
    }
}

template <typename H, int NI>
__device__ inline void g16d_store_b(const G16BStage<NI>& st, H (*sB)[LROW64], int tid) {
    constexpr int NB = 16 * NI * KC16 / 8;
#pragma unroll
    for (int j = 0; j < (NB + kT - 1) / kT; ++j) {
        const int e = tid + j * kT;
        if (e < NB) *reinterpret_cast<u4*>(&sB[e >> 3][swz(e >> 3, e & 7)]) = st.b[j];
    }
}

template <typename H, int TM>
__device__ inline void g16d_load_a(u4 (&fa)[TM][KC16 / KS], const H* __restrict__ A, int64_t ldd, int64_t rs,
                                   int64_t row0, int64_t k0, int lane) {
#pragma unroll
    for (int t = 0; t < TM; ++t) {
        const int64_t row = row0 + t * 16 + (lane & 15);
#pragma unroll
        for (int ks = 0; ks < KC16 / KS; ++ks) {
            const int64_t k = k0 + ks * KS + 8 * (lane >> 4);
            fa[t][ks] = (row < ldd && k < ldd) ? *reinterpret_cast<const u4*>(A + row * rs + k)
                                               : u4{0u, 0u, 0u, 0u};
        }
    }
}

template <typename H, int TM, int NI>
__global__ __launch_bounds__(kT) void g1_16d(const H* __restrict__ Bd, int64_t ldd, int64_t rs, int64_t nao,
                                              const H* __restrict__ Ct, int64_t ncol, int64_t ncp,
                                              H* __restrict__ X, int64_t nib, int64_t nmb, int64_t nblk) {
    constexpr int BI = 16 * NI, BM = 64 * TM, NKS = KC16 / KS;
    __shared__ H sB[2][BI][LROW64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t lid = xcd_lid(blockIdx.x, nblk);
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ib * BI, row0 = mb * BM + wave * 16 * TM;
    const H* A = Bd + P * ldd * rs;
    v4f acc[TM][NI];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t nk = ldd / KC16 + (ldd % KC16 ? 1 : 0);
    u4 fa[TM][NKS], fn[TM][NKS];
    G16BStage<NI> st;
    g16d_load_a<H, TM>(fa, A, ldd, rs, row0, 0, lane);
    g16d_load_b<H, NI>(st, Ct, ldd, rs, ncp, i0, 0, tid);
    g16d_store_b<H, NI>(st, sB[0], tid);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) {
            g16d_load_a<H, TM>(fn, A, ldd, rs, row0, (kc + 1) * KC16, lane);
            g16d_load_b<H, NI>(st, Ct, ldd, rs, ncp, i0, (kc + 1) * KC16, tid);
        }
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
            for (int n = 0; n < NI; ++n) {
                const int r = n * 16 + (lane & 15);
                const u4 b = *reinterpret_cast<const u4*>(&sB[buf][r][swz(r, ks * (KS / 8) + (lane >> 4))]);
#pragma unroll
                for (int t = 0; t < TM; ++t) acc[t][n] = Mma16<H>::step(fa[t][ks], b, acc[t][n]);
            }
        }
        if (more) {
            g16d_store_b<H, NI>(st, sB[buf ^ 1], tid);
#pragma unroll
            for (int t = 0; t < TM; ++t)
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) fa[t][ks] = fn[t][ks];
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < TM; ++t)
#pragma unroll
        for (int n = 0; n < NI; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t mu = row0 + t * 16 + 4 * (lane >> 4) + r;
                const int64_t i = i0 + n * 16 + (lane & 15);
                if (mu < nao && i < ncp)
                    X[(P * nao + mu) * ncp + i] = Mma16<H>::from_float(i < ncol ? acc[t][n][r] : 0.f);
            }
}

// ---------------------------------------------------------------- GEMM2
// Lower tile (I >= J) of 128 x 128 of K; 2 x 2 waves of 64 x 64; the
// contraction over (P, i) runs in 32-wide steps inside each P, staged two
// steps at a time with the next pair prefetched into registers.
struct S16Stage {
    u4 a[2], b[2];  // 2 x 128 rows x 32 halves = 1024 pieces / 256 threads... per operand 512: 2 each
};

template <typename H>
__device__ inline void s16_load(S16Stage& st, const H* __restrict__ X, int64_t nao, int64_t ncp,
                                int64_t P, int64_t k0, int64_t mu0, int64_t nu0, int tid) {
    const H* XP = X + P * nao * ncp;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int e = tid + j * kT;  // 512 pieces: row e>>2, quarter e&3
        const int r = e >> 2, q = e & 3;
        st.a[j] = (mu0 + r < nao) ? *reinterpret_cast<const u4*>(XP + (mu0 + r) * ncp + k0 + 8 * q)
                                  : u4{0u, 0u, 0u, 0u};
        st.b[j] = (nu0 + r < nao) ? *reinterpret_cast<const u4*>(XP + (nu0 + r) * ncp + k0 + 8 * q)
                                  : u4{0u, 0u, 0u, 0u};
    }
}

template <typename H>
__device__ inline void s16_store(const S16Stage& st, H (*sA)[LROW], H (*sB)[LROW], int tid) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int e = tid + j * kT;
        *reinterpret_cast<u4*>(&sA[e >> 2][swz4(e >> 2, e & 3)]) = st.a[j];
        *reinterpret_cast<u4*>(&sB[e >> 2][swz4(e >> 2, e & 3)]) = st.b[j];
    }
}

template <typename H>
__device__ __attribute__((always_inline)) inline void syrk16_body(int64_t lid, const H* __restrict__ X, int64_t nao, int64_t ncp, int64_t naux,
                                   int64_t pchunk, int64_t ntl, float* __restrict__ part) {
    __shared__ H sA[2][128][LROW];
    __shared__ H sB[2][128][LROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t t = lid % ntl, s = lid / ntl;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t mu0 = I * 128, nu0 = J * 128;
    const int64_t P0 = s * pchunk, P1 = P0 + pchunk < naux ? P0 + pchunk : naux;
    v4f acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t nks = ncp / KS;
    const int64_t nsteps = (P1 > P0 ? P1 - P0 : 0) * nks;  // (P, 32-wide step) in order
    if (nsteps > 0) {
        S16Stage st;
        s16_load<H>(st, X, nao, ncp, P0, 0, mu0, nu0, tid);
        s16_store<H>(st, sA[0], sB[0], tid);
        __syncthreads();
        for (int64_t step = 0; step < nsteps; ++step) {
            const int buf = step & 1;
            const bool more = step + 1 < nsteps;
            if (more) {
                const int64_t nx = step + 1;
                s16_load<H>(st, X, nao, ncp, P0 + nx / nks, (nx % nks) * KS, mu0, nu0, tid);
            }
            u4 a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ra = wm * 64 + q * 16 + (lane & 15), rb = wn * 64 + q * 16 + (lane & 15);
                a[q] = *reinterpret_cast<const u4*>(&sA[buf][ra][swz4(ra, lane >> 4)]);
                b[q] = *reinterpret_cast<const u4*>(&sB[buf][rb][swz4(rb, lane >> 4)]);
            }
#pragma unroll
            for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = Mma16<H>::step(a[ti], b[tj], acc[ti][tj]);
            if (more) s16_store<H>(st, sA[buf ^ 1], sB[buf ^ 1], tid);
            __syncthreads();
        }
    }
    float* out = part + (s * ntl + t) * (int64_t)(128 * 128);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * 64 + ti * 16 + 4 * (lane >> 4) + r;
                const int n = wn * 64 + tj * 16 + (lane & 15);
                out[m * 128 + n] = acc[ti][tj][r];
            }
}

template <typename H>
__global__ __launch_bounds__(kT) void syrk_16(const H* __restrict__ X, int64_t nao, int64_t ncp,
                                               int64_t naux, int64_t pchunk, int64_t ntl, int64_t nblk,
                                               float* __restrict__ part) {
    syrk16_body<H>(xcd_lid(blockIdx.x, nblk), X, nao, ncp, naux, pchunk, ntl, part);
}

// Lower tile (I >= J) of 256 x 256 of K; 2 x 2 waves of 128 x 128 (64
// accumulator blocks per wave, held in the matrix-core registers): per
// 32-wide step each wave reads 16 operand fragments from LDS for 64
// matrix-core steps, half the LDS and L2 traffic per step of the 128 tile.
struct S16WStage {
    u4 a[4], b[4];  // 256 rows x 4 pieces per operand = 1024 pieces / 256 threads
};

template <typename H>
__global__ __launch_bounds__(kT, 1) void syrk_16w(const H* __restrict__ X, int64_t nao, int64_t ncp,
                                                   int64_t naux, int64_t pchunk, int64_t ntl, int64_t nblk,
                                                   float* __restrict__ part) {
    __shared__ H sA[2][256][LROW];
    __shared__ H sB[2][256][LROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t lid = xcd_lid(blockIdx.x, nblk);
    const int64_t t = lid % ntl, s = lid / ntl;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t mu0 = I * 256, nu0 = J * 256;
    const int64_t P0 = s * pchunk, P1 = P0 + pchunk < naux ? P0 + pchunk : naux;
    v4f acc[8][8];
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
        for (int b = 0; b < 8; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    // rows past nao read row nao-1: they only feed output rows and columns
    // past nao, which the finish discards
    int64_t roff_a[4], roff_b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t r = (tid >> 2) + 64 * j;
        roff_a[j] = (mu0 + r < nao ? mu0 + r : nao - 1) * ncp + 8 * (tid & 3);
        roff_b[j] = (nu0 + r < nao ? nu0 + r : nao - 1) * ncp + 8 * (tid & 3);
    }
    const int64_t nks = ncp / KS;
    const int64_t nsteps = (P1 > P0 ? P1 - P0 : 0) * nks;  // (P, 32-wide step) in order
    if (nsteps > 0) {
        S16WStage st;
        const H* Pb = X + P0 * nao * ncp;
        int64_t kk = 0;
        auto load = [&]() {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                st.a[j] = *reinterpret_cast<const u4*>(Pb + kk + roff_a[j]);
                st.b[j] = *reinterpret_cast<const u4*>(Pb + kk + roff_b[j]);
            }
            kk += KS;
            if (kk == ncp) {
                kk = 0;
                Pb += nao * ncp;
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = (tid >> 2) + 64 * j, q = tid & 3;
                *reinterpret_cast<u4*>(&sA[buf][r][swz4(r, q)]) = st.a[j];
                *reinterpret_cast<u4*>(&sB[buf][r][swz4(r, q)]) = st.b[j];
            }
        };
        load();
        store(0);
        __syncthreads();
        for (int64_t step = 0; step < nsteps; ++step) {
            const int buf = step & 1;
            const bool more = step + 1 < nsteps;
            if (more) load();
            u4 a[8], b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int ra = wm * 128 + q * 16 + (lane & 15), rb = wn * 128 + q * 16 + (lane & 15);
                a[q] = *reinterpret_cast<const u4*>(&sA[buf][ra][swz4(ra, lane >> 4)]);
                b[q] = *reinterpret_cast<const u4*>(&sB[buf][rb][swz4(rb, lane >> 4)]);
            }
#pragma unroll
            for (int ti = 0; ti < 8; ++ti)
#pragma unroll
                for (int tj = 0; tj < 8; ++tj) acc[ti][tj] = Mma16<H>::step(a[ti], b[tj], acc[ti][tj]);
            // all 16 operand reads before the first product: left to itself
            // the compiler re-read 7 of the fragments into one register set,
            // each read waited for before its 8 products
            __builtin_amdgcn_sched_group_barrier(0x100, 16, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 64, 0);
            if (more) store(buf ^ 1);
            __syncthreads();
        }
    }
    float* out = part + (s * ntl + t) * (int64_t)(256 * 256);
#pragma unroll
    for (int ti = 0; ti < 8; ++ti)
#pragma unroll
        for (int tj = 0; tj < 8; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = wm * 128 + ti * 16 + 4 * (lane >> 4) + r;
                const int n = wn * 128 + tj * 16 + (lane & 15);
                out[m * 256 + n] = acc[ti][tj][r];
            }
}

// ---------------------------------------------------------------- 32 x 32 forms
// v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies A[l%32][8(l/32)+j] and
// B[8(l/32)+j][l%32] (j < 8, one 16-byte piece each); result register r of
// lane l is row 8(r/4) + 4(l/32) + r%4, column l%32.  Twice the work of a
// 16 x 16 x 32 step per operand piece, and on MI355X the register-only rate
// of this shape sustains 0.96-0.98 of the published peak against 0.87 for
// the 16 x 16 one (measured).
typedef float v16f __attribute__((ext_vector_type(16)));

template <typename H>
struct Mma32;
template <>
struct Mma32<uint16_t> {
    __device__ static v16f step(u4 a, u4 b, v16f c) {
        v8bf av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
    }
};
template <>
struct Mma32<_Float16> {
    __device__ static v16f step(u4 a, u4 b, v16f c) {
        v8h av, bv;
        __builtin_memcpy(&av, &a, 16);
        __builtin_memcpy(&bv, &b, 16);
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
    }
};
__device__ inline int mrow32(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__device__ inline v16f zero16() {
    v16f z;
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = 0.f;
    return z;
}

// 64-byte rows for 32 x 32 operand reads: piece p of row r at p ^ f(r), f
// from bits 2 and 4 of the row, free of bank conflicts when lanes l and
// l + 16 (l < 8) are served together and read rows 16 apart at one piece.
__device__ inline int swz4c(int row, int piece) {
    const int f = ((row >> 2) & 1) | (((row >> 4) & 1) << 1);
    return (piece ^ f) * 8;
}
// Staging order of those panels: thread t stores piece t & 3 of row
// st_row(t), so that lanes l and l + 16 store rows whose r % 4 differ (lane
// bit 4 becomes row bit 1).  Measured on MI355X (SQ_LDS_BANK_CONFLICT): the
// swz4 layout with rows t >> 2 spent 37.5% of LDS cycles in conflicts with
// 32 x 32 operand reads, this one none.
__device__ inline int st_row(int t) {
    return ((t >> 2) & 1) | (((t >> 4) & 1) << 1) | (((t >> 3) & 1) << 2) | ((t >> 5) << 3);
}

// GEMM1, X[P][mu][i] = sum_nu Bd_P[mu][nu] Ct[i][nu], wide form: workgroup =
// 8 wavefronts, 4 along mu (32 rows each) x 2 along i (16*NI columns each),
// i.e. a 128 x 32*NI output tile per P; with 32*NI >= the padded orbital
// count every element of Bd_P is read from memory once.  Per 64-deep chunk
// the 128 rows of Bd_P and the 32*NI rows of Ct are staged in LDS (128-byte
// rows, piece p of row r at p ^ (r & 7)), double-buffered, the next chunk
// loaded into registers while the current one is multiplied on
// 16 x 16 x 32 steps (2 x NI result blocks per wavefront).
constexpr int kT8 = 512;
constexpr int GW_M = 128;

template <int NI>
struct GwStage {
    static constexpr int NP = (GW_M + 32 * NI) * 8;        // 16-byte pieces per chunk
    static constexpr int PER = (NP + kT8 - 1) / kT8;       // per thread
    u4 v[PER];
};

template <typename H, int NI, bool PRE, bool SCHED = false>
__global__ __launch_bounds__(kT8, 1) void g1_w(const H* __restrict__ Bd, int64_t ldd, int64_t rs, int64_t nao,
                                                const H* __restrict__ Ct, int64_t ncol, int64_t ncp,
                                                H* __restrict__ X, int64_t nib, int64_t nmb, int64_t nblk) {
    constexpr int BI = 32 * NI, ROWS = GW_M + BI;
    __shared__ uint16_t sT[2][ROWS][LROW64];  // rows 0..127: Bd_P; rows 128..: Ct
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 3, wn = wave >> 2;
    const int64_t lid = xcd_lid(blockIdx.x, nblk);
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ib * BI, mu0 = mb * GW_M;
    const uint16_t* A = reinterpret_cast<const uint16_t*>(Bd) + P * ldd * rs;
    const uint16_t* Bt = reinterpret_cast<const uint16_t*>(Ct);
    using St = GwStage<NI>;
    // piece e = tid + j*512: row e>>3, piece e&7 of the 64-deep chunk
    const uint16_t* src[St::PER];
    bool ok[St::PER];
#pragma unroll
    for (int j = 0; j < St::PER; ++j) {
        const int e = tid + j * kT8, r = e >> 3;
        if (r < GW_M) {
            const int64_t row = mu0 + r;
            ok[j] = e < St::NP && row < ldd;
            src[j] = A + (ok[j] ? row : 0) * rs + 8 * (e & 7);
        } else {
            const int64_t row = i0 + (r - GW_M);
            ok[j] = e < St::NP && row < ncp;
            src[j] = Bt + (ok[j] ? row : 0) * rs + 8 * (e & 7);
        }
    }
    const u4 z4 = u4{0u, 0u, 0u, 0u};
    St st;
    // loads always read a valid address (row 0 stands in for rows outside the
    // operands); the pieces of such rows are replaced by zeros when stored
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int j = 0; j < St::PER; ++j) st.v[j] = *reinterpret_cast<const u4*>(src[j] + k0);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int j = 0; j < St::PER; ++j) {
            const int e = tid + j * kT8;
            if (e < St::NP) *reinterpret_cast<u4*>(&sT[buf][e >> 3][swz(e >> 3, e & 7)]) = ok[j] ? st.v[j] : z4;
        }
    };
    v4f acc[2][NI];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NI; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t nk = ldd / KC16;  // ldd is a multiple of 64
    load(0);
    store(0);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        const bool more = kc + 1 < nk;
        if (more) load((kc + 1) * KC16);
#pragma unroll
        for (int ks = 0; ks < KC16 / KS; ++ks) {
            const int pc = ks * (KS / 8) + (lane >> 4);
            u4 a[2];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int r = wm * 32 + t * 16 + (lane & 15);
                a[t] = *reinterpret_cast<const u4*>(&sT[buf][r][swz(r, pc)]);
            }
            if constexpr (PRE) {
                // every operand piece of the step is requested before the first
                // product, so the LDS latency is paid once per step
                u4 b[NI];
#pragma unroll
                for (int n = 0; n < NI; ++n) {
                    const int r = GW_M + wn * 16 * NI + n * 16 + (lane & 15);
                    b[n] = *reinterpret_cast<const u4*>(&sT[buf][r][swz(r, pc)]);
                }
#pragma unroll
                for (int n = 0; n < NI; ++n)
#pragma unroll
                    for (int t = 0; t < 2; ++t) acc[t][n] = Mma16<H>::step(a[t], b[n], acc[t][n]);
                if constexpr (SCHED) {
                    // keep several operand reads in flight ahead of the products:
                    // 6 reads, then (2 products, 1 read) until the reads run out
                    constexpr int R0 = 6 < NI + 2 ? 6 : NI + 2;
                    __builtin_amdgcn_sched_group_barrier(0x100, R0, 0);
#pragma unroll
                    for (int g = 0; g < NI + 2 - R0; ++g) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x008, 2 * NI - 2 * (NI + 2 - R0), 0);
                }
            } else {
#pragma unroll
                for (int n = 0; n < NI; ++n) {
                    const int r = GW_M + wn * 16 * NI + n * 16 + (lane & 15);
                    const u4 b = *reinterpret_cast<const u4*>(&sT[buf][r][swz(r, pc)]);
#pragma unroll
                    for (int t = 0; t < 2; ++t) acc[t][n] = Mma16<H>::step(a[t], b, acc[t][n]);
                }
            }
        }
        if (more) store(buf ^ 1);
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int n = 0; n < NI; ++n)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t mu = mu0 + wm * 32 + t * 16 + 4 * (lane >> 4) + r;
                const int64_t i = i0 + wn * 16 * NI + n * 16 + (lane & 15);
                if (mu < nao && i < ncp)
                    X[(P * nao + mu) * ncp + i] = Mma16<H>::from_float(i < ncol ? acc[t][n][r] : 0.f);
            }
}

// ---------------------------------------------------------------- GEMM1 on the packed triangle
// X[P][mu][i] = sum_nu B_P[mu][nu] Ct[i][nu] with B_P read straight from the
// packed lower triangle (element (a, b), a >= b, at a(a+1)/2 + b): no dense
// copy.  Workgroup: WM x WN wavefronts of FM x FN result blocks of 16 x 16,
// i.e. a BM = 16 FM WM by BI = 16 FN WN output tile of one P.  Per 64-deep
// chunk of nu the BM rows of B_P are staged in LDS as rows mu, nu contiguous:
//   below the diagonal (every nu <= every mu) packed row mu holds the chunk
//     contiguously: 16-byte loads at any 2-byte alignment, stored as loaded;
//   above it (every nu >= every mu) packed row nu holds mu contiguously: rows
//     nu and nu + 1 are loaded at 8 consecutive mu and interleaved into the
//     8 words (B[mu][nu], B[mu][nu + 1]), one 4-byte LDS store each;
//   the chunks crossing the diagonal element by element.
// Piece p of LDS row r sits at p ^ (r & 7) ^ ((r >> 3) & 7): the operand
// reads (16 consecutive rows, one piece) keep one row per piece within each
// 8 rows, and the word stores of 8 row-octets at one column land in 8
// different pieces.
constexpr int KCP = 64;
__device__ inline int swzp(int row, int piece) { return (piece ^ (row & 7) ^ ((row >> 3) & 7)) * 8; }

template <int WM, int WN, int FM, int FN>
struct G1P {
    static constexpr int NT = 64 * WM * WN, BM = 16 * FM * WM, BI = 16 * FN * WN;
    static constexpr int PB = 8 * BM / NT;             // B pieces per thread (two per above-diagonal unit)
    static constexpr int PC = (8 * BI + NT - 1) / NT;  // Ct pieces per thread
    static_assert((8 * BM) % NT == 0 && PB % 2 == 0, "tile shape");
};

template <typename H, int WM, int WN, int FM, int FN>
__device__ __attribute__((always_inline)) inline void g1p_body(int64_t lid, const H* __restrict__ Bp, int64_t ldB, int64_t nao,
                                const H* __restrict__ Ct, int64_t rs, int64_t ncol, int64_t ncp,
                                H* __restrict__ X, int64_t nib, int64_t nmb) {
    using G = G1P<WM, WN, FM, FN>;
    constexpr int BM = G::BM, BI = G::BI, NT = G::NT, PB = G::PB, PC = G::PC, OCT = BM / 8;
    __shared__ __attribute__((aligned(16))) uint16_t sA[2][BM][KCP];
    __shared__ __attribute__((aligned(16))) uint16_t sC[2][BI][KCP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WM, wn = wave / WM;
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ib * BI, mu0 = mb * BM;
    const uint16_t* Bw = reinterpret_cast<const uint16_t*>(Bp) + P * ldB;
    const uint16_t* Cw = reinterpret_cast<const uint16_t*>(Ct);
    // Ct pieces e = tid + j NT: row i0 + e/8, piece e%8 (rows past ncp read
    // row 0 and are stored as zeros)
    const uint16_t* csrc[PC];
    bool cok[PC];
#pragma unroll
    for (int j = 0; j < PC; ++j) {
        const int e = tid + j * NT;
        cok[j] = e < 8 * BI && i0 + (e >> 3) < ncp;
        csrc[j] = Cw + (cok[j] ? i0 + (e >> 3) : 0) * rs + 8 * (e & 7);
    }
    // below-diagonal pieces e = tid + j NT: packed row mu0 + e/8 (rows past
    // nao read row 0, which holds the chunk too, and are stored as zeros)
    int64_t trow[PB];
    bool rok[PB];
#pragma unroll
    for (int j = 0; j < PB; ++j) {
        const int64_t mu = mu0 + ((tid + j * NT) >> 3);
        rok[j] = mu < nao;
        trow[j] = rok[j] ? mu * (mu + 1) / 2 : 0;
    }
    const u4 z4 = u4{0u, 0u, 0u, 0u};
    u4 sb[PB], sc[PC];
    auto below = [&](int64_t nu0) { return nu0 + KCP <= mu0 + 1; };
    auto above = [&](int64_t nu0) { return nu0 >= mu0 + BM - 1; };
    auto load = [&](int64_t nu0) {
#pragma unroll
        for (int j = 0; j < PC; ++j) sc[j] = *reinterpret_cast<const u4*>(csrc[j] + nu0);
        if (below(nu0)) {
#pragma unroll
            for (int j = 0; j < PB; ++j) __builtin_memcpy(&sb[j], Bw + trow[j] + nu0 + 8 * ((tid + j * NT) & 7), 16);
        } else if (above(nu0)) {
            // unit u: rows nu0 + 2q, + 1 at mu0 + 8o .. + 7 (q < 32, o < BM/8);
            // rows past nao read row 0 at the same columns, which lie below
            // nu0 <= nao - 1, and are stored as zeros
#pragma unroll
            for (int u = 0; u < PB / 2; ++u) {
                const int e = tid + u * NT, o = e % OCT, q = e / OCT;
                const int64_t nu = nu0 + 2 * q;
                const int64_t t0 = nu < nao ? nu * (nu + 1) / 2 : 0;
                const int64_t t1 = nu + 1 < nao ? (nu + 1) * (nu + 2) / 2 : 0;
                __builtin_memcpy(&sb[2 * u], Bw + t0 + mu0 + 8 * o, 16);
                __builtin_memcpy(&sb[2 * u + 1], Bw + t1 + mu0 + 8 * o, 16);
            }
        } else if constexpr (BM == KCP) {
            // the diagonal block (nu0 == mu0): its lower triangle from the packed
            // rows (whole pieces as 16-byte loads, the piece holding the
            // diagonal element by element); the upper part is mirrored in LDS
            // after the store
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int e = tid + j * NT;
                const int64_t mu = mu0 + (e >> 3), nb = nu0 + 8 * (e & 7);
                if (mu < nao && nb + 7 <= mu) {
                    __builtin_memcpy(&sb[j], Bw + trow[j] + nb, 16);
                } else {
                    uint32_t w[4];
#pragma unroll
                    for (int t = 0; t < 8; t += 2) {
                        const uint32_t lo = (mu < nao && nb + t <= mu) ? (uint32_t)Bw[trow[j] + nb + t] : 0u;
                        const uint32_t hi = (mu < nao && nb + t + 1 <= mu) ? (uint32_t)Bw[trow[j] + nb + t + 1] : 0u;
                        w[t >> 1] = lo | (hi << 16);
                    }
                    sb[j] = u4{w[0], w[1], w[2], w[3]};
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int e = tid + j * NT;
                const int64_t mu = mu0 + (e >> 3);
                uint32_t w[4];
#pragma unroll
                for (int t = 0; t < 8; t += 2) {
                    uint32_t h2[2];
#pragma unroll
                    for (int d = 0; d < 2; ++d) {
                        const int64_t nu = nu0 + 8 * (e & 7) + t + d;
                        const int64_t a = mu > nu ? mu : nu, b = mu > nu ? nu : mu;
                        h2[d] = (mu < nao && nu < nao) ? (uint32_t)Bw[a * (a + 1) / 2 + b] : 0u;
                    }
                    w[t >> 1] = h2[0] | (h2[1] << 16);
                }
                sb[j] = u4{w[0], w[1], w[2], w[3]};
            }
        }
    };
    auto store = [&](int buf, int64_t nu0) {
#pragma unroll
        for (int j = 0; j < PC; ++j) {
            const int e = tid + j * NT;
            if (e < 8 * BI) *reinterpret_cast<u4*>(&sC[buf][e >> 3][swz(e >> 3, e & 7)]) = cok[j] ? sc[j] : z4;
        }
        if (above(nu0)) {
#pragma unroll
            for (int u = 0; u < PB / 2; ++u) {
                const int e = tid + u * NT, o = e % OCT, q = e / OCT;
                const int64_t nu = nu0 + 2 * q;
                const u4 a = nu < nao ? sb[2 * u] : z4, b = nu + 1 < nao ? sb[2 * u + 1] : z4;
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const uint32_t lo = (a[m >> 1] >> (16 * (m & 1))) & 0xffffu;
                    const uint32_t hi = (b[m >> 1] >> (16 * (m & 1))) & 0xffffu;
                    const int r = 8 * o + m;
                    *reinterpret_cast<uint32_t*>(&sA[buf][r][swzp(r, q >> 2) + 2 * (q & 3)]) = lo | (hi << 16);
                }
            }
        } else {
            const bool bl = below(nu0);
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                const int e = tid + j * NT, r = e >> 3;
                *reinterpret_cast<u4*>(&sA[buf][r][swzp(r, e & 7)]) = (!bl || rok[j]) ? sb[j] : z4;
            }
            if constexpr (BM == KCP) {
                if (!bl) {
                    // diagonal block: B[mu][nu] = B[nu][mu] above the diagonal
                    __syncthreads();
#pragma unroll 1
                    for (int k = 0; k < KCP * KCP / NT; ++k) {
                        const int e = tid + k * NT, r = e / KCP, c = e % KCP;
                        if (c > r) sA[buf][r][swzp(r, c >> 3) + (c & 7)] = sA[buf][c][swzp(c, r >> 3) + (r & 7)];
                    }
                }
            }
        }
    };
    v4f acc[FM][FN];
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int64_t nk = cdiv(nao, KCP);  // Ct holds zeros from nao to the next multiple of 64
    auto compute = [&](int buf) {
#pragma unroll
        for (int ks = 0; ks < KCP / KS; ++ks) {
            const int pc = ks * (KS / 8) + (lane >> 4);
            u4 a[FM], b[FN];
#pragma unroll
            for (int f = 0; f < FM; ++f) {
                const int r = wm * 16 * FM + f * 16 + (lane & 15);
                a[f] = *reinterpret_cast<const u4*>(&sA[buf][r][swzp(r, pc)]);
            }
#pragma unroll
            for (int n = 0; n < FN; ++n) {
                const int r = wn * 16 * FN + n * 16 + (lane & 15);
                b[n] = *reinterpret_cast<const u4*>(&sC[buf][r][swz(r, pc)]);
            }
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int f = 0; f < FM; ++f) acc[f][n] = Mma16<H>::step(a[f], b[n], acc[f][n]);
            if constexpr (FN >= 8) {
                // wide tiles: several operand reads in flight ahead of the
                // products: R0 reads, then (FM products, 1 read) until the
                // reads run out (narrow tiles keep the compiler's order, which
                // measured the same)
                constexpr int NR = FM + FN, R0 = 6 < NR ? 6 : NR;
                __builtin_amdgcn_sched_group_barrier(0x100, R0, 0);
#pragma unroll
                for (int g = 0; g < NR - R0; ++g) {
                    __builtin_amdgcn_sched_group_barrier(0x008, FM, 0);
                    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                }
                __builtin_amdgcn_sched_group_barrier(0x008, FM * FN - FM * (NR - R0), 0);
            }
        }
    };
    load(0);
    store(0, 0);
    __syncthreads();
    for (int64_t kc = 0; kc < nk; ++kc) {
        const bool more = kc + 1 < nk;
        if (more) load((kc + 1) * KCP);
        compute(kc & 1);
        if (more) store((kc & 1) ^ 1, (kc + 1) * KCP);
        __syncthreads();
    }
    if constexpr (BM * BI <= 2 * BM * KCP) {
        // the output tile through LDS (free after the last barrier), then
        // written as 16-byte pieces of the X rows
        uint16_t* sO = &sA[0][0][0];
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm * 16 * FM + f * 16 + 4 * (lane >> 4) + r;
                    const int col = wn * 16 * FN + n * 16 + (lane & 15);
                    const H v = Mma16<H>::from_float(i0 + col < ncol ? acc[f][n][r] : 0.f);
                    __builtin_memcpy(&sO[row * BI + col], &v, 2);
                }
        __syncthreads();
#pragma unroll
        for (int e = tid; e < BM * BI / 8; e += NT) {
            const int row = e / (BI / 8), pc = e % (BI / 8);
            const int64_t mu = mu0 + row, i = i0 + 8 * pc;
            if (mu < nao && i < ncp)
                *reinterpret_cast<u4*>(&X[(P * nao + mu) * ncp + i]) = *reinterpret_cast<const u4*>(&sO[row * BI + 8 * pc]);
        }
    } else {
#pragma unroll
        for (int f = 0; f < FM; ++f)
#pragma unroll
            for (int n = 0; n < FN; ++n)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t mu = mu0 + wm * 16 * FM + f * 16 + 4 * (lane >> 4) + r;
                    const int64_t i = i0 + wn * 16 * FN + n * 16 + (lane & 15);
                    if (mu < nao && i < ncp)
                        X[(P * nao + mu) * ncp + i] = Mma16<H>::from_float(i < ncol ? acc[f][n][r] : 0.f);
                }
    }
}

template <typename H, int WM, int WN, int FM, int FN>
__global__ __launch_bounds__(64 * WM * WN) void g1_p(const H* __restrict__ Bp, int64_t ldB, int64_t nao,
                                                      const H* __restrict__ Ct, int64_t rs, int64_t ncol,
                                                      int64_t ncp, H* __restrict__ X, int64_t nib, int64_t nmb,
                                                      int64_t nblk) {
    g1p_body<H, WM, WN, FM, FN>(xcd_lid(blockIdx.x, nblk), Bp, ldB, nao, Ct, rs, ncol, ncp, X, nib, nmb);
}

// GEMM2 on 256 x 256 lower tiles of K with 8 wavefronts (4 along mu x 2
// along nu, 64 x 128 each = 2 x 4 result blocks of 32 x 32 on 32 x 32 x 16
// steps).  The contraction over (P, i) runs in 32-wide steps inside each P;
// two steps (possibly of consecutive P) are staged per barrier, both
// 256-row panels of each in LDS, double-buffered, the next pair prefetched
// into registers.  Rows past nao read row nao-1: they only feed output rows
// and columns past nao, which the finish discards.
constexpr int kSyNS = 2;  // 32-wide steps per barrier

template <typename H>
__global__ __launch_bounds__(kT8, 1) void syrk_32(const H* __restrict__ X, int64_t nao, int64_t ncp,
                                                   int64_t naux, int64_t pchunk, int64_t ntl, int64_t nblk,
                                                   float* __restrict__ part) {
    __shared__ uint16_t sA[2][kSyNS][256][LROW];
    __shared__ uint16_t sB[2][kSyNS][256][LROW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t lid = xcd_lid(blockIdx.x, nblk);
    const int64_t t = lid % ntl, s = lid / ntl;
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t mu0 = I * 256, nu0 = J * 256;
    const int64_t P0 = s * pchunk, P1 = P0 + pchunk < naux ? P0 + pchunk : naux;
    v16f acc[2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = zero16();
    // staging: each panel of one step is 256 rows x 4 pieces = 1024 pieces, 2 per thread
    int64_t roff_a[2], roff_b[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t r = st_row(tid) + 128 * j;
        roff_a[j] = (mu0 + r < nao ? mu0 + r : nao - 1) * ncp + 8 * (tid & 3);
        roff_b[j] = (nu0 + r < nao ? nu0 + r : nao - 1) * ncp + 8 * (tid & 3);
    }
    const int64_t nks = ncp / KS;
    const int64_t nsteps = (P1 > P0 ? P1 - P0 : 0) * nks;  // (P, 32-wide step) in order
    const int64_t nchunks = (nsteps + kSyNS - 1) / kSyNS;
    if (nchunks > 0) {
        u4 sta[kSyNS][2], stb[kSyNS][2];
        const uint16_t* Pb = reinterpret_cast<const uint16_t*>(X) + P0 * nao * ncp;
        int64_t kk = 0, left = nsteps;
        const u4 z4 = u4{0u, 0u, 0u, 0u};
        auto load = [&]() {
#pragma unroll
            for (int q = 0; q < kSyNS; ++q) {
                const bool live = left > 0;
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    sta[q][j] = live ? *reinterpret_cast<const u4*>(Pb + kk + roff_a[j]) : z4;
                    stb[q][j] = live ? *reinterpret_cast<const u4*>(Pb + kk + roff_b[j]) : z4;
                }
                if (live) {
                    --left;
                    kk += KS;
                    if (kk == ncp) {
                        kk = 0;
                        Pb += nao * ncp;
                    }
                }
            }
        };
        auto store = [&](int buf) {
#pragma unroll
            for (int q = 0; q < kSyNS; ++q)
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const int r = st_row(tid) + 128 * j, p = tid & 3;
                    *reinterpret_cast<u4*>(&sA[buf][q][r][swz4c(r, p)]) = sta[q][j];
                    *reinterpret_cast<u4*>(&sB[buf][q][r][swz4c(r, p)]) = stb[q][j];
                }
        };
        load();
        store(0);
        __syncthreads();
        for (int64_t c = 0; c < nchunks; ++c) {
            const int buf = c & 1;
            const bool more = c + 1 < nchunks;
            if (more) load();
#pragma unroll
            for (int q = 0; q < kSyNS; ++q)
#pragma unroll
                for (int ks = 0; ks < KS / 16; ++ks) {
                    const int pc = 2 * ks + (lane >> 5);
                    u4 a[2], b[4];
#pragma unroll
                    for (int u = 0; u < 2; ++u) {
                        const int r = wm * 64 + u * 32 + (lane & 31);
                        a[u] = *reinterpret_cast<const u4*>(&sA[buf][q][r][swz4c(r, pc)]);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int r = wn * 128 + u * 32 + (lane & 31);
                        b[u] = *reinterpret_cast<const u4*>(&sB[buf][q][r][swz4c(r, pc)]);
                    }
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int tj = 0; tj < 4; ++tj) acc[ti][tj] = Mma32<H>::step(a[ti], b[tj], acc[ti][tj]);
                }
            if (more) store(buf ^ 1);
            __syncthreads();
        }
    }
    float* out = part + (s * ntl + t) * (int64_t)(256 * 256);
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = wm * 64 + ti * 32 + mrow32(lane, r);
                const int n = wn * 128 + tj * 32 + (lane & 31);
                out[m * 256 + n] = acc[ti][tj][r];
            }
}

// K = scale * sum_s part[s][t] over the lower triangle, mirrored (diagonal
// tiles use m >= n only, so K is exactly symmetric).
// grid: kFin16 blocks per lower tile, each adding up a contiguous slice of it
// (kFin16 workgroups per 128 x 128 block of the tile)
template <int TS>
__device__ __attribute__((always_inline)) inline void syrk16_finish_body(int64_t bid, const float* __restrict__ part, int64_t nsplit, int64_t ntl,
                                          int64_t nao, double scale, double* __restrict__ K) {
    constexpr int nsub = kFin16 * (TS / 128) * (TS / 128);
    constexpr int per = TS * TS / nsub;
    const int64_t t = bid / nsub;
    const int sub = (int)(bid % nsub);
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t stride = ntl * (int64_t)(TS * TS);
    for (int e = sub * per + (int)threadIdx.x; e < (sub + 1) * per; e += kT) {
        const int m = e / TS, n = e % TS;
        const int64_t mu = I * TS + m, nu = J * TS + n;
        if (mu >= nao || nu >= nao || (I == J && m < n)) continue;
        const float* p = part + t * (int64_t)(TS * TS) + e;
        double v = 0.0;
#pragma unroll 8
        for (int64_t s = 0; s < nsplit; ++s) v += (double)p[s * stride];  // fixed order
        v *= scale;
        K[mu * nao + nu] = v;
        K[nu * nao + mu] = v;
    }
}

template <int TS>
__global__ __launch_bounds__(kT) void syrk16_finish(const float* __restrict__ part, int64_t nsplit,
                                                     int64_t ntl, int64_t nao, double scale,
                                                     double* __restrict__ K) {
    syrk16_finish_body<TS>(blockIdx.x, part, nsplit, ntl, nao, scale, K);
}

template <typename H, int NI>
void launch_g1(hipStream_t st, const H* Bd, int64_t ldd, int64_t rs, int64_t nao, const H* Ct, int64_t ncol,
               int64_t ncp, H* X, int64_t naux) {
    const int64_t nib = cdiv(ncp, 16 * NI), nmb = cdiv(nao, 128);
    const int64_t nblk = nib * nmb * naux;
    g1_16<H, NI><<<dim3((unsigned)nblk), kT, 0, st>>>(Bd, ldd, rs, nao, Ct, ncol, ncp, X, nib, nmb, nblk);
}

template <typename H, int TM, int NI>
void launch_g1d(hipStream_t st, const H* Bd, int64_t ldd, int64_t rs, int64_t nao, const H* Ct, int64_t ncol,
                int64_t ncp, H* X, int64_t naux) {
    const int64_t nib = cdiv(ncp, 16 * NI), nmb = cdiv(nao, 64 * TM);
    const int64_t nblk = nib * nmb * naux;
    g1_16d<H, TM, NI><<<dim3((unsigned)nblk), kT, 0, st>>>(Bd, ldd, rs, nao, Ct, ncol, ncp, X, nib, nmb, nblk);
}

template <typename H, int NI, bool PRE = true, bool SCHED = false>
void launch_gw(hipStream_t st, const H* Bd, int64_t ldd, int64_t rs, int64_t nao, const H* Ct, int64_t ncol,
               int64_t ncp, H* X, int64_t naux) {
    const int64_t nib = cdiv(ncp, 32 * NI), nmb = cdiv(nao, GW_M);
    const int64_t nblk = nib * nmb * naux;
    g1_w<H, NI, PRE, SCHED><<<dim3((unsigned)nblk), kT8, 0, st>>>(Bd, ldd, rs, nao, Ct, ncol, ncp, X, nib, nmb, nblk);
}

template <typename H, int WM, int WN, int FM, int FN>
void launch_gp(hipStream_t st, const H* Bp, int64_t ldB, int64_t nao, const H* Ct, int64_t rs, int64_t ncol,
               int64_t ncp, H* X, int64_t naux) {
    using G = G1P<WM, WN, FM, FN>;
    const int64_t nib = cdiv(ncp, G::BI), nmb = cdiv(nao, G::BM);
    const int64_t nblk = nib * nmb * naux;
    g1_p<H, WM, WN, FM, FN><<<dim3((unsigned)nblk), G::NT, 0, st>>>(Bp, ldB, nao, Ct, rs, ncol, ncp, X, nib, nmb,
                                                                     nblk);
}

// Compiled 16-bit GEMM1 tiles: (orbital columns, basis-function rows) per
// workgroup; the first three stage both operands in LDS, the rest load A
// straight into registers.
template <typename H>
using G16Launch = void (*)(hipStream_t, const H*, int64_t, int64_t, const H*, int64_t, int64_t, H*, int64_t);
struct G16Tile {
    int cols, rows;
};
constexpr G16Tile kG16Tiles[] = {{64, 128}, {128, 128}, {208, 128}, {128, 128}, {208, 128},
                                 {128, 256}, {64, 256}, {416, 128}, {416, 128}, {256, 128},
                                 {96, 64},   {64, 64},   {32, 64}};
// 7: g1_w, 8 wavefronts, both operands staged in LDS, 416 columns, operand
// reads scheduled ahead of the products.  8 and up: g1_p on the packed
// triangle (no dense copy of B).
constexpr int kFirstPackedG16 = 8;
constexpr int kNumG16Tiles = sizeof(kG16Tiles) / sizeof(kG16Tiles[0]);

// Default tile: least padded orbital columns per unit of measured rate.  On
// MI355X at nao=2048, naux=1024, nocc=400 (BF16) the tiles of 64, 128 and 208
// columns (indices 0, 1, 4) executed 468, 740 and 741 TFLOP/s counting the
// padded columns (435, 578 and 713 of useful work).
inline int pick_g16_tile_16(int64_t ncp);

// Default: the 416-column g1_w tile when it pads the orbital columns by at
// most 10% more than the best of the other tiles (at nao=2048, naux=8192,
// nocc=400 on MI355X it took 35.7-36.2 ms against 37.0-37.3 for the
// 208-column direct tile); else that other tile.
inline int pick_g16_tile(int64_t ncp) {
    const int other = pick_g16_tile_16(ncp);
    const int64_t wo = kG16Tiles[other].cols;
    const double pad_other = (double)(cdiv(ncp, wo) * wo), pad_w = (double)(cdiv(ncp, 416) * 416);
    return pad_w <= 1.1 * pad_other ? 7 : other;
}

// The choice among the 16 x 16 x 32 tiles 0..6.
inline int pick_g16_tile_16(int64_t ncp) {
    static const int cand[3] = {0, 1, 4};
    static const double rate[3] = {468.0, 740.0, 741.0};
    int best = 1;
    double best_cost = 1e300;
    for (int c = 0; c < 3; ++c) {
        const int64_t w = kG16Tiles[cand[c]].cols;
        const double cost = (double)(cdiv(ncp, w) * w) / rate[c];
        if (cost < best_cost) {
            best_cost = cost;
            best = cand[c];
        }
    }
    return best;
}

// Bd / ldd: the dense copy (tiles below kFirstPackedG16); Bp / ldB: the
// packed triangle (tiles from kFirstPackedG16 on).
template <typename H>
void launch_g16(int t, hipStream_t st, const H* Bd, int64_t ldd, const H* Bp, int64_t ldB, int64_t rs, int64_t nao,
                const H* Ct, int64_t ncol, int64_t ncp, H* X, int64_t naux) {
    switch (t) {
        case 8: launch_gp<H, 4, 2, 2, 13>(st, Bp, ldB, nao, Ct, rs, ncol, ncp, X, naux); return;
        case 9: launch_gp<H, 4, 2, 2, 8>(st, Bp, ldB, nao, Ct, rs, ncol, ncp, X, naux); return;
        case 10: launch_gp<H, 2, 2, 2, 3>(st, Bp, ldB, nao, Ct, rs, ncol, ncp, X, naux); return;
        case 11: launch_gp<H, 2, 2, 2, 2>(st, Bp, ldB, nao, Ct, rs, ncol, ncp, X, naux); return;
        case 12: launch_gp<H, 2, 2, 2, 1>(st, Bp, ldB, nao, Ct, rs, ncol, ncp, X, naux); return;
        default: break;
    }
    switch (t) {
        case 0: launch_g1<H, 4>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 1: launch_g1<H, 8>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 2: launch_g1<H, 13>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 3: launch_g1d<H, 2, 8>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 4: launch_g1d<H, 2, 13>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 5: launch_g1d<H, 4, 8>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        case 6: launch_g1d<H, 4, 4>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
        default: launch_gw<H, 13, true, true>(st, Bd, ldd, rs, nao, Ct, ncol, ncp, X, naux); break;
    }
}

// 16-bit GEMM2 output tiles (edge).  At nao=2048, naux=8192, nocc=400 the
// 256 tile ran 687-695 TFLOP/s against 523-531 for the 128 tile; below
// nao=1024 it would leave few tiles to split over, so the 128 tile stays.
// Index 2: the 256 tile on 32 x 32 x 16 steps (syrk_32, 8 wavefronts); at
// nao=2048, naux=8192, nocc=400 it took 19.3-19.4 ms against 18.7-18.9 for
// the 16 x 16 x 32 256 tile, which stays the default.
constexpr int kSyrk16Tiles[] = {128, 256, 256};
constexpr int kNumSyrk16Tiles = 3;
inline int pick_syrk16_tile(int64_t nao) { return nao >= 1024 ? 1 : 0; }

// Dense row length of the 16-bit copy (64-deep chunks) and the GEMM2 split:
// about 2048 workgroups, and no FP32 running sum longer than kMaxSum16 terms
// (the split partials are added in FP64).
inline int64_t k16_ldd(int64_t nao) { return cdiv(nao, KC16) * KC16; }
// Row stride of the dense copy and of Ct: ldd plus 64 elements, so that rows
// are not a power-of-two number of bytes apart (at nao = 2048 a 4096-byte
// stride sends the same chunk of every row to the same memory channel).
inline int64_t k16_rs(int64_t ldd) { return ldd + 64; }

struct K16Plan {
    int64_t ncp, T, ntl, nsplit, pchunk;
    int kind;  // GEMM2 tile index
    size_t Bdense, Cw, X, kpart;  // bytes
};

K16Plan k16_plan(const dfjk_ctx* h, int64_t ncol) {
    K16Plan p;
    const int64_t nao = h->nao, naux = h->naux, ldd = k16_ldd(nao);
    p.ncp = cdiv(ncol, KS) * KS;
    int ts = h->k16_syrk_tile;
    if (ts < 0 || ts >= kNumSyrk16Tiles) ts = pick_syrk16_tile(nao);
    p.T = kSyrk16Tiles[ts];
    p.kind = ts;
    const int64_t nt = cdiv(nao, p.T);
    p.ntl = nt * (nt + 1) / 2;
    int64_t nsplit = cdiv(2048, p.ntl);
    if (nsplit < cdiv(naux * p.ncp, kMaxSum16)) nsplit = cdiv(naux * p.ncp, kMaxSum16);
    if (nsplit > naux) nsplit = naux;
    p.pchunk = cdiv(naux, nsplit);
    p.nsplit = cdiv(naux, p.pchunk);
    p.Bdense = 2 * (size_t)naux * (size_t)(ldd * k16_rs(ldd));
    p.Cw = 2 * (size_t)(p.ncp * k16_rs(ldd));
    p.X = 2 * (size_t)(naux * nao * p.ncp);
    p.kpart = sizeof(float) * (size_t)(p.nsplit * p.ntl) * p.T * p.T;
    return p;
}

template <typename H>
int make_dense_t(dfjk_ctx* h) {
    const int64_t ldd = k16_ldd(h->nao);
    int rc;
    if ((rc = h->Bdense.ensure(k16_plan(h, 1).Bdense))) return rc;
    const int64_t nt = cdiv(ldd, 64), ntile = nt * (nt + 1) / 2;
    dense_copy<H><<<dim3((unsigned)ntile, (unsigned)h->naux), kT, 0, h->stream>>>(
        static_cast<const H*>(h->B), h->ldB, h->nao, ldd, k16_rs(ldd), ntile, static_cast<H*>(h->Bdense.ptr));
    DFJK_LAUNCH_CHECK("dense_copy");
    h->dense_ready = true;
    return DFJK_OK;
}

template <typename H>
int k16_t(dfjk_ctx* h, const double* C, int64_t ncol, double scale, double* K) {
    const hipStream_t st = h->stream;
    const int64_t nao = h->nao, naux = h->naux;
    const int64_t ldd = k16_ldd(nao);
    const K16Plan plan = k16_plan(h, ncol);
    const int64_t ncp = plan.ncp;
    int rc;
    if ((rc = h->Cw.ensure(plan.Cw)) || (rc = h->X.ensure(plan.X)) || (rc = h->kpart.ensure(plan.kpart)))
        return rc;
    int t = h->k16_tile;
    if (t < 0 || t >= kNumG16Tiles) t = pick_g16_tile(ncp);
    if (t < kFirstPackedG16 && !h->dense_ready && (rc = make_dense_t<H>(h))) return rc;
    H* Ct = static_cast<H*>(h->Cw.ptr);
    H* X = static_cast<H*>(h->X.ptr);
    const H* Bd = static_cast<const H*>(h->Bdense.ptr);
    h->prof.begin(PH_K, st);
    c_transpose<H><<<dim3((unsigned)cdiv(ncp * ldd, 256)), 256, 0, st>>>(C, nao, ncol, ncp, ldd, k16_rs(ldd), Ct);
    DFJK_LAUNCH_CHECK("c_transpose");
    h->prof.begin(PH_K_GEMM1, st);
    launch_g16<H>(t, st, Bd, ldd, static_cast<const H*>(h->B), h->ldB, k16_rs(ldd), nao, Ct, ncol, ncp, X, naux);
    h->prof.end(PH_K_GEMM1, st);
    DFJK_LAUNCH_CHECK("g1_16");
    const int64_t T = plan.T, ntl = plan.ntl, nsplit = plan.nsplit, pchunk = plan.pchunk;
    float* part = static_cast<float*>(h->kpart.ptr);
    const dim3 grid((unsigned)(ntl * nsplit));
    h->prof.begin(PH_K_SYRK, st);
    if (plan.kind == 2)
        syrk_32<H><<<grid, kT8, 0, st>>>(X, nao, ncp, naux, pchunk, ntl, ntl * nsplit, part);
    else if (T == 256)
        syrk_16w<H><<<grid, kT, 0, st>>>(X, nao, ncp, naux, pchunk, ntl, ntl * nsplit, part);
    else
        syrk_16<H><<<grid, kT, 0, st>>>(X, nao, ncp, naux, pchunk, ntl, ntl * nsplit, part);
    h->prof.end(PH_K_SYRK, st);
    DFJK_LAUNCH_CHECK("syrk_16");
    h->prof.begin(PH_K_FINISH, st);
    if (T == 256)
        syrk16_finish<256><<<dim3((unsigned)(ntl * kFin16 * 4)), kT, 0, st>>>(part, nsplit, ntl, nao, scale, K);
    else
        syrk16_finish<128><<<dim3((unsigned)(ntl * kFin16)), kT, 0, st>>>(part, nsplit, ntl, nao, scale, K);
    h->prof.end(PH_K_FINISH, st);
    h->prof.end(PH_K, st);
    DFJK_LAUNCH_CHECK("syrk16_finish");
    return DFJK_OK;
}

// ---------------------------------------------------------------- batched
// The 16-bit exchange over many molecules: every phase is one launch over
// all molecules' blocks; a block finds its molecule by binary search in the
// phase's prefix table (molecules longest first).
__device__ inline int find_mol16(const int64_t* __restrict__ prefix, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename H>
__global__ __launch_bounds__(kT) void kb16_kernel(int kind, const MolDesc* __restrict__ mols, PhaseList pl) {
    const int64_t b = kind == BP_SYRK16 ? xcd_lid(blockIdx.x, pl.nblk) : (int64_t)blockIdx.x;
    const int j = find_mol16(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    const int64_t lid = b - pl.prefix[j];
    if (kind == BP_CT16) {
        const int64_t e = lid * kT + threadIdx.x;
        if (e < d.ncp16 * d.ldd16) {
            const int64_t i = e / d.ldd16, nu = e % d.ldd16;
            const double v = (i < d.nocc && nu < d.nao) ? d.C[nu * d.nocc + i] : 0.0;
            static_cast<H*>(d.Ct16)[i * d.rs16 + nu] = Mma16<H>::from_double(v);
        }
    } else if (kind == BP_SYRK16) {
        syrk16_body<H>(lid, static_cast<const H*>(d.X16), d.nao, d.ncp16, d.naux, d.pchunk16, d.ntl, d.kpart16);
    } else if (kind == BP_KFIN16) {
        syrk16_finish_body<128>(lid, d.kpart16, d.nsplit16, d.ntl, d.nao, 2.0, d.K);
    }
}

// GEMM1 of bucket FN - 1: 32 kG16WM rows x 32 FN columns per workgroup,
// on the packed triangle.
constexpr int kG16WM = 2;
template <typename H, int FN>
__global__ __launch_bounds__(128 * kG16WM, 4) void kb16_gemm1(const MolDesc* __restrict__ mols, PhaseList pl) {
    using G = G1P<kG16WM, 2, 2, FN>;
    const int64_t b = xcd_lid(blockIdx.x, pl.nblk);
    const int j = find_mol16(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    g1p_body<H, kG16WM, 2, 2, FN>(b - pl.prefix[j], static_cast<const H*>(d.B), d.ldB, d.nao,
                                  static_cast<const H*>(d.Ct16), d.rs16, d.nocc, d.ncp16,
                                  static_cast<H*>(d.X16), cdiv(d.ncp16, G::BI), cdiv(d.nao, G::BM));
}

template <typename H>
int k16_batch_phase_t(hipStream_t st, int kind, int bucket, const MolDesc* mols, const PhaseList& pl) {
    const dim3 grid((unsigned)pl.nblk);
    if (kind == BP_G16) {
        switch (bucket) {
            case 0: kb16_gemm1<H, 1><<<grid, 128 * kG16WM, 0, st>>>(mols, pl); break;
            case 1: kb16_gemm1<H, 2><<<grid, 128 * kG16WM, 0, st>>>(mols, pl); break;
            default: kb16_gemm1<H, 3><<<grid, 128 * kG16WM, 0, st>>>(mols, pl); break;
        }
        DFJK_LAUNCH_CHECK("kb16_gemm1");
    } else {
        kb16_kernel<H><<<grid, kT, 0, st>>>(kind, mols, pl);
        DFJK_LAUNCH_CHECK("kb16_kernel");
    }
    return DFJK_OK;
}

}  // namespace

int k_build_16(dfjk_ctx* h, const double* C, int64_t ncol, double scale, double* K) {
    if (h->dtype == DFJK_BF16) return k16_t<uint16_t>(h, C, ncol, scale, K);
    if (h->dtype == DFJK_F16) return k16_t<_Float16>(h, C, ncol, scale, K);
    set_error("16-bit exchange needs BF16 or FP16 B");
    return DFJK_E_DTYPE;
}

int k16_make_dense(dfjk_ctx* h) {
    if (h->dtype == DFJK_BF16) return make_dense_t<uint16_t>(h);
    if (h->dtype == DFJK_F16) return make_dense_t<_Float16>(h);
    return DFJK_OK;
}

int k16_reserve(dfjk_ctx* h, int64_t max_ncol) {
    // the SYRK tile may be changed later with dfjk_set_tile: reserve for both
    const int keep = h->k16_syrk_tile;
    size_t kp = 0;
    K16Plan p{};
    for (int t = 0; t < kNumSyrk16Tiles; ++t) {
        h->k16_syrk_tile = t;
        p = k16_plan(h, max_ncol);
        if (p.kpart > kp) kp = p.kpart;
    }
    h->k16_syrk_tile = keep;
    int rc;
    if ((rc = h->Bdense.ensure(p.Bdense)) || (rc = h->Cw.ensure(p.Cw)) || (rc = h->X.ensure(p.X)) ||
        (rc = h->kpart.ensure(kp)))
        return rc;
    return DFJK_OK;
}

int k16_tile_count() { return kNumG16Tiles; }

int k16_syrk_tile_count() { return kNumSyrk16Tiles; }

int k16_syrk_tile_size(int t) { return t >= 0 && t < kNumSyrk16Tiles ? kSyrk16Tiles[t] : 0; }

int k16_tile_info(int index, int* cols, int* rows) {
    if (index < 0 || index >= kNumG16Tiles) return DFJK_E_INVALID;
    *cols = kG16Tiles[index].cols;
    *rows = kG16Tiles[index].rows;
    return DFJK_OK;
}

// Batch geometry: C^T and X padded to 32 orbital columns; the GEMM2 split
// gives every molecule at least 32 workgroups and no workgroup more than
// about kBatch16SyrkTerms (P, i) terms (which also bounds its FP32 running
// sums).  Every workgroup writes a 64 KB partial tile, so fewer, longer
// splits save partial traffic.
constexpr int64_t kBatch16SyrkTerms = 4096;
void k16_batch_geometry(MolDesc& d, size_t* ct_bytes, size_t* x_bytes, size_t* kpart_bytes) {
    d.ldd16 = k16_ldd(d.nao);
    d.rs16 = k16_rs(d.ldd16);
    d.ncp16 = cdiv(d.nocc, KS) * KS;
    int64_t pchunk = kBatch16SyrkTerms / d.ncp16;
    const int64_t want = cdiv(32, d.ntl);
    if (pchunk > cdiv(d.naux, want)) pchunk = cdiv(d.naux, want);
    if (pchunk < 1) pchunk = 1;
    d.pchunk16 = pchunk;
    d.nsplit16 = cdiv(d.naux, pchunk);
    *ct_bytes = 2 * (size_t)(d.ncp16 * d.rs16);
    *x_bytes = 2 * (size_t)(d.naux * d.nao * d.ncp16);
    *kpart_bytes = sizeof(float) * (size_t)(d.nsplit16 * d.ntl) * 128 * 128;
}

// GEMM1 buckets: 32, 64 and at least 96 padded orbital columns.
int k16_batch_bucket(const MolDesc& d) {
    const int64_t w = d.ncp16 / KS;
    return (int)(w < 3 ? w : 3) - 1;
}

int64_t k16_batch_blocks(int kind, int bucket, const MolDesc& d) {
    switch (kind) {
        case BP_CT16: return cdiv(d.ncp16 * d.ldd16, kT);
        case BP_G16: return cdiv(d.ncp16, (int64_t)KS * (bucket + 1)) * cdiv(d.nao, 32 * kG16WM) * d.naux;
        case BP_SYRK16: return d.ntl * d.nsplit16;
        case BP_KFIN16: return d.ntl * kFin16;
        default: return 0;
    }
}

int k16_batch_phase(hipStream_t st, int kind, int bucket, int dtype, const MolDesc* mols, const PhaseList& pl) {
    if (pl.nblk <= 0) return DFJK_OK;
    if (dtype == DFJK_BF16) return k16_batch_phase_t<uint16_t>(st, kind, bucket, mols, pl);
    if (dtype == DFJK_F16) return k16_batch_phase_t<_Float16>(st, kind, bucket, mols, pl);
    set_error("16-bit exchange needs BF16 or FP16 B");
    return DFJK_E_DTYPE;
}

}  // namespace dfjk
