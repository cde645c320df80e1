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
#include "mma.h"

namespace dfjk {

namespace {

constexpr int kThreads = 256;
constexpr int KC = 16;      // contraction chunk held in LDS
constexpr int SY_T = 128;   // SYRK output tile
constexpr int64_t kMaxSum32 = 16384;  // longest FP32 running sum in the SYRK
constexpr int kFinSub = 16;           // SYRK finish: workgroups per output tile

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline int64_t pidx(int64_t a, int64_t b) {
    const int64_t hi = a > b ? a : b, lo = a > b ? b : a;
    return hi * (hi + 1) / 2 + lo;
}

// Storage element of B -> compute type (exact for every pair used here).
template <typename T, typename TS>
__device__ inline T to_compute(TS x) {
    return (T)x;
}
template <>
__device__ inline float to_compute<float, uint16_t>(uint16_t x) {  // bfloat16 bits
    return __uint_as_float((uint32_t)x << 16);
}
template <>
__device__ inline float to_compute<float, _Float16>(_Float16 x) {
    return (float)x;
}

// ---------------------------------------------------------------- GEMM1
// Workgroup tile: BI = 16*NI rows i (all waves) x BM = 64*WM columns mu
// (each of the 4 waves owns 16*WM columns).  Per 16-deep nu chunk each thread
// stages its share of C (VC consecutive orbitals of a row per load) and of
// B_P (VB consecutive elements of a packed row per load: along nu below the
// diagonal, along mu above it) in registers, then LDS.  VC = VB = 1 is one
// element per load; the wider forms use 16-byte loads of C where its rows
// are 16-byte aligned and loads of up to 16 bytes of B at any alignment (the
// GPU's global loads take unaligned addresses), with element loads at the
// edges (past ncol or nao).
//
// Address arithmetic is incremental: a thread's C elements and its
// below-diagonal B elements (packed row mu, column nu) advance by a constant
// per chunk; its above-diagonal B elements (packed row nu, column mu) follow
// the triangular row starts T(nu + 16) = T(nu) + 16 nu + 136.
template <typename T, int NI, int VC>
struct G1C {
    static constexpr int V = VC;                  // orbitals per load
    static constexpr int VPR = 16 * NI / V;       // loads per row of the C tile
    static constexpr int NV = KC * VPR;           // loads per chunk
    static constexpr int NCV = (NV + kThreads - 1) / kThreads;  // per thread
};

// B elements per load: with wide C staging, 16 bytes' worth, at most the
// 4*WM elements a thread stages per chunk
template <typename TS, int WM, int VC>
constexpr int g1_vb() {
    return VC == 1 ? 1 : (4 * WM < (int)(16 / sizeof(TS)) ? 4 * WM : (int)(16 / sizeof(TS)));
}

template <int WM, int VB>
struct G1B {
    static constexpr int NP = 4 * WM / VB;        // loads per thread per chunk
    static constexpr int TLO = KC / VB;           // below: threads per packed row mu
    static constexpr int RLO = kThreads / TLO;    // below: rows mu per pass
    static constexpr int TUP = 64 * WM / VB;      // above: threads per packed row nu
    static constexpr int RUP = kThreads / TUP;    // above: rows nu per pass
};

template <typename T, int NI, int WM, int VC, int VB>
struct G1Stage {
    T b[G1B<WM, VB>::NP][VB];
    T c[G1C<T, NI, VC>::NCV][VC];
};

template <typename T, int NI, int WM, int VC, int VB>
struct G1Addr {
    int64_t c_off[G1C<T, NI, VC>::NCV];  // offset of C[nu0 + k][i] for the current chunk
    int c_lim[G1C<T, NI, VC>::NCV];      // orbitals below ncol among the VC (0 for no load)
    int64_t lo_off[G1B<WM, VB>::NP];     // below-diagonal: mu(mu+1)/2 + nu0 + k
    int64_t up_row[G1B<WM, VB>::NP];     // above-diagonal: T(nu0 + k)
    bool mu_ok_lo[G1B<WM, VB>::NP];
    int up_lim;                          // above: columns mu below nao among the VB
};

template <typename T, int NI, int WM, int VC, int VB>
__device__ inline void g1_addr_init(G1Addr<T, NI, WM, VC, VB>& ad, int64_t nao, int64_t ldc, int64_t ncol,
                                    int64_t mu0, int64_t i0, int tid) {
    using G = G1C<T, NI, VC>;
    using GB = G1B<WM, VB>;
#pragma unroll
    for (int j = 0; j < G::NCV; ++j) {
        const int e = tid + j * kThreads;
        const int k = e / G::VPR, ii = (e % G::VPR) * G::V;
        const int64_t lim = ncol - (i0 + ii);
        ad.c_off[j] = (int64_t)k * ldc + i0 + ii;
        ad.c_lim[j] = e < G::NV ? (int)(lim < 0 ? 0 : lim > G::V ? G::V : lim) : 0;
    }
#pragma unroll
    for (int j = 0; j < GB::NP; ++j) {
        const int64_t mu = mu0 + tid / GB::TLO + GB::RLO * j;
        ad.lo_off[j] = mu * (mu + 1) / 2 + (tid % GB::TLO) * VB;
        ad.mu_ok_lo[j] = mu < nao;
        const int64_t nu = tid / GB::TUP + GB::RUP * j;
        ad.up_row[j] = nu * (nu + 1) / 2;
    }
    const int64_t ul = nao - (mu0 + (tid % GB::TUP) * VB);
    ad.up_lim = (int)(ul < 0 ? 0 : ul > VB ? VB : ul);
}

// n consecutive elements of B (n = VB, or fewer: zeros after them), converted
template <typename T, typename TS, int VB>
__device__ inline void g1_bvec(T (&v)[VB], const TS* __restrict__ src, int n) {
    if (VB > 1 && n == VB) {
        TS w[VB];
        __builtin_memcpy(w, src, VB * sizeof(TS));
#pragma unroll
        for (int e = 0; e < VB; ++e) v[e] = to_compute<T, TS>(w[e]);
    } else {
#pragma unroll
        for (int e = 0; e < VB; ++e) v[e] = e < n ? to_compute<T, TS>(src[e]) : T(0);
    }
}

template <typename T, typename TS, int NI, int WM, int VC, int VB>
__device__ inline void g1_load(G1Stage<T, NI, WM, VC, VB>& st, const G1Addr<T, NI, WM, VC, VB>& ad,
                               const TS* __restrict__ Bp, int64_t nao,
                               const T* __restrict__ C, bool cvec, int64_t nu0, int64_t mu0, int tid) {
    using G = G1C<T, NI, VC>;
    using GB = G1B<WM, VB>;
    constexpr int BM = 64 * WM;
#pragma unroll
    for (int j = 0; j < G::NCV; ++j) {
        const int k = (tid + j * kThreads) / G::VPR;
        const int lim = nu0 + k < nao ? ad.c_lim[j] : 0;
        if (VC > 1 && cvec && lim == VC) {
            __builtin_memcpy(st.c[j], C + ad.c_off[j], VC * sizeof(T));
        } else {
#pragma unroll
            for (int e = 0; e < G::V; ++e) st.c[j][e] = e < lim ? C[ad.c_off[j] + e] : T(0);
        }
    }
    if (nu0 + KC <= mu0) {
        // every nu < mu: packed row mu, columns nu0 .. nu0+15
#pragma unroll
        for (int j = 0; j < GB::NP; ++j) g1_bvec<T, TS, VB>(st.b[j], Bp + ad.lo_off[j], ad.mu_ok_lo[j] ? VB : 0);
    } else if (nu0 >= mu0 + BM - 1) {
        // every nu >= mu: packed row nu, columns mu0 .. mu0+BM-1
        const int m = (tid % GB::TUP) * VB;
#pragma unroll
        for (int j = 0; j < GB::NP; ++j) {
            const int64_t nu = nu0 + tid / GB::TUP + GB::RUP * j;
            g1_bvec<T, TS, VB>(st.b[j], Bp + ad.up_row[j] + mu0 + m, nu < nao ? ad.up_lim : 0);
        }
    } else {
        // chunk crossing the diagonal (above-diagonal layout, element loads)
        const int m = (tid % GB::TUP) * VB;
#pragma unroll
        for (int j = 0; j < GB::NP; ++j) {
            const int64_t nu = nu0 + tid / GB::TUP + GB::RUP * j;
#pragma unroll
            for (int e = 0; e < VB; ++e) {
                const int64_t mu = mu0 + m + e;
                st.b[j][e] = (nu < nao && mu < nao) ? to_compute<T, TS>(Bp[pidx(nu, mu)]) : T(0);
            }
        }
    }
}

// Move the addresses from chunk nu0 to chunk nu0 + KC.
template <typename T, int NI, int WM, int VC, int VB>
__device__ inline void g1_addr_next(G1Addr<T, NI, WM, VC, VB>& ad, int64_t nu0, int64_t ldc, int tid) {
    using GB = G1B<WM, VB>;
#pragma unroll
    for (int j = 0; j < G1C<T, NI, VC>::NCV; ++j) ad.c_off[j] += (int64_t)KC * ldc;
#pragma unroll
    for (int j = 0; j < GB::NP; ++j) {
        ad.lo_off[j] += KC;
        const int64_t nu = nu0 + tid / GB::TUP + GB::RUP * j;
        ad.up_row[j] += (int64_t)KC * nu + (KC * (KC + 1)) / 2;
    }
}

// LDS row pitches of the GEMM1 tiles.  An FP32 operand read covers 4 rows x
// 16 consecutive columns (64 lanes, 64 banks): a pitch of 16 or 48 modulo 64
// words puts the four rows on disjoint banks.  The B tile is also written
// transposed (16 rows x 4 columns per wavefront), so its columns are XOR-ed
// with g1_swz(row) < 16, which keeps every 16-column group in place for the
// reads and spreads the transposed writes over all banks.  FP64 reads go 16
// lanes at a time, so the FP64 tiles keep a pitch of one extra element.  The
// per-row XOR costs address registers: on MI355X the bank-free layout was
// faster only for FP32 storage and the (5, 1) tile (26.0 -> 25.0 ms at
// nao=1024, naux=4096, nocc=200); for the (13, 1) tile it ran 22.1 against
// 21.6 ms (FP32 B) and 460 against 450 ms (BF16 B, nao=2048, nocc=400), so
// the other tiles keep the padded layout.
template <typename T, typename TS, int NI, int WM>
constexpr bool g1_bankfree() { return sizeof(T) == 4 && sizeof(TS) == 4 && WM == 1 && NI <= 5; }
template <typename T, typename TS, int NI, int WM>
constexpr int g1_pitch_c() {
    return g1_bankfree<T, TS, NI, WM>() ? ((16 * NI) % 32 == 16 ? 16 * NI : 16 * NI + 16) : 16 * NI + 1;
}
template <typename T, typename TS, int NI, int WM>
constexpr int g1_pitch_b() { return g1_bankfree<T, TS, NI, WM>() ? 64 * WM + 16 : 64 * WM + 1; }
template <typename T, typename TS, int NI, int WM>
__device__ inline int g1_swz(int row) { return g1_bankfree<T, TS, NI, WM>() ? 2 * ((row >> 1) & 7) : 0; }

template <typename T, typename TS, int NI, int WM, int VC, int VB>
__device__ inline void g1_store(const G1Stage<T, NI, WM, VC, VB>& st, T (*sC)[g1_pitch_c<T, TS, NI, WM>()],
                                T (*sB)[g1_pitch_b<T, TS, NI, WM>()], bool lower, int tid) {
    using G = G1C<T, NI, VC>;
    using GB = G1B<WM, VB>;
#pragma unroll
    for (int j = 0; j < G::NCV; ++j) {
        const int e = tid + j * kThreads;
        if (G::NV % kThreads == 0 || e < G::NV) {
            const int k = e / G::VPR, ii = (e % G::VPR) * G::V;
#pragma unroll
            for (int q = 0; q < G::V; ++q) sC[k][ii + q] = st.c[j][q];
        }
    }
    if (lower) {
        // element e of load j: row nu0 + (tid % TLO) * VB + e, column mu
#pragma unroll
        for (int j = 0; j < GB::NP; ++j) {
            const int m = tid / GB::TLO + GB::RLO * j;
#pragma unroll
            for (int e = 0; e < VB; ++e) {
                const int r = (tid % GB::TLO) * VB + e;
                sB[r][m ^ g1_swz<T, TS, NI, WM>(r)] = st.b[j][e];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < GB::NP; ++j) {
            const int r = tid / GB::TUP + GB::RUP * j, m = (tid % GB::TUP) * VB;
#pragma unroll
            for (int e = 0; e < VB; ++e) sB[r][(m + e) ^ g1_swz<T, TS, NI, WM>(r)] = st.b[j][e];
        }
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
// Columns [ioff, iend) of the ncol orbital columns (a launch may cover part of
// them with one tile and the rest with another).
// VC: orbitals of C per load (1, or 16 bytes' worth).
template <typename T, typename TS, int NI, int WM, int VC = 1, int VB = g1_vb<TS, WM, VC>()>
__device__ __attribute__((always_inline)) inline void k_gemm1_body(int64_t lid, const TS* __restrict__ B, int64_t ldB, int64_t nao,
                                    const T* __restrict__ C, int64_t ldc, int64_t ncol,
                                    T* __restrict__ X, int64_t ldx, int64_t nib, int64_t nmb,
                                    int64_t ioff = 0, int64_t iend = -1) {
    constexpr int BI = 16 * NI, BM = 64 * WM;
    if (iend < 0) iend = ncol;
    __shared__ T sC[2][KC][g1_pitch_c<T, TS, NI, WM>()];
    __shared__ T sB[2][KC][g1_pitch_b<T, TS, NI, WM>()];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ioff + ib * BI, mu0 = mb * BM;
    const TS* Bp = B + P * ldB;

    typename Mma<T>::acc_t acc[NI][WM];
#pragma unroll
    for (int a = 0; a < NI; ++a)
#pragma unroll
        for (int b = 0; b < WM; ++b) acc[a][b] = Mma<T>::zero();

    const int64_t nchunks = cdiv(nao, KC);
    G1Stage<T, NI, WM, VC, VB> st;
    G1Addr<T, NI, WM, VC, VB> ad;
    // 16-byte loads of C where its rows are 16-byte aligned
    const bool cvec = VC > 1 && ldc % VC == 0 && i0 % VC == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
    g1_addr_init<T, NI, WM, VC, VB>(ad, nao, ldc, iend, mu0, i0, tid);
    g1_load<T, TS, NI, WM, VC, VB>(st, ad, Bp, nao, C, cvec, 0, mu0, tid);
    g1_store<T, TS, NI, WM, VC, VB>(st, sC[0], sB[0], KC <= mu0, tid);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        const int64_t nnext = (ch + 1) * KC;
        const bool more = ch + 1 < nchunks;
        if (more) {
            g1_addr_next<T, NI, WM, VC, VB>(ad, ch * KC, ldc, tid);
            g1_load<T, TS, NI, WM, VC, VB>(st, ad, Bp, nao, C, cvec, nnext, mu0, tid);
        }
#pragma unroll
        for (int kk = 0; kk < KC / 4; ++kk) {
            const int kr = kk * 4 + (lane >> 4);
            T a[NI], b[WM];
#pragma unroll
            for (int t = 0; t < NI; ++t) a[t] = sC[buf][kr][t * 16 + (lane & 15)];
#pragma unroll
            for (int t = 0; t < WM; ++t) b[t] = sB[buf][kr][(wave * 16 * WM + t * 16 + (lane & 15)) ^ g1_swz<T, TS, NI, WM>(kr)];
#pragma unroll
            for (int ti = 0; ti < NI; ++ti)
#pragma unroll
                for (int tj = 0; tj < WM; ++tj) acc[ti][tj] = Mma<T>::step(a[ti], b[tj], acc[ti][tj]);
        }
        if (more) g1_store<T, TS, NI, WM, VC, VB>(st, sC[buf ^ 1], sB[buf ^ 1], nnext + KC <= mu0, tid);
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < NI; ++ti)
#pragma unroll
        for (int tj = 0; tj < WM; ++tj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t i = i0 + ti * 16 + Mma<T>::row(lane, r);
                const int64_t mu = mu0 + wave * 16 * WM + tj * 16 + (lane & 15);
                if (i < iend && mu < nao) X[(P * ncol + i) * ldx + mu] = acc[ti][tj][r];
            }
}

// FP32 form on v_mfma_f32_32x32x2f32 (4096 flop per step; lane l supplies
// A[l%32][l/32] and B[l/32][l%32], result register r of lane l is row
// 8(r/4) + 4(l/32) + r%4, column l%32): wavefront tile 32*NJ orbital columns
// x 32*WJ basis functions, the four wavefronts stacked along mu.  Staging as
// k_gemm1_body with (NI, WM) = (2 NJ, 2 WJ).  A wavefront holds NJ*WJ
// independent 32 x 32 accumulators, whose longer steps keep the FP32 matrix
// cores busy with far fewer chains than the 16 x 16 x 4 form needs (measured
// register-only: 0.98 of the FP32 peak with 4 chains per wavefront).
typedef float v16f_k __attribute__((ext_vector_type(16)));

template <typename TS, int NJ, int WJ, int VC = 1>
__device__ __attribute__((always_inline)) inline void k_gemm1w_body(int64_t lid, const TS* __restrict__ B, int64_t ldB, int64_t nao,
                                     const float* __restrict__ C, int64_t ldc, int64_t ncol,
                                     float* __restrict__ X, int64_t ldx, int64_t nib, int64_t nmb,
                                     int64_t ioff = 0, int64_t iend = -1) {
    constexpr int NI = 2 * NJ, WM = 2 * WJ;
    constexpr int BI = 16 * NI, BM = 64 * WM;
    if (iend < 0) iend = ncol;
    __shared__ float sC[2][KC][g1_pitch_c<float, TS, NI, WM>()];
    __shared__ float sB[2][KC][g1_pitch_b<float, TS, NI, WM>()];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t ib = lid % nib, mb = (lid / nib) % nmb, P = lid / (nib * nmb);
    const int64_t i0 = ioff + ib * BI, mu0 = mb * BM;
    const TS* Bp = B + P * ldB;

    v16f_k acc[NJ][WJ];
#pragma unroll
    for (int a = 0; a < NJ; ++a)
#pragma unroll
        for (int b = 0; b < WJ; ++b)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

    const int64_t nchunks = cdiv(nao, KC);
    constexpr int VB = g1_vb<TS, WM, VC>();
    G1Stage<float, NI, WM, VC, VB> st;
    G1Addr<float, NI, WM, VC, VB> ad;
    // 16-byte loads of C where its rows are 16-byte aligned
    const bool cvec = VC > 1 && ldc % VC == 0 && i0 % VC == 0 && (reinterpret_cast<uintptr_t>(C) & 15) == 0;
    g1_addr_init<float, NI, WM, VC, VB>(ad, nao, ldc, iend, mu0, i0, tid);
    g1_load<float, TS, NI, WM, VC, VB>(st, ad, Bp, nao, C, cvec, 0, mu0, tid);
    g1_store<float, TS, NI, WM, VC, VB>(st, sC[0], sB[0], KC <= mu0, tid);
    __syncthreads();
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        const int64_t nnext = (ch + 1) * KC;
        const bool more = ch + 1 < nchunks;
        if (more) {
            g1_addr_next<float, NI, WM, VC, VB>(ad, ch * KC, ldc, tid);
            g1_load<float, TS, NI, WM, VC, VB>(st, ad, Bp, nao, C, cvec, nnext, mu0, tid);
        }
#pragma unroll
        for (int kp = 0; kp < KC / 2; ++kp) {
            const int kr = kp * 2 + (lane >> 5);
            float a[NJ], b[WJ];
#pragma unroll
            for (int t = 0; t < NJ; ++t) a[t] = sC[buf][kr][t * 32 + (lane & 31)];
#pragma unroll
            for (int t = 0; t < WJ; ++t)
                b[t] = sB[buf][kr][(wave * 32 * WJ + t * 32 + (lane & 31)) ^ g1_swz<float, TS, NI, WM>(kr)];
#pragma unroll
            for (int ti = 0; ti < NJ; ++ti)
#pragma unroll
                for (int tj = 0; tj < WJ; ++tj)
                    acc[ti][tj] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
        if (more) g1_store<float, TS, NI, WM, VC, VB>(st, sC[buf ^ 1], sB[buf ^ 1], nnext + KC <= mu0, tid);
        __syncthreads();
    }
#pragma unroll
    for (int ti = 0; ti < NJ; ++ti)
#pragma unroll
        for (int tj = 0; tj < WJ; ++tj)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int64_t i = i0 + ti * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
                const int64_t mu = mu0 + wave * 32 * WJ + tj * 32 + (lane & 31);
                if (i < iend && mu < nao) X[(P * ncol + i) * ldx + mu] = acc[ti][tj][r];
            }
}

template <typename TS, int NJ, int WJ>
__global__ __launch_bounds__(kThreads) void k_gemm1w(const TS* __restrict__ B, int64_t ldB, int64_t nao,
                                                      const float* __restrict__ C, int64_t ldc, int64_t ncol,
                                                      float* __restrict__ X, int64_t ldx, int64_t nib,
                                                      int64_t nmb, int64_t nblk, int64_t ioff, int64_t iend) {
    k_gemm1w_body<TS, NJ, WJ, 4>(xcd_logical(blockIdx.x, nblk), B, ldB, nao, C, ldc, ncol, X, ldx, nib, nmb,
                              ioff, iend);
}

// Waves per SIMD the register allocation is held to (LDS allows them):
// FP64 (7,1) 3 instead of 2 (nao=1024, nocc=200: 35.5 -> 34.6 ms for the
// GEMM1 phase); FP32 (13,1) on 16-bit B 4 instead of 3 (nao=2048, nocc=400:
// 309 -> 299 ms, with a 48-byte spill; on FP32 B the same bound ran slower,
// 18.95 -> 19.70 ms, so that tile keeps 3).
template <typename T, typename TS, int NI, int WM>
constexpr int g1_waves() {
    return (sizeof(T) == 8 && NI == 7 && WM == 1) ? 3
           : (sizeof(T) == 4 && sizeof(TS) == 2 && NI == 13 && WM == 1) ? 4
                                                                          : 1;
}

template <typename T, typename TS, int NI, int WM>
__global__ __launch_bounds__(kThreads, (g1_waves<T, TS, NI, WM>())) void k_gemm1(const TS* __restrict__ B, int64_t ldB, int64_t nao,
                                                     const T* __restrict__ C, int64_t ldc, int64_t ncol,
                                                     T* __restrict__ X, int64_t ldx, int64_t nib,
                                                     int64_t nmb, int64_t nblk, int64_t ioff, int64_t iend) {
    // FP32: C and B staged up to 16 bytes per load (measured faster: 21.5 ->
    // 19.05 ms for the (13,1) tile at nao=1024, nocc=200); FP64 keeps one
    // element per load (wide C ran 36.9 against 35.7 ms, wide B no faster)
    k_gemm1_body<T, TS, NI, WM, sizeof(T) == 4 ? 4 : 1>(xcd_logical(blockIdx.x, nblk), B, ldB, nao, C, ldc, ncol, X, ldx, nib,
                                nmb, ioff, iend);
}

// ---------------------------------------------------------------- GEMM2 (SYRK)
// Staging of one KC-deep chunk of the two 128-wide operand panels, 8
// elements of each per thread.  Vector form (rows 16-byte aligned): each
// load moves V = 16 / sizeof(T) consecutive elements of a row, rows RPP
// apart.  Element form (any row stride): one element per load, the 256
// threads covering two rows of 128 per pass.
template <typename T>
struct SyStage {
    static constexpr int V = 16 / sizeof(T);          // elements per vector load
    static constexpr int TPR = SY_T / V;              // threads per panel row
    static constexpr int RPP = kThreads / TPR;        // rows per pass
    static constexpr int NP = KC / RPP;               // passes per chunk
    T a[8], b[8];
};

// GEMM2 modes.  SY_SYM: K = sum_k s_k x_k x_k^T over the rows of one X,
// lower tiles.  For two factors (D = L R^T) X holds X_L (rows 0..n) and then
// X_R (rows n..2n), and row k of the second operand is row (k + n) mod 2n:
// SY_PAIR_FULL contracts k < n over all tiles (sum_k xL_k xR_k^T);
// SY_PAIR_LOWER contracts k < 2n over the lower tiles, which adds the
// transpose (sum_k xL_k xR_k^T + xR_k xL_k^T, a symmetric result).
enum { SY_SYM = 0, SY_PAIR_LOWER = 1, SY_PAIR_FULL = 2 };

// V elements of row xr from column c0 (zeros at or past nao); one 16-byte
// load when all of them are below nao
template <typename T>
__device__ inline void sy_vec(T* v, const T* __restrict__ xr, int64_t c0, int64_t nao, bool ok) {
    constexpr int V = SyStage<T>::V;
    if (ok && c0 + V <= nao) {
        __builtin_memcpy(v, xr + c0, 16);
    } else {
#pragma unroll
        for (int e = 0; e < V; ++e) v[e] = (ok && c0 + e < nao) ? xr[c0 + e] : T(0);
    }
}

template <typename T, int MODE, bool VEC>
__device__ inline void sy_load(SyStage<T>& st, const T* __restrict__ X, int64_t ldx,
                               int64_t nrows, int64_t nao, int64_t ncol, const double* __restrict__ sign,
                               int64_t k0, int64_t kend, int64_t mu0, int64_t nu0, int64_t boff, int tid) {
    using S = SyStage<T>;
    auto rows = [&](int k, const T*& xr, const T*& xb, bool& ok, bool& neg) {
        const int64_t row = k0 + k;
        ok = row < kend;
        xr = X + row * ldx;
        xb = xr;
        if constexpr (MODE != SY_SYM) {
            const int64_t rb = row + boff;
            xb = X + (rb >= 2 * boff ? rb - 2 * boff : rb) * ldx;
        }
        neg = sign && ok && sign[row % ncol] < 0;
    };
    if constexpr (VEC) {
#pragma unroll
        for (int p = 0; p < S::NP; ++p) {
            const int k = tid / S::TPR + S::RPP * p, m = (tid % S::TPR) * S::V;
            const T *xr, *xb;
            bool ok, neg;
            rows(k, xr, xb, ok, neg);
            sy_vec<T>(&st.a[p * S::V], xr, mu0 + m, nao, ok);
            sy_vec<T>(&st.b[p * S::V], xb, nu0 + m, nao, ok);
#pragma unroll
            for (int e = 0; e < S::V; ++e)
                if (neg) st.b[p * S::V + e] = -st.b[p * S::V + e];
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = tid / SY_T + 2 * j, m = tid % SY_T;
            const T *xr, *xb;
            bool ok, neg;
            rows(k, xr, xb, ok, neg);
            st.a[j] = (ok && mu0 + m < nao) ? xr[mu0 + m] : T(0);
            const T bv = (ok && nu0 + m < nao) ? xb[nu0 + m] : T(0);
            st.b[j] = neg ? -bv : bv;
        }
    }
}

template <typename T, bool VEC>
__device__ inline void sy_store(const SyStage<T>& st, T (*sA)[SY_T + (sizeof(T) == 4 ? 16 : 1)],
                                T (*sB)[SY_T + (sizeof(T) == 4 ? 16 : 1)], int tid) {
    using S = SyStage<T>;
    if constexpr (VEC) {
#pragma unroll
        for (int p = 0; p < S::NP; ++p) {
            const int k = tid / S::TPR + S::RPP * p, m = (tid % S::TPR) * S::V;
#pragma unroll
            for (int e = 0; e < S::V; ++e) {
                sA[k][m + e] = st.a[p * S::V + e];
                sB[k][m + e] = st.b[p * S::V + e];
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sA[tid / SY_T + 2 * j][tid % SY_T] = st.a[j];
            sB[tid / SY_T + 2 * j][tid % SY_T] = st.b[j];
        }
    }
}

// partial[(s*ntl + t)][m][n] = sum_{k in split s} X[k][mu0+m] * sign_k * X[k'][nu0+n]
// (k' = k, or the row paired with k for two factors); block id = s*ntl + t,
// t a lower tile (I >= J) or, for SY_PAIR_FULL, any tile (I = t / nt).
// VEC: staging with 16-byte loads (X and ldx * sizeof(T) 16-byte aligned).
template <typename T, int MODE = SY_SYM, bool VEC = false>
__device__ __attribute__((always_inline)) inline void k_syrk_body(int64_t lid, const T* __restrict__ X, int64_t ldx, int64_t nrows,
                                   int64_t nao, int64_t ncol, const double* __restrict__ sign,
                                   int64_t kchunk, int64_t ntl, T* __restrict__ part, int64_t boff = 0) {
    // FP32 reads cover 4 rows x 16 columns over 64 banks: pitch 144 = 16 mod 64
    constexpr int PS = sizeof(T) == 4 ? SY_T + 16 : SY_T + 1;
    __shared__ T sA[2][KC][PS];
    __shared__ T sB[2][KC][PS];
    const int tid = threadIdx.x, lane = tid & 63;
    // the wave index is the same in all lanes: keep it (and what follows from
    // it) in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t t = lid % ntl;
    int64_t I, J;
    if constexpr (MODE == SY_PAIR_FULL) {
        const int64_t nt = cdiv(nao, SY_T);
        I = t / nt;
        J = t % nt;
    } else {
        I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > t) --I;
        while ((I + 1) * (I + 2) / 2 <= t) ++I;
        J = t - I * (I + 1) / 2;
    }
    const int64_t mu0 = I * SY_T, nu0 = J * SY_T;
    const int64_t s = lid / ntl;
    const int64_t kbeg = s * kchunk;
    const int64_t kend = kbeg + kchunk < nrows ? kbeg + kchunk : nrows;

    // Wave -> 64 x 64 sub-tile (rows ab.., columns bb.. of the tile) and the
    // 16 x 16 blocks of it that are computed: those the finish reads (rows
    // and columns below nao, on or below the diagonal of K).  Off the
    // diagonal the four waves take the 2 x 2 sub-tiles; a diagonal tile of a
    // symmetric result needs 36 of the 64 blocks, spread as the two halves
    // of its lower-left sub-tile (8 blocks each) and the lower block
    // triangles of the two diagonal sub-tiles (10 each).  The blocks computed
    // come out bitwise as with the plain 2 x 2 split.
    const bool diag = MODE != SY_PAIR_FULL && I == J;
    int ab = wm * 64, bb = wn * 64;
    uint32_t pat = 0xFFFFu;
    if (diag) {
        ab = wave == 2 ? 0 : 64;
        bb = wave == 3 ? 64 : 0;
        pat = wave == 0 ? 0x00FFu : wave == 1 ? 0xFF00u : 0xF731u;
    }
    uint32_t live = 0;
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            const bool on = mu0 + ab + ti * 16 < nao && nu0 + bb + tj * 16 < nao;
            live |= (uint32_t)on << (ti * 4 + tj);
        }
    live &= pat;

    typename Mma<T>::acc_t acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = Mma<T>::zero();

    if (kbeg < kend) {
        const int64_t nchunks = cdiv(kend - kbeg, KC);
        SyStage<T> st;
        sy_load<T, MODE, VEC>(st, X, ldx, nrows, nao, ncol, sign, kbeg, kend, mu0, nu0, boff, tid);
        sy_store<T, VEC>(st, sA[0], sB[0], tid);
        __syncthreads();
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            const int buf = ch & 1;
            const bool more = ch + 1 < nchunks;
            if (more)
                sy_load<T, MODE, VEC>(st, X, ldx, nrows, nao, ncol, sign, kbeg + (ch + 1) * KC, kend, mu0,
                                      nu0, boff, tid);
#pragma unroll
            for (int kk = 0; kk < KC / 4; ++kk) {
                const int kr = kk * 4 + (lane >> 4);
                T a[4], b[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a[q] = sA[buf][kr][ab + q * 16 + (lane & 15)];
                    b[q] = sB[buf][kr][bb + q * 16 + (lane & 15)];
                }
#pragma unroll
                for (int ti = 0; ti < 4; ++ti)
#pragma unroll
                    for (int tj = 0; tj < 4; ++tj)
                        if ((live >> (ti * 4 + tj)) & 1u) acc[ti][tj] = Mma<T>::step(a[ti], b[tj], acc[ti][tj]);
            }
            if (more) sy_store<T, VEC>(st, sA[buf ^ 1], sB[buf ^ 1], tid);
            __syncthreads();
        }
    }
    T* out = part + (s * ntl + t) * (int64_t)(SY_T * SY_T);
#pragma unroll
    for (int ti = 0; ti < 4; ++ti)
#pragma unroll
        for (int tj = 0; tj < 4; ++tj) {
            if (!((live >> (ti * 4 + tj)) & 1u)) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = ab + ti * 16 + Mma<T>::row(lane, r);
                const int n = bb + tj * 16 + (lane & 15);
                out[m * SY_T + n] = acc[ti][tj][r];
            }
        }
}

// FP32 held to 4 waves per SIMD (3 by its registers otherwise; LDS allows 4):
// nao=1024, nocc=200: 8.26 -> 7.50 ms.
template <typename T, int MODE = SY_SYM, bool VEC = false>
__global__ __launch_bounds__(kThreads, (sizeof(T) == 4 ? 4 : 1)) void k_syrk(const T* __restrict__ X, int64_t ldx, int64_t nrows,
                                                    int64_t nao, int64_t ncol,
                                                    const double* __restrict__ sign, int64_t kchunk,
                                                    int64_t ntl, int64_t nblk, T* __restrict__ part,
                                                    int64_t boff) {
    // all tiles of one split run on one XCD and share its L2 copy of the X rows
    k_syrk_body<T, MODE, VEC>(xcd_logical(blockIdx.x, nblk), X, ldx, nrows, nao, ncol, sign, kchunk, ntl, part,
                         boff);
}

// K[mu][nu] = K[nu][mu] = scale * sum_s partial[s][t][m][n] over the lower
// triangle (on diagonal tiles only m >= n is used, so K is exactly symmetric).
template <typename T>
__device__ __attribute__((always_inline)) inline void k_syrk_finish_body(int64_t t, int e0, int e1, const T* __restrict__ part,
                                          int64_t nsplit, int64_t ntl, int64_t nao, double scale,
                                          double* __restrict__ K) {
    int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > t) --I;
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    const int64_t J = t - I * (I + 1) / 2;
    const int64_t stride = ntl * (int64_t)(SY_T * SY_T);
    for (int e = e0 + (int)threadIdx.x; e < e1; e += kThreads) {
        const int m = e / SY_T, n = e % SY_T;
        const int64_t mu = I * SY_T + m, nu = J * SY_T + n;
        if (mu >= nao || nu >= nao) continue;
        if (I == J && m < n) continue;
        const T* p = part + t * (int64_t)(SY_T * SY_T) + e;
        double v = 0.0;
#pragma unroll 8
        for (int64_t s = 0; s < nsplit; ++s) v += (double)p[s * stride];  // fixed order
        v *= scale;
        K[mu * nao + nu] = v;
        K[nu * nao + mu] = v;
    }
}

// grid: kFinSub blocks per lower tile, each adding up a contiguous slice of it
template <typename T>
__global__ __launch_bounds__(kThreads) void k_syrk_finish(const T* __restrict__ part, int64_t nsplit,
                                                           int64_t ntl, int64_t nao, double scale,
                                                           double* __restrict__ K) {
    constexpr int per = SY_T * SY_T / kFinSub;
    const int sub = (int)(blockIdx.x % kFinSub);
    k_syrk_finish_body<T>(blockIdx.x / kFinSub, sub * per, (sub + 1) * per, part, nsplit, ntl, nao, scale,
                          K);
}

// Full-tile finish (two factors, no symmetry): K[mu][nu] = scale * sum_s
// partial[s][t][m][n] with t = I * nt + J.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pair_finish(const T* __restrict__ part, int64_t nsplit,
                                                           int64_t nt, int64_t nao, double scale,
                                                           double* __restrict__ K) {
    constexpr int per = SY_T * SY_T / kFinSub;
    const int64_t t = blockIdx.x / kFinSub;
    const int sub = (int)(blockIdx.x % kFinSub);
    const int64_t I = t / nt, J = t % nt;
    const int64_t stride = nt * nt * (int64_t)(SY_T * SY_T);
    for (int e = sub * per + (int)threadIdx.x; e < (sub + 1) * per; e += kThreads) {
        const int m = e / SY_T, n = e % SY_T;
        const int64_t mu = I * SY_T + m, nu = J * SY_T + n;
        if (mu >= nao || nu >= nao) continue;
        const T* p = part + t * (int64_t)(SY_T * SY_T) + e;
        double v = 0.0;
#pragma unroll 8
        for (int64_t s = 0; s < nsplit; ++s) v += (double)p[s * stride];  // fixed order
        K[mu * nao + nu] = v * scale;
    }
}

template <typename T, typename TS, int NI, int WM>
int launch_gemm1(const dfjk_ctx* h, const void* C, int64_t ncol, void* X, int64_t ldx, int64_t ioff,
                 int64_t iend) {
    const int64_t nib = cdiv(iend - ioff, 16 * NI), nmb = cdiv(h->nao, 64 * WM);
    const int64_t nblk = nib * nmb * h->naux;
    k_gemm1<T, TS, NI, WM><<<dim3((unsigned)nblk), kThreads, 0, h->stream>>>(
        static_cast<const TS*>(h->B), h->ldB, h->nao, static_cast<const T*>(C), ncol, ncol,
        static_cast<T*>(X), ldx, nib, nmb, nblk, ioff, iend);
    DFJK_LAUNCH_CHECK("k_gemm1");
    return DFJK_OK;
}

template <typename TS, int NJ, int WJ>
int launch_gemm1w(const dfjk_ctx* h, const void* C, int64_t ncol, void* X, int64_t ldx, int64_t ioff,
                  int64_t iend) {
    const int64_t nib = cdiv(iend - ioff, 32 * NJ), nmb = cdiv(h->nao, 128 * WJ);
    const int64_t nblk = nib * nmb * h->naux;
    k_gemm1w<TS, NJ, WJ><<<dim3((unsigned)nblk), kThreads, 0, h->stream>>>(
        static_cast<const TS*>(h->B), h->ldB, h->nao, static_cast<const float*>(C), ncol, ncol,
        static_cast<float*>(X), ldx, nib, nmb, nblk, ioff, iend);
    DFJK_LAUNCH_CHECK("k_gemm1w");
    return DFJK_OK;
}

// Compiled GEMM1 tiles: (NI, WM) = (i tiles of 16, mu tiles of 16 per wave),
// one launcher per B storage type (FP64 on the FP64 matrix cores; FP32, BF16
// and FP16 dequantised exactly on load and run on the FP32 matrix cores).
typedef int (*G1Launch)(const dfjk_ctx*, const void*, int64_t, void*, int64_t, int64_t, int64_t);
struct G1Tile {
    int ni, wm;
    G1Launch by_dtype[4];  // indexed by dfjk_dtype
};
#define G1T(a, b)                                                                              \
    {                                                                                          \
        a, b, {                                                                                \
            launch_gemm1<double, double, a, b>, launch_gemm1<float, float, a, b>,              \
                launch_gemm1<float, uint16_t, a, b>, launch_gemm1<float, _Float16, a, b>       \
        }                                                                                      \
    }
// Tiles 14..16: the FP32 32 x 32 x 2 form, (NI, WM) = (2 NJ, 2 WJ); no FP64
// launcher (FP64 has no 32 x 32 step).  Not defaults: at nao=1024,
// naux=4096, nocc=200 (FP32 B) on MI355X they took 24.9 / 29.7 / 28.0 ms
// against 21.5 ms for (13,1) on 16 x 16 x 4 steps (both with one element
// per staging load; (13,1) takes 19.1-19.3 ms with the wide staging).
#define G1W(a, b)                                                                              \
    {                                                                                          \
        2 * a, 2 * b, {                                                                        \
            nullptr, launch_gemm1w<float, a, b>, launch_gemm1w<uint16_t, a, b>,                \
                launch_gemm1w<_Float16, a, b>                                                  \
        }                                                                                      \
    }
const G1Tile kG1Tiles[] = {
    G1T(1, 2), G1T(2, 2), G1T(3, 2), G1T(4, 2), G1T(5, 2), G1T(6, 2),
    G1T(7, 2), G1T(8, 2), G1T(13, 1), G1T(4, 4), G1T(7, 1), G1T(5, 1), G1T(6, 1), G1T(3, 1),
    G1W(2, 1), G1W(1, 2), G1W(2, 2),
};
#undef G1T
#undef G1W
constexpr int kNumG1Tiles = sizeof(kG1Tiles) / sizeof(kG1Tiles[0]);
constexpr int kFirstRestTile = 12;  // (6,1) and (3,1): defaults only for the rest of a split

// FP64 -> FP32 copy of C (one rounding per element).
__global__ void to_f32(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (float)x[i];
}

// Default tile: least padded work, where each extra i block costs another
// read of the B tile (weight 1/2 of a padded column block), among the tiles
// that keep two waves per SIMD (FP64 sweep on MI355X, nao=1024, nocc=200:
// (7,1) 43.8 TFLOP/s, (5,2) 43.5, (13,1) 40.4, (1,2) 32.6).
// FP32 compute (FP32/BF16/FP16 storage) allows up to 14 accumulator tiles
// (sweep at nocc=200, FP32 B, one element per staging load: (13,1) and
// (7,2) 79.7 TFLOP/s, (5,2) 76.6, (7,1) 76.0, (5,1) 68.7, (8,2) 72.5,
// (4,4) 62.5).
int pick_g1_tile(int64_t ncol, bool f32 = false) {
    int best = 0;
    double best_cost = 1e300;
    for (int t = 0; t < kFirstRestTile; ++t) {
        const int ni = kG1Tiles[t].ni, wm = kG1Tiles[t].wm;
        if (ni * wm > (f32 ? 14 : 7)) continue;  // larger accumulator sets leave one wave per SIMD
        const double padded = (double)(cdiv(ncol, 16 * ni) * 16 * ni);
        const double cost = padded * (1.0 + 0.5 / ni);
        if (cost < best_cost) {
            best_cost = cost;
            best = t;
        }
    }
    return best;
}

// Default for the single build: one tile, or the default tile over the
// first columns (a whole number of its widths) and the narrowest tile with
// one wavefront row (WM = 1) over the rest, when that pads fewer columns
// (nocc=200: FP64 112 + 96 = 208 columns computed instead of 224; FP32
// 160 + 48 = 208 instead of 240).
struct G1Split {
    int t0, t1;
    int64_t n0;  // columns [0, n0) with tile t0, [n0, ncol) with t1
};
G1Split pick_g1_split(int64_t ncol, bool f32) {
    const int single = pick_g1_tile(ncol, f32);
    G1Split sp{single, single, ncol};
    const int64_t w = 16 * kG1Tiles[single].ni;
    if (kG1Tiles[single].wm != 1) return sp;
    const int64_t padded_single = cdiv(ncol, w) * w;
    const int64_t n0 = (ncol / w) * w, rest = ncol - n0;
    if (n0 == 0 || rest == 0) return sp;
    int best = -1;
    for (int t = 0; t < kNumG1Tiles; ++t) {
        const int ni = kG1Tiles[t].ni;
        if (kG1Tiles[t].wm != 1 || 16 * ni < rest || ni > kG1Tiles[single].ni) continue;
        if (best < 0 || ni < kG1Tiles[best].ni) best = t;
    }
    if (best >= 0 && n0 + 16 * kG1Tiles[best].ni < padded_single) sp = G1Split{single, best, n0};
    return sp;
}

// X = (B_P C)^T for every P, with the handle's forced tile or the default
// split (profiled as the GEMM1 phase).
int run_gemm1(dfjk_ctx* h, const void* C, int64_t ncol, void* X, int64_t ldx, bool f32) {
    if (h->g1_tile >= 0 && h->g1_tile < kNumG1Tiles) {
        const G1Launch f = kG1Tiles[h->g1_tile].by_dtype[h->dtype];
        if (!f) {
            set_error("GEMM1 tile %d has no FP64 form", h->g1_tile);
            return DFJK_E_INVALID;
        }
        return f(h, C, ncol, X, ldx, 0, ncol);
    }
    G1Split sp = pick_g1_split(ncol, f32);
    int rc = kG1Tiles[sp.t0].by_dtype[h->dtype](h, C, ncol, X, ldx, 0, sp.n0);
    if (!rc && sp.n0 < ncol) rc = kG1Tiles[sp.t1].by_dtype[h->dtype](h, C, ncol, X, ldx, sp.n0, ncol);
    return rc;
}

// Splits of a GEMM2 contraction of nrows terms over ntl output tiles: about
// 8192 workgroups (FP64) or 16384 (FP32, whose partials are half the size),
// and for FP32 no running sum longer than kMaxSum32 terms (the split partials
// are added in FP64).  On MI355X at nao=1024, naux=4096, nocc=200 the FP64
// SYRK took 20.4 / 18.4 / 17.4 / 16.8 / 16.5 ms for about 1024 / 2048 / 4096 /
// 8192 / 16384 workgroups while the finish, which reads every partial tile,
// grew from 0.07 ms (2048) to 0.24 (8192) and 0.44 (16384); the FP32 SYRK took
// 10.3 / 9.45 / 9.24 ms for 2048 / 8192 / 16384 (finish 0.04 / 0.14 / 0.25).
void syrk_splits(int64_t nrows, int64_t ntl, bool f32, int64_t* nsplit_out, int64_t* kchunk_out) {
    int64_t nsplit = cdiv(f32 ? 16384 : 8192, ntl);
    if (f32 && nsplit < cdiv(nrows, kMaxSum32)) nsplit = cdiv(nrows, kMaxSum32);
    const int64_t max_split = cdiv(nrows, 384);  // splits of at least 384 rows (short contractions)
    if (nsplit > max_split) nsplit = max_split;
    if (nsplit < 1) nsplit = 1;
    const int64_t kchunk = cdiv(cdiv(nrows, nsplit), KC) * KC;
    *nsplit_out = cdiv(nrows, kchunk);
    *kchunk_out = kchunk;
}

// Workspace of one K build: X rows of nao elements and the GEMM2 split
// partials (nrows contraction terms over ntl output tiles), in bytes.
struct KBytes {
    size_t X, kpart;
};
KBytes k_bytes(const dfjk_ctx* h, size_t elem, int64_t xrows, int64_t nrows, int64_t ntl) {
    int64_t nsplit, kchunk;
    syrk_splits(nrows, ntl, elem == 4, &nsplit, &kchunk);
    return KBytes{elem * (size_t)xrows * (size_t)h->nao, elem * (size_t)(nsplit * ntl) * SY_T * SY_T};
}

template <typename T>
int k_build_t(dfjk_ctx* h, const void* C, int64_t ncol, const double* sign, double scale, double* K) {
    const int64_t ldx = h->nao;
    const int64_t nrows = h->naux * ncol;
    const int64_t nt = cdiv(h->nao, SY_T);
    const int64_t ntl = nt * (nt + 1) / 2;
    const KBytes need = k_bytes(h, sizeof(T), nrows, nrows, ntl);
    int rc;
    if ((rc = h->X.ensure(need.X)) || (rc = h->kpart.ensure(need.kpart))) return rc;
    T* X = static_cast<T*>(h->X.ptr);

    h->prof.begin(PH_K, h->stream);
    h->prof.begin(PH_K_GEMM1, h->stream);
    rc = run_gemm1(h, C, ncol, X, ldx, sizeof(T) == 4);
    h->prof.end(PH_K_GEMM1, h->stream);
    if (rc) return rc;

    int64_t nsplit, kchunk;
    syrk_splits(nrows, ntl, sizeof(T) == 4, &nsplit, &kchunk);
    T* part = static_cast<T*>(h->kpart.ptr);
    h->prof.begin(PH_K_SYRK, h->stream);
    if (ldx % SyStage<T>::V == 0)
        k_syrk<T, SY_SYM, true><<<dim3((unsigned)(ntl * nsplit)), kThreads, 0, h->stream>>>(
            X, ldx, nrows, h->nao, ncol, sign, kchunk, ntl, ntl * nsplit, part, 0);
    else
        k_syrk<T><<<dim3((unsigned)(ntl * nsplit)), kThreads, 0, h->stream>>>(
            X, ldx, nrows, h->nao, ncol, sign, kchunk, ntl, ntl * nsplit, part, 0);
    h->prof.end(PH_K_SYRK, h->stream);
    DFJK_LAUNCH_CHECK("k_syrk");
    h->prof.begin(PH_K_FINISH, h->stream);
    k_syrk_finish<T><<<dim3((unsigned)(ntl * kFinSub)), kThreads, 0, h->stream>>>(part, nsplit, ntl, h->nao,
                                                                                   scale, K);
    h->prof.end(PH_K_FINISH, h->stream);
    h->prof.end(PH_K, h->stream);
    DFJK_LAUNCH_CHECK("k_syrk_finish");
    return DFJK_OK;
}

// Two factors, D = L R^T (L, R: nao x ncol): X_L = (B_P L)^T and X_R =
// (B_P R)^T are stored one after the other, then
//   sym = 0: K = scale * sum_P X_L^T X_R            (all output tiles)
//   sym = 1: K = scale * sum_P (X_L^T X_R + X_R^T X_L)  (lower tiles, mirrored)
template <typename T>
int k_build_pair_t(dfjk_ctx* h, const void* L, const void* R, int64_t ncol, int sym, double scale, double* K) {
    const int64_t ldx = h->nao;
    const int64_t n1 = h->naux * ncol;  // rows of X_L (and of X_R)
    const int64_t nt = cdiv(h->nao, SY_T);
    const int64_t ntl = sym ? nt * (nt + 1) / 2 : nt * nt;
    const int64_t nrows = sym ? 2 * n1 : n1;  // contraction length
    const KBytes need = k_bytes(h, sizeof(T), 2 * n1, nrows, ntl);
    int rc;
    if ((rc = h->X.ensure(need.X)) || (rc = h->kpart.ensure(need.kpart))) return rc;
    T* X = static_cast<T*>(h->X.ptr);

    h->prof.begin(PH_K, h->stream);
    h->prof.begin(PH_K_GEMM1, h->stream);
    rc = run_gemm1(h, L, ncol, X, ldx, sizeof(T) == 4);
    if (!rc) rc = run_gemm1(h, R, ncol, X + n1 * ldx, ldx, sizeof(T) == 4);
    h->prof.end(PH_K_GEMM1, h->stream);
    if (rc) return rc;

    int64_t nsplit, kchunk;
    syrk_splits(nrows, ntl, sizeof(T) == 4, &nsplit, &kchunk);
    T* part = static_cast<T*>(h->kpart.ptr);
    const dim3 grid((unsigned)(ntl * nsplit));
    h->prof.begin(PH_K_SYRK, h->stream);
    const bool vec = ldx % SyStage<T>::V == 0;
    if (sym && vec)
        k_syrk<T, SY_PAIR_LOWER, true><<<grid, kThreads, 0, h->stream>>>(X, ldx, nrows, h->nao, ncol, nullptr,
                                                                           kchunk, ntl, ntl * nsplit, part, n1);
    else if (sym)
        k_syrk<T, SY_PAIR_LOWER><<<grid, kThreads, 0, h->stream>>>(X, ldx, nrows, h->nao, ncol, nullptr, kchunk,
                                                                     ntl, ntl * nsplit, part, n1);
    else if (vec)
        k_syrk<T, SY_PAIR_FULL, true><<<grid, kThreads, 0, h->stream>>>(X, ldx, nrows, h->nao, ncol, nullptr,
                                                                          kchunk, ntl, ntl * nsplit, part, n1);
    else
        k_syrk<T, SY_PAIR_FULL><<<grid, kThreads, 0, h->stream>>>(X, ldx, nrows, h->nao, ncol, nullptr, kchunk,
                                                                    ntl, ntl * nsplit, part, n1);
    h->prof.end(PH_K_SYRK, h->stream);
    DFJK_LAUNCH_CHECK("k_syrk (two factors)");
    h->prof.begin(PH_K_FINISH, h->stream);
    if (sym)
        k_syrk_finish<T><<<dim3((unsigned)(ntl * kFinSub)), kThreads, 0, h->stream>>>(part, nsplit, ntl,
                                                                                       h->nao, scale, K);
    else
        k_pair_finish<T><<<dim3((unsigned)(ntl * kFinSub)), kThreads, 0, h->stream>>>(part, nsplit, nt, h->nao,
                                                                                       scale, K);
    h->prof.end(PH_K_FINISH, h->stream);
    h->prof.end(PH_K, h->stream);
    DFJK_LAUNCH_CHECK("k finish (two factors)");
    return DFJK_OK;
}

// ---------------------------------------------------------------- batched
__device__ inline int find_mol_k(const int64_t* __restrict__ prefix, int n, int64_t b) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// 4 waves per SIMD, as the FP32 GEMM2 it runs (256 molecules: 69.2 -> 67.0 ms
// per eager build)
__global__ __launch_bounds__(kThreads, 4) void kb_kernel(int kind, const MolDesc* __restrict__ mols,
                                                       PhaseList pl) {
    // SYRK blocks are renumbered so runs of consecutive ids share an XCD
    const int64_t b = kind == BP_SYRK ? xcd_logical(blockIdx.x, pl.nblk) : (int64_t)blockIdx.x;
    const int j = find_mol_k(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    const int64_t lid = b - pl.prefix[j];
    switch (kind) {
        case BP_CF32: {
            const int64_t e = lid * kThreads + threadIdx.x;
            if (e < d.nao * d.nocc) d.Cf[e / d.nocc * d.ldcf + e % d.nocc] = (float)d.C[e];
            break;
        }
        case BP_SYRK:
            k_syrk_body<float, SY_SYM, true>(lid, d.X, d.ldx, d.naux * d.nocc, d.nao, d.nocc, nullptr, d.kchunk,
                                             d.ntl,
                               d.kpart);
            break;
        case BP_KFIN:
            k_syrk_finish_body<float>(lid, 0, SY_T * SY_T, d.kpart, d.nsplit, d.ntl, d.nao, 2.0, d.K);
            break;
        default:
            break;
    }
}

// Batched GEMM1 tiles with at most 8 accumulator blocks are held to 5 waves
// per SIMD (their LDS allows 6); larger ones would spill.
template <int NI, int WM>
constexpr int kb_g1_waves() { return NI * WM <= 8 ? 5 : 1; }

template <typename TS, int NI, int WM>
__global__ __launch_bounds__(kThreads, (kb_g1_waves<NI, WM>())) void kb_gemm1(const MolDesc* __restrict__ mols,
                                                                             PhaseList pl) {
    const int64_t b = xcd_logical(blockIdx.x, pl.nblk);
    const int j = find_mol_k(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    k_gemm1_body<float, TS, NI, WM, 4>(b - pl.prefix[j], static_cast<const TS*>(d.B), d.ldB, d.nao, d.Cf,
                                        d.ldcf, d.nocc, d.X, d.ldx, d.g1_nib, d.g1_nmb);
}

template <int NI, int WM>
int launch_kb_gemm1(hipStream_t st, int dtype, const MolDesc* mols, const PhaseList& pl) {
    const dim3 grid((unsigned)pl.nblk);
    switch (dtype) {
        case DFJK_F32: kb_gemm1<float, NI, WM><<<grid, kThreads, 0, st>>>(mols, pl); break;
        case DFJK_BF16: kb_gemm1<uint16_t, NI, WM><<<grid, kThreads, 0, st>>>(mols, pl); break;
        case DFJK_F16: kb_gemm1<_Float16, NI, WM><<<grid, kThreads, 0, st>>>(mols, pl); break;
        default: set_error("batched builds take FP32, BF16 or FP16 B"); return DFJK_E_DTYPE;
    }
    DFJK_LAUNCH_CHECK("kb_gemm1");
    return DFJK_OK;
}

template <typename TS, int NJ, int WJ>
__global__ __launch_bounds__(kThreads) void kb_gemm1w(const MolDesc* __restrict__ mols, PhaseList pl) {
    const int64_t b = xcd_logical(blockIdx.x, pl.nblk);
    const int j = find_mol_k(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    k_gemm1w_body<TS, NJ, WJ, 4>(b - pl.prefix[j], static_cast<const TS*>(d.B), d.ldB, d.nao, d.Cf, d.ldcf,
                                 d.nocc, d.X, d.ldx, d.g1_nib, d.g1_nmb);
}

template <int NJ, int WJ>
int launch_kb_gemm1w(hipStream_t st, int dtype, const MolDesc* mols, const PhaseList& pl) {
    const dim3 grid((unsigned)pl.nblk);
    switch (dtype) {
        case DFJK_F32: kb_gemm1w<float, NJ, WJ><<<grid, kThreads, 0, st>>>(mols, pl); break;
        case DFJK_BF16: kb_gemm1w<uint16_t, NJ, WJ><<<grid, kThreads, 0, st>>>(mols, pl); break;
        case DFJK_F16: kb_gemm1w<_Float16, NJ, WJ><<<grid, kThreads, 0, st>>>(mols, pl); break;
        default: set_error("batched builds take FP32, BF16 or FP16 B"); return DFJK_E_DTYPE;
    }
    DFJK_LAUNCH_CHECK("kb_gemm1w");
    return DFJK_OK;
}

typedef int (*KbLaunch)(hipStream_t, int, const MolDesc*, const PhaseList&);
#define KBT(a, b) launch_kb_gemm1<a, b>
const KbLaunch kKbTiles[] = {KBT(1, 2), KBT(2, 2), KBT(3, 2), KBT(4, 2), KBT(5, 2), KBT(6, 2),
                             KBT(7, 2), KBT(8, 2), KBT(13, 1), KBT(4, 4), KBT(7, 1), KBT(5, 1),
                             KBT(6, 1), KBT(3, 1), launch_kb_gemm1w<2, 1>, launch_kb_gemm1w<1, 2>,
                             launch_kb_gemm1w<2, 2>};
#undef KBT
static_assert(sizeof(kKbTiles) / sizeof(kKbTiles[0]) == kNumG1Tiles, "tile tables differ");

}  // namespace

int k_batch_phase(hipStream_t st, int kind, int dtype, const MolDesc* mols, const PhaseList& pl) {
    (void)dtype;
    if (pl.nblk <= 0) return DFJK_OK;
    kb_kernel<<<dim3((unsigned)pl.nblk), kThreads, 0, st>>>(kind, mols, pl);
    DFJK_LAUNCH_CHECK("kb_kernel");
    return DFJK_OK;
}

int k_batch_gemm1(hipStream_t st, int dtype, int tile, const MolDesc* mols, const PhaseList& pl) {
    if (pl.nblk <= 0) return DFJK_OK;
    if (tile < 0 || tile >= kNumG1Tiles) {
        set_error("tile %d out of range", tile);
        return DFJK_E_INVALID;
    }
    return kKbTiles[tile](st, dtype, mols, pl);
}

int pick_tile(int64_t ncol) { return pick_g1_tile(ncol, true); }

int tile_nb(int tile, int64_t nao, int64_t ncol, int64_t* nib, int64_t* nmb) {
    if (tile < 0 || tile >= kNumG1Tiles) return DFJK_E_INVALID;
    *nib = cdiv(ncol, 16 * kG1Tiles[tile].ni);
    *nmb = cdiv(nao, 64 * kG1Tiles[tile].wm);
    return DFJK_OK;
}

int k_build_factored(dfjk_ctx* h, const double* C, int64_t ncol, const double* sign, double scale,
                     double* K) {
    if (h->dtype == DFJK_F64) return k_build_t<double>(h, C, ncol, sign, scale, K);
    if ((h->dtype == DFJK_BF16 || h->dtype == DFJK_F16) && h->opts.k16 && !sign)
        return k_build_16(h, C, ncol, scale, K);
    {  // FP32 compute for FP32, BF16 and FP16 storage of B
        int rc;
        if ((rc = h->Cw.ensure(sizeof(float) * (size_t)(h->nao * ncol)))) return rc;
        float* Cf = static_cast<float*>(h->Cw.ptr);
        to_f32<<<dim3((unsigned)cdiv(h->nao * ncol, 256)), 256, 0, h->stream>>>(C, h->nao * ncol, Cf);
        DFJK_LAUNCH_CHECK("to_f32");
        return k_build_t<float>(h, Cf, ncol, sign, scale, K);
    }
}

int k_build_pair(dfjk_ctx* h, const double* L, const double* R, int64_t ncol, int sym, double scale, double* K) {
    if (h->dtype == DFJK_F64) return k_build_pair_t<double>(h, L, R, ncol, sym, scale, K);
    // FP32 compute for FP32, BF16 and FP16 storage of B (also with the k16
    // option: the 16-bit exchange takes one factor)
    int rc;
    const int64_t n = h->nao * ncol;
    if ((rc = h->Cw.ensure(sizeof(float) * (size_t)(2 * n)))) return rc;
    float* Lf = static_cast<float*>(h->Cw.ptr);
    float* Rf = Lf + n;
    to_f32<<<dim3((unsigned)cdiv(n, 256)), 256, 0, h->stream>>>(L, n, Lf);
    to_f32<<<dim3((unsigned)cdiv(n, 256)), 256, 0, h->stream>>>(R, n, Rf);
    DFJK_LAUNCH_CHECK("to_f32");
    return k_build_pair_t<float>(h, Lf, Rf, ncol, sym, scale, K);
}


int k_reserve(dfjk_ctx* h, int64_t max_ncol) {
    const size_t elem = h->dtype == DFJK_F64 ? 8 : 4;
    const int64_t nt = cdiv(h->nao, SY_T), lower = nt * (nt + 1) / 2;
    const int64_t n1 = h->naux * max_ncol, half = h->naux * (max_ncol / 2);
    // one factor of max_ncol columns; two factors of max_ncol / 2 each (the
    // symmetric form contracts both over the lower tiles, the general one
    // half of the rows over every tile)
    const KBytes a = k_bytes(h, elem, n1, n1, lower);
    const KBytes b = k_bytes(h, elem, 2 * half, 2 * half, lower);
    const KBytes c = k_bytes(h, elem, 2 * half, half, nt * nt);
    size_t kp = a.kpart > b.kpart ? a.kpart : b.kpart;
    kp = kp > c.kpart ? kp : c.kpart;
    int rc;
    if ((rc = h->X.ensure(a.X > b.X ? a.X : b.X))) return rc;
    if ((rc = h->kpart.ensure(kp))) return rc;
    if (h->dtype != DFJK_F64 && (rc = h->Cw.ensure(sizeof(float) * (size_t)(h->nao * max_ncol)))) return rc;
    return DFJK_OK;
}

int k_tile_count() { return kNumG1Tiles; }

bool k_tile_has_dtype(int t, int dtype) {
    return t >= 0 && t < kNumG1Tiles && dtype >= 0 && dtype < 4 && kG1Tiles[t].by_dtype[dtype] != nullptr;
}

int k_tile_info(int t, int* ni, int* wm) {
    if (t < 0 || t >= kNumG1Tiles) return DFJK_E_INVALID;
    *ni = kG1Tiles[t].ni;
    *wm = kG1Tiles[t].wm;
    return DFJK_OK;
}

}  // namespace dfjk
