// Coulomb matrix J from the packed three-index tensor B.
//
// J[mu,nu] = sum_P rho_P B_P[mu,nu],  rho_P = sum_{ka,la} B_P[ka,la] D[ka,la]
// (Eq. eq:df:eri contracted with the density).  Because B_P is symmetric,
// rho_P = sum_p B[P,p] dt[p] over the packed pairs with
// dt[p(mu,nu)] = D[mu,nu] + D[nu,mu] (mu != nu) and D[mu,mu] on the diagonal.
//
// Two streaming passes over B, both bound by HBM bandwidth:
//   pass 1 (j_rho):  each workgroup takes R rows of B and one column chunk,
//                    reusing each dt element R times from registers; partial
//                    sums per (row, chunk) are added in a fixed order.
//   pass 2 (j_out):  each thread owns a few packed columns and walks a
//                    slice of the rows; slices are added in a fixed order and
//                    unpacked into both triangles of J.
// No atomics anywhere, so J is bitwise reproducible.
#include "internal.h"
#include "numerics.h"

namespace dfjk {

namespace {

typedef double d2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;
constexpr int kRhoRows = 4;     // rows of B per workgroup in pass 1
constexpr int kOutVec = 2;      // double2 loads per row per thread in pass 2
constexpr int kOutCols = kThreads * 2 * kOutVec;  // columns per workgroup in pass 2

// dt[p(mu,nu)] for all mu <= nu; one block per row nu of the packed triangle.
__global__ __launch_bounds__(kThreads) void pack_density(const double* __restrict__ D, int64_t nao,
                                                          double* __restrict__ dt) {
    const int64_t nu = blockIdx.x;
    const int64_t base = nu * (nu + 1) / 2;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += kThreads) {
        const double v = (mu == nu) ? D[nu * nao + nu] : D[mu * nao + nu] + D[nu * nao + mu];
        dt[base + mu] = v;
    }
}

// Sum of `v` over the 256 threads of the block; result valid in thread 0.
__device__ inline double block_sum(double v, double* lds) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return s;
}

template <int R, bool VEC>
__global__ __launch_bounds__(kThreads) void j_rho_f64(const double* __restrict__ B, int64_t ldB,
                                                       int64_t naux, int64_t npair,
                                                       const double* __restrict__ dt, int64_t chunk,
                                                       int nchunk, double* __restrict__ part) {
    __shared__ double lds[4];
    const int64_t P0 = (int64_t)blockIdx.x * R;
    const int c = blockIdx.y;
    const int64_t c0 = (int64_t)c * chunk;
    const int64_t c1 = c0 + chunk < npair ? c0 + chunk : npair;
    const double* rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t P = P0 + r < naux ? P0 + r : naux - 1;  // clamped rows are discarded below
        rows[r] = B + P * ldB;
    }
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    if (VEC) {
        // c0 is even and rows start 16-byte aligned: pairs (p, p+1) load as one double2.
        int64_t p = c0 + 2 * (int64_t)threadIdx.x;
#pragma unroll 2
        for (; p + 1 < c1; p += 2 * kThreads) {
            const d2 d = *reinterpret_cast<const d2*>(dt + p);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2*>(rows[r] + p));
                acc[r] = fma(b.x, d.x, acc[r]);
                acc[r] = fma(b.y, d.y, acc[r]);
            }
        }
        if (p < c1) {
            const double d = dt[p];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = fma(rows[r][p], d, acc[r]);
        }
    } else {
#pragma unroll 4
        for (int64_t p = c0 + threadIdx.x; p < c1; p += kThreads) {
            const double d = dt[p];
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = fma(__builtin_nontemporal_load(rows[r] + p), d, acc[r]);
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double s = block_sum(acc[r], lds);
        if (threadIdx.x == 0 && P0 + r < naux) part[(P0 + r) * nchunk + c] = s;
    }
}

__global__ void j_rho_finish(const double* __restrict__ part, int64_t naux, int nchunk,
                             double* __restrict__ rho, double* __restrict__ rho_out) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= naux) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[P * nchunk + c];
    rho[P] = s;
    if (rho_out) rho_out[P] = s;
}

template <bool VEC>
__global__ __launch_bounds__(kThreads) void j_out_f64(const double* __restrict__ B, int64_t ldB,
                                                       int64_t naux, int64_t npair,
                                                       const double* __restrict__ rho, int64_t prows,
                                                       double* __restrict__ jpart) {
    const int s = blockIdx.y;
    const int64_t P0 = (int64_t)s * prows;
    const int64_t P1 = P0 + prows < naux ? P0 + prows : naux;
    const int64_t base = (int64_t)blockIdx.x * kOutCols;
    double acc[2 * kOutVec];
#pragma unroll
    for (int u = 0; u < 2 * kOutVec; ++u) acc[u] = 0.0;
    // columns of this thread: base + u*2*kThreads + 2*tid + {0,1}
    const int64_t col0 = base + 2 * (int64_t)threadIdx.x;
    const bool full = base + kOutCols <= npair;
    if (VEC && full) {
#pragma unroll 4
        for (int64_t P = P0; P < P1; ++P) {
            const double r = rho[P];
            const double* row = B + P * ldB + col0;
#pragma unroll
            for (int u = 0; u < kOutVec; ++u) {
                const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2*>(row + u * 2 * kThreads));
                acc[2 * u] = fma(b.x, r, acc[2 * u]);
                acc[2 * u + 1] = fma(b.y, r, acc[2 * u + 1]);
            }
        }
    } else {
        for (int64_t P = P0; P < P1; ++P) {
            const double r = rho[P];
            const double* row = B + P * ldB;
#pragma unroll
            for (int u = 0; u < kOutVec; ++u) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t col = col0 + u * 2 * kThreads + e;
                    if (col < npair) acc[2 * u + e] = fma(row[col], r, acc[2 * u + e]);
                }
            }
        }
    }
    double* out = jpart + (int64_t)s * npair;
#pragma unroll
    for (int u = 0; u < kOutVec; ++u) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t col = col0 + u * 2 * kThreads + e;
            if (col < npair) out[col] = acc[2 * u + e];
        }
    }
}

// J[nu,mu] = J[mu,nu] = sum_s jpart[s][p(mu,nu)]; one block per packed row nu.
__global__ __launch_bounds__(kThreads) void j_finish(const double* __restrict__ jpart, int64_t npair,
                                                      int nsplit, int64_t nao, double* __restrict__ J) {
    const int64_t nu = blockIdx.x;
    const int64_t base = nu * (nu + 1) / 2;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += kThreads) {
        double v = 0.0;
        for (int s = 0; s < nsplit; ++s) v += jpart[(int64_t)s * npair + base + mu];
        J[nu * nao + mu] = v;
        J[mu * nao + nu] = v;
    }
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

int j_setup(dfjk_ctx* h) {
    const int64_t rowblocks = cdiv(h->naux, kRhoRows);
    // pass 1: enough (row block, chunk) workgroups to cover the chip several times
    int64_t chunks = cdiv(4096, rowblocks);
    chunks = chunks < 1 ? 1 : chunks;
    const int64_t max_chunks = cdiv(h->npair, 2 * kThreads * 4);
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    h->j_chunks = (int)chunks;
    // pass 2: row slices so that (column blocks x slices) covers the chip
    const int64_t colblocks = cdiv(h->npair, kOutCols);
    int64_t splits = cdiv(4096, colblocks);
    if (splits > h->naux) splits = h->naux;
    if (splits < 1) splits = 1;
    if (splits > 64) splits = 64;
    h->j_splits = (int)splits;
    int rc;
    if ((rc = h->dt.ensure(sizeof(double) * (size_t)h->npair * 3))) return rc;
    if ((rc = h->rho_part.ensure(sizeof(double) * (size_t)h->naux * (size_t)chunks))) return rc;
    if ((rc = h->rho.ensure(sizeof(double) * (size_t)h->naux))) return rc;
    if ((rc = h->jpart.ensure(sizeof(double) * (size_t)h->npair * (size_t)splits))) return rc;
    return DFJK_OK;
}

int j_build_reduced(dfjk_ctx* h, const double* D, double* J, double* rho_out) {
    (void)D;
    (void)J;
    (void)rho_out;
    set_error("J for dtype %d is not built yet", h->dtype);
    return DFJK_E_DTYPE;
}

int j_build(dfjk_ctx* h, const double* D, double* J, double* rho_out) {
    if (h->dtype != DFJK_F64) return j_build_reduced(h, D, J, rho_out);
    const double* B = static_cast<const double*>(h->B);
    double* dt = static_cast<double*>(h->dt.ptr);
    double* part = static_cast<double*>(h->rho_part.ptr);
    double* rho = static_cast<double*>(h->rho.ptr);
    double* jpart = static_cast<double*>(h->jpart.ptr);
    const hipStream_t st = h->stream;

    h->prof.begin(PH_J, st);
    pack_density<<<dim3((unsigned)h->nao), dim3(kThreads), 0, st>>>(D, h->nao, dt);
    DFJK_LAUNCH_CHECK("pack_density");

    const bool vec = (h->ldB % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    int64_t chunk = cdiv(h->npair, h->j_chunks);
    chunk = cdiv(chunk, 2) * 2;  // even, so every chunk starts 16-byte aligned
    const dim3 g1((unsigned)cdiv(h->naux, kRhoRows), (unsigned)h->j_chunks);
    h->prof.begin(PH_J_RHO, st);
    if (vec)
        j_rho_f64<kRhoRows, true><<<g1, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, dt, chunk,
                                                            h->j_chunks, part);
    else
        j_rho_f64<kRhoRows, false><<<g1, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, dt, chunk,
                                                             h->j_chunks, part);
    h->prof.end(PH_J_RHO, st);
    DFJK_LAUNCH_CHECK("j_rho_f64");
    j_rho_finish<<<dim3((unsigned)cdiv(h->naux, 256)), 256, 0, st>>>(part, h->naux, h->j_chunks, rho,
                                                                       rho_out);
    DFJK_LAUNCH_CHECK("j_rho_finish");

    const int64_t prows = cdiv(h->naux, h->j_splits);
    const dim3 g2((unsigned)cdiv(h->npair, kOutCols), (unsigned)h->j_splits);
    h->prof.begin(PH_J_OUT, st);
    if (vec)
        j_out_f64<true><<<g2, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, rho, prows, jpart);
    else
        j_out_f64<false><<<g2, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, rho, prows, jpart);
    h->prof.end(PH_J_OUT, st);
    DFJK_LAUNCH_CHECK("j_out_f64");
    j_finish<<<dim3((unsigned)h->nao), kThreads, 0, st>>>(jpart, h->npair, h->j_splits, h->nao, J);
    h->prof.end(PH_J, st);
    DFJK_LAUNCH_CHECK("j_finish");
    return DFJK_OK;
}

}  // namespace dfjk
