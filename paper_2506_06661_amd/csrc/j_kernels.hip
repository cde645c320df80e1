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

// dt[p(mu,nu)] for all mu <= nu; one block per row nu of the packed triangle.
__device__ __attribute__((always_inline)) inline void pack_density_body(int64_t nu, const double* __restrict__ D, int64_t nao,
                                         double* __restrict__ dt) {
    const int64_t base = nu * (nu + 1) / 2;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += kThreads) {
        const double v = (mu == nu) ? D[nu * nao + nu] : D[mu * nao + nu] + D[nu * nao + mu];
        dt[base + mu] = v;
    }
}

__global__ __launch_bounds__(kThreads) void pack_density(const double* __restrict__ D, int64_t nao,
                                                          double* __restrict__ dt) {
    pack_density_body(blockIdx.x, D, nao, dt);
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

__device__ __attribute__((always_inline)) inline void rho_finish_body(int64_t P, const double* __restrict__ part, int64_t naux,
                                       int nchunk, double* __restrict__ rho,
                                       double* __restrict__ rho_out) {
    if (P >= naux) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[P * nchunk + c];
    rho[P] = s;
    if (rho_out) rho_out[P] = s;
}

__global__ void j_rho_finish(const double* __restrict__ part, int64_t naux, int nchunk,
                             double* __restrict__ rho, double* __restrict__ rho_out) {
    rho_finish_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, part, naux, nchunk, rho, rho_out);
}

// U = double2 loads per row per thread: a workgroup owns 512*U packed columns
// (a 4U-KB run of each row it visits).  With DG the same stream also sums
// B[P,p]^2 (the DF diagonal) into dpart.
template <bool VEC, int U, bool DG>
__global__ __launch_bounds__(kThreads) void j_out_f64(const double* __restrict__ B, int64_t ldB,
                                                       int64_t naux, int64_t npair,
                                                       const double* __restrict__ rho, int64_t prows,
                                                       double* __restrict__ jpart, double* __restrict__ dpart) {
    constexpr int64_t COLS = (int64_t)kThreads * 2 * U;
    const int s = blockIdx.y;
    const int64_t P0 = (int64_t)s * prows;
    const int64_t P1 = P0 + prows < naux ? P0 + prows : naux;
    const int64_t base = (int64_t)blockIdx.x * COLS;
    double acc[2 * U], sq[2 * U];  // sq is dead code without DG
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) acc[u] = sq[u] = 0.0;
    // columns of this thread: base + u*2*kThreads + 2*tid + {0,1}
    const int64_t col0 = base + 2 * (int64_t)threadIdx.x;
    const bool full = base + COLS <= npair;
    if (VEC && full) {
#pragma unroll 2
        for (int64_t P = P0; P < P1; ++P) {
            const double r = rho[P];
            const double* row = B + P * ldB + col0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const d2 b = __builtin_nontemporal_load(reinterpret_cast<const d2*>(row + u * 2 * kThreads));
                acc[2 * u] = fma(b.x, r, acc[2 * u]);
                acc[2 * u + 1] = fma(b.y, r, acc[2 * u + 1]);
                if (DG) {
                    sq[2 * u] = fma(b.x, b.x, sq[2 * u]);
                    sq[2 * u + 1] = fma(b.y, b.y, sq[2 * u + 1]);
                }
            }
        }
    } else {
        for (int64_t P = P0; P < P1; ++P) {
            const double r = rho[P];
            const double* row = B + P * ldB;
#pragma unroll
            for (int u = 0; u < U; ++u) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t col = col0 + u * 2 * kThreads + e;
                    if (col < npair) {
                        const double b = row[col];
                        acc[2 * u + e] = fma(b, r, acc[2 * u + e]);
                        if (DG) sq[2 * u + e] = fma(b, b, sq[2 * u + e]);
                    }
                }
            }
        }
    }
    double* out = jpart + (int64_t)s * npair;
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int64_t col = col0 + u * 2 * kThreads + e;
            if (col < npair) {
                out[col] = acc[2 * u + e];
                if (DG) dpart[(int64_t)s * npair + col] = sq[2 * u + e];
            }
        }
    }
}

template <int U>
void launch_j_out(bool vec, dim3 g, hipStream_t st, const double* B, int64_t ldB, int64_t naux,
                  int64_t npair, const double* rho, int64_t prows, double* jpart, double* dpart) {
    if (dpart) {
        if (vec)
            j_out_f64<true, U, true><<<g, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, jpart, dpart);
        else
            j_out_f64<false, U, true><<<g, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, jpart, dpart);
    } else {
        if (vec)
            j_out_f64<true, U, false><<<g, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, jpart, nullptr);
        else
            j_out_f64<false, U, false><<<g, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, jpart, nullptr);
    }
}

// diag[p] = sum_s dpart[s][p], splits in order
__global__ __launch_bounds__(256) void diag_finish(const double* __restrict__ dpart, int64_t npair, int nsplit,
                                                   double* __restrict__ diag) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= npair) return;
    double v = 0.0;
    for (int s = 0; s < nsplit; ++s) v += dpart[(int64_t)s * npair + p];
    diag[p] = v;
}

constexpr int kJOutU[] = {2, 4, 8, 16};
constexpr int kNumJOut = 4;

// J[nu,mu] = J[mu,nu] = sum_s jpart[s][p(mu,nu)]; one block per packed row nu.
__device__ __attribute__((always_inline)) inline void j_finish_body(int64_t nu, const double* __restrict__ jpart, int64_t npair,
                                     int nsplit, int64_t nao, double* __restrict__ J) {
    const int64_t base = nu * (nu + 1) / 2;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += kThreads) {
        double v = 0.0;
        for (int s = 0; s < nsplit; ++s) v += jpart[(int64_t)s * npair + base + mu];
        J[nu * nao + mu] = v;
        J[mu * nao + nu] = v;
    }
}

__global__ __launch_bounds__(kThreads) void j_finish(const double* __restrict__ jpart, int64_t npair,
                                                      int nsplit, int64_t nao, double* __restrict__ J) {
    j_finish_body(blockIdx.x, jpart, npair, nsplit, nao, J);
}

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- reduced B
// B in FP32, BF16 or FP16.  Every element converts exactly to FP32.  Three
// accumulation modes (the `compensated_j` option):
//   ACC_F64  products and sums in FP64 (the FP64 VALU runs at full rate on
//            MI355X, so this costs about one instruction per element);
//   ACC_DOT2 FP32 compensated dot product (Dot2: TwoProduct + TwoSum) with the
//            FP64 multiplier split into FP32 hi + lo parts;
//   ACC_F32  plain FP32 fused multiply-add with the hi part.
enum { ACC_F32 = 0, ACC_DOT2 = 1, ACC_F64 = 2 };

template <typename TB>
struct Elem;
template <>
struct Elem<float> {
    static constexpr int V = 4;  // elements per 16-byte load
    __device__ static float f(float x) { return x; }
};
template <>
struct Elem<uint16_t> {  // bfloat16 bit pattern
    static constexpr int V = 8;
    __device__ static float f(uint16_t x) { return __uint_as_float((uint32_t)x << 16); }
};
template <>
struct Elem<_Float16> {
    static constexpr int V = 8;
    __device__ static float f(_Float16 x) { return (float)x; }
};

// 16 bytes of B from any element-aligned address (the rows of a packed B
// with ldB not a multiple of V start at any element; the GPU's global loads
// take unaligned addresses).
template <typename TB>
__device__ inline void load16(const TB* p, float* out) {
    constexpr int V = Elem<TB>::V;
    typedef uint32_t u4 __attribute__((ext_vector_type(4), aligned(2)));
    const u4 raw = __builtin_nontemporal_load(reinterpret_cast<const u4*>(p));
    const TB* e = reinterpret_cast<const TB*>(&raw);
#pragma unroll
    for (int v = 0; v < V; ++v) out[v] = Elem<TB>::f(e[v]);
}

template <int ACC>
struct Acc {
    double d = 0.0;
    float s = 0.f, c = 0.f;
    __device__ inline void add(float b, double m, float mhi, float mlo) {
        if (ACC == ACC_F64) {
            d = fma((double)b, m, d);
        } else if (ACC == ACC_F32) {
            s = __builtin_fmaf(b, mhi, s);
        } else {
            dot2_step(b, mhi, s, c);
            c = __builtin_fmaf(b, mlo, c);
        }
    }
    __device__ inline double value() const {
        if (ACC == ACC_F64) return d;
        if (ACC == ACC_F32) return (double)s;
        return (double)s + (double)c;
    }
};

// dt_hi = fl32(dt), dt_lo = fl32(dt - dt_hi)
__global__ void split_f64(const double* __restrict__ x, int64_t n, float* __restrict__ hi,
                          float* __restrict__ lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float h = (float)x[i];
    hi[i] = h;
    lo[i] = (float)(x[i] - (double)h);
}

template <typename TB, int R, int ACC>
__device__ __attribute__((always_inline)) inline void j_rho_red_body(int64_t bx, int c, const TB* __restrict__ B, int64_t ldB,
                                      int64_t naux, int64_t npair, const double* __restrict__ dt,
                                      const float* __restrict__ dhi, const float* __restrict__ dlo,
                                      int64_t chunk, int nchunk, bool vec, double* __restrict__ part) {
    constexpr int V = Elem<TB>::V;
    __shared__ double lds[4];
    const int64_t P0 = bx * R;
    const int64_t c0 = (int64_t)c * chunk;
    const int64_t c1 = c0 + chunk < npair ? c0 + chunk : npair;
    const TB* rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rows[r] = B + (P0 + r < naux ? P0 + r : naux - 1) * ldB;
    Acc<ACC> acc[R];
    int64_t p = c0;
    if (vec) {
        // c0 is a multiple of V; rows may start at any element
        for (p = c0 + (int64_t)V * threadIdx.x; p + V <= c1; p += (int64_t)V * kThreads) {
            double m[V];
            float mh[V], ml[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                if (ACC == ACC_F64) m[v] = dt[p + v];
                else {
                    mh[v] = dhi[p + v];
                    ml[v] = ACC == ACC_DOT2 ? dlo[p + v] : 0.f;
                }
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                float b[V];
                load16<TB>(rows[r] + p, b);
#pragma unroll
                for (int v = 0; v < V; ++v) acc[r].add(b[v], ACC == ACC_F64 ? m[v] : 0.0, mh[v], ml[v]);
            }
        }
        // the last partial vector of the chunk: element by element
        p = c0 + ((c1 - c0) / V) * V + threadIdx.x;
    } else {
        p = c0 + threadIdx.x;
    }
    for (; p < c1; p += kThreads) {
        const double m = dt[p];
        const float mh = ACC == ACC_F64 ? 0.f : dhi[p];
        const float ml = ACC == ACC_DOT2 ? dlo[p] : 0.f;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r].add(Elem<TB>::f(rows[r][p]), m, mh, ml);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const double sum = block_sum(acc[r].value(), lds);
        if (threadIdx.x == 0 && P0 + r < naux) part[(P0 + r) * nchunk + c] = sum;
    }
}

template <typename TB, int R, int ACC>
__global__ __launch_bounds__(kThreads) void j_rho_red(const TB* __restrict__ B, int64_t ldB, int64_t naux,
                                                       int64_t npair, const double* __restrict__ dt,
                                                       const float* __restrict__ dhi,
                                                       const float* __restrict__ dlo, int64_t chunk,
                                                       int nchunk, bool vec, double* __restrict__ part) {
    j_rho_red_body<TB, R, ACC>(blockIdx.x, blockIdx.y, B, ldB, naux, npair, dt, dhi, dlo, chunk, nchunk,
                               vec, part);
}

// With DG the stream also sums B[P,p]^2 in FP64 (exact products of the
// stored values) into dpart: the DF diagonal.
template <typename TB, int ACC, bool DG = false>
__device__ __attribute__((always_inline)) inline void j_out_red_body(int64_t bx, int s, const TB* __restrict__ B, int64_t ldB,
                                      int64_t naux, int64_t npair, const double* __restrict__ rho,
                                      const float* __restrict__ rhi, const float* __restrict__ rlo,
                                      int64_t prows, bool vec, double* __restrict__ jpart,
                                      double* __restrict__ dpart = nullptr) {
    constexpr int V = Elem<TB>::V;
    const int64_t P0 = (int64_t)s * prows;
    const int64_t P1 = P0 + prows < naux ? P0 + prows : naux;
    const int64_t col0 = (bx * kThreads + threadIdx.x) * V;
    Acc<ACC> acc[V];
    double sq[V];  // dead code without DG
#pragma unroll
    for (int v = 0; v < V; ++v) sq[v] = 0.0;
    if (vec && col0 + V <= npair) {
#pragma unroll 4
        for (int64_t P = P0; P < P1; ++P) {
            const double m = rho[P];
            const float mh = ACC == ACC_F64 ? 0.f : rhi[P];
            const float ml = ACC == ACC_DOT2 ? rlo[P] : 0.f;
            float b[V];
            load16<TB>(B + P * ldB + col0, b);
#pragma unroll
            for (int v = 0; v < V; ++v) {
                acc[v].add(b[v], m, mh, ml);
                if (DG) sq[v] = fma((double)b[v], (double)b[v], sq[v]);
            }
        }
    } else {
        for (int64_t P = P0; P < P1; ++P) {
            const double m = rho[P];
            const float mh = ACC == ACC_F64 ? 0.f : rhi[P];
            const float ml = ACC == ACC_DOT2 ? rlo[P] : 0.f;
#pragma unroll
            for (int v = 0; v < V; ++v)
                if (col0 + v < npair) {
                    const float bv = Elem<TB>::f(B[P * ldB + col0 + v]);
                    acc[v].add(bv, m, mh, ml);
                    if (DG) sq[v] = fma((double)bv, (double)bv, sq[v]);
                }
        }
    }
    double* out = jpart + (int64_t)s * npair;
#pragma unroll
    for (int v = 0; v < V; ++v)
        if (col0 + v < npair) {
            out[col0 + v] = acc[v].value();
            if (DG) dpart[(int64_t)s * npair + col0 + v] = sq[v];
        }
}

template <typename TB, int ACC, bool DG>
__global__ __launch_bounds__(kThreads) void j_out_red(const TB* __restrict__ B, int64_t ldB, int64_t naux,
                                                       int64_t npair, const double* __restrict__ rho,
                                                       const float* __restrict__ rhi,
                                                       const float* __restrict__ rlo, int64_t prows,
                                                       bool vec, double* __restrict__ jpart,
                                                       double* __restrict__ dpart) {
    j_out_red_body<TB, ACC, DG>(blockIdx.x, blockIdx.y, B, ldB, naux, npair, rho, rhi, rlo, prows, vec, jpart,
                                dpart);
}

template <typename TB, int ACC>
int j_build_red_t(dfjk_ctx* h, double* J, double* rho_out, double* diag) {
    constexpr int V = Elem<TB>::V;
    // rows per workgroup in pass 1: each FP64 (or FP32 hi/lo) weight is loaded
    // once per R rows, so 16-bit B uses more rows to keep that traffic small
    constexpr int R = sizeof(TB) == 2 ? 16 : 8;
    const TB* B = static_cast<const TB*>(h->B);
    double* dt = static_cast<double*>(h->dt.ptr);
    float* dhi = reinterpret_cast<float*>(dt + h->npair);
    float* dlo = dhi + h->npair;
    double* part = static_cast<double*>(h->rho_part.ptr);
    double* rho = static_cast<double*>(h->rho.ptr);
    float* rhi = reinterpret_cast<float*>(rho + h->naux);
    float* rlo = rhi + h->naux;
    double* jpart = static_cast<double*>(h->jpart.ptr);
    const hipStream_t st = h->stream;
    if (ACC != ACC_F64) {
        split_f64<<<dim3((unsigned)cdiv(h->npair, 256)), 256, 0, st>>>(dt, h->npair, dhi, dlo);
        DFJK_LAUNCH_CHECK("split_f64");
    }
    const bool vec = true;  // 16-byte loads at any element alignment (load16)
    int64_t chunk = cdiv(h->npair, h->j_chunks);
    chunk = cdiv(chunk, V) * V;
    const dim3 g1((unsigned)cdiv(h->naux, R), (unsigned)h->j_chunks);
    h->prof.begin(PH_J_RHO, st);
    j_rho_red<TB, R, ACC><<<g1, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, dt, dhi, dlo, chunk,
                                                    h->j_chunks, vec, part);
    h->prof.end(PH_J_RHO, st);
    DFJK_LAUNCH_CHECK("j_rho_red");
    j_rho_finish<<<dim3((unsigned)cdiv(h->naux, 256)), 256, 0, st>>>(part, h->naux, h->j_chunks, rho,
                                                                       rho_out);
    DFJK_LAUNCH_CHECK("j_rho_finish");
    if (ACC != ACC_F64) {
        split_f64<<<dim3((unsigned)cdiv(h->naux, 256)), 256, 0, st>>>(rho, h->naux, rhi, rlo);
        DFJK_LAUNCH_CHECK("split_f64");
    }
    const int64_t prows = cdiv(h->naux, h->j_splits);
    const dim3 g2((unsigned)cdiv(h->npair, (int64_t)kThreads * V), (unsigned)h->j_splits);
    double* dpart = nullptr;
    if (diag) {
        int rc;
        if ((rc = h->dpart.ensure(sizeof(double) * (size_t)h->npair * (size_t)h->j_splits))) return rc;
        dpart = static_cast<double*>(h->dpart.ptr);
    }
    h->prof.begin(PH_J_OUT, st);
    if (dpart)
        j_out_red<TB, ACC, true><<<g2, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, rho, rhi, rlo, prows,
                                                          vec, jpart, dpart);
    else
        j_out_red<TB, ACC, false><<<g2, kThreads, 0, st>>>(B, h->ldB, h->naux, h->npair, rho, rhi, rlo, prows,
                                                           vec, jpart, nullptr);
    h->prof.end(PH_J_OUT, st);
    DFJK_LAUNCH_CHECK("j_out_red");
    j_finish<<<dim3((unsigned)h->nao), kThreads, 0, st>>>(jpart, h->npair, h->j_splits, h->nao, J);
    DFJK_LAUNCH_CHECK("j_finish");
    if (dpart) {
        diag_finish<<<dim3((unsigned)cdiv(h->npair, 256)), 256, 0, st>>>(dpart, h->npair, h->j_splits, diag);
        DFJK_LAUNCH_CHECK("diag_finish");
    }
    h->prof.end(PH_J, st);
    return DFJK_OK;
}

template <typename TB>
int j_build_red(dfjk_ctx* h, double* J, double* rho_out, double* diag) {
    switch (h->opts.compensated_j) {
        case ACC_F32: return j_build_red_t<TB, ACC_F32>(h, J, rho_out, diag);
        case ACC_DOT2: return j_build_red_t<TB, ACC_DOT2>(h, J, rho_out, diag);
        default: return j_build_red_t<TB, ACC_F64>(h, J, rho_out, diag);
    }
}

// ---------------------------------------------------------------- batched
__device__ inline int find_mol(const int64_t* __restrict__ prefix, int n, int64_t b) {
    int lo = 0, hi = n - 1;  // largest j with prefix[j] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

constexpr int kBatchR = 8;

template <typename TB>
__global__ __launch_bounds__(kThreads) void jb_kernel(int kind, const MolDesc* __restrict__ mols,
                                                       PhaseList pl) {
    const int64_t b = blockIdx.x;
    const int j = find_mol(pl.prefix, pl.n, b);
    const MolDesc& d = mols[pl.ids[j]];
    const int64_t lid = b - pl.prefix[j];
    const TB* B = static_cast<const TB*>(d.B);
    switch (kind) {
        case BP_PACK:
            pack_density_body(lid, d.D, d.nao, d.dt);
            break;
        case BP_RHO: {
            const int64_t nrb = cdiv(d.naux, kBatchR);
            j_rho_red_body<TB, kBatchR, ACC_F64>(lid % nrb, (int)(lid / nrb), B, d.ldB, d.naux, d.npair,
                                                 d.dt, nullptr, nullptr, d.chunk, (int)d.j_chunks,
                                                 d.vec != 0, d.rho_part);
            break;
        }
        case BP_RHO_FIN:
            rho_finish_body(lid * kThreads + threadIdx.x, d.rho_part, d.naux, (int)d.j_chunks, d.rho,
                            nullptr);
            break;
        case BP_OUT: {
            const int64_t ncb = cdiv(d.npair, (int64_t)kThreads * Elem<TB>::V);
            j_out_red_body<TB, ACC_F64>(lid % ncb, (int)(lid / ncb), B, d.ldB, d.naux, d.npair, d.rho,
                                        nullptr, nullptr, d.prows, d.vec != 0, d.jpart);
            break;
        }
        case BP_JFIN:
            j_finish_body(lid, d.jpart, d.npair, (int)d.j_splits, d.nao, d.J);
            break;
        default:
            break;
    }
}

// ---------------------------------------------------------------- several densities
// J for M densities from one pass over B per pass (FP64 B): pass 1 reads each
// B element once for all M packed densities, pass 2 once for all M rho.
constexpr int kMaxDm = 8;     // densities fused per pass
constexpr int kRhoRowsM = 8;  // rows of B per workgroup in pass 1 (M/R packed-density loads per B element)

__global__ __launch_bounds__(kThreads) void pack_density_m(const double* __restrict__ D, int64_t nao,
                                                            int64_t npair, double* __restrict__ dt) {
    const int64_t m = blockIdx.y;
    pack_density_body(blockIdx.x, D + m * nao * nao, nao, dt + m * npair);
}

// part[m][P][c] = sum over chunk c of B[P,p] dt_m[p]
template <int M, bool VEC>
__global__ __launch_bounds__(kThreads) void j_rho_f64m(const double* __restrict__ B, int64_t ldB,
                                                        int64_t naux, int64_t npair,
                                                        const double* __restrict__ dt, int64_t chunk,
                                                        int nchunk, double* __restrict__ part) {
    constexpr int R = kRhoRowsM;
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
    double acc[M][R];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int r = 0; r < R; ++r) acc[m][r] = 0.0;
    if (VEC) {
        int64_t p = c0 + 2 * (int64_t)threadIdx.x;
        for (; p + 1 < c1; p += 2 * kThreads) {
            d2 b[R];
#pragma unroll
            for (int r = 0; r < R; ++r) b[r] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(rows[r] + p));
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const d2 d = *reinterpret_cast<const d2*>(dt + m * npair + p);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    acc[m][r] = fma(b[r].x, d.x, acc[m][r]);
                    acc[m][r] = fma(b[r].y, d.y, acc[m][r]);
                }
            }
        }
        if (p < c1) {
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double d = dt[m * npair + p];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[m][r] = fma(rows[r][p], d, acc[m][r]);
            }
        }
    } else {
        for (int64_t p = c0 + threadIdx.x; p < c1; p += kThreads) {
            double b[R];
#pragma unroll
            for (int r = 0; r < R; ++r) b[r] = __builtin_nontemporal_load(rows[r] + p);
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double d = dt[m * npair + p];
#pragma unroll
                for (int r = 0; r < R; ++r) acc[m][r] = fma(b[r], d, acc[m][r]);
            }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double sum = block_sum(acc[m][r], lds);
            if (threadIdx.x == 0 && P0 + r < naux) part[(m * naux + P0 + r) * nchunk + c] = sum;
        }
}

__global__ void j_rho_finish_m(const double* __restrict__ part, int64_t naux, int nchunk,
                               double* __restrict__ rho, double* __restrict__ rho_out) {
    const int64_t m = blockIdx.y;
    rho_finish_body((int64_t)blockIdx.x * blockDim.x + threadIdx.x, part + m * naux * nchunk, naux, nchunk,
                    rho + m * naux, rho_out ? rho_out + m * naux : nullptr);
}

// jpart[m][s][p] = sum over the row slice s of B[P,p] rho_m[P]; 1024 columns per workgroup
template <int M, bool VEC>
__global__ __launch_bounds__(kThreads) void j_out_f64m(const double* __restrict__ B, int64_t ldB,
                                                        int64_t naux, int64_t npair,
                                                        const double* __restrict__ rho, int64_t prows,
                                                        int64_t nsplit, double* __restrict__ jpart) {
    constexpr int U = 2;
    constexpr int64_t COLS = (int64_t)kThreads * 2 * U;
    const int s = blockIdx.y;
    const int64_t P0 = (int64_t)s * prows;
    const int64_t P1 = P0 + prows < naux ? P0 + prows : naux;
    const int64_t base = (int64_t)blockIdx.x * COLS;
    double acc[M][2 * U];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
        for (int u = 0; u < 2 * U; ++u) acc[m][u] = 0.0;
    const int64_t col0 = base + 2 * (int64_t)threadIdx.x;
    const bool full = base + COLS <= npair;
    if (VEC && full) {
        for (int64_t P = P0; P < P1; ++P) {
            const double* row = B + P * ldB + col0;
            d2 b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) b[u] = __builtin_nontemporal_load(reinterpret_cast<const d2*>(row + u * 2 * kThreads));
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const double r = rho[m * naux + P];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    acc[m][2 * u] = fma(b[u].x, r, acc[m][2 * u]);
                    acc[m][2 * u + 1] = fma(b[u].y, r, acc[m][2 * u + 1]);
                }
            }
        }
    } else {
        for (int64_t P = P0; P < P1; ++P) {
            const double* row = B + P * ldB;
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t col = col0 + u * 2 * kThreads + e;
                    if (col < npair) {
                        const double b = row[col];
#pragma unroll
                        for (int m = 0; m < M; ++m) acc[m][2 * u + e] = fma(b, rho[m * naux + P], acc[m][2 * u + e]);
                    }
                }
        }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        double* out = jpart + (m * nsplit + s) * npair;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const int64_t col = col0 + u * 2 * kThreads + e;
                if (col < npair) out[col] = acc[m][2 * u + e];
            }
    }
}

__global__ __launch_bounds__(kThreads) void j_finish_m(const double* __restrict__ jpart, int64_t npair,
                                                        int nsplit, int64_t nao, double* __restrict__ J) {
    const int64_t m = blockIdx.y;
    j_finish_body(blockIdx.x, jpart + m * nsplit * npair, npair, nsplit, nao, J + m * nao * nao);
}

template <int M>
void launch_j_multi(bool vec, dim3 g1, dim3 g2, hipStream_t st, const double* B, int64_t ldB, int64_t naux,
                    int64_t npair, const double* dt, int64_t chunk, int nchunk, double* part,
                    const double* rho, int64_t prows, int64_t nsplit, double* jpart, bool pass1) {
    if (pass1) {
        if (vec)
            j_rho_f64m<M, true><<<g1, kThreads, 0, st>>>(B, ldB, naux, npair, dt, chunk, nchunk, part);
        else
            j_rho_f64m<M, false><<<g1, kThreads, 0, st>>>(B, ldB, naux, npair, dt, chunk, nchunk, part);
    } else {
        if (vec)
            j_out_f64m<M, true><<<g2, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, nsplit, jpart);
        else
            j_out_f64m<M, false><<<g2, kThreads, 0, st>>>(B, ldB, naux, npair, rho, prows, nsplit, jpart);
    }
}

void dispatch_j_multi(int M, bool vec, dim3 g1, dim3 g2, hipStream_t st, const double* B, int64_t ldB,
                      int64_t naux, int64_t npair, const double* dt, int64_t chunk, int nchunk, double* part,
                      const double* rho, int64_t prows, int64_t nsplit, double* jpart, bool pass1) {
    switch (M) {
#define DFJK_JM(k) \
    case k: launch_j_multi<k>(vec, g1, g2, st, B, ldB, naux, npair, dt, chunk, nchunk, part, rho, prows, nsplit, jpart, pass1); break;
        DFJK_JM(1) DFJK_JM(2) DFJK_JM(3) DFJK_JM(4) DFJK_JM(5) DFJK_JM(6) DFJK_JM(7) DFJK_JM(8)
#undef DFJK_JM
        default: break;
    }
}

}  // namespace

int j_batch_phase(hipStream_t st, int kind, int dtype, const MolDesc* mols, const PhaseList& pl) {
    if (pl.nblk <= 0) return DFJK_OK;
    const dim3 grid((unsigned)pl.nblk);
    switch (dtype) {
        case DFJK_F32: jb_kernel<float><<<grid, kThreads, 0, st>>>(kind, mols, pl); break;
        case DFJK_BF16: jb_kernel<uint16_t><<<grid, kThreads, 0, st>>>(kind, mols, pl); break;
        case DFJK_F16: jb_kernel<_Float16><<<grid, kThreads, 0, st>>>(kind, mols, pl); break;
        default: set_error("batched builds take FP32, BF16 or FP16 B"); return DFJK_E_DTYPE;
    }
    DFJK_LAUNCH_CHECK("jb_kernel");
    return DFJK_OK;
}

// Pass-2 geometry for column width U: (column blocks) x (row slices) ~ 4096.
static void j_out_geometry(const dfjk_ctx* h, int U, int64_t* splits_out) {
    const int64_t colblocks = cdiv(h->npair, (int64_t)kThreads * 2 * U);
    int64_t splits = cdiv(4096, colblocks);
    if (splits > h->naux) splits = h->naux;
    if (splits < 1) splits = 1;
    if (splits > 128) splits = 128;
    *splits_out = splits;
}

int j_out_count() { return kNumJOut; }

void j_plan(dfjk_ctx* h, JWork* w) {
    const int64_t rowblocks = cdiv(h->naux, kRhoRows);
    // pass 1: enough (row block, chunk) workgroups to cover the chip several times
    int64_t chunks = cdiv(4096, rowblocks);
    chunks = chunks < 1 ? 1 : chunks;
    const int64_t max_chunks = cdiv(h->npair, 2 * kThreads * 4);
    if (chunks > max_chunks) chunks = max_chunks;
    if (chunks < 1) chunks = 1;
    h->j_chunks = (int)chunks;
    // pass 2: the largest row slice count any column width needs
    int64_t splits = 1;
    for (int t = 0; t < kNumJOut; ++t) {
        int64_t sp;
        j_out_geometry(h, kJOutU[t], &sp);
        if (sp > splits) splits = sp;
    }
    h->j_splits = (int)splits;
    w->dt = sizeof(double) * (size_t)h->npair * 3;  // FP64 packed density + FP32 hi/lo
    w->rho_part = sizeof(double) * (size_t)h->naux * (size_t)chunks;
    w->rho = sizeof(double) * (size_t)h->naux * 2;  // rho + FP32 hi/lo
    w->jpart = sizeof(double) * (size_t)h->npair * (size_t)splits;
}

int64_t j_splits_used(const dfjk_ctx* h) {
    if (h->dtype != DFJK_F64) return h->j_splits;
    const int t = h->jout_tile >= 0 && h->jout_tile < kNumJOut ? h->jout_tile : 1;
    int64_t splits;
    j_out_geometry(h, kJOutU[t], &splits);
    return splits;
}

// DF-diagonal partials (one row slice of npair sums per pass-2 split)
static size_t j_diag_bytes(const dfjk_ctx* h) {
    return sizeof(double) * (size_t)h->npair * (size_t)(h->dtype == DFJK_F64 ? j_splits_used(h) : h->j_splits);
}

int j_setup(dfjk_ctx* h) {
    JWork w;
    j_plan(h, &w);
    int rc;
    if ((rc = h->dt.ensure(w.dt))) return rc;
    if ((rc = h->rho_part.ensure(w.rho_part))) return rc;
    if ((rc = h->rho.ensure(w.rho))) return rc;
    if ((rc = h->jpart.ensure(w.jpart))) return rc;
    return DFJK_OK;
}

int j_build(dfjk_ctx* h, const double* D, double* J, double* rho_out, double* diag) {
    double* dt = static_cast<double*>(h->dt.ptr);
    const hipStream_t st = h->stream;
    h->prof.begin(PH_J, st);
    pack_density<<<dim3((unsigned)h->nao), dim3(kThreads), 0, st>>>(D, h->nao, dt);
    DFJK_LAUNCH_CHECK("pack_density");
    switch (h->dtype) {
        case DFJK_F32: return j_build_red<float>(h, J, rho_out, diag);
        case DFJK_BF16: return j_build_red<uint16_t>(h, J, rho_out, diag);
        case DFJK_F16: return j_build_red<_Float16>(h, J, rho_out, diag);
        default: break;
    }
    const double* B = static_cast<const double*>(h->B);
    double* part = static_cast<double*>(h->rho_part.ptr);
    double* rho = static_cast<double*>(h->rho.ptr);
    double* jpart = static_cast<double*>(h->jpart.ptr);

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

    // default width 2048 columns (sweep at nao=1024, naux=4096 FP64: total J
    // 5.33 / 5.27 / 5.29 / 5.32 ms for 1024 / 2048 / 4096 / 8192 columns)
    const int t = h->jout_tile >= 0 && h->jout_tile < kNumJOut ? h->jout_tile : 1;
    const int U = kJOutU[t];
    int64_t splits;
    j_out_geometry(h, U, &splits);
    const int64_t prows = cdiv(h->naux, splits);
    const dim3 g2((unsigned)cdiv(h->npair, (int64_t)kThreads * 2 * U), (unsigned)splits);
    double* dpart = nullptr;
    if (diag) {
        int rc;
        if ((rc = h->dpart.ensure(j_diag_bytes(h)))) return rc;
        dpart = static_cast<double*>(h->dpart.ptr);
    }
    h->prof.begin(PH_J_OUT, st);
    switch (U) {
        case 2: launch_j_out<2>(vec, g2, st, B, h->ldB, h->naux, h->npair, rho, prows, jpart, dpart); break;
        case 4: launch_j_out<4>(vec, g2, st, B, h->ldB, h->naux, h->npair, rho, prows, jpart, dpart); break;
        case 8: launch_j_out<8>(vec, g2, st, B, h->ldB, h->naux, h->npair, rho, prows, jpart, dpart); break;
        default: launch_j_out<16>(vec, g2, st, B, h->ldB, h->naux, h->npair, rho, prows, jpart, dpart); break;
    }
    h->prof.end(PH_J_OUT, st);
    DFJK_LAUNCH_CHECK("j_out_f64");
    j_finish<<<dim3((unsigned)h->nao), kThreads, 0, st>>>(jpart, h->npair, (int)splits, h->nao, J);
    DFJK_LAUNCH_CHECK("j_finish");
    if (dpart) {
        diag_finish<<<dim3((unsigned)cdiv(h->npair, 256)), 256, 0, st>>>(dpart, h->npair, (int)splits, diag);
        DFJK_LAUNCH_CHECK("diag_finish");
    }
    h->prof.end(PH_J, st);
    return DFJK_OK;
}

// several-density geometry: pass 1 (8-row block, chunk) workgroups covering
// the chip several times; pass 2 1024 columns per workgroup
static void j_multi_geometry(const dfjk_ctx* h, int64_t* nchunk_out, int64_t* nsplit_out) {
    const int64_t rowblocks = cdiv(h->naux, kRhoRowsM);
    int64_t nchunk = cdiv(4096, rowblocks);
    const int64_t max_chunks = cdiv(h->npair, 2 * kThreads * 4);
    if (nchunk > max_chunks) nchunk = max_chunks;
    if (nchunk < 1) nchunk = 1;
    *nchunk_out = nchunk;
    j_out_geometry(h, 2, nsplit_out);
}

static int j_multi_ensure(dfjk_ctx* h, int64_t mmax, int64_t nchunk, int64_t nsplit) {
    const int64_t naux = h->naux, npair = h->npair;
    int rc;
    if ((rc = h->mdt.ensure(sizeof(double) * (size_t)(mmax * npair))) ||
        (rc = h->mpart.ensure(sizeof(double) * (size_t)(mmax * naux * nchunk))) ||
        (rc = h->mrho.ensure(sizeof(double) * (size_t)(mmax * naux))) ||
        (rc = h->mjpart.ensure(sizeof(double) * (size_t)(mmax * nsplit * npair))))
        return rc;
    return DFJK_OK;
}

int j_reserve(dfjk_ctx* h, int64_t max_ndm) {
    int rc;
    // the pass-2 width may be changed later with dfjk_set_tile: reserve the
    // DF-diagonal partials for the widest split count any width uses
    if ((rc = h->dpart.ensure(sizeof(double) * (size_t)h->npair * (size_t)h->j_splits))) return rc;
    if (h->dtype != DFJK_F64) return DFJK_OK;  // reduced B: one density at a time, no extra buffers
    int64_t nchunk, nsplit;
    j_multi_geometry(h, &nchunk, &nsplit);
    return j_multi_ensure(h, max_ndm < kMaxDm ? max_ndm : kMaxDm, nchunk, nsplit);
}

int j_build_multi(dfjk_ctx* h, int64_t ndm, const double* D, double* J, double* rho_out) {
    const int64_t nao = h->nao, naux = h->naux, npair = h->npair;
    if (h->dtype != DFJK_F64) {  // reduced B: one J stream per density
        for (int64_t m = 0; m < ndm; ++m) {
            int rc = j_build(h, D + m * nao * nao, J + m * nao * nao, rho_out ? rho_out + m * naux : nullptr,
                             nullptr);
            if (rc) return rc;
        }
        return DFJK_OK;
    }
    const hipStream_t st = h->stream;
    const double* B = static_cast<const double*>(h->B);
    const bool vec = (h->ldB % 2 == 0) && ((reinterpret_cast<uintptr_t>(B) & 15) == 0);
    const int64_t mmax = ndm < kMaxDm ? ndm : kMaxDm;
    const int64_t rowblocks = cdiv(naux, kRhoRowsM);
    int64_t nchunk, nsplit;
    j_multi_geometry(h, &nchunk, &nsplit);
    int64_t chunk = cdiv(cdiv(npair, nchunk), 2) * 2;
    const int64_t prows = cdiv(naux, nsplit);
    int rc;
    if ((rc = j_multi_ensure(h, mmax, nchunk, nsplit))) return rc;
    double* dt = static_cast<double*>(h->mdt.ptr);
    double* part = static_cast<double*>(h->mpart.ptr);
    double* rho = static_cast<double*>(h->mrho.ptr);
    double* jpart = static_cast<double*>(h->mjpart.ptr);
    const dim3 g1((unsigned)rowblocks, (unsigned)nchunk);
    const dim3 g2((unsigned)cdiv(npair, (int64_t)kThreads * 4), (unsigned)nsplit);
    h->prof.begin(PH_J, st);
    for (int64_t m0 = 0; m0 < ndm; m0 += kMaxDm) {
        const int M = (int)(ndm - m0 < kMaxDm ? ndm - m0 : kMaxDm);
        pack_density_m<<<dim3((unsigned)nao, (unsigned)M), kThreads, 0, st>>>(D + m0 * nao * nao, nao, npair, dt);
        DFJK_LAUNCH_CHECK("pack_density_m");
        h->prof.begin(PH_J_RHO, st);
        dispatch_j_multi(M, vec, g1, g2, st, B, h->ldB, naux, npair, dt, chunk, (int)nchunk, part, rho, prows,
                         nsplit, jpart, true);
        h->prof.end(PH_J_RHO, st);
        DFJK_LAUNCH_CHECK("j_rho_f64m");
        j_rho_finish_m<<<dim3((unsigned)cdiv(naux, 256), (unsigned)M), 256, 0, st>>>(
            part, naux, (int)nchunk, rho, rho_out ? rho_out + m0 * naux : nullptr);
        DFJK_LAUNCH_CHECK("j_rho_finish_m");
        h->prof.begin(PH_J_OUT, st);
        dispatch_j_multi(M, vec, g1, g2, st, B, h->ldB, naux, npair, dt, chunk, (int)nchunk, part, rho, prows,
                         nsplit, jpart, false);
        h->prof.end(PH_J_OUT, st);
        DFJK_LAUNCH_CHECK("j_out_f64m");
        j_finish_m<<<dim3((unsigned)nao, (unsigned)M), kThreads, 0, st>>>(jpart, npair, (int)nsplit, nao,
                                                                           J + m0 * nao * nao);
        DFJK_LAUNCH_CHECK("j_finish_m");
    }
    h->prof.end(PH_J, st);
    return DFJK_OK;
}

}  // namespace dfjk
