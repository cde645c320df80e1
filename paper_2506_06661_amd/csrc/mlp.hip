// Learned initial guess: a three-layer perceptron (d_in -> H -> H -> 1, SiLU)
// that maps features of a basis-function pair to a correction of the
// core-Hamiltonian guess density.  The paper's mean-field runs accept any
// guess density (Sec. IV.A.1), so the prediction is used as given.
//
// All arithmetic is FP32 on the matrix cores (products) and vector units
// (activations, reductions, Adam); with the BF16 compute mode the three
// hidden-layer products (forward, input gradient, weight gradient) round
// their FP32 operands to bfloat16 and run on the 16-bit matrix cores with
// FP32 sums.  Weight gradients contract over the batch
// with the batch split into slabs whose partial products are added in a fixed
// order, so a training step is bitwise reproducible.
#include <new>
#include <vector>

#include "dense.h"
#include "numerics.h"

namespace dfjk {
namespace {

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__device__ inline float silu(float z) { return z / (1.f + __expf(-z)); }
__device__ inline float dsilu(float z) {
    const float s = 1.f / (1.f + __expf(-z));
    return s * (1.f + z * (1.f - s));
}

// Z += b (row broadcast), A = silu(Z)
__global__ void bias_silu(float* __restrict__ Z, const float* __restrict__ b, int64_t n, int h,
                          float* __restrict__ A) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h) return;
    const float z = Z[e] + b[e % h];
    Z[e] = z;
    A[e] = silu(z);
}

// y[i] = H2[i,:] . w + b   (one wavefront per row)
__global__ void rowdot(const float* __restrict__ H2, const float* __restrict__ w,
                       const float* __restrict__ b, int64_t n, int h, float* __restrict__ y) {
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n) return;
    float s = 0.f;
    for (int k = lane; k < h; k += 64) s = __builtin_fmaf(H2[row * h + k], w[k], s);
    s = wave_sum(s);
    if (lane == 0) y[row] = s + b[0];
}

// gy = 2 (y - t) / n; per-block partial sums of (y - t)^2 for the loss
__global__ void mse_grad(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                         float* __restrict__ gy, float* __restrict__ part) {
    __shared__ float red[4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float d = 0.f;
    if (i < n) {
        d = y[i] - t[i];
        gy[i] = 2.f * d / (float)n;
    }
    float s = wave_sum(d * d);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ void sum_parts(const float* __restrict__ part, int64_t np, float scale,
                          float* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < np; ++i) s += part[i];
    out[0] = (float)(s * scale);
}

// gZ2[i,h] = gy[i] * w3[h] * dsilu(Z2[i,h])
__global__ void back_out(const float* __restrict__ gy, const float* __restrict__ w3,
                         const float* __restrict__ Z2, int64_t n, int h, float* __restrict__ gZ2) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * h) return;
    gZ2[e] = gy[e / h] * w3[e % h] * dsilu(Z2[e]);
}

// G *= dsilu(Z) elementwise
__global__ void mul_dsilu(float* __restrict__ G, const float* __restrict__ Z, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) G[e] *= dsilu(Z[e]);
}

// out[c] = sum_i w_i A[i, c] (w = 1 when null): per-slab partials, then a
// fixed-order sum.  part: nslab x cols.
__global__ void col_partial(const float* __restrict__ A, const float* __restrict__ w, int64_t n,
                            int cols, int64_t slab, float* __restrict__ part) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = blockIdx.y;
    if (c >= cols) return;
    const int64_t i0 = s * slab, i1 = i0 + slab < n ? i0 + slab : n;
    float acc = 0.f;
    for (int64_t i = i0; i < i1; ++i) acc = __builtin_fmaf(w ? w[i] : 1.f, A[i * cols + c], acc);
    part[s * cols + c] = acc;
}

__global__ void col_finish(const float* __restrict__ part, int64_t nslab, int cols,
                           float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float acc = 0.f;
    for (int64_t s = 0; s < nslab; ++s) acc += part[s * cols + c];
    out[c] = acc;
}

// out[m][k] = sum_i A[i][m] B[i][k] over batch slabs (m < M, k < K), each slab
// a separate product into part, then added in order.
__global__ void slab_finish(const float* __restrict__ part, int64_t nslab, int64_t mk,
                            float* __restrict__ out) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= mk) return;
    float acc = 0.f;
    for (int64_t s = 0; s < nslab; ++s) acc += part[s * mk + e];
    out[e] = acc;
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Pair features of one system (mu <= nu, packed order p = nu(nu+1)/2 + mu):
// [Dcore_mn, H_mn, (H_mm + H_nn)/2, |H_mm - H_nn|, r/10, exp(-r^2),
//  delta_mn, (rank_m + rank_n) / (2 nao)] with rank = position of H_mm in
// ascending order of the diagonal of H.
__global__ void pair_features(const double* __restrict__ H, const double* __restrict__ Dc,
                              const double* __restrict__ R, int64_t nao, float* __restrict__ X) {
    const int64_t nu = blockIdx.x;
    const double hnn = H[nu * nao + nu];
    int rn = 0;
    for (int64_t k = 0; k < nao; ++k) {
        const double hk = H[k * nao + k];
        rn += (hk < hnn || (hk == hnn && k < nu)) ? 1 : 0;
    }
    for (int64_t mu = threadIdx.x; mu <= nu; mu += blockDim.x) {
        const double hmm = H[mu * nao + mu];
        int rm = 0;
        for (int64_t k = 0; k < nao; ++k) {
            const double hk = H[k * nao + k];
            rm += (hk < hmm || (hk == hmm && k < mu)) ? 1 : 0;
        }
        const double dx = R[3 * mu] - R[3 * nu], dy = R[3 * mu + 1] - R[3 * nu + 1],
                     dz = R[3 * mu + 2] - R[3 * nu + 2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        float* x = X + (nu * (nu + 1) / 2 + mu) * 8;
        x[0] = (float)Dc[mu * nao + nu];
        x[1] = (float)H[mu * nao + nu];
        x[2] = (float)(0.5 * (hmm + hnn));
        x[3] = (float)fabs(hmm - hnn);
        x[4] = (float)(sqrt(r2) * 0.1);
        x[5] = (float)exp(-r2);
        x[6] = mu == nu ? 1.f : 0.f;
        x[7] = (float)((rm + rn) * 0.5 / (double)nao);
    }
}

// D[mu][nu] = D[nu][mu] = Dcore[mu][nu] + y[p(mu,nu)]
__global__ void assemble_guess(const float* __restrict__ y, const double* __restrict__ Dc, int64_t nao,
                               double* __restrict__ D) {
    const int64_t nu = blockIdx.x;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += blockDim.x) {
        const double v = Dc[mu * nao + nu] + (double)y[nu * (nu + 1) / 2 + mu];
        D[mu * nao + nu] = v;
        D[nu * nao + mu] = v;
    }
}

// t[p(mu,nu)] = D[mu][nu] - Dcore[mu][nu] for mu <= nu (FP32 training target)
__global__ void guess_target(const double* __restrict__ D, const double* __restrict__ Dc, int64_t nao,
                             float* __restrict__ t) {
    const int64_t nu = blockIdx.x;
    for (int64_t mu = threadIdx.x; mu <= nu; mu += blockDim.x)
        t[nu * (nu + 1) / 2 + mu] = (float)(D[mu * nao + nu] - Dc[mu * nao + nu]);
}

// One workgroup: out[0] = tr D (fixed-order sum), out[1] = number of
// non-finite entries of D.
__global__ __launch_bounds__(256) void guess_check(const double* __restrict__ D, int64_t nao,
                                                   double* __restrict__ out) {
    __shared__ double s_tr[256];
    __shared__ double s_bad[256];
    double tr = 0.0, bad = 0.0;
    for (int64_t e = threadIdx.x; e < nao * nao; e += 256) {
        const double v = D[e];
        if (!isfinite(v)) bad += 1.0;
        if (e / nao == e % nao) tr += v;
    }
    s_tr[threadIdx.x] = tr;
    s_bad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_tr[threadIdx.x] += s_tr[threadIdx.x + w];
            s_bad[threadIdx.x] += s_bad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s_tr[0];
        out[1] = s_bad[0];
    }
}

// Y[r][:] = X[idx[r]][:] (rows of d FP32 values)
__global__ void gather_rows(const float* __restrict__ X, const int64_t* __restrict__ idx, int64_t n, int d,
                            float* __restrict__ Y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * d) return;
    const int64_t r = e / d;
    Y[e] = X[idx[r] * d + (e - r * d)];
}

constexpr int64_t kSlab = 2048;

}  // namespace
}  // namespace dfjk

struct dfjk_mlp_ctx {
    hipStream_t stream = nullptr;
    int d_in = 0, hidden = 0;
    int64_t max_batch = 0, nparam = 0;
    dfjk::DevBuf params, grads, m1, m2, act, part;
    int64_t step = 0;
    int compute = DFJK_F32;  // DFJK_BF16: hidden-layer products on the 16-bit matrix cores
    // parameter blocks inside `params` / `grads`
    int64_t oW1, ob1, oW2, ob2, oW3, ob3;
};

using namespace dfjk;

namespace {

struct Act {
    float *Z1, *A1, *Z2, *A2, *y, *gy, *gZ2, *gA1, *loss;
};

Act act_of(dfjk_mlp_ctx* m) {
    const int64_t nH = m->max_batch * m->hidden;
    float* b = static_cast<float*>(m->act.ptr);
    Act a;
    a.Z1 = b;
    a.A1 = b + nH;
    a.Z2 = b + 2 * nH;
    a.A2 = b + 3 * nH;
    a.gZ2 = b + 4 * nH;
    a.gA1 = b + 5 * nH;
    a.y = b + 6 * nH;
    a.gy = a.y + m->max_batch;
    a.loss = a.gy + m->max_batch;
    return a;
}

int forward(dfjk_mlp_ctx* m, const float* X, int64_t n, Act& a) {
    const hipStream_t st = m->stream;
    const float* P = static_cast<const float*>(m->params.ptr);
    const int H = m->hidden;
    int rc;
    if ((rc = sgemm(st, false, true, n, H, m->d_in, 1.f, X, m->d_in, P + m->oW1, m->d_in, 0.f, a.Z1, H)))
        return rc;
    bias_silu<<<dim3((unsigned)cdiv(n * H, 256)), 256, 0, st>>>(a.Z1, P + m->ob1, n, H, a.A1);
    DFJK_LAUNCH_CHECK("bias_silu");
    if (m->compute == DFJK_BF16)
        rc = bgemm(st, false, true, n, H, H, a.A1, H, P + m->oW2, H, a.Z2, H);
    else
        rc = sgemm(st, false, true, n, H, H, 1.f, a.A1, H, P + m->oW2, H, 0.f, a.Z2, H);
    if (rc) return rc;
    bias_silu<<<dim3((unsigned)cdiv(n * H, 256)), 256, 0, st>>>(a.Z2, P + m->ob2, n, H, a.A2);
    DFJK_LAUNCH_CHECK("bias_silu");
    rowdot<<<dim3((unsigned)cdiv(n, 4)), 256, 0, st>>>(a.A2, P + m->oW3, P + m->ob3, n, H, a.y);
    DFJK_LAUNCH_CHECK("rowdot");
    return DFJK_OK;
}

// out (M x K) = sum over the batch of A[i][:]^T B[i][:] in slabs (with bf16
// true, the slab products round A and B to bfloat16)
int batch_outer(dfjk_mlp_ctx* m, const float* A, int M, const float* B, int K, int64_t n, float* out,
                bool bf16 = false) {
    const hipStream_t st = m->stream;
    float* part = static_cast<float*>(m->part.ptr);
    const int64_t nslab = cdiv(n, kSlab);
    for (int64_t s = 0; s < nslab; ++s) {
        const int64_t i0 = s * kSlab, len = i0 + kSlab < n ? kSlab : n - i0;
        float* ps = part + s * (int64_t)M * K;
        int rc = bf16 ? bgemm(st, true, false, M, K, len, A + i0 * M, M, B + i0 * K, K, ps, K)
                      : sgemm(st, true, false, M, K, len, 1.f, A + i0 * M, M, B + i0 * K, K, 0.f, ps, K);
        if (rc) return rc;
    }
    slab_finish<<<dim3((unsigned)cdiv((int64_t)M * K, 256)), 256, 0, st>>>(part, nslab, (int64_t)M * K, out);
    DFJK_LAUNCH_CHECK("slab_finish");
    return DFJK_OK;
}

int colsum(dfjk_mlp_ctx* m, const float* A, const float* w, int cols, int64_t n, float* out) {
    const hipStream_t st = m->stream;
    float* part = static_cast<float*>(m->part.ptr);
    const int64_t nslab = cdiv(n, kSlab);
    col_partial<<<dim3((unsigned)cdiv(cols, 256), (unsigned)nslab), 256, 0, st>>>(A, w, n, cols, kSlab, part);
    DFJK_LAUNCH_CHECK("col_partial");
    col_finish<<<dim3((unsigned)cdiv(cols, 256)), 256, 0, st>>>(part, nslab, cols, out);
    DFJK_LAUNCH_CHECK("col_finish");
    return DFJK_OK;
}

int check(const dfjk_mlp_ctx* m, int64_t n) {
    if (!m) {
        set_error("null MLP handle");
        return DFJK_E_INVALID;
    }
    if (n < 1 || n > m->max_batch) {
        set_error("batch of %lld rows outside [1, %lld]", (long long)n, (long long)m->max_batch);
        return DFJK_E_INVALID;
    }
    return DFJK_OK;
}

}  // namespace

extern "C" {

int dfjk_mlp_init(dfjk_mlp* out, int d_in, int hidden, int64_t max_batch, void* stream) {
    clear_error();
    if (!out || d_in < 1 || d_in > 64 || hidden < 16 || hidden > 1024 || max_batch < 1 ||
        max_batch > (int64_t(1) << 24)) {
        set_error("dfjk_mlp_init: sizes out of range");
        return DFJK_E_INVALID;
    }
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_mlp_init: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    dfjk_mlp_ctx* m = new (std::nothrow) dfjk_mlp_ctx();
    if (!m) {
        set_error("dfjk_mlp_init: host allocation failed");
        return DFJK_E_OOM;
    }
    m->stream = (hipStream_t)stream;
    m->d_in = d_in;
    m->hidden = hidden;
    m->max_batch = max_batch;
    const int64_t H = hidden;
    m->oW1 = 0;
    m->ob1 = m->oW1 + H * d_in;
    m->oW2 = m->ob1 + H;
    m->ob2 = m->oW2 + H * H;
    m->oW3 = m->ob2 + H;
    m->ob3 = m->oW3 + H;
    m->nparam = m->ob3 + 1;
    const size_t pb = sizeof(float) * (size_t)m->nparam;
    const int64_t nslab = cdiv(max_batch, kSlab);
    int rc;
    if ((rc = m->params.ensure(pb)) || (rc = m->grads.ensure(pb)) || (rc = m->m1.ensure(pb)) ||
        (rc = m->m2.ensure(pb)) ||
        (rc = m->act.ensure(sizeof(float) * (size_t)(6 * max_batch * H + 2 * max_batch + 64))) ||
        (rc = m->part.ensure(sizeof(float) * (size_t)(nslab * (H * H + H + 64))))) {
        dfjk_mlp_destroy(m);
        return rc;
    }
    *out = m;
    return DFJK_OK;
}

int64_t dfjk_mlp_nparam(dfjk_mlp m) { return m ? m->nparam : -1; }

int dfjk_mlp_set_params(dfjk_mlp m, const float* host) {
    clear_error();
    if (!m || !host) {
        set_error("dfjk_mlp_set_params: null argument");
        return DFJK_E_INVALID;
    }
    const size_t pb = sizeof(float) * (size_t)m->nparam;
    DFJK_HIP_TRY(hipMemcpy(m->params.ptr, host, pb, hipMemcpyHostToDevice));
    std::vector<float> zero((size_t)m->nparam, 0.f);
    DFJK_HIP_TRY(hipMemcpy(m->m1.ptr, zero.data(), pb, hipMemcpyHostToDevice));
    DFJK_HIP_TRY(hipMemcpy(m->m2.ptr, zero.data(), pb, hipMemcpyHostToDevice));
    m->step = 0;
    return DFJK_OK;
}

int dfjk_mlp_get(dfjk_mlp m, int which, float* host) {
    clear_error();
    if (!m || !host || which < 0 || which > 1) {
        set_error("dfjk_mlp_get: bad arguments");
        return DFJK_E_INVALID;
    }
    DFJK_HIP_TRY(hipStreamSynchronize(m->stream));
    DFJK_HIP_TRY(hipMemcpy(host, which == 0 ? m->params.ptr : m->grads.ptr,
                           sizeof(float) * (size_t)m->nparam, hipMemcpyDeviceToHost));
    return DFJK_OK;
}

int dfjk_mlp_forward(dfjk_mlp m, const float* X_dev, int64_t n, float* y_dev) {
    clear_error();
    if (int rc = check(m, n)) return rc;
    if (!X_dev || !y_dev) {
        set_error("dfjk_mlp_forward: null argument");
        return DFJK_E_INVALID;
    }
    Act a = act_of(m);
    if (int rc = forward(m, X_dev, n, a)) return rc;
    DFJK_HIP_TRY(hipMemcpyAsync(y_dev, a.y, sizeof(float) * n, hipMemcpyDeviceToDevice, m->stream));
    return DFJK_OK;
}

int dfjk_mlp_loss_grad(dfjk_mlp m, const float* X, const float* t, int64_t n, float* loss_dev) {
    clear_error();
    if (int rc = check(m, n)) return rc;
    if (!X || !t) {
        set_error("dfjk_mlp_loss_grad: null argument");
        return DFJK_E_INVALID;
    }
    const hipStream_t st = m->stream;
    Act a = act_of(m);
    int rc;
    if ((rc = forward(m, X, n, a))) return rc;
    const int H = m->hidden;
    const float* P = static_cast<const float*>(m->params.ptr);
    float* G = static_cast<float*>(m->grads.ptr);
    float* part = static_cast<float*>(m->part.ptr);
    const int64_t nb = cdiv(n, 256);
    mse_grad<<<dim3((unsigned)nb), 256, 0, st>>>(a.y, t, n, a.gy, part);
    DFJK_LAUNCH_CHECK("mse_grad");
    sum_parts<<<1, 64, 0, st>>>(part, nb, 1.f / (float)n, a.loss);
    DFJK_LAUNCH_CHECK("sum_parts");
    // layer 3
    if ((rc = colsum(m, a.A2, a.gy, H, n, G + m->oW3))) return rc;
    if ((rc = colsum(m, a.gy, nullptr, 1, n, G + m->ob3))) return rc;
    // layer 2
    back_out<<<dim3((unsigned)cdiv(n * H, 256)), 256, 0, st>>>(a.gy, P + m->oW3, a.Z2, n, H, a.gZ2);
    DFJK_LAUNCH_CHECK("back_out");
    const bool bf = m->compute == DFJK_BF16;
    if ((rc = batch_outer(m, a.gZ2, H, a.A1, H, n, G + m->oW2, bf))) return rc;
    if ((rc = colsum(m, a.gZ2, nullptr, H, n, G + m->ob2))) return rc;
    // layer 1
    rc = bf ? bgemm(st, false, false, n, H, H, a.gZ2, H, P + m->oW2, H, a.gA1, H)
            : sgemm(st, false, false, n, H, H, 1.f, a.gZ2, H, P + m->oW2, H, 0.f, a.gA1, H);
    if (rc) return rc;
    mul_dsilu<<<dim3((unsigned)cdiv(n * H, 256)), 256, 0, st>>>(a.gA1, a.Z1, n * H);
    DFJK_LAUNCH_CHECK("mul_dsilu");
    if ((rc = batch_outer(m, a.gA1, H, X, m->d_in, n, G + m->oW1))) return rc;
    if ((rc = colsum(m, a.gA1, nullptr, H, n, G + m->ob1))) return rc;
    if (loss_dev)
        DFJK_HIP_TRY(hipMemcpyAsync(loss_dev, a.loss, sizeof(float), hipMemcpyDeviceToDevice, st));
    return DFJK_OK;
}

int dfjk_mlp_set_compute(dfjk_mlp m, int dtype) {
    clear_error();
    if (!m || (dtype != DFJK_F32 && dtype != DFJK_BF16)) {
        set_error("dfjk_mlp_set_compute: null handle or dtype other than DFJK_F32 / DFJK_BF16");
        return DFJK_E_INVALID;
    }
    m->compute = dtype;
    return DFJK_OK;
}

int dfjk_mlp_adam(dfjk_mlp m, float lr, float beta1, float beta2, float eps) {
    clear_error();
    if (!m || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f)) {
        set_error("dfjk_mlp_adam: bad arguments");
        return DFJK_E_INVALID;
    }
    m->step += 1;
    const float c1 = 1.f - powf(beta1, (float)m->step), c2 = 1.f - powf(beta2, (float)m->step);
    adam_kernel<<<dim3((unsigned)cdiv(m->nparam, 256)), 256, 0, m->stream>>>(
        static_cast<float*>(m->params.ptr), static_cast<const float*>(m->grads.ptr),
        static_cast<float*>(m->m1.ptr), static_cast<float*>(m->m2.ptr), m->nparam, lr, beta1, beta2, eps,
        c1, c2);
    DFJK_LAUNCH_CHECK("adam_kernel");
    return DFJK_OK;
}

int dfjk_guess_features(const double* H, const double* Dcore, const double* R, int64_t nao, float* X,
                        void* stream) {
    clear_error();
    if (!H || !Dcore || !R || !X || nao < 1 || nao > 65535) {
        set_error("dfjk_guess_features: bad arguments");
        return DFJK_E_INVALID;
    }
    pair_features<<<dim3((unsigned)nao), 128, 0, (hipStream_t)stream>>>(H, Dcore, R, nao, X);
    DFJK_LAUNCH_CHECK("pair_features");
    return DFJK_OK;
}

int dfjk_guess_assemble(const float* y, const double* Dcore, int64_t nao, double* D, void* stream) {
    clear_error();
    if (!y || !Dcore || !D || nao < 1 || nao > 65535) {
        set_error("dfjk_guess_assemble: bad arguments");
        return DFJK_E_INVALID;
    }
    assemble_guess<<<dim3((unsigned)nao), 128, 0, (hipStream_t)stream>>>(y, Dcore, nao, D);
    DFJK_LAUNCH_CHECK("assemble_guess");
    return DFJK_OK;
}

int dfjk_guess_target(const double* D, const double* Dcore, int64_t nao, float* t, void* stream) {
    clear_error();
    if (!D || !Dcore || !t || nao < 1 || nao > 65535) {
        set_error("dfjk_guess_target: bad arguments");
        return DFJK_E_INVALID;
    }
    guess_target<<<dim3((unsigned)nao), 128, 0, (hipStream_t)stream>>>(D, Dcore, nao, t);
    DFJK_LAUNCH_CHECK("guess_target");
    return DFJK_OK;
}

int dfjk_guess_check(const double* D, int64_t nao, double* out, void* stream) {
    clear_error();
    if (!D || !out || nao < 1 || nao > 65535) {
        set_error("dfjk_guess_check: bad arguments");
        return DFJK_E_INVALID;
    }
    guess_check<<<1, 256, 0, (hipStream_t)stream>>>(D, nao, out);
    DFJK_LAUNCH_CHECK("guess_check");
    return DFJK_OK;
}

int dfjk_gather_rows(const float* X, const int64_t* idx, int64_t n, int d, float* Y, void* stream) {
    clear_error();
    if (!X || !idx || !Y || n < 0 || d < 1) {
        set_error("dfjk_gather_rows: bad arguments");
        return DFJK_E_INVALID;
    }
    if (n == 0) return DFJK_OK;
    gather_rows<<<dim3((unsigned)cdiv(n * d, 256)), 256, 0, (hipStream_t)stream>>>(X, idx, n, d, Y);
    DFJK_LAUNCH_CHECK("gather_rows");
    return DFJK_OK;
}

void dfjk_mlp_destroy(dfjk_mlp m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    m->params.release();
    m->grads.release();
    m->m1.release();
    m->m2.release();
    m->act.release();
    m->part.release();
    delete m;
}

}  // extern "C"
