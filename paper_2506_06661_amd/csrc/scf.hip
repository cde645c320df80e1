// One restricted closed-shell SCF iteration on the GPU (FP64), and the
// exchange matrix of a general symmetric density.
//
// Iteration k with density D_k (paper Sec. IV.A: a mean-field run takes a
// guess density dm0, which need not be idempotent; Sec. IV.B: DIIS is the
// default accelerator):
//   J, K from D_k (K through C when D_k = 2 C C^T, else through the signed
//   eigen-factors of D_k); F = H + J - K/2;
//   E_k = tr(D H) + tr(D J)/2 - tr(D K)/4 = tr(D (H + F))/2;
//   e = F D - D F = G - G^T with G = F D (F, D symmetric);
//   Pulay DIIS over the last `diis_space` (F, e): minimise |sum c_i e_i| with
//   sum c_i = 1 through the bordered Gram system, solved by Gaussian
//   elimination with partial pivoting, after dropping the oldest pairs while
//   the Gram matrix's condition number exceeds 1e12; F' = sum c_i F_i;
//   aufbau on F' (Jacobi eigensolver): C = the nocc lowest eigenvectors,
//   D_{k+1} = 2 C C^T.
// Everything stays on the device; the host reads the iteration record only
// when the caller asks for it.
#include "dense.h"

namespace dfjk {

namespace {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

__global__ void fock_kernel(const double* __restrict__ H, const double* __restrict__ J,
                            const double* __restrict__ K, int64_t n2, double* __restrict__ F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n2) F[i] = H[i] + J[i] - 0.5 * K[i];
}

// e = G - G^T
__global__ void antisym_kernel(const double* __restrict__ G, int64_t n, double* __restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int64_t r = i / n, c = i % n;
    e[i] = G[r * n + c] - G[c * n + r];
}

__global__ void identity_kernel(int64_t n, double* __restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * n) Y[i] = (i / n == i % n) ? 1.0 : 0.0;
}

__global__ void symmetrize_kernel(const double* __restrict__ X, int64_t n, double* __restrict__ Y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * n) return;
    const int64_t r = i / n, c = i % n;
    Y[i] = 0.5 * (X[r * n + c] + X[c * n + r]);
}

struct Slots {
    int s[16];
};

// Gram matrix row/column of the newest error vector: dots[j] = <e_new, e_slot[j]>.
__global__ void gram_update(double* __restrict__ gram, int space, int snew, Slots order, int m,
                            const double* __restrict__ dotv) {
    const int j = threadIdx.x;
    if (j >= m) return;
    const int sj = order.s[j];
    gram[snew * space + sj] = dotv[j];
    gram[sj * space + snew] = dotv[j];
}

constexpr double kDiisMaxCond = 1e12;

// Extreme eigenvalues of a symmetric k x k matrix (k <= 15) by cyclic Jacobi
// rotations (Golub & Van Loan, Sec. 8.5), on one thread.
__device__ void small_eig_range(const double (*g)[16], int k, double* lo, double* hi) {
    double a[16][16];
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) a[i][j] = g[i][j];
    for (int sweep = 0; sweep < 30; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) {
                tot += a[i][j] * a[i][j];
                if (i != j) off += a[i][j] * a[i][j];
            }
        if (off <= 1e-30 * tot) break;
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int r = 0; r < k; ++r) {  // columns p, q
                    const double ap = a[r][p], aq = a[r][q];
                    a[r][p] = c * ap - sn * aq;
                    a[r][q] = sn * ap + c * aq;
                }
                for (int r = 0; r < k; ++r) {  // rows p, q
                    const double ap = a[p][r], aq = a[q][r];
                    a[p][r] = c * ap - sn * aq;
                    a[q][r] = sn * ap + c * aq;
                }
            }
    }
    double l = a[0][0], h = a[0][0];
    for (int i = 1; i < k; ++i) {
        l = fmin(l, a[i][i]);
        h = fmax(h, a[i][i]);
    }
    *lo = l;
    *hi = h;
}

// Bordered DIIS system for the stored vectors in chronological order, solved
// by Gaussian elimination with partial pivoting (one thread; m <= 15).  The
// oldest vectors are dropped, for this and every later iteration, while the
// Gram matrix of the remaining error vectors has a 2-norm condition number
// above kDiisMaxCond (or is singular); at least the newest stays.  first[0]
// holds the oldest iteration still in use (reset on iteration 1).  coef gets
// m entries in the order of `order`, zero for dropped vectors.
__global__ void diis_solve(const double* __restrict__ gram, int space, Slots order, int m, int iter,
                          double* __restrict__ first, double* __restrict__ coef) {
    if (threadIdx.x != 0) return;
    const int it0 = iter - m + 1;  // iteration of order.s[0]
    int k0 = 0;                     // first index of order still kept
    if (iter > 1) {
        const int f = (int)first[0];
        k0 = f > it0 ? f - it0 : 0;
    }
    if (k0 > m - 1) k0 = m - 1;
    double g[16][16];
    while (k0 < m - 1) {
        const int k = m - k0;
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j) g[i][j] = gram[order.s[k0 + i] * space + order.s[k0 + j]];
        double lo, hi;
        small_eig_range(g, k, &lo, &hi);
        if (lo > 0.0 && hi / lo <= kDiisMaxCond) break;
        ++k0;
    }
    first[0] = (double)(it0 + k0);
    for (int j = 0; j < k0; ++j) coef[j] = 0.0;
    const int mk = m - k0;  // vectors kept: order.s[k0 .. m-1]
    double a[16][17];
    const int n = mk + 1;
    for (int i = 0; i < mk; ++i) {
        for (int j = 0; j < mk; ++j) a[i][j] = gram[order.s[k0 + i] * space + order.s[k0 + j]];
        a[i][mk] = -1.0;
        a[i][n] = 0.0;
    }
    for (int j = 0; j < mk; ++j) a[mk][j] = -1.0;
    a[mk][mk] = 0.0;
    a[mk][n] = -1.0;
    bool singular = false;
    for (int col = 0; col < n && !singular; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (a[piv][col] == 0.0) {
            singular = true;
            break;
        }
        if (piv != col)
            for (int c = 0; c <= n; ++c) {
                const double t = a[col][c];
                a[col][c] = a[piv][c];
                a[piv][c] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            const double f = a[r][col] / a[col][col];
            for (int c = col; c <= n; ++c) a[r][c] -= f * a[col][c];
        }
    }
    double x[16];
    if (!singular) {
        for (int r = n - 1; r >= 0; --r) {
            double t = a[r][n];
            for (int c = r + 1; c < n; ++c) t -= a[r][c] * x[c];
            x[r] = t / a[r][r];
        }
        for (int j = 0; j < mk; ++j) coef[k0 + j] = x[j];
    } else {
        for (int j = 0; j < mk; ++j) coef[k0 + j] = j == mk - 1 ? 1.0 : 0.0;
    }
}

struct FList {
    const double* f[16];
};

__global__ void diis_combine(FList fl, const double* __restrict__ coef, int m, int64_t n2,
                             double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n2) return;
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += coef[j] * fl.f[j][i];
    out[i] = s;
}

struct ScfRecord {  // mirrors dfjk_scf_info
    double e_tot, e_1e, e_j, e_k, err_norm, d_e;
    int iter, converged;
};

// en = [tr(DH), tr(DJ), tr(DK)]; gram diagonal of the newest slot = |e|^2.
__global__ void scf_record(const double* __restrict__ en, const double* __restrict__ gram, int space,
                           int snew, int iter, double conv_tol, double conv_tol_grad,
                           double* __restrict__ e_prev, ScfRecord* __restrict__ rec) {
    if (threadIdx.x != 0) return;
    ScfRecord r;
    r.e_1e = en[0];
    r.e_j = 0.5 * en[1];
    r.e_k = -0.25 * en[2];
    r.e_tot = r.e_1e + r.e_j + r.e_k;
    r.err_norm = sqrt(gram[snew * space + snew]);
    r.d_e = iter > 1 ? r.e_tot - *e_prev : r.e_tot;
    r.iter = iter;
    r.converged = (iter > 1 && fabs(r.d_e) < conv_tol && r.err_norm < conv_tol_grad) ? 1 : 0;
    *e_prev = r.e_tot;
    *rec = r;
}

}  // namespace

// Workspace carved from h->eig: see scf_ws().
struct ScfWs {
    double *A, *V, *w, *work, *Cf, *sign;  // eigen-work (also used by the D path of K)
    int* iwork;
    double *J, *K, *F, *G, *Fx;            // SCF matrices
    double *Fh, *Eh;                       // DIIS history: space x n^2 each
    double *gram, *coef, *dotv, *part, *en, *e_prev, *diis_first;
    void* rec;
};

static int scf_ws(dfjk_ctx* h, bool scf, ScfWs& ws) {
    const int64_t n = h->nao, n2 = n * n;
    const int space = h->opts.diis_space;
    size_t need = 0;
    auto take = [&](size_t elems) {
        const size_t off = need;
        need += (elems + 31) / 32 * 32;
        return off;
    };
    const size_t oA = take(n2), oV = take(n2), ow = take(n), owork = take(n + 2), oCf = take(n2),
                 osign = take(n), oiw = take((n + 2 + 1) / 2);
    size_t oJ = 0, oK = 0, oF = 0, oG = 0, oFx = 0, oFh = 0, oEh = 0, ogr = 0, oco = 0, odv = 0,
           opart = 0, oen = 0, oep = 0, orec = 0, ofirst = 0;
    if (scf) {
        oJ = take(n2), oK = take(n2), oF = take(n2), oG = take(n2), oFx = take(n2);
        oFh = take((size_t)space * n2), oEh = take((size_t)space * n2);
        ogr = take((size_t)space * space), oco = take(16), odv = take(16),
        opart = take(dots_part_elems(kMaxDots)), oen = take(16), oep = take(1),
        orec = take(sizeof(ScfRecord) / sizeof(double) + 1), ofirst = take(1);
    }
    if (need * sizeof(double) > h->eig.bytes) h->scf_v_warm = false;  // fresh buffer
    int rc = h->eig.ensure(need * sizeof(double));
    if (rc) return rc;
    double* base = static_cast<double*>(h->eig.ptr);
    ws.A = base + oA;
    ws.V = base + oV;
    ws.w = base + ow;
    ws.work = base + owork;
    ws.Cf = base + oCf;
    ws.sign = base + osign;
    ws.iwork = reinterpret_cast<int*>(base + oiw);
    if (scf) {
        ws.J = base + oJ;
        ws.K = base + oK;
        ws.F = base + oF;
        ws.G = base + oG;
        ws.Fx = base + oFx;
        ws.Fh = base + oFh;
        ws.Eh = base + oEh;
        ws.gram = base + ogr;
        ws.coef = base + oco;
        ws.dotv = base + odv;
        ws.part = base + opart;
        ws.en = base + oen;
        ws.e_prev = base + oep;
        ws.rec = base + orec;
        ws.diis_first = base + ofirst;
    }
    return DFJK_OK;
}

// From this nao on, K of a density goes through the two factors (D, I)
// instead of D's eigen-factors.
constexpr int64_t kPairFromD = 256;

int k_build_from_D(dfjk_ctx* h, const double* D, double* K) {
    const int64_t n = h->nao;
    h->scf_v_warm = false;  // the eigensolver buffer is reused below
    if (n > kMaxEighN) {
        set_error("K from a density needs nao <= %d (got %lld); pass Cocc", kMaxEighN, (long long)n);
        return DFJK_E_INVALID;
    }
    // the SCF workspace also holds the eigen-work; keep it if it exists
    ScfWs ws;
    int rc = scf_ws(h, h->scf_ready, ws);
    if (rc) return rc;
    const hipStream_t st = h->stream;
    symmetrize_kernel<<<dim3((unsigned)cdiv(n * n, 256)), 256, 0, st>>>(D, n, ws.A);
    DFJK_LAUNCH_CHECK("symmetrize_kernel");
    if (n >= kPairFromD && h->opts.max_ncol == 0) {
        // K = 1/2 sum_P [(B_P D)(B_P I)^T + (B_P I)(B_P D)^T]: two factors of
        // nao columns each, no eigensolver (whose one-workgroup sweeps take
        // seconds from nao ~ 500 on); a reserved workspace (at most nao
        // columns) keeps the eigen-factor path, which fits it
        identity_kernel<<<dim3((unsigned)cdiv(n * n, 256)), 256, 0, st>>>(n, ws.V);
        DFJK_LAUNCH_CHECK("identity_kernel");
        return k_build_pair(h, ws.A, ws.V, n, 1, 0.5, K);
    }
    if ((rc = eigh(st, ws.A, ws.V, (int)n, true, ws.work, ws.iwork, ws.w))) return rc;
    // D = sum_c w_c v_c v_c^T = sum_c sign_c (sqrt|w_c| v_c)(sqrt|w_c| v_c)^T
    if ((rc = eig_gather(st, ws.V, (int)n, ws.iwork, (int)n, ws.w, 1, ws.Cf, ws.sign))) return rc;
    return k_build_factored(h, ws.Cf, n, ws.sign, 1.0, K);
}

int aufbau(dfjk_ctx* h, const double* F, int64_t nocc, double* C, double* D) {
    const int64_t n = h->nao;
    h->scf_v_warm = false;
    if (n > kMaxEighN) {
        set_error("dfjk_aufbau: nao=%lld above %d", (long long)n, kMaxEighN);
        return DFJK_E_INVALID;
    }
    ScfWs ws;
    int rc = scf_ws(h, h->scf_ready, ws);
    if (rc) return rc;
    const hipStream_t st = h->stream;
    symmetrize_kernel<<<dim3((unsigned)cdiv(n * n, 256)), 256, 0, st>>>(F, n, ws.A);
    DFJK_LAUNCH_CHECK("symmetrize_kernel");
    if ((rc = eigh(st, ws.A, ws.V, (int)n, true, ws.work, ws.iwork, ws.w))) return rc;
    if ((rc = eig_gather(st, ws.V, (int)n, ws.iwork, (int)nocc, ws.w, 0, C, nullptr))) return rc;
    if (D) return dgemm(st, false, true, n, n, nocc, 2.0, C, nocc, C, nocc, 0.0, D, n);
    return DFJK_OK;
}

int scf_reserve(dfjk_ctx* h) {
    ScfWs ws;
    return scf_ws(h, true, ws);
}

int scf_reset(dfjk_ctx* h) {
    h->scf_v_warm = false;
    h->scf_iter = 0;
    h->scf_count = 0;
    return DFJK_OK;
}

int scf_step(dfjk_ctx* h, const double* H, double* D, double* C, int64_t nocc, int flags,
             dfjk_scf_info* info) {
    const int64_t n = h->nao;
    if (n > kMaxEighN) {
        set_error("dfjk_scf_step: nao=%lld above %d", (long long)n, kMaxEighN);
        return DFJK_E_INVALID;
    }
    ScfWs ws;
    int rc = scf_ws(h, true, ws);
    if (rc) return rc;
    h->scf_ready = true;
    // J and K of the current density
    if ((rc = j_build(h, D, ws.J, nullptr, nullptr))) return rc;
    if (flags & DFJK_SCF_C_VALID)
        rc = k_build_factored(h, C, nocc, nullptr, 2.0, ws.K);
    else
        rc = k_build_from_D(h, D, ws.K);
    if (rc) return rc;
    const void* rec = nullptr;
    if ((rc = scf_tail(h, H, D, C, nocc, ws.J, ws.K, &rec))) return rc;
    if (info) return scf_read_info(h, rec, info);
    return DFJK_OK;
}

int scf_read_info(dfjk_ctx* h, const void* rec, dfjk_scf_info* info) {
    DFJK_HIP_TRY(hipMemcpyAsync(info, rec, sizeof(ScfRecord), hipMemcpyDeviceToHost, h->stream));
    DFJK_HIP_TRY(hipStreamSynchronize(h->stream));
    if (!(info->e_tot == info->e_tot)) {
        set_error("dfjk_scf_step: non-finite energy at iteration %d", info->iter);
        return DFJK_E_NONFINITE;
    }
    return info->converged ? DFJK_OK : DFJK_W_NOT_CONVERGED;
}

// Everything of an SCF iteration after J and K: Fock matrix, energies,
// commutator, DIIS, aufbau, next D and C, on the handle's stream.  *rec gets
// the device address of the iteration record.
int scf_tail(dfjk_ctx* h, const double* H, double* D, double* C, int64_t nocc, const double* J,
             const double* K, const void** rec) {
    const int64_t n = h->nao, n2 = n * n;
    const int space = h->opts.diis_space;
    ScfWs ws;
    int rc = scf_ws(h, true, ws);
    if (rc) return rc;
    h->scf_ready = true;
    const hipStream_t st = h->stream;
    const unsigned g2 = (unsigned)cdiv(n2, 256);
    fock_kernel<<<g2, 256, 0, st>>>(H, J, K, n2, ws.F);
    DFJK_LAUNCH_CHECK("fock_kernel");
    {
        DotList l{};
        l.a[0] = D, l.b[0] = H;
        l.a[1] = D, l.b[1] = J;
        l.a[2] = D, l.b[2] = K;
        if ((rc = dots(st, l, 3, n2, ws.part, ws.en))) return rc;
    }

    // DIIS history: slot of this iteration, chronological order of stored slots
    const int iter = h->scf_iter + 1;
    const int snew = (iter - 1) % space;
    const int m = h->scf_count + 1 < space ? h->scf_count + 1 : space;
    Slots order{};
    for (int j = 0; j < m; ++j) order.s[j] = (iter - m + j) % space;
    double* Fnew = ws.Fh + (size_t)snew * n2;
    double* enew = ws.Eh + (size_t)snew * n2;
    if ((rc = dgemm(st, false, false, n, n, n, 1.0, ws.F, n, D, n, 0.0, ws.G, n))) return rc;
    antisym_kernel<<<g2, 256, 0, st>>>(ws.G, n, enew);
    DFJK_LAUNCH_CHECK("antisym_kernel");
    DFJK_HIP_TRY(hipMemcpyAsync(Fnew, ws.F, n2 * sizeof(double), hipMemcpyDeviceToDevice, st));
    {
        DotList l{};
        for (int j = 0; j < m; ++j) l.a[j] = enew, l.b[j] = ws.Eh + (size_t)order.s[j] * n2;
        if ((rc = dots(st, l, m, n2, ws.part, ws.dotv))) return rc;
    }
    gram_update<<<1, 64, 0, st>>>(ws.gram, space, snew, order, m, ws.dotv);
    DFJK_LAUNCH_CHECK("gram_update");
    scf_record<<<1, 64, 0, st>>>(ws.en, ws.gram, space, snew, iter, h->opts.conv_tol,
                                 h->opts.conv_tol_grad, ws.e_prev, static_cast<ScfRecord*>(ws.rec));
    DFJK_LAUNCH_CHECK("scf_record");
    diis_solve<<<1, 64, 0, st>>>(ws.gram, space, order, m, iter, ws.diis_first, ws.coef);
    DFJK_LAUNCH_CHECK("diis_solve");
    {
        FList fl{};
        for (int j = 0; j < m; ++j) fl.f[j] = ws.Fh + (size_t)order.s[j] * n2;
        diis_combine<<<g2, 256, 0, st>>>(fl, ws.coef, m, n2, ws.Fx);
        DFJK_LAUNCH_CHECK("diis_combine");
    }

    // aufbau on the extrapolated Fock matrix; from the second iteration on the
    // Jacobi sweeps start in the previous eigenbasis (rows of V): V F V^T is
    // then nearly diagonal and needs few sweeps; V accumulates the rotations
    const bool warm = h->scf_v_warm;
    if (warm) {
        if ((rc = dgemm(st, false, true, n, n, n, 1.0, ws.Fx, n, ws.V, n, 0.0, ws.G, n))) return rc;
        if ((rc = dgemm(st, false, false, n, n, n, 1.0, ws.V, n, ws.G, n, 0.0, ws.Fx, n))) return rc;
    }
    symmetrize_kernel<<<g2, 256, 0, st>>>(ws.Fx, n, ws.A);
    DFJK_LAUNCH_CHECK("symmetrize_kernel");
    if ((rc = eigh(st, ws.A, ws.V, (int)n, !warm, ws.work, ws.iwork, ws.w))) return rc;
    h->scf_v_warm = true;
    if ((rc = eig_gather(st, ws.V, (int)n, ws.iwork, (int)nocc, ws.w, 0, C, nullptr))) return rc;
    if ((rc = dgemm(st, false, true, n, n, nocc, 2.0, C, nocc, C, nocc, 0.0, D, n))) return rc;

    h->scf_iter = iter;
    h->scf_count = m;
    *rec = ws.rec;
    return DFJK_OK;
}

}  // namespace dfjk
