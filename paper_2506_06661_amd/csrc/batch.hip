// Batched J/K builds over many molecules of uneven size.
//
// Every phase of the single-molecule build (pack density, J pass 1, rho
// reduction, J pass 2, J unpack, C to FP32, GEMM1, SYRK, K reduction) runs as
// ONE launch over all molecules: the grid is the concatenation of every
// molecule's blocks, molecules in longest-processing-time-first order (cost
// naux * nao^2 * nocc), and each block finds its molecule by binary search in
// a prefix table.  GEMM1 runs once per tile bucket (molecules grouped by
// ceil(nocc/16)), with the tile of each bucket chosen by the autotuner.  The
// whole sequence can be captured once into a HIP graph and replayed: no
// allocation, host synchronisation or memset is enqueued by a build.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <vector>

#include "internal.h"

namespace dfjk {
namespace {

constexpr int kT = 256;
constexpr int kBuckets = 8;
constexpr int64_t kBatchJRows = 256;      // most B rows one J pass-2 workgroup walks
constexpr int64_t kBatchSyrkRows = 1024;  // most (P, i) rows one SYRK workgroup sums

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline int bucket_of(int64_t nocc) {
    const int64_t b = cdiv(nocc, 16) - 1;
    return (int)(b < kBuckets - 1 ? b : kBuckets - 1);
}

struct Phase {
    int kind;  // BatchPhaseKind, or -1 for GEMM1
    int bucket;
    std::vector<int> ids;
    std::vector<int64_t> prefix;
    int64_t off_ids = 0, off_prefix = 0;  // byte offsets in the list buffer
};

}  // namespace
}  // namespace dfjk

struct dfjk_batch_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;  // private stream for graph capture
    int dtype = DFJK_F32;
    int nmol = 0;
    std::vector<dfjk::MolDesc> mols;
    std::vector<double> cost;
    std::vector<int> order;  // molecules, longest first
    dfjk::DevBuf d_mols, work, lists;
    std::vector<dfjk::Phase> phases;
    int tile[dfjk::kBuckets];
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // SCF iterations over the batch: one handle per molecule without B (its
    // DIIS history and eigensolver state), and worker streams for the
    // molecules' dense steps
    std::vector<dfjk_ctx*> scf;
    std::vector<hipStream_t> workers;
    std::vector<hipEvent_t> worker_done;
    hipEvent_t built = nullptr;
    // exchange on the 16-bit matrix cores (BF16 / FP16 B), off by default
    bool k16 = false;
    dfjk::DevBuf work16;
};

namespace dfjk {
namespace {

int64_t phase_blocks(int kind, const MolDesc& d, int dtype) {
    const int64_t V = dtype == DFJK_F32 ? 4 : 8;
    switch (kind) {
        case BP_PACK: return d.nao;
        case BP_RHO: return cdiv(d.naux, 8) * d.j_chunks;
        case BP_RHO_FIN: return cdiv(d.naux, kT);
        case BP_OUT: return cdiv(d.npair, kT * V) * d.j_splits;
        case BP_JFIN: return d.nao;
        case BP_CF32: return cdiv(d.nao * d.nocc, kT);
        case BP_SYRK: return d.ntl * d.nsplit;
        case BP_KFIN: return d.ntl;
        case BP_CT16:
        case BP_SYRK16:
        case BP_KFIN16: return k16_batch_blocks(kind, 0, d);
        default: return 0;
    }
}

// (Re)build the GEMM1 geometry and the phase lists for the current tiles.
int build_phases(dfjk_batch_ctx* b) {
    for (auto& d : b->mols) {
        const int t = b->tile[bucket_of(d.nocc)];
        tile_nb(t, d.nao, d.nocc, &d.g1_nib, &d.g1_nmb);
    }
    b->phases.clear();
    auto add = [&](int kind, int bucket) {
        Phase ph;
        ph.kind = kind;
        ph.bucket = bucket;
        int64_t acc = 0;
        for (int m : b->order) {
            const MolDesc& d = b->mols[m];
            int64_t nb;
            if (kind < 0) {
                if (bucket_of(d.nocc) != bucket) continue;
                nb = d.g1_nib * d.g1_nmb * d.naux;
            } else if (kind == BP_G16) {
                if (k16_batch_bucket(d) != bucket) continue;
                nb = k16_batch_blocks(BP_G16, bucket, d);
            } else {
                nb = phase_blocks(kind, d, b->dtype);
            }
            ph.ids.push_back(m);
            ph.prefix.push_back(acc);
            acc += nb;
        }
        ph.prefix.push_back(acc);
        if (!ph.ids.empty()) b->phases.push_back(ph);
    };
    for (int k : {BP_PACK, BP_RHO, BP_RHO_FIN, BP_OUT, BP_JFIN}) add(k, 0);
    if (b->k16) {
        add(BP_CT16, 0);
        for (int bk = 0; bk < 3; ++bk) add(BP_G16, bk);
        for (int k : {BP_SYRK16, BP_KFIN16}) add(k, 0);
    } else {
        add(BP_CF32, 0);
        for (int bk = 0; bk < kBuckets; ++bk) add(-1, bk);
        for (int k : {BP_SYRK, BP_KFIN}) add(k, 0);
    }
    size_t bytes = 0;
    for (auto& ph : b->phases) {
        ph.off_ids = (int64_t)bytes;
        bytes += (ph.ids.size() * sizeof(int) + 255) / 256 * 256;
        ph.off_prefix = (int64_t)bytes;
        bytes += (ph.prefix.size() * sizeof(int64_t) + 255) / 256 * 256;
    }
    int rc = b->lists.ensure(bytes);
    if (rc) return rc;
    char* base = static_cast<char*>(b->lists.ptr);
    for (auto& ph : b->phases) {
        DFJK_HIP_TRY(hipMemcpy(base + ph.off_ids, ph.ids.data(), ph.ids.size() * sizeof(int),
                               hipMemcpyHostToDevice));
        DFJK_HIP_TRY(hipMemcpy(base + ph.off_prefix, ph.prefix.data(), ph.prefix.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice));
    }
    DFJK_HIP_TRY(hipMemcpy(b->d_mols.ptr, b->mols.data(), b->mols.size() * sizeof(MolDesc),
                           hipMemcpyHostToDevice));
    return DFJK_OK;
}

PhaseList list_of(const dfjk_batch_ctx* b, const Phase& ph) {
    const char* base = static_cast<const char*>(b->lists.ptr);
    PhaseList pl;
    pl.ids = reinterpret_cast<const int*>(base + ph.off_ids);
    pl.prefix = reinterpret_cast<const int64_t*>(base + ph.off_prefix);
    pl.n = (int)ph.ids.size();
    pl.nblk = ph.prefix.back();
    return pl;
}

int run_phase(dfjk_batch_ctx* b, const Phase& ph, hipStream_t st) {
    const MolDesc* mols = static_cast<const MolDesc*>(b->d_mols.ptr);
    const PhaseList pl = list_of(b, ph);
    if (ph.kind < 0) return k_batch_gemm1(st, b->dtype, b->tile[ph.bucket], mols, pl);
    if (ph.kind <= BP_JFIN) return j_batch_phase(st, ph.kind, b->dtype, mols, pl);
    if (ph.kind >= BP_CT16) return k16_batch_phase(st, ph.kind, ph.bucket, b->dtype, mols, pl);
    return k_batch_phase(st, ph.kind, b->dtype, mols, pl);
}

int run_all(dfjk_batch_ctx* b, hipStream_t st) {
    for (const auto& ph : b->phases)
        if (int rc = run_phase(b, ph, st)) return rc;
    return DFJK_OK;
}

void drop_graph(dfjk_batch_ctx* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Time every compiled GEMM1 tile on each occupied bucket's launch (best of
// reps after one warm-up) and keep the fastest per bucket.
int time_tiles(dfjk_batch_ctx* b, int reps, double* best_ms) {
    int rc = DFJK_OK;
    hipEvent_t e0, e1;
    DFJK_HIP_TRY(hipEventCreate(&e0));
    DFJK_HIP_TRY(hipEventCreate(&e1));
    for (int bk = 0; bk < kBuckets; ++bk) {
        bool present = false;
        for (const auto& d : b->mols) present |= bucket_of(d.nocc) == bk;
        if (!present) continue;
        double best = 1e300;
        int best_t = b->tile[bk];
        for (int t = 0; t < k_tile_count(); ++t) {
            b->tile[bk] = t;
            if ((rc = build_phases(b))) break;
            const Phase* ph = nullptr;
            for (const auto& p : b->phases)
                if (p.kind < 0 && p.bucket == bk) ph = &p;
            if (!ph) continue;
            if ((rc = run_phase(b, *ph, b->stream))) break;  // warm-up
            double tmin = 1e300;
            for (int r = 0; r < reps; ++r) {
                (void)hipEventRecord(e0, b->stream);
                if ((rc = run_phase(b, *ph, b->stream))) break;
                (void)hipEventRecord(e1, b->stream);
                (void)hipEventSynchronize(e1);
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                tmin = std::min(tmin, (double)ms);
            }
            if (rc) break;
            if (tmin < best) {
                best = tmin;
                best_t = t;
            }
        }
        if (rc) break;
        b->tile[bk] = best_t;
        if (best_ms) best_ms[bk] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// Per-molecule SCF handles and worker streams, made on first use.
int scf_setup(dfjk_batch b) {
    if (!b->scf.empty()) return DFJK_OK;
    const int nw = std::min(b->nmol, 8);
    for (int w = 0; w < nw; ++w) {
        hipStream_t s = nullptr;
        hipEvent_t e = nullptr;
        DFJK_HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        b->workers.push_back(s);
        DFJK_HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->worker_done.push_back(e);
    }
    DFJK_HIP_TRY(hipEventCreateWithFlags(&b->built, hipEventDisableTiming));
    for (int i = 0; i < b->nmol; ++i) {
        dfjk_ctx* h = new (std::nothrow) dfjk_ctx();
        if (!h) {
            ::dfjk::set_error("dfjk_batch_scf: host allocation failed");
            return DFJK_E_OOM;
        }
        const MolDesc& d = b->mols[i];
        h->device = b->device;
        h->nao = d.nao;
        h->naux = d.naux;
        h->npair = d.npair;
        h->dtype = b->dtype;
        dfjk_default_options(&h->opts);
        b->scf.push_back(h);
    }
    // molecules longest first, dealt round-robin to the worker streams
    for (int j = 0; j < b->nmol; ++j) b->scf[b->order[j]]->stream = b->workers[j % nw];
    return DFJK_OK;
}

// Fork the worker streams off the batch stream, run fn(i) for every molecule
// on its worker stream, and join them back.
template <typename F>
int on_workers(dfjk_batch b, F fn) {
    DFJK_HIP_TRY(hipEventRecord(b->built, b->stream));
    for (hipStream_t s : b->workers) DFJK_HIP_TRY(hipStreamWaitEvent(s, b->built, 0));
    int rc = DFJK_OK;
    for (int j = 0; j < b->nmol && !rc; ++j) rc = fn(b->order[j]);
    for (size_t w = 0; w < b->workers.size(); ++w) {
        DFJK_HIP_TRY(hipEventRecord(b->worker_done[w], b->workers[w]));
        DFJK_HIP_TRY(hipStreamWaitEvent(b->stream, b->worker_done[w], 0));
    }
    return rc;
}

}  // namespace
}  // namespace dfjk

using namespace dfjk;

extern "C" {

int dfjk_batch_init(dfjk_batch* out, const dfjk_mol* mols, int nmol, int dtype, void* stream) {
    clear_error();
    if (!out || !mols || nmol < 1 || nmol > (1 << 20)) {
        set_error("dfjk_batch_init: null pointer or nmol=%d out of range", nmol);
        return DFJK_E_INVALID;
    }
    *out = nullptr;
    if (dtype != DFJK_F32 && dtype != DFJK_BF16 && dtype != DFJK_F16) {
        set_error("dfjk_batch_init: dtype %d; batched builds take FP32, BF16 or FP16 B", dtype);
        return DFJK_E_DTYPE;
    }
    for (int i = 0; i < nmol; ++i) {
        const dfjk_mol& m = mols[i];
        const int64_t npair = m.nao * (m.nao + 1) / 2;
        if (!m.B || !m.D || !m.Cocc || !m.J || !m.K || m.nao < 1 || m.nao > 65535 || m.naux < 1 ||
            m.ldB < npair || m.nocc < 1 || m.nocc > m.nao) {
            set_error("dfjk_batch_init: molecule %d has a null pointer or sizes out of range", i);
            return DFJK_E_INVALID;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        (void)hipGetLastError();
        set_error("dfjk_batch_init: no HIP device available");
        return DFJK_E_NO_DEVICE;
    }
    dfjk_batch_ctx* b = new (std::nothrow) dfjk_batch_ctx();
    if (!b) {
        set_error("dfjk_batch_init: host allocation failed");
        return DFJK_E_OOM;
    }
    (void)hipGetDevice(&b->device);
    b->stream = (hipStream_t)stream;
    b->dtype = dtype;
    b->nmol = nmol;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        set_error("dfjk_batch_init: hipStreamCreate failed");
        return DFJK_E_HIP;
    }
    const int64_t V = dtype == DFJK_F32 ? 4 : 8;
    const size_t esz = dtype == DFJK_F32 ? 4 : 2;
    // per-molecule geometry and workspace layout
    size_t total = 0;
    auto take = [&](size_t bytes) {
        const size_t off = total;
        total += (bytes + 255) / 256 * 256;
        return off;
    };
    std::vector<size_t> offs;
    b->mols.resize(nmol);
    for (int i = 0; i < nmol; ++i) {
        const dfjk_mol& m = mols[i];
        MolDesc& d = b->mols[i];
        d = MolDesc{};
        d.B = m.B;
        d.ldB = m.ldB;
        d.nao = m.nao;
        d.naux = m.naux;
        d.npair = m.nao * (m.nao + 1) / 2;
        d.nocc = m.nocc;
        d.D = m.D;
        d.C = m.Cocc;
        d.J = m.J;
        d.K = m.K;
        d.vec = 1;  // 16-byte loads of B at any element alignment
        (void)esz;
        const int64_t rowblocks = cdiv(d.naux, 8);
        int64_t chunks = cdiv(64, rowblocks);
        const int64_t max_chunks = std::max<int64_t>(1, cdiv(d.npair, kT * V * 2));
        d.j_chunks = std::min(std::max<int64_t>(chunks, 1), max_chunks);
        d.chunk = cdiv(cdiv(d.npair, d.j_chunks), V) * V;
        const int64_t colblocks = cdiv(d.npair, kT * V);
        // pass 2: at least 64 workgroups per molecule, and none walking more
        // than kBatchJRows rows of B (long serial walks left the pass at
        // 3.8 TB/s on MI355X)
        d.j_splits = std::min<int64_t>(
            std::min<int64_t>(std::max<int64_t>(std::max<int64_t>(cdiv(64, colblocks), cdiv(d.naux, kBatchJRows)), 1),
                              64),
            d.naux);
        d.prows = cdiv(d.naux, d.j_splits);
        const int64_t nt = cdiv(d.nao, 128);
        d.ntl = nt * (nt + 1) / 2;
        const int64_t nrows = d.naux * d.nocc;
        // SYRK: at least 32 workgroups per molecule, and none longer than
        // kBatchSyrkRows rows of the (P, i) contraction: bounds the FP32 running
        // sums and the launch's tail (with 4 splits per molecule the largest
        // molecules' blocks ran alone at the end: 56 ms of a 130 ms build; at
        // 256 molecules a graph replay took 79.6 / 77.8 / 77.3 ms with 4096 /
        // 2048 / 1024 rows per split)
        int64_t nsplit = std::min<int64_t>(std::max<int64_t>(std::max<int64_t>(cdiv(32, d.ntl), cdiv(nrows, kBatchSyrkRows)), 1),
                                           cdiv(nrows, 256));
        nsplit = std::max<int64_t>(nsplit, 1);
        d.kchunk = cdiv(cdiv(nrows, nsplit), 16) * 16;
        d.nsplit = cdiv(nrows, d.kchunk);
        offs.push_back(take(sizeof(double) * d.npair));
        offs.push_back(take(sizeof(double) * d.naux * d.j_chunks));
        offs.push_back(take(sizeof(double) * d.naux));
        offs.push_back(take(sizeof(double) * d.npair * d.j_splits));
        // FP32 C and X rows padded to whole 16-byte vectors (the exchange
        // kernels then stage them with 16-byte loads)
        d.ldcf = cdiv(d.nocc, 4) * 4;
        d.ldx = cdiv(d.nao, 4) * 4;
        offs.push_back(take(sizeof(float) * d.nao * d.ldcf));
        offs.push_back(take(sizeof(float) * nrows * d.ldx));
        offs.push_back(take(sizeof(float) * d.nsplit * d.ntl * 128 * 128));
        b->cost.push_back((double)d.naux * d.nao * d.nao * d.nocc);
    }
    int rc;
    if ((rc = b->work.ensure(total)) || (rc = b->d_mols.ensure(sizeof(MolDesc) * nmol))) {
        dfjk_batch_destroy(b);
        return rc;
    }
    char* base = static_cast<char*>(b->work.ptr);
    for (int i = 0; i < nmol; ++i) {
        MolDesc& d = b->mols[i];
        const size_t* o = &offs[7 * (size_t)i];
        d.dt = reinterpret_cast<double*>(base + o[0]);
        d.rho_part = reinterpret_cast<double*>(base + o[1]);
        d.rho = reinterpret_cast<double*>(base + o[2]);
        d.jpart = reinterpret_cast<double*>(base + o[3]);
        d.Cf = reinterpret_cast<float*>(base + o[4]);
        d.X = reinterpret_cast<float*>(base + o[5]);
        d.kpart = reinterpret_cast<float*>(base + o[6]);
    }
    b->order.resize(nmol);
    for (int i = 0; i < nmol; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(),
                     [&](int x, int y) { return b->cost[x] > b->cost[y]; });
    for (int k = 0; k < kBuckets; ++k) b->tile[k] = pick_tile(16 * (k + 1));
    if ((rc = build_phases(b))) {
        dfjk_batch_destroy(b);
        return rc;
    }
    *out = b;
    return DFJK_OK;
}

int dfjk_batch_build(dfjk_batch b) {
    clear_error();
    if (!b) {
        set_error("null batch handle");
        return DFJK_E_INVALID;
    }
    return run_all(b, b->stream);
}

int dfjk_batch_capture(dfjk_batch b) {
    clear_error();
    if (!b) {
        set_error("null batch handle");
        return DFJK_E_INVALID;
    }
    drop_graph(b);
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    DFJK_HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    int rc = run_all(b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(b->cap, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(e));
        return DFJK_E_HIP;
    }
    b->graph = g;
    DFJK_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return DFJK_OK;
}

int dfjk_batch_launch(dfjk_batch b) {
    clear_error();
    if (!b) {
        set_error("null batch handle");
        return DFJK_E_INVALID;
    }
    if (!b->exec) {
        set_error("dfjk_batch_launch: no captured graph (call dfjk_batch_capture)");
        return DFJK_E_INVALID;
    }
    DFJK_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    return DFJK_OK;
}

int dfjk_batch_get_tile(dfjk_batch b, int bucket, int* tile) {
    clear_error();
    if (!b || !tile || bucket < 0 || bucket >= kBuckets) {
        set_error("dfjk_batch_get_tile: bad arguments");
        return DFJK_E_INVALID;
    }
    *tile = b->tile[bucket];
    return DFJK_OK;
}

int dfjk_batch_set_tile(dfjk_batch b, int bucket, int tile) {
    clear_error();
    if (!b || bucket < 0 || bucket >= kBuckets || tile < 0 || tile >= k_tile_count()) {
        set_error("dfjk_batch_set_tile: bad arguments");
        return DFJK_E_INVALID;
    }
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    b->tile[bucket] = tile;
    drop_graph(b);
    return build_phases(b);
}

int dfjk_batch_autotune(dfjk_batch b, int reps, const char* cache_path, double* best_ms) {
    clear_error();
    if (!b || reps < 1 || reps > 100) {
        set_error("dfjk_batch_autotune: bad arguments");
        return DFJK_E_INVALID;
    }
    int rc;
    // a graph recorded with the old tiles must never replay over new geometry
    drop_graph(b);
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    // reference K of every molecule with the default tiles
    int default_tile[kBuckets];
    for (int k = 0; k < kBuckets; ++k) default_tile[k] = b->tile[k] = pick_tile(16 * (k + 1));
    if ((rc = build_phases(b)) || (rc = run_all(b, b->stream))) return rc;
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    std::vector<std::vector<double>> Kref(b->nmol);
    for (int i = 0; i < b->nmol; ++i) {
        const MolDesc& d = b->mols[i];
        Kref[i].resize((size_t)(d.nao * d.nao));
        DFJK_HIP_TRY(hipMemcpy(Kref[i].data(), d.K, Kref[i].size() * 8, hipMemcpyDeviceToHost));
    }
    // cached choices for this dtype replace the timing, not the parity check
    bool cached = false;
    if (cache_path) {
        if (FILE* f = fopen(cache_path, "r")) {
            int dt, bk, t;
            double ms;
            while (fscanf(f, "%d %d %d %lf", &dt, &bk, &t, &ms) == 4)
                if (dt == b->dtype && bk >= 0 && bk < kBuckets && t >= 0 && t < k_tile_count()) {
                    b->tile[bk] = t;
                    if (best_ms) best_ms[bk] = ms;
                    cached = true;
                }
            fclose(f);
        }
    }
    if (!cached && (rc = time_tiles(b, reps, best_ms))) return rc;
    // keep a bucket's choice only if its molecules reproduce the reference K
    if ((rc = build_phases(b)) || (rc = run_all(b, b->stream))) return rc;
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    bool changed = false;
    for (int i = 0; i < b->nmol; ++i) {
        const MolDesc& d = b->mols[i];
        std::vector<double> K((size_t)(d.nao * d.nao));
        DFJK_HIP_TRY(hipMemcpy(K.data(), d.K, K.size() * 8, hipMemcpyDeviceToHost));
        double err = 0, ref = 0;
        for (size_t e = 0; e < K.size(); ++e) {
            err = std::max(err, std::fabs(K[e] - Kref[i][e]));
            ref = std::max(ref, std::fabs(Kref[i][e]));
        }
        const int bk = bucket_of(d.nocc);
        if (err > 1e-5 * ref && b->tile[bk] != default_tile[bk]) {
            b->tile[bk] = default_tile[bk];
            changed = true;
        }
    }
    if (changed && (rc = build_phases(b))) return rc;
    if (cache_path && (!cached || changed)) {
        if (FILE* f = fopen(cache_path, "w")) {
            for (int bk = 0; bk < kBuckets; ++bk)
                fprintf(f, "%d %d %d %.6f\n", b->dtype, bk, b->tile[bk], best_ms ? best_ms[bk] : 0.0);
            fclose(f);
        }
    }
    return DFJK_OK;
}

int dfjk_batch_set_k16(dfjk_batch b, int on) {
    clear_error();
    if (!b || (on != 0 && on != 1)) {
        set_error("dfjk_batch_set_k16: null batch or flag not 0/1");
        return DFJK_E_INVALID;
    }
    if (on && b->dtype != DFJK_BF16 && b->dtype != DFJK_F16) {
        set_error("dfjk_batch_set_k16: the 16-bit exchange needs BF16 or FP16 B");
        return DFJK_E_DTYPE;
    }
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    drop_graph(b);
    if (on && !b->work16.ptr) {
        size_t total = 0;
        auto take = [&](size_t bytes) {
            const size_t off = total;
            total += (bytes + 255) / 256 * 256;
            return off;
        };
        std::vector<size_t> offs;
        for (auto& d : b->mols) {
            size_t ct, x, kp;
            k16_batch_geometry(d, &ct, &x, &kp);
            offs.push_back(take(ct));
            offs.push_back(take(x));
            offs.push_back(take(kp));
        }
        int rc;
        if ((rc = b->work16.ensure(total))) return rc;
        char* base = static_cast<char*>(b->work16.ptr);
        for (size_t i = 0; i < b->mols.size(); ++i) {
            MolDesc& d = b->mols[i];
            d.Ct16 = base + offs[3 * i];
            d.X16 = base + offs[3 * i + 1];
            d.kpart16 = reinterpret_cast<float*>(base + offs[3 * i + 2]);
        }
    }
    b->k16 = on != 0;
    return build_phases(b);
}

int dfjk_batch_workspace_bytes(dfjk_batch b, size_t* bytes) {
    clear_error();
    if (!b || !bytes) {
        set_error("dfjk_batch_workspace_bytes: bad arguments");
        return DFJK_E_INVALID;
    }
    *bytes = b->work.bytes + b->work16.bytes + b->d_mols.bytes + b->lists.bytes;
    return DFJK_OK;
}

int dfjk_batch_scf_guess(dfjk_batch b, const double* const* H_list) {
    clear_error();
    if (!b || !H_list) {
        set_error("dfjk_batch_scf_guess: null batch or H list");
        return DFJK_E_INVALID;
    }
    for (int i = 0; i < b->nmol; ++i)
        if (!H_list[i] || b->mols[i].nao > 4096) {
            set_error("dfjk_batch_scf_guess: molecule %d has a null H or nao above 4096", i);
            return DFJK_E_INVALID;
        }
    int rc;
    if ((rc = scf_setup(b))) return rc;
    return on_workers(b, [&](int i) {
        const MolDesc& d = b->mols[i];
        scf_reset(b->scf[i]);
        return aufbau(b->scf[i], H_list[i], d.nocc, const_cast<double*>(d.C), const_cast<double*>(d.D));
    });
}

int dfjk_batch_scf_reset(dfjk_batch b) {
    clear_error();
    if (!b) {
        set_error("null batch handle");
        return DFJK_E_INVALID;
    }
    for (dfjk_ctx* h : b->scf) scf_reset(h);
    return DFJK_OK;
}

int dfjk_batch_scf_step(dfjk_batch b, const double* const* H_list, dfjk_scf_info* info) {
    static_assert(sizeof(dfjk_scf_info) == 6 * sizeof(double) + 2 * sizeof(int), "record layout");
    clear_error();
    if (!b || !H_list) {
        set_error("dfjk_batch_scf_step: null batch or H list");
        return DFJK_E_INVALID;
    }
    for (int i = 0; i < b->nmol; ++i)
        if (!H_list[i] || b->mols[i].nao > 4096) {
            set_error("dfjk_batch_scf_step: molecule %d has a null H or nao above 4096", i);
            return DFJK_E_INVALID;
        }
    int rc;
    if ((rc = scf_setup(b))) return rc;
    // J(D) and K(Cocc) of every molecule, the batch's phases on its stream
    if ((rc = run_all(b, b->stream))) return rc;
    std::vector<const void*> rec((size_t)b->nmol, nullptr);
    rc = on_workers(b, [&](int i) {
        const MolDesc& d = b->mols[i];
        return scf_tail(b->scf[i], H_list[i], const_cast<double*>(d.D), const_cast<double*>(d.C), d.nocc, d.J,
                        d.K, &rec[i]);
    });
    if (rc || !info) return rc;
    for (int i = 0; i < b->nmol; ++i)
        DFJK_HIP_TRY(hipMemcpyAsync(&info[i], rec[i], sizeof(dfjk_scf_info), hipMemcpyDeviceToHost, b->stream));
    DFJK_HIP_TRY(hipStreamSynchronize(b->stream));
    bool all = true;
    for (int i = 0; i < b->nmol; ++i) {
        if (!(info[i].e_tot == info[i].e_tot)) {
            set_error("dfjk_batch_scf_step: non-finite energy for molecule %d", i);
            return DFJK_E_NONFINITE;
        }
        all = all && info[i].converged;
    }
    return all ? DFJK_OK : DFJK_W_NOT_CONVERGED;
}

void dfjk_batch_destroy(dfjk_batch b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (hipStream_t s : b->workers) (void)hipStreamSynchronize(s);
    for (dfjk_ctx* h : b->scf) dfjk_destroy(h);
    for (hipEvent_t e : b->worker_done) (void)hipEventDestroy(e);
    for (hipStream_t s : b->workers) (void)hipStreamDestroy(s);
    if (b->built) (void)hipEventDestroy(b->built);
    drop_graph(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    b->work.release();
    b->work16.release();
    b->d_mols.release();
    b->lists.release();
    delete b;
}

}  // extern "C"
