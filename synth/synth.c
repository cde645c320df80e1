/*
 * Seeded synthetic inputs for the density-fitted J/K build: the 3-index
 * tensor B[P, mu<=nu], and the plain random streams (uniform, normal) from
 * which the Python side builds lattices, C_occ and core Hamiltonians.
 *
 * This file holds no J/K, SCF or model arithmetic.  It is shared by the
 * oracle side and the GPU side only as a source of inputs.
 *
 * Random numbers: Philox-4x32-10, the counter-based generator of
 * Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
 * 1, 2, 3" (SC'11), written out here from its published definition.
 * Key = (seed low 32 bits, seed high 32 bits); counter words =
 * (index low, index high, stream id, 0).  A 53-bit uniform in [0,1) takes two
 * output words; a normal takes one Box-Muller draw from the four words of
 * one counter (the cosine branch only).
 *
 * Packed pair order: p(mu, nu) = nu*(nu+1)/2 + mu for mu <= nu, i.e. the lower
 * triangle listed row by row, the order numpy.tril_indices gives and the one
 * the paper's aosym='s2' three-index arrays use.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

/* One Philox-4x32-10 block: ten rounds, key bumped by the Weyl constants
 * between rounds. */
void synth_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(PHILOX_M0, c0, &hi0, &lo0);
        mulhilo32(PHILOX_M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static inline void draw(uint64_t seed, uint32_t stream, uint64_t index, uint32_t out[4]) {
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), stream, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    synth_philox4x32_10(ctr, key, out);
}

static inline double u53(uint32_t hi, uint32_t lo) {
    uint64_t x = (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
    return (double)x * 0x1.0p-53;
}

static inline double uniform_at(uint64_t seed, uint32_t stream, uint64_t index) {
    uint32_t w[4];
    draw(seed, stream, index, w);
    return u53(w[0], w[1]);
}

static inline double normal_at(uint64_t seed, uint32_t stream, uint64_t index) {
    uint32_t w[4];
    draw(seed, stream, index, w);
    double u1 = 1.0 - u53(w[0], w[1]); /* (0, 1] */
    double u2 = u53(w[2], w[3]);       /* [0, 1) */
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

void synth_uniform(uint64_t seed, uint32_t stream, uint64_t start, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = uniform_at(seed, stream, start + (uint64_t)i);
}

void synth_normal(uint64_t seed, uint32_t stream, uint64_t start, int64_t n, double* out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = normal_at(seed, stream, start + (uint64_t)i);
}

/* Stream ids used for B. */
#define STREAM_AUX_SCALE 1u
#define STREAM_B_NORMAL 2u

/*
 * Rows P0 .. P0+nrows-1 of B, written to out[(P-P0)*ldB + p] in FP64:
 *   B[P, p(mu,nu)] = a_P * exp(-|R_mu - R_nu|^2 / 2) * z_{P,p},
 *   a_P ~ U(0.1, 1) (stream 1, counter P), z ~ N(0,1) (stream 2, counter
 *   P*npair + p).
 * R is nao x 3 row-major (bohr).  Pad columns p >= npair are set to zero.
 * The value of every element depends only on (seed, P, p), so any block of
 * rows can be produced on its own.
 */
void synth_B_rows(uint64_t seed, int64_t nao, const double* R, int64_t P0, int64_t nrows,
                  int64_t ldB, double* out) {
    const int64_t npair = nao * (nao + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t P = P0 + r;
        const double aP = 0.1 + 0.9 * uniform_at(seed, STREAM_AUX_SCALE, (uint64_t)P);
        double* row = out + r * ldB;
        for (int64_t nu = 0; nu < nao; ++nu) {
            const int64_t base = nu * (nu + 1) / 2;
            for (int64_t mu = 0; mu <= nu; ++mu) {
                const double dx = R[3 * mu + 0] - R[3 * nu + 0];
                const double dy = R[3 * mu + 1] - R[3 * nu + 1];
                const double dz = R[3 * mu + 2] - R[3 * nu + 2];
                const double decay = exp(-0.5 * (dx * dx + dy * dy + dz * dz));
                const uint64_t idx = (uint64_t)P * (uint64_t)npair + (uint64_t)(base + mu);
                row[base + mu] = aP * decay * normal_at(seed, STREAM_B_NORMAL, idx);
            }
        }
        for (int64_t p = npair; p < ldB; ++p) row[p] = 0.0;
    }
}

/*
 * Sampled columns of B: out[P*ncols + j] = B[P, p_j] for all P < naux.
 * Lets a checker build single outputs at sizes where B does not fit in
 * host memory.
 */
void synth_B_cols(uint64_t seed, int64_t nao, const double* R, int64_t naux, const int64_t* cols,
                  int64_t ncols, double* out) {
    const int64_t npair = nao * (nao + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t P = 0; P < naux; ++P) {
        const double aP = 0.1 + 0.9 * uniform_at(seed, STREAM_AUX_SCALE, (uint64_t)P);
        for (int64_t j = 0; j < ncols; ++j) {
            const int64_t p = cols[j];
            /* invert p -> (mu, nu) */
            int64_t nu = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
            while (nu * (nu + 1) / 2 > p) --nu;
            while ((nu + 1) * (nu + 2) / 2 <= p) ++nu;
            const int64_t mu = p - nu * (nu + 1) / 2;
            const double dx = R[3 * mu + 0] - R[3 * nu + 0];
            const double dy = R[3 * mu + 1] - R[3 * nu + 1];
            const double dz = R[3 * mu + 2] - R[3 * nu + 2];
            const double decay = exp(-0.5 * (dx * dx + dy * dy + dz * dz));
            const uint64_t idx = (uint64_t)P * (uint64_t)npair + (uint64_t)p;
            out[P * ncols + j] = aP * decay * normal_at(seed, STREAM_B_NORMAL, idx);
        }
    }
}
