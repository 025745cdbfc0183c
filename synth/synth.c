/*
 * Seeded synthetic inputs: counter-based random numbers, BPSK/AWGN channel
 * LLRs, and a GF(2) systematic encoder for quasi-cyclic parity-check
 * matrices.
 *
 * This file produces what is transmitted and received; it is not part of any
 * decoder.
 *
 * Random numbers: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011):
 * ten rounds of two 32x32->64-bit multiplications by 0xD2511F53 and
 * 0xCD9E8D57, the key bumped by the Weyl constants 0x9E3779B9 and
 * 0xBB67AE85 between rounds.
 *
 * Encoder:
 * The parity-check matrix is lifted from a base matrix of circulant shifts
 * (the paper's Eq. 2: block (j,l) is the p x p identity with its columns
 * shifted cyclically right a[j][l] times, so row r of that block has its one
 * in column (r + a) mod p; a = -1 is the zero block).  Gauss-Jordan
 * elimination over GF(2) brings H to reduced row echelon form R with pivot
 * columns P; the remaining columns F carry the information bits.  A codeword
 * takes c_F = u and c_{P_i} = sum_f R[i][f] u_f (mod 2), so H c^T = 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static void philox_round(uint32_t c[4], const uint32_t k[2]) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

/* out[4] = Philox-4x32-10(ctr, key) */
void synth_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k[0] += 0x9E3779B9u; k[1] += 0xBB67AE85u; }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* many counters at once: ctr [count][4], out [count][4] */
void synth_philox_many(const uint32_t* ctr, int64_t count, uint64_t seed, uint32_t* out) {
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) synth_philox(ctr + 4 * i, key, out + 4 * i);
}

static double uniform_open(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/*
 * Standard normal samples z [gamma][n] (double): sample (g, i) depends only
 * on (seed, frame0 + g, i).  Block b = i / 4 of frame f uses the counter
 * (b, f mod 2^32, tag, f >> 32); its four words (u0, u1, u2, u3) give two
 * Box-Muller pairs: r0 = sqrt(-2 ln u0) (cos, sin)(2 pi u1) and likewise
 * for (u2, u3).
 */
void synth_gaussian(uint64_t seed, int64_t frame0, int64_t gamma, int64_t n, uint32_t tag, double* z) {
    const int64_t nblk = (n + 3) / 4;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559;
    #pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < gamma; ++g) {
        const uint64_t f = (uint64_t)(frame0 + g);
        for (int64_t b = 0; b < nblk; ++b) {
            uint32_t ctr[4] = {(uint32_t)b, (uint32_t)f, tag, (uint32_t)(f >> 32)}, w[4];
            synth_philox(ctr, key, w);
            double r0 = sqrt(-2.0 * log(uniform_open(w[0])));
            double r1 = sqrt(-2.0 * log(uniform_open(w[2])));
            double v[4] = {r0 * cos(two_pi * uniform_open(w[1])), r0 * sin(two_pi * uniform_open(w[1])),
                           r1 * cos(two_pi * uniform_open(w[3])), r1 * sin(two_pi * uniform_open(w[3]))};
            for (int q = 0; q < 4; ++q) {
                int64_t i = 4 * b + q;
                if (i < n) z[g * n + i] = v[q];
            }
        }
    }
}

/* Channel LLRs mu = 2 y / sigma^2 with y = (1 - 2c) + sigma z, as float.
 * cw: [gamma][n] bits or NULL for the all-zero codeword. */
void synth_llr(uint64_t seed, int64_t frame0, int64_t gamma, int64_t n, uint32_t tag, const uint8_t* cw,
               double sigma2, float* llr) {
    const int64_t nblk = (n + 3) / 4;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two_pi = 6.283185307179586476925286766559, sigma = sqrt(sigma2);
    #pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < gamma; ++g) {
        const uint64_t f = (uint64_t)(frame0 + g);
        for (int64_t b = 0; b < nblk; ++b) {
            uint32_t ctr[4] = {(uint32_t)b, (uint32_t)f, tag, (uint32_t)(f >> 32)}, w[4];
            synth_philox(ctr, key, w);
            double r0 = sqrt(-2.0 * log(uniform_open(w[0])));
            double r1 = sqrt(-2.0 * log(uniform_open(w[2])));
            double v[4] = {r0 * cos(two_pi * uniform_open(w[1])), r0 * sin(two_pi * uniform_open(w[1])),
                           r1 * cos(two_pi * uniform_open(w[3])), r1 * sin(two_pi * uniform_open(w[3]))};
            for (int q = 0; q < 4; ++q) {
                int64_t i = 4 * b + q;
                if (i >= n) break;
                double x = (cw && (cw[g * n + i] & 1)) ? -1.0 : 1.0;
                llr[g * n + i] = (float)(2.0 * (x + sigma * v[q]) / sigma2);
            }
        }
    }
}

typedef struct {
    int n, m, rank, words;
    uint64_t* R;       /* rank x words, reduced row echelon form */
    int32_t* pivot;    /* rank pivot columns */
    int32_t* free_cols;/* n - rank information columns, ascending */
} gf2_code;

static inline int getbit(const uint64_t* row, int c) { return (int)((row[c >> 6] >> (c & 63)) & 1u); }

/* Returns an opaque handle, or NULL on bad input / allocation failure. */
void* gf2_qc_create(const int32_t* shifts, int J, int L, int p) {
    if (J <= 0 || L <= 0 || p <= 0) return NULL;
    int n = L * p, m = J * p, words = (n + 63) / 64;
    uint64_t* H = (uint64_t*)calloc((size_t)m * words, sizeof(uint64_t));
    if (!H) return NULL;
    for (int j = 0; j < J; ++j)
        for (int l = 0; l < L; ++l) {
            int a = shifts[j * L + l];
            if (a < 0) continue;
            if (a >= p) { free(H); return NULL; }
            for (int r = 0; r < p; ++r) {
                int row = j * p + r, col = l * p + (r + a) % p;
                H[(size_t)row * words + (col >> 6)] ^= (uint64_t)1 << (col & 63);
            }
        }
    int32_t* pivot = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m < n ? m : n));
    char* is_pivot = (char*)calloc((size_t)n, 1);
    if (!pivot || !is_pivot) { free(H); free(pivot); free(is_pivot); return NULL; }
    int rank = 0;
    for (int col = 0; col < n && rank < m; ++col) {
        int sel = -1;
        for (int r = rank; r < m; ++r)
            if (getbit(H + (size_t)r * words, col)) { sel = r; break; }
        if (sel < 0) continue;
        if (sel != rank) {
            uint64_t* a = H + (size_t)sel * words;
            uint64_t* b = H + (size_t)rank * words;
            for (int w = 0; w < words; ++w) { uint64_t t = a[w]; a[w] = b[w]; b[w] = t; }
        }
        const uint64_t* prow = H + (size_t)rank * words;
        #pragma omp parallel for schedule(static)
        for (int r = 0; r < m; ++r) {
            if (r == rank) continue;
            uint64_t* row = H + (size_t)r * words;
            if (getbit(row, col))
                for (int w = 0; w < words; ++w) row[w] ^= prow[w];
        }
        pivot[rank] = col;
        is_pivot[col] = 1;
        ++rank;
    }
    gf2_code* c = (gf2_code*)calloc(1, sizeof(gf2_code));
    int32_t* fr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n - rank > 0 ? n - rank : 1));
    if (!c || !fr) { free(H); free(pivot); free(is_pivot); free(c); free(fr); return NULL; }
    int k = 0;
    for (int col = 0; col < n; ++col)
        if (!is_pivot[col]) fr[k++] = col;
    free(is_pivot);
    c->n = n; c->m = m; c->rank = rank; c->words = words;
    c->R = H; c->pivot = pivot; c->free_cols = fr;
    return c;
}

int gf2_rank(const void* h) { return ((const gf2_code*)h)->rank; }
int gf2_n(const void* h) { return ((const gf2_code*)h)->n; }

/* info: [count][n - rank] bytes (0/1); out: [count][n] bytes (0/1). */
void gf2_encode(const void* h, const uint8_t* info, int count, uint8_t* out) {
    const gf2_code* c = (const gf2_code*)h;
    int n = c->n, k = n - c->rank, words = c->words;
    #pragma omp parallel
    {
        uint64_t* cw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)words);
        #pragma omp for schedule(static)
        for (int f = 0; f < count; ++f) {
            memset(cw, 0, sizeof(uint64_t) * (size_t)words);
            const uint8_t* u = info + (size_t)f * k;
            for (int i = 0; i < k; ++i)
                if (u[i] & 1) cw[c->free_cols[i] >> 6] |= (uint64_t)1 << (c->free_cols[i] & 63);
            for (int i = 0; i < c->rank; ++i) {
                const uint64_t* row = c->R + (size_t)i * words;
                uint64_t acc = 0;
                for (int w = 0; w < words; ++w) acc ^= row[w] & cw[w];
                int bit = __builtin_popcountll(acc) & 1;
                if (bit) cw[c->pivot[i] >> 6] |= (uint64_t)1 << (c->pivot[i] & 63);
            }
            uint8_t* o = out + (size_t)f * n;
            for (int i = 0; i < n; ++i) o[i] = (uint8_t)getbit(cw, i);
        }
        free(cw);
    }
}

void gf2_destroy(void* h) {
    gf2_code* c = (gf2_code*)h;
    if (!c) return;
    free(c->R); free(c->pivot); free(c->free_cols); free(c);
}
