/*
 * FP64 reference sum-product decoder.
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that the GPU decoder can be
 * checked against a plain, slow, obviously correct implementation of the
 * paper's Algorithm 1.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it; the GPU library never does, and the
 * two share no code (only their seeded inputs).
 *
 * The decoder works on an explicit parity-check matrix H in compressed rows
 * (column indices ascending within each row).  Per frame, independently:
 *
 *   Initialization (Algorithm 1):   beta_mn = clip(mu_n) on every edge.
 *   Horizontal step (Eq. 3):        alpha_mn = 2 atanh( prod_{n' in N(m)\n} tanh(beta_mn' / 2) ),
 *                                   the product taken directly over the other
 *                                   edges of the row in ascending column order.
 *   Vertical step (Eq. 4):          beta_mn = clip( mu_n + sum_{m' in M(n)\m} alpha_m'n ),
 *                                   a direct sum in ascending row order.
 *   A-posteriori LLR (Eq. 5):       L_n = mu_n + sum_{m in M(n)} alpha_mn.
 *   Hard decision (Eq. 6):          c_n = 0 if L_n >= 0, else 1.
 *
 * One iteration is one full horizontal pass followed by one full vertical
 * pass (the two-phase flooding schedule of Sec. II-B).  Readings of points the
 * paper leaves open:
 *   - clip(x) = max(-lmax, min(lmax, x)) with lmax = 30 by default (the paper
 *     states no saturation; +inf disables it);
 *   - with early stopping enabled, the syndrome H c^T is tested after every
 *     complete iteration i >= 1 and the frame stops at the first i with a zero
 *     syndrome (the paper always runs I_max iterations);
 *   - the posterior output is clip(L_n).
 *
 * The window decoder for terminated LDPC convolutional codes (Sec. II-C/E)
 * runs the same two steps restricted to a sliding window of check layers and
 * code positions; see oracle_decode_window below.  The pipelined decoder of
 * Algorithm 2 runs them on a stream of code frames with I processors; see
 * oracle_decode_pipeline.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static double clipd(double x, double lmax) {
    if (x > lmax) return lmax;
    if (x < -lmax) return -lmax;
    return x;
}

/* column-wise view: for every column, its edges (indices into the row-major
 * edge list) in ascending row order */
typedef struct {
    int32_t* col_ptr;   /* n + 1 */
    int32_t* col_edge;  /* ne */
    int32_t* edge_row;  /* ne */
} colview;

static int build_colview(int n, int m, const int32_t* row_ptr, const int32_t* col_idx, colview* cv) {
    int ne = row_ptr[m];
    cv->col_ptr = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    cv->col_edge = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    cv->edge_row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ne > 0 ? ne : 1));
    int32_t* fill = (int32_t*)calloc((size_t)n + 1, sizeof(int32_t));
    if (!cv->col_ptr || !cv->col_edge || !cv->edge_row || !fill) { free(fill); return -1; }
    for (int e = 0; e < ne; ++e) {
        int c = col_idx[e];
        if (c < 0 || c >= n) { free(fill); return -1; }
        cv->col_ptr[c + 1]++;
    }
    for (int c = 0; c < n; ++c) cv->col_ptr[c + 1] += cv->col_ptr[c];
    /* rows visited in ascending order, so each column's list is row-ascending */
    for (int r = 0; r < m; ++r)
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            int c = col_idx[e];
            cv->col_edge[cv->col_ptr[c] + fill[c]++] = e;
            cv->edge_row[e] = r;
        }
    free(fill);
    return 0;
}

static void free_colview(colview* cv) {
    free(cv->col_ptr); free(cv->col_edge); free(cv->edge_row);
}

/* Horizontal step (Eq. 3) for one row: every outgoing alpha from the other
 * edges' beta, product taken directly (no division, no "total minus own").
 * th is caller scratch of at least the row weight. */
static void check_update(const int32_t* row_ptr, int r, const double* beta, double* alpha, double* th) {
    int e0 = row_ptr[r], e1 = row_ptr[r + 1];
    for (int f = e0; f < e1; ++f) th[f - e0] = tanh(beta[f] / 2.0);
    for (int e = e0; e < e1; ++e) {
        double prod = 1.0;
        for (int f = e0; f < e1; ++f)
            if (f != e) prod *= th[f - e0];
        alpha[e] = 2.0 * atanh(prod);
    }
}

static int max_row_weight(int m, const int32_t* row_ptr) {
    int w = 1;
    for (int r = 0; r < m; ++r)
        if (row_ptr[r + 1] - row_ptr[r] > w) w = row_ptr[r + 1] - row_ptr[r];
    return w;
}

/* Syndrome of hard decisions c: returns 1 if every row has even parity. */
static int syndrome_zero(int m, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* c) {
    for (int r = 0; r < m; ++r) {
        int par = 0;
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) par ^= c[col_idx[e]];
        if (par) return 0;
    }
    return 1;
}

/*
 * Could flipping some of the decisions whose |L| is below `near` change
 * whether the syndrome of c is zero?  Flipping a set of variables toggles the
 * parity of every check they meet, so: if the syndrome is zero, yes as soon as
 * one such variable meets a check; if not, only if every unsatisfied check
 * meets such a variable (a necessary condition, so the answer errs towards
 * yes).  Returns 1 for yes.  touched is caller scratch of m bytes.
 */
static int syndrome_fragile(int n, int m, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* c,
                            const double* L, double near, uint8_t* touched) {
    int any_near = 0;
    for (int v = 0; v < n; ++v)
        if (fabs(L[v]) < near) { any_near = 1; break; }
    if (!any_near) return 0;
    int unsat = 0, all_covered = 1, near_checked = 0;
    for (int r = 0; r < m; ++r) {
        int par = 0;
        touched[r] = 0;
        for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e) {
            par ^= c[col_idx[e]];
            if (fabs(L[col_idx[e]]) < near) touched[r] = 1;
        }
        if (touched[r]) near_checked = 1;
        if (par) {
            unsat = 1;
            if (!touched[r]) all_covered = 0;
        }
    }
    return unsat ? all_covered : near_checked;
}

/*
 * Block decoder (Algorithm 1, flooding).
 *   llr       [gamma][n] float channel LLRs (read as double)
 *   post      [gamma][n] double, clip(L) of the stopping iteration
 *   bits      [gamma][n] hard decisions of the stopping iteration
 *   iters     [gamma] iterations run (first zero-syndrome iteration with early
 *             stopping, else max_iters)
 *   converged [gamma] 1 if the syndrome of the returned decisions is zero
 *   min_abs   [gamma] or NULL: min |L_n| over every decision made (all n, all
 *             iterations up to the stopping one)
 *   syn_trace [gamma][max_iters] or NULL: 1 where iteration i's decisions have
 *             a zero syndrome (filled up to the stopping iteration, rest 0)
 *   fragile   [gamma] or NULL: the first iteration (up to the returned one) at
 *             which decisions with |L_n| < near could change whether the
 *             syndrome is zero, else 0 (see syndrome_fragile); a diagnostic for
 *             comparing decoders that round differently, not part of decoding
 *   L_trace   [gamma][max_iters][n] or NULL: the unclipped L of every
 *             iteration (filled up to the stopping iteration)
 * Returns 0, or -1 on invalid input.
 */
int oracle_decode_block(int n, int m, const int32_t* row_ptr, const int32_t* col_idx,
                        const float* llr, int gamma, int max_iters, int early_stop,
                        double lmax, int nthreads,
                        double* post, uint8_t* bits, int32_t* iters, uint8_t* converged,
                        double* min_abs, uint8_t* syn_trace, double near, int32_t* fragile,
                        double* L_trace) {
    if (n < 0 || m < 0 || gamma < 0 || max_iters < 1) return -1;
    colview cv;
    if (build_colview(n, m, row_ptr, col_idx, &cv)) { free_colview(&cv); return -1; }
    int ne = row_ptr[m];
    int status = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    #pragma omp parallel
    {
        double* mu = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        double* beta = (double*)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
        double* alpha = (double*)malloc(sizeof(double) * (size_t)(ne > 0 ? ne : 1));
        double* L = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
        uint8_t* c = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
        double* th = (double*)malloc(sizeof(double) * (size_t)max_row_weight(m, row_ptr));
        uint8_t* touched = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
        if (!mu || !beta || !alpha || !L || !c || !th || !touched) {
            #pragma omp atomic write
            status = -1;
        } else {
            #pragma omp for schedule(dynamic, 1)
            for (int g = 0; g < gamma; ++g) {
                const float* y = llr + (size_t)g * n;
                for (int v = 0; v < n; ++v) mu[v] = (double)y[v];
                /* Initialization: beta_mn = mu_n on every edge */
                for (int r = 0; r < m; ++r)
                    for (int e = row_ptr[r]; e < row_ptr[r + 1]; ++e)
                        beta[e] = clipd(mu[col_idx[e]], lmax);
                double mina = INFINITY;
                int it_done = max_iters, zero = 0, frag = 0;
                if (syn_trace) memset(syn_trace + (size_t)g * max_iters, 0, (size_t)max_iters);
                for (int it = 1; it <= max_iters; ++it) {
                    /* horizontal step */
                    for (int r = 0; r < m; ++r) check_update(row_ptr, r, beta, alpha, th);
                    /* vertical step, a-posteriori LLR and hard decision */
                    for (int v = 0; v < n; ++v) {
                        int k0 = cv.col_ptr[v], k1 = cv.col_ptr[v + 1];
                        double tot = mu[v];
                        for (int k = k0; k < k1; ++k) tot += alpha[cv.col_edge[k]];
                        L[v] = tot;
                        for (int k = k0; k < k1; ++k) {
                            double s = mu[v];
                            for (int q = k0; q < k1; ++q)
                                if (q != k) s += alpha[cv.col_edge[q]];
                            beta[cv.col_edge[k]] = clipd(s, lmax);
                        }
                        c[v] = (uint8_t)(tot < 0.0);
                        double a = fabs(tot);
                        if (a < mina) mina = a;
                    }
                    zero = syndrome_zero(m, row_ptr, col_idx, c);
                    if (syn_trace) syn_trace[(size_t)g * max_iters + (it - 1)] = (uint8_t)zero;
                    if (L_trace) memcpy(L_trace + ((size_t)g * max_iters + (it - 1)) * n, L, sizeof(double) * (size_t)n);
                    if (fragile && frag == 0 && syndrome_fragile(n, m, row_ptr, col_idx, c, L, near, touched))
                        frag = it;
                    if (early_stop && zero) { it_done = it; break; }
                }
                for (int v = 0; v < n; ++v) {
                    post[(size_t)g * n + v] = clipd(L[v], lmax);
                    bits[(size_t)g * n + v] = c[v];
                }
                iters[g] = it_done;
                converged[g] = (uint8_t)zero;
                if (min_abs) min_abs[g] = mina;
                if (fragile) fragile[g] = frag;
            }
        }
        free(mu); free(beta); free(alpha); free(L); free(c); free(th); free(touched);
    }
    free_colview(&cv);
    return status;
}

/*
 * Sliding-window decoder for a terminated LDPC convolutional code.
 *
 * H is the explicit terminated parity-check matrix; layer_of_row[r] is the
 * check layer (time index of the block row of Eq. (ldpcccH)) of row r and
 * pos_of_col[v] the code position (frame) of column v.  Any two variables
 * sharing a check lie at most m_s positions apart (Sec. II-E), which is what
 * makes a window decoder possible.
 *
 * Window schedule for target position s = 0 .. npos-1 (the window decoder of
 * Iyengar et al., IEEE Trans. IT 2012, with flooding inside the window):
 *   window layers    s .. s+W-1 (those that exist)
 *   active positions s .. s+W-1 (those that exist)
 *   positions entering the window (all of 0..W-1 at s = 0, else s+W-1) start
 *   with beta = clip(mu) and alpha = 0 on all their edges; everything else is
 *   kept from the previous window (warm start), and positions before s keep
 *   their last beta (frozen);
 *   K iterations of: horizontal step over the window layers, then vertical
 *   step over the active positions, where only alphas from window layers are
 *   summed;
 *   decide position s: L_n = mu_n + sum of alphas from window layers,
 *   post = clip(L), bit = (L < 0).
 */
int oracle_decode_window(int n, int m, const int32_t* row_ptr, const int32_t* col_idx,
                         const int32_t* layer_of_row, const int32_t* pos_of_col,
                         int nlayers, int npos, const float* llr, int gamma, int W, int K,
                         double lmax, int nthreads, double* post, uint8_t* bits) {
    if (n < 0 || m < 0 || gamma < 0 || W < 1 || K < 1 || npos < 0 || nlayers < 0) return -1;
    colview cv;
    if (build_colview(n, m, row_ptr, col_idx, &cv)) { free_colview(&cv); return -1; }
    int ne = row_ptr[m];
    /* rows of each layer, columns of each position (both ascending) */
    int32_t* lay_ptr = (int32_t*)calloc((size_t)nlayers + 1, sizeof(int32_t));
    int32_t* lay_row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* pos_ptr = (int32_t*)calloc((size_t)npos + 1, sizeof(int32_t));
    int32_t* pos_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int status = 0;
    if (!lay_ptr || !lay_row || !pos_ptr || !pos_col) status = -1;
    for (int r = 0; r < m && !status; ++r) {
        if (layer_of_row[r] < 0 || layer_of_row[r] >= nlayers) status = -1;
        else lay_ptr[layer_of_row[r] + 1]++;
    }
    for (int v = 0; v < n && !status; ++v) {
        if (pos_of_col[v] < 0 || pos_of_col[v] >= npos) status = -1;
        else pos_ptr[pos_of_col[v] + 1]++;
    }
    if (!status) {
        for (int t = 0; t < nlayers; ++t) lay_ptr[t + 1] += lay_ptr[t];
        for (int t = 0; t < npos; ++t) pos_ptr[t + 1] += pos_ptr[t];
        int32_t* fl = (int32_t*)calloc((size_t)nlayers + 1, sizeof(int32_t));
        int32_t* fp = (int32_t*)calloc((size_t)npos + 1, sizeof(int32_t));
        for (int r = 0; r < m; ++r) lay_row[lay_ptr[layer_of_row[r]] + fl[layer_of_row[r]]++] = r;
        for (int v = 0; v < n; ++v) pos_col[pos_ptr[pos_of_col[v]] + fp[pos_of_col[v]]++] = v;
        free(fl); free(fp);
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    if (!status) {
        #pragma omp parallel
        {
            double* beta = (double*)calloc((size_t)(ne > 0 ? ne : 1), sizeof(double));
            double* alpha = (double*)calloc((size_t)(ne > 0 ? ne : 1), sizeof(double));
            double* th = (double*)malloc(sizeof(double) * (size_t)max_row_weight(m, row_ptr));
            if (beta && alpha && th) {
                #pragma omp for schedule(dynamic, 1)
                for (int g = 0; g < gamma; ++g) {
                    const float* y = llr + (size_t)g * n;
                    memset(beta, 0, sizeof(double) * (size_t)ne);
                    memset(alpha, 0, sizeof(double) * (size_t)ne);
                    for (int s = 0; s < npos; ++s) {
                        int lay_lo = s, lay_hi = s + W - 1;
                        if (lay_hi > nlayers - 1) lay_hi = nlayers - 1;
                        int pos_hi = s + W - 1;
                        if (pos_hi > npos - 1) pos_hi = npos - 1;
                        int in_lo = (s == 0) ? 0 : s + W - 1, in_hi = pos_hi;
                        for (int t = in_lo; t <= in_hi; ++t)
                            for (int q = pos_ptr[t]; q < pos_ptr[t + 1]; ++q) {
                                int v = pos_col[q];
                                for (int k = cv.col_ptr[v]; k < cv.col_ptr[v + 1]; ++k) {
                                    int e = cv.col_edge[k];
                                    beta[e] = clipd((double)y[v], lmax);
                                    alpha[e] = 0.0;
                                }
                            }
                        for (int it = 0; it < K; ++it) {
                            for (int t = lay_lo; t <= lay_hi; ++t)
                                for (int q = lay_ptr[t]; q < lay_ptr[t + 1]; ++q)
                                    check_update(row_ptr, lay_row[q], beta, alpha, th);
                            for (int t = s; t <= pos_hi; ++t)
                                for (int q = pos_ptr[t]; q < pos_ptr[t + 1]; ++q) {
                                    int v = pos_col[q];
                                    int k0 = cv.col_ptr[v], k1 = cv.col_ptr[v + 1];
                                    for (int k = k0; k < k1; ++k) {
                                        double acc = (double)y[v];
                                        for (int j = k0; j < k1; ++j) {
                                            if (j == k) continue;
                                            int lay = layer_of_row[cv.edge_row[cv.col_edge[j]]];
                                            if (lay >= lay_lo && lay <= lay_hi) acc += alpha[cv.col_edge[j]];
                                        }
                                        beta[cv.col_edge[k]] = clipd(acc, lmax);
                                    }
                                }
                        }
                        for (int q = pos_ptr[s]; q < pos_ptr[s + 1]; ++q) {
                            int v = pos_col[q];
                            double tot = (double)y[v];
                            for (int k = cv.col_ptr[v]; k < cv.col_ptr[v + 1]; ++k) {
                                int e = cv.col_edge[k];
                                int lay = layer_of_row[cv.edge_row[e]];
                                if (lay >= lay_lo && lay <= lay_hi) tot += alpha[e];
                            }
                            post[(size_t)g * n + v] = clipd(tot, lmax);
                            bits[(size_t)g * n + v] = (uint8_t)(tot < 0.0);
                        }
                    }
                }
            } else {
                #pragma omp atomic write
                status = -1;
            }
            free(beta); free(alpha); free(th);
        }
    }
    free(lay_ptr); free(lay_row); free(pos_ptr); free(pos_col);
    free_colview(&cv);
    return status;
}

/*
 * Pipelined decoder of Algorithm 2 (Sec. II-E, IV-B) on a terminated LDPC
 * convolutional code: I processors, each spanning m_s + 1 code frames.
 * At time slot t = 0, 1, ...:
 *   - frame t enters processor 1 (if it exists): beta = clip(mu) on its edges;
 *   - horizontal step: processor i (i = 1..I) updates check layer
 *     t - (i-1)(m_s+1) (if it exists) from the current beta of its edges;
 *   - vertical step: processor i updates frame t - (i-1)(m_s+1) - m_s (if it
 *     exists) from the current alpha of all its edges;
 *   - the frame leaving processor I is decided from its a-posteriori LLR.
 * All horizontal steps of a slot precede all vertical steps.  Slots run until
 * the last frame has left processor I.
 */
int oracle_decode_pipeline(int n, int m, const int32_t* row_ptr, const int32_t* col_idx,
                           const int32_t* layer_of_row, const int32_t* pos_of_col,
                           int nlayers, int npos, int ms, const float* llr, int gamma, int I,
                           double lmax, int nthreads, double* post, uint8_t* bits) {
    if (n < 0 || m < 0 || gamma < 0 || I < 1 || ms < 0 || npos < 0 || nlayers < 0) return -1;
    colview cv;
    if (build_colview(n, m, row_ptr, col_idx, &cv)) { free_colview(&cv); return -1; }
    int ne = row_ptr[m];
    int32_t* lay_ptr = (int32_t*)calloc((size_t)nlayers + 1, sizeof(int32_t));
    int32_t* lay_row = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int32_t* pos_ptr = (int32_t*)calloc((size_t)npos + 1, sizeof(int32_t));
    int32_t* pos_col = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int status = 0;
    if (!lay_ptr || !lay_row || !pos_ptr || !pos_col) status = -1;
    for (int r = 0; r < m && !status; ++r) {
        if (layer_of_row[r] < 0 || layer_of_row[r] >= nlayers) status = -1;
        else lay_ptr[layer_of_row[r] + 1]++;
    }
    for (int v = 0; v < n && !status; ++v) {
        if (pos_of_col[v] < 0 || pos_of_col[v] >= npos) status = -1;
        else pos_ptr[pos_of_col[v] + 1]++;
    }
    if (!status) {
        for (int t = 0; t < nlayers; ++t) lay_ptr[t + 1] += lay_ptr[t];
        for (int t = 0; t < npos; ++t) pos_ptr[t + 1] += pos_ptr[t];
        int32_t* fl = (int32_t*)calloc((size_t)nlayers + 1, sizeof(int32_t));
        int32_t* fp = (int32_t*)calloc((size_t)npos + 1, sizeof(int32_t));
        for (int r = 0; r < m; ++r) lay_row[lay_ptr[layer_of_row[r]] + fl[layer_of_row[r]]++] = r;
        for (int v = 0; v < n; ++v) pos_col[pos_ptr[pos_of_col[v]] + fp[pos_of_col[v]]++] = v;
        free(fl); free(fp);
    }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    const int last_slot = npos - 1 + ms + (I - 1) * (ms + 1);
    if (!status) {
        #pragma omp parallel
        {
            double* beta = (double*)calloc((size_t)(ne > 0 ? ne : 1), sizeof(double));
            double* alpha = (double*)calloc((size_t)(ne > 0 ? ne : 1), sizeof(double));
            double* th = (double*)malloc(sizeof(double) * (size_t)max_row_weight(m, row_ptr));
            if (beta && alpha && th) {
                #pragma omp for schedule(dynamic, 1)
                for (int g = 0; g < gamma; ++g) {
                    const float* y = llr + (size_t)g * n;
                    memset(beta, 0, sizeof(double) * (size_t)ne);
                    memset(alpha, 0, sizeof(double) * (size_t)ne);
                    for (int t = 0; t <= last_slot; ++t) {
                        if (t < npos)
                            for (int q = pos_ptr[t]; q < pos_ptr[t + 1]; ++q) {
                                int v = pos_col[q];
                                for (int k = cv.col_ptr[v]; k < cv.col_ptr[v + 1]; ++k)
                                    beta[cv.col_edge[k]] = clipd((double)y[v], lmax);
                            }
                        for (int i = 1; i <= I; ++i) {
                            int tau = t - (i - 1) * (ms + 1);
                            if (tau < 0 || tau >= nlayers) continue;
                            for (int q = lay_ptr[tau]; q < lay_ptr[tau + 1]; ++q)
                                check_update(row_ptr, lay_row[q], beta, alpha, th);
                        }
                        for (int i = 1; i <= I; ++i) {
                            int f = t - (i - 1) * (ms + 1) - ms;
                            if (f < 0 || f >= npos) continue;
                            for (int q = pos_ptr[f]; q < pos_ptr[f + 1]; ++q) {
                                int v = pos_col[q];
                                int k0 = cv.col_ptr[v], k1 = cv.col_ptr[v + 1];
                                double tot = (double)y[v];
                                for (int k = k0; k < k1; ++k) tot += alpha[cv.col_edge[k]];
                                for (int k = k0; k < k1; ++k) {
                                    double acc = (double)y[v];
                                    for (int j = k0; j < k1; ++j)
                                        if (j != k) acc += alpha[cv.col_edge[j]];
                                    beta[cv.col_edge[k]] = clipd(acc, lmax);
                                }
                                if (i == I) {
                                    post[(size_t)g * n + v] = clipd(tot, lmax);
                                    bits[(size_t)g * n + v] = (uint8_t)(tot < 0.0);
                                }
                            }
                        }
                    }
                }
            } else {
                #pragma omp atomic write
                status = -1;
            }
            free(beta); free(alpha); free(th);
        }
    }
    free(lay_ptr); free(lay_row); free(pos_ptr); free(pos_col);
    free_colview(&cv);
    return status;
}
